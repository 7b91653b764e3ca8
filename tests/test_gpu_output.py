"""GPU tests of the output rows: the energy-averaged flavor content (the
paper's second dump mode) against the oracle, and snapshot files (first dump
mode and resume) through the C ABI."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import nuosc, workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,ne,na,prec", [
    (3, 37, 13, W.FP64), (2, 100, 0, W.FP64), (3, 200, 6, W.FP64), (3, 1, 1, W.FP64), (2, 65, 5, W.FP64),
    (3, 37, 13, W.FP32_AMP), (3, 70, 9, W.FP32_AMP_FP64_MATH),
])
def test_energy_average_of_random_states_matches_the_oracle(n, ne, na, prec):
    w = W.multi_angle_3f(ne, na)
    w.update(n_flavors=n, precision=prec, lum_erg_s=[1.3e51, 0.6e51, 0.9e51, 1.1e51])
    say(f"case: energy average n={n} NE={ne} NA={na} prec={prec}")
    with nuosc.Run(w) as run:
        psi = W.random_states(n, run.nb, seed=300 + ne)
        if prec != W.FP64:
            psi = psi.astype(np.float32).astype(np.float64)
        run.set_state(psi, W.random_phases(n, run.na, seed=7), 14.0)
        avg = run.energy_average()
    ref = O.Run(w)
    ref.set_state(psi, None, 14.0)
    np.testing.assert_allclose(avg, ref.energy_average(), rtol=0, atol=1e-14)


@pytest.mark.parametrize("prec", [W.FP32_AMP, W.FP64])
def test_energy_average_at_the_bench_grid_matches_the_oracle(prec):
    """The 400 x 4000 x 2 grid the bench times the average on (3.2M beams),
    from a seeded random state."""
    w = W.multi_angle_3f_large(prec)
    say(f"case: energy average 400x4000 prec={prec}")
    with nuosc.Run(w) as run:
        psi = W.random_states(3, run.nb, seed=311)
        if prec != W.FP64:
            psi = psi.astype(np.float32).astype(np.float64)
        run.set_state(psi, None, 10.0)
        avg = run.energy_average()
    ref = O.Run(w)
    ref.set_state(psi, None, 10.0)
    np.testing.assert_allclose(avg, ref.energy_average(), rtol=0, atol=1e-14)


def test_energy_average_after_evolution_matches_the_oracle():
    w = W.multi_angle_3f(24, 6)
    say("case: energy average after 40 adaptive attempts")
    ref = O.Run(w)
    with nuosc.Run(w) as run:
        run.step(40)
        r = run.stats()["r_km"]
        ref.evolve_dp54(r)
        avg = run.energy_average()
    np.testing.assert_allclose(avg, ref.energy_average(), rtol=1e-10, atol=1e-13)


def test_energy_average_with_a_species_without_flux():
    w = dict(W.multi_angle_3f(20, 3), lum_erg_s=[1e51, 0.0, 1e51, 1e51])
    with nuosc.Run(w) as run:
        psi = W.random_states(3, run.nb, seed=9)
        run.set_state(psi, None, 12.0)
        avg = run.energy_average()
    ref = O.Run(w)
    ref.set_state(psi, None, 12.0)
    np.testing.assert_allclose(avg, ref.energy_average(), rtol=0, atol=1e-14)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_AMP])
def test_snapshot_resume_continues_the_run(tmp_path, prec):
    w = dict(W.multi_angle_3f(40, 8), precision=prec)
    path = str(tmp_path / "run.snap")
    say(f"case: snapshot resume prec={prec}")
    with nuosc.Run(w) as a:
        a.step(30)
        a.snapshot_write(path)
        s_mid = a.stats()
        a.step(25)
        p_a, s_a = a.probabilities(), a.stats()
        st_a = a.get_state()
    info = nuosc.snapshot_info(path)
    assert (info["n_flavors"], info["n_energy"], info["n_angle"], info["precision"]) == (3, 40, 8, prec)
    assert info["r_km"] == s_mid["r_km"] and info["accepted"] == s_mid["accepted"]
    with nuosc.Run(w) as b:
        b.snapshot_read(path)
        assert b.stats()["r_km"] == s_mid["r_km"] and b.stats()["accepted"] == s_mid["accepted"]
        b.step(25)
        p_b, s_b = b.probabilities(), b.stats()
        st_b = b.get_state()
    assert s_b["r_km"] == s_a["r_km"] and s_b["accepted"] == s_a["accepted"]
    np.testing.assert_array_equal(p_a, p_b)
    np.testing.assert_array_equal(st_a[0], st_b[0])
    np.testing.assert_array_equal(st_a[1], st_b[1])


def test_snapshot_of_another_grid_is_refused_and_leaves_the_run(tmp_path):
    path = str(tmp_path / "other.snap")
    with nuosc.Run(W.multi_angle_3f(30, 4)) as a:
        a.step(5)
        a.snapshot_write(path)
    w = W.multi_angle_3f(30, 5)
    with nuosc.Run(w) as b:
        b.step(3)
        before = b.get_state(), b.stats()
        with pytest.raises(nuosc.NuoscError) as e:
            b.snapshot_read(path)
        assert e.value.status == nuosc.E_INVALID
        after = b.get_state(), b.stats()
    np.testing.assert_array_equal(before[0][0], after[0][0])
    assert before[1] == after[1]


def test_fp64_snapshot_restores_into_an_fp32_run(tmp_path):
    path = str(tmp_path / "fp64.snap")
    w = W.multi_angle_3f(30, 4)
    with nuosc.Run(w) as a:
        a.step(20)
        a.snapshot_write(path)
        p64 = a.probabilities()
    with nuosc.Run(dict(w, precision=W.FP32_AMP)) as b:
        b.snapshot_read(path)
        p32 = b.probabilities()
    np.testing.assert_allclose(p32, p64, rtol=0, atol=5e-7)
