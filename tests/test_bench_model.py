"""Host logic of bench.py's roofline models (no GPU): the method's byte floor
per beam-step, 7 S for the first-same-as-last Dormand-Prince pair with
S = 2n amplitude reals; the per-launch algorithmic bytes (the state update
reads psi_n and writes psi_{n+1}, the power-moment launch reads the new state,
the per-trajectory launches touch no beam data); and the bound chosen against
the unpacked vector peak."""

import bench

NB = 3200000


def _form(prec, value=1e10, launch_us=None):
    amp = 8 if prec == 0 else 4
    launch_us = launch_us or [10.0] * 7 + [60.0, 45.0]
    return dict(n=3, amp_bytes=amp, value=value, precision=prec, beams=NB, launch_us=launch_us,
                names=bench.kernel_names(prec))


def test_alg_bytes_per_beam_step():
    assert bench.step_roofline(_form(1))["alg_bytes_per_beam_step"] == 7 * 24
    assert bench.step_roofline(_form(0))["alg_bytes_per_beam_step"] == 7 * 48


def test_fraction_of_the_floor():
    r = bench.step_roofline(_form(1, value=1e10))
    assert abs(r["frac_alg"] - 1e10 * 168 / 8e12) < 1e-4
    assert abs(r["alg_ceiling"] - 8e12 / 168) < 1.0


def test_launch_bytes_follow_the_floor():
    f = _form(1)
    state = 6 * 4 * NB
    assert [bench.beam_model(f, i)[0] for i in range(9)] == [0] * 7 + [2 * state, state]
    # the FP32 state update moves 153.6 MB: a read of psi_n and a write of psi_{n+1}
    assert bench.beam_model(f, 7)[0] == 153_600_000
    assert bench.beam_model(_form(0), 7)[0] == 307_200_000


def test_dominant_kernel_and_its_hbm_fraction():
    f = _form(1, launch_us=[10.0] * 7 + [66.5, 48.0])
    r = bench.roofline(f)
    assert r["kernel"] == "k_final<float,float,3,DP54,2>"
    assert abs(r["hbm"]["frac"] - 153.6e6 / 66.5e-6 / 8e12) < 1e-4
    assert r["mean_launch_us"] == 66.5
    # the bound is the view with the larger fraction of its own peak (unpacked VALU peak)
    assert r["alu"]["peak"] == 78.6
    assert r["bound"] == ("alu" if r["alu"]["frac"] > r["hbm"]["frac"] else "hbm")
    assert r["frac"] == max(r["alu"]["frac"], r["hbm"]["frac"])


def test_update_flops_count_both_polynomials():
    # per beam: the update polynomial (degree 6) and the FP64 error polynomial
    # (degree 7) of a 3 x 3 complex matrix, each 2 n^2 (D + 1) + 4 n^2 FMAs
    f64 = bench.beam_model(_form(0), 7)[1] / NB
    assert f64 >= 2 * (18 * 7 + 36) + 2 * (18 * 8 + 36)
    # FP32 amplitudes add the renormalisation
    assert bench.beam_model(_form(1), 7)[1] / NB > f64


def test_kernel_names_of_the_three_forms():
    assert bench.kernel_names(0)[7] == "k_final<double,double,3,DP54,2>"
    assert bench.kernel_names(2)[7] == "k_final<float,double,3,DP54,2>"
    assert bench.kernel_names(1)[0] == "k_traj<3,DP54,2,1,double>"
    assert bench.kernel_names(1)[6] == "k_traj<3,DP54,2,7,float>"
    assert bench.kernel_names(2)[8] == "k_power<float,3,DP54,2,false>"


def test_power_moment_flops_pair_the_species():
    # per energy bin: both densities (24 flops each for three flavors), their
    # even and odd combinations (5 n^2), the 13 powers and 13 n^2 FMAs; half
    # of that per beam
    f = _form(1)
    assert bench.beam_model(f, 8)[1] / NB == (2 * 24 + 5 * 9 + 13 + 2 * 13 * 9) / 2 == 170
    assert bench.beam_model(f, 8)[0] == 6 * 4 * NB


def test_more_than_one_gpu_is_refused_with_a_message():
    # the timed path runs on one GPU; asking for more exits before any device work
    import subprocess, sys, os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")
