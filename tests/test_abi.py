"""CPU checks of the C ABI: the library loads, exports every declared symbol,
lays out nuosc_params as the header does, and rejects invalid parameters
before touching a device.  No kernel is launched here."""

import ctypes as C
import os
import re

import pytest

from paper_1907_05560_amd import nuosc, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nuosc.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nuosc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = nuosc.lib()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(nuosc.EXPORTS)


def test_params_layout_matches_the_header_defaults():
    p = nuosc.Params()
    nuosc.lib().nuosc_default_params(C.byref(p))
    assert (p.n_flavors, p.n_energy, p.n_angle) == (2, 100, 0)
    assert (p.e_min_mev, p.e_max_mev) == (1.0, 60.0)
    assert list(p.mean_e_mev) == [11.0, 16.0, 25.0, 25.0]
    assert p.dm2_ev2 == -2.4e-3 and p.theta == 0.1
    assert p.lambda0_km == 1e4 and p.lambda_power == 3.0 and p.mu0_km == 1e5
    assert (p.r_start_km, p.r_end_km) == (10.0, 250.0)
    assert p.integrator == 0 and p.n_fixed_steps == 10000
    assert p.safety == 0.9 and p.max_steps == 0 and p.max_wall_s == 0.0
    assert p.precision == 0 and p.frame == 0


def test_footprint_scales_with_the_grid_and_precision():
    w64 = W.multi_angle_3f_large(W.FP64)
    w32 = W.multi_angle_3f_large(W.FP32_AMP)
    f64, f32 = nuosc.footprint_bytes(w64), nuosc.footprint_bytes(w32)
    nb = W.n_beams(w64)
    assert f64 > 2 * 6 * nb * 8  # two FP64 state buffers of 3 complex amplitudes
    assert f32 > 2 * 6 * nb * 4
    assert f32 < f64
    assert nuosc.footprint_bytes(W.single_angle_2f()) < 1 << 20


@pytest.mark.parametrize("bad", [
    dict(n_flavors=4), dict(n_energy=0), dict(n_angle=-1), dict(e_max_mev=0.5),
    dict(r_start_km=5.0), dict(r_end_km=10.0), dict(integrator=7), dict(n_fixed_steps=0),
    dict(integrator=1, rtol=0.0), dict(integrator=1, safety=1.5), dict(precision=3), dict(frame=2),
    dict(mean_e_mev=[11.0, 0.0, 25.0, 25.0]),
    dict(n_energy=1 << 27, n_angle=4),               # one amplitude component above 4 GiB
    dict(n_energy=1 << 27, n_angle=4, precision=1),
])
def test_invalid_parameters_are_rejected_without_a_device(bad):
    w = W.single_angle_2f()
    w.update(bad)
    assert nuosc.footprint_bytes(w) == 0
    with pytest.raises(nuosc.NuoscError) as e:
        nuosc.Run(w)
    assert e.value.status == nuosc.E_INVALID


def test_static_runs_beyond_the_static_scratch_are_rejected_without_a_device():
    big = W.multi_angle_3f_large(W.FP32_AMP)
    need = nuosc.footprint_bytes(big)
    assert need > nuosc.STATIC_SCRATCH_BYTES
    with pytest.raises(nuosc.NuoscError) as e:
        nuosc.Run(big, static=True)
    assert e.value.status == nuosc.E_INVALID
    assert str(need) in str(e.value) and str(nuosc.STATIC_SCRATCH_BYTES) in str(e.value)
    with pytest.raises(nuosc.NuoscError) as e:
        nuosc.Run(dict(W.single_angle_2f(), n_flavors=4), static=True)
    assert e.value.status == nuosc.E_INVALID


@pytest.mark.parametrize("args", [
    (0, 3, W.FP32_AMP, W.RK_DP54, 1 << 20),      # no slots
    (2000, 3, W.FP32_AMP, W.RK_DP54, 1 << 30),   # too many slots
    (4, 4, W.FP32_AMP, W.RK_DP54, 1 << 20),      # flavors
    (4, 3, 9, W.RK_DP54, 1 << 20),               # precision
    (4, 3, W.FP64, 5, 1 << 20),                  # integrator
    (64, 3, W.FP64, W.RK_DP54, 1024),            # budget below the run-constant table
])
def test_invalid_batches_are_rejected_without_a_device(args):
    with pytest.raises(nuosc.NuoscError) as e:
        nuosc.Batch(*args)
    assert e.value.status == nuosc.E_INVALID


def test_footprint_of_a_serving_mix_is_what_admission_checks():
    ws = W.serving_requests(duration_s=2.0)
    assert len(ws) > 10
    sizes = [nuosc.footprint_bytes(w) for w in ws]
    assert all(s > 2 * 6 * W.n_beams(w) * 4 for s, w in zip(sizes, ws))
