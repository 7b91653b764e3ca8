"""Seeded synthetic workloads for the bulb-model flavor-evolution path.

This module only holds physics parameter sets and seeded random draws.  It
contains none of the method's arithmetic, so both the HIP path (through the
binding) and the CPU oracle (through its test wrapper) can take their inputs
from here without sharing any computation.

A workload is a plain ``dict`` whose keys mirror the fields of ``nuosc_params``
in ``include/nuosc.h``.  Parameter names follow the paper's configuration
keywords (Appendix A.3: ``Flvs``, ``Ebins``, ``E0``/``E1``, ``Abins``,
``dm2``, ``theta``, ``R0``/``Rn``, ``dr``, ``max_dr``, ``eps0``, ``ksi``,
``Rv``, ``Lve``..., ``eta_ve``...).

Workloads (all inputs are synthetic: the paper's workloads are parameter sets,
not datasets):

* ``single_angle_2f``: two flavors, single-angle bulb model (eq 3.16-3.17),
  100 energy bins on 1-60 MeV, fixed-step classic RK4 with 1e4 radial steps
  from 10 km to 250 km, FP64.
* ``multi_angle_3f``: three flavors, multi-angle bulb model (eq 3.13-3.15),
  200 energies x 1000 emission angles, embedded adaptive RK, rtol 1e-9, FP64.
* ``multi_angle_3f_large``: 400 energies x 4000 angles (3.2M beams), FP32
  amplitudes with FP64 moments, step error and phases.
* ``exp_stepper_3f`` / ``exp_stepper_2f``: the paper's own stepper on the
  multi-angle three-flavor and single-angle two-flavor bulb models.
* ``batched_runs``: 64 independent multi-angle runs with seeded uneven grids.
* ``serving_requests``: a seeded Poisson arrival stream of such runs, each
  evolved over a short radius window from the neutrinosphere.
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

# Integrator and precision codes (same values as include/nuosc.h).
RK4_FIXED = 0
RK_DP54 = 1
EXP_STEPPER = 2
FP64 = 0
FP32_AMP = 1
FP32_AMP_FP64_MATH = 2
FRAME_COROTATING = 0
FRAME_LAB = 1

SEED_BASE = 20190705


def base_bulb() -> Dict:
    """Shared physics of every workload (before per-workload overrides).

    Fermi-Dirac spectra with eta = 0 and mean energies 11 / 16 / 25 / 25 MeV
    (nu_e, nubar_e, nu_x, nubar_x), luminosity 1e51 erg/s per flavor, matter
    potential lambda(r) = 1e4 km^-1 (10 km / r)^3, self-coupling 1e5 km^-1
    diluted by the bulb geometry, neutrinosphere at 10 km, pure-flavor start.
    """
    return dict(
        n_flavors=2,
        n_energy=100,
        e_min_mev=1.0,
        e_max_mev=60.0,
        n_angle=0,  # 0 => single-angle model
        lum_erg_s=[1e51, 1e51, 1e51, 1e51],
        mean_e_mev=[11.0, 16.0, 25.0, 25.0],
        eta=[0.0, 0.0, 0.0, 0.0],
        dm2_ev2=-2.4e-3,
        theta=0.1,
        dm2_21_ev2=7.5e-5,
        dm2_31_ev2=-2.4e-3,
        theta12=0.59,
        theta13=0.15,
        theta23=math.pi / 4,
        delta_cp=0.0,
        lambda0_km=1.0e4,
        lambda_rref_km=10.0,
        lambda_power=3.0,
        mu0_km=1.0e5,
        r_nu_km=10.0,
        r_start_km=10.0,
        r_end_km=250.0,
        integrator=RK4_FIXED,
        n_fixed_steps=10000,
        rtol=1e-9,
        dr_init_km=1e-5,
        dr_max_km=1.0,
        safety=0.9,
        max_steps=0,
        precision=FP64,
        frame=FRAME_COROTATING,
    )


def single_angle_2f() -> Dict:
    """Two-flavor single-angle run: 200 beams, RK4 with 1e4 fixed steps."""
    return base_bulb()


def multi_angle_3f(n_energy: int = 200, n_angle: int = 1000) -> Dict:
    """Three-flavor multi-angle run with the embedded adaptive pair, FP64."""
    w = base_bulb()
    w.update(
        n_flavors=3,
        n_energy=n_energy,
        n_angle=n_angle,
        integrator=RK_DP54,
        rtol=1e-9,
        precision=FP64,
    )
    return w


def multi_angle_3f_large(precision: int = FP32_AMP) -> Dict:
    """400 x 4000 x {nu, nubar} = 3.2M beams, three flavors, adaptive pair."""
    w = multi_angle_3f(400, 4000)
    w["precision"] = precision
    return w


def extended_bulb_3f(n_energy: int = 100, n_angle: int = 100, n_azimuth: int = 32,
                     precision: int = FP32_AMP) -> Dict:
    """Three-flavor extended bulb model (eq 3.18): n_angle emission angles x
    n_azimuth azimuth bins per angle, adaptive pair; the physics of the bulb
    workloads.  Starts from azimuth_perturbed_states (the seed that breaks the
    azimuthal symmetry)."""
    w = multi_angle_3f(n_energy, n_angle)
    w.update(n_azimuth=n_azimuth, precision=precision)
    return w


def exp_stepper_3f(n_energy: int = 200, n_angle: int = 1000) -> Dict:
    """The paper's own stepper (exponential steps of eq 3.10-3.12 in the
    half/full-step loop with averaging and max-error control) on the
    three-flavor multi-angle bulb model, lab frame, FP64, rtol 1e-9."""
    w = multi_angle_3f(n_energy, n_angle)
    w.update(integrator=EXP_STEPPER, frame=FRAME_LAB, precision=FP64)
    return w


def exp_stepper_2f() -> Dict:
    """The paper's own stepper on the two-flavor single-angle model (eq 3.11
    is then the closed-form 2x2 exponential), lab frame, FP64."""
    w = base_bulb()
    w.update(integrator=EXP_STEPPER, frame=FRAME_LAB, precision=FP64)
    return w


# Radius windows (km) of the FP32-versus-FP64 accuracy measurement, both
# started from pure flavor states with the physics of multi_angle_3f: from
# 50 km about 2000 accepted steps in which survival probabilities move by a few
# 1e-2 (matter-suppressed oscillations); from 110 km about 4000 steps through
# the region where the matter potential falls to the vacuum frequencies of the
# lowest energy bins, with complete flavor conversion of some beams.
ACCURACY_WINDOWS = ((50.0, 56.7), (110.0, 178.0))


def window(w: Dict, r0: float, r1: float) -> Dict:
    """The workload w started at r0 (pure flavor states) with end radius r1."""
    w = dict(w)
    w.update(r_start_km=r0, r_end_km=r1)
    return w


def error_subsample(n_beams: int, count: int = 4096) -> np.ndarray:
    """Sorted seeded subsample of beam indices used to report FP32 error."""
    rng = np.random.default_rng(SEED_BASE + 2)
    count = min(count, n_beams)
    return np.sort(rng.choice(n_beams, count, replace=False))


def _draw_run(rng: np.random.Generator, large: bool = False) -> Dict:
    w = multi_angle_3f()
    if large:
        w["n_energy"], w["n_angle"] = 400, 4000
    else:
        w["n_energy"] = int(rng.integers(50, 401))
        w["n_angle"] = int(round(math.exp(rng.uniform(math.log(100), math.log(4000)))))
    w["lum_erg_s"] = [float(x) for x in rng.uniform(0.5e51, 2e51, 4)]
    normal = bool(rng.random() < 0.5)
    w["dm2_31_ev2"] = 2.4e-3 if normal else -2.4e-3
    w["theta13"] = float(rng.uniform(0.14, 0.16))
    w["precision"] = FP32_AMP
    return w


def batched_runs(count: int = 64) -> List[Dict]:
    """64 independent three-flavor multi-angle runs with uneven grids.

    Energy bins uniform in [50, 400], angle bins log-uniform in [100, 4000],
    four luminosities uniform in 0.5-2e51 erg/s, normal or inverted hierarchy
    with probability 1/2, theta13 uniform in [0.14, 0.16].
    """
    rng = np.random.default_rng(SEED_BASE + 3)
    return [_draw_run(rng) for _ in range(count)]


def serving_requests(rate_per_s: float = 20.0, duration_s: float = 120.0,
                     large_fraction: float = 0.1, window_km: float = 3e-5,
                     precision: int = FP32_AMP) -> List[Dict]:
    """Poisson arrivals; each request is a batched-runs draw, 10% large.

    Each request evolves from the neutrinosphere over a radius window of
    `window_km` (its r_end).  Near R the adaptive step of a multi-angle run is
    about 1e-5 km / N_A at rtol 1e-9 (nearly tangential trajectories have
    1 / cos(theta) up to 2 N_A), so a request costs about 2 N_E N_A^2 x
    window / 1e-5 km beam-steps: with the draws below, measured ~6e13 x
    window (km) on average.  At 20 requests/s and a window of 3e-5 km the
    offered load is ~3e10 beam-steps/s, above what one GPU serves (~1.2e10),
    so the queue grows over the arrival period.  The draws of every request (and so the sequence) do
    not depend on the window or the precision."""
    rng = np.random.default_rng(SEED_BASE + 4)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        large = bool(rng.random() < large_fraction)
        w = _draw_run(rng, large=large)
        w["arrival_s"] = t
        w["r_end_km"] = w["r_start_km"] + window_km
        w["precision"] = precision
        out.append(w)
    return out


def random_states(n_flavors: int, n_beams: int, seed: int) -> np.ndarray:
    """Seeded random unit-norm amplitudes, shape (n_flavors, 2, n_beams).

    Layout: component-major, then (re, im), then beam index -- the host state
    layout of ``nuosc_get_state`` / ``nuosc_set_state``.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_flavors, n_beams)) + 1j * rng.standard_normal((n_flavors, n_beams))
    z /= np.sqrt((np.abs(z) ** 2).sum(axis=0, keepdims=True))
    out = np.empty((n_flavors, 2, n_beams))
    out[:, 0, :] = z.real
    out[:, 1, :] = z.imag
    return out


def azimuth_perturbed_states(n_flavors: int, n_beams: int, n_traj: int, seed: int,
                             amplitude: float = 1e-6) -> np.ndarray:
    """Birth-flavor states (component 0) with seeded complex perturbations of
    size `amplitude` in the other components, different for every beam: the
    small symmetry-breaking seed the extended bulb model's azimuth bins need.
    Unit norm; host state layout, shape (n_flavors, 2, n_beams)."""
    rng = np.random.default_rng(seed)
    z = np.zeros((n_flavors, n_beams), complex)
    z[0] = 1.0
    z[1:] = amplitude * (rng.standard_normal((n_flavors - 1, n_beams))
                         + 1j * rng.standard_normal((n_flavors - 1, n_beams)))
    z /= np.sqrt((np.abs(z) ** 2).sum(axis=0, keepdims=True))
    out = np.empty((n_flavors, 2, n_beams))
    out[:, 0, :] = z.real
    out[:, 1, :] = z.imag
    return out


def random_phases(n_flavors: int, n_traj: int, seed: int, scale: float = 10.0) -> np.ndarray:
    """Seeded co-rotating phases, shape (n_traj, n_flavors), each row sums to 0."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(-scale, scale, (n_traj, n_flavors))
    ph -= ph.mean(axis=1, keepdims=True)
    return ph


def n_beams(w: Dict) -> int:
    return 2 * int(w["n_energy"]) * max(1, int(w["n_angle"]))
