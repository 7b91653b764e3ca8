"""Pins of the oracle's energy-averaged output (the paper's second dump mode,
Section 4.2.4; reading O: bins weighted by the number flux of the beam's
birth flavor).  The expected values come from closed forms: the two-flavor
vacuum probability and Fermi-Dirac spectra at eta = 0, whose temperature
T = <E> F2(0) / F3(0) uses F2(0) = 3 zeta(3) / 2 and F3(0) = 7 pi^4 / 120."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W

ZETA3 = 1.2020569031595942


def _fd_weights(e, mean_e):
    """Number flux per bin up to a constant (eq 4.1 at eta = 0)."""
    t = mean_e * (1.5 * ZETA3) / (7 * math.pi ** 4 / 120)
    return e ** 2 / (np.exp(e / t) + 1.0)


def test_pure_flavor_state_averages_to_its_birth_flavor():
    run = O.Run(W.multi_angle_3f(12, 5))
    avg = run.energy_average()
    assert avg.shape == (2, 5, 3)
    np.testing.assert_array_equal(avg[:, :, 0], 1.0)
    np.testing.assert_array_equal(avg[:, :, 1:], 0.0)


@pytest.mark.parametrize("species", [0, 1])
def test_two_flavor_vacuum_average_is_the_flux_weighted_closed_form(species):
    w = dict(W.single_angle_2f(), mu0_km=0.0, lambda_power=0.0, lambda0_km=0.0,
             r_start_km=10.0, r_end_km=12.0, n_fixed_steps=20000)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    ne = w["n_energy"]
    de = (w["e_max_mev"] - w["e_min_mev"]) / ne
    e = w["e_min_mev"] + (np.arange(ne) + 0.5) * de
    delta = O.vacuum_coefficient() * w["dm2_ev2"] / e
    p_ee = 1 - math.sin(2 * w["theta"]) ** 2 * np.sin(delta * 2.0 / 2) ** 2
    f = _fd_weights(e, w["mean_e_mev"][species])
    expect = np.sum(f * p_ee) / np.sum(f)
    avg = run.energy_average()
    assert avg.shape == (2, 1, 2)
    assert abs(avg[species, 0, 0] - expect) <= 1e-10
    assert abs(avg[species, 0, 1] - (1 - expect)) <= 1e-10


def test_bins_with_equal_content_give_that_content_for_any_spectrum():
    w = dict(W.multi_angle_3f(9, 4), lum_erg_s=[0.7e51, 1.9e51, 1.1e51, 0.4e51], mean_e_mev=[9.0, 14.0, 22.0, 22.0])
    run = O.Run(w)
    rng = np.random.default_rng(11)
    amp = rng.standard_normal((3, 2)) + 0.0
    amp /= np.linalg.norm(amp)
    psi = np.zeros((3, 2, run.nb))
    psi[:, :, :] = amp[:, :, None]          # every beam in the same state
    run.set_state(psi, None, 12.0)
    avg = run.energy_average()
    np.testing.assert_allclose(avg, np.broadcast_to((amp ** 2).sum(axis=1), avg.shape), rtol=0, atol=1e-15)


def test_a_species_without_flux_gets_the_plain_mean():
    w = dict(W.multi_angle_3f(7, 3), lum_erg_s=[1e51, 0.0, 1e51, 1e51])
    run = O.Run(w)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((3, 2, run.nb))
    psi /= np.sqrt((psi ** 2).sum(axis=(0, 1)))
    run.set_state(psi, None, 12.0)
    p = (psi ** 2).sum(axis=1).reshape(3, 2, 3, 7)      # [a][s][j][k]
    avg = run.energy_average()
    np.testing.assert_allclose(avg[1], p[:, 1].mean(axis=2).T, rtol=0, atol=1e-14)
    assert not np.allclose(avg[0], p[:, 0].mean(axis=2).T, atol=1e-6)   # flux-weighted
