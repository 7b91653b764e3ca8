"""Pins of the oracle's spectra and beam weights (eq 4.1-4.2, Section 4.5).

Each check compares the oracle with something it does not compute itself:
closed forms of the Fermi integrals, the temperatures the paper prints, and
the normalisation and mean energy that eq 4.1 implies.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fermi_integrals_closed_forms_at_zero_degeneracy():
    # F_k(0) = (1 - 2^-k) k! zeta(k+1):  F_2(0) = 3 zeta(3) / 2,  F_3(0) = 7 pi^4 / 120.
    assert O.fermi_integral(2, 0.0) == pytest.approx(1.5 * special.zeta(3), rel=1e-14)
    assert O.fermi_integral(3, 0.0) == pytest.approx(7 * math.pi ** 4 / 120, rel=1e-14)


@pytest.mark.parametrize("eta", [-1.0, -3.0])
@pytest.mark.parametrize("k", [2, 3])
def test_fermi_integrals_series_for_negative_degeneracy(k, eta):
    # For eta < 0: F_k(eta) = k! sum_{n>=1} (-1)^(n+1) exp(n eta) / n^(k+1).
    series = math.factorial(k) * sum((-1) ** (m + 1) * math.exp(m * eta) / m ** (k + 1) for m in range(1, 200))
    assert O.fermi_integral(k, eta) == pytest.approx(series, rel=1e-14)


def test_temperatures_match_values_printed_in_the_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_temperatures.json")))
    half_digit = 0.5 * 10 ** -g["printed_digits_after_point"]
    for mean_e, t_printed in zip(g["mean_e_mev"], g["temperature_mev"]):
        t = O.temperature(mean_e, g["eta"])
        assert abs(t - t_printed) <= half_digit + 1e-12, (mean_e, t, t_printed)


@pytest.mark.parametrize("mean_e,eta", [(11.0, 0.0), (16.0, 0.0), (25.0, 3.0)])
def test_spectrum_is_normalised_with_the_requested_mean_energy(mean_e, eta):
    t = O.temperature(mean_e, eta)
    f = lambda e: O.spectrum(e, t, eta)  # noqa: E731
    norm, _ = integrate.quad(f, 0.0, 60 * t, limit=400, epsabs=1e-14, epsrel=1e-13)
    mean, _ = integrate.quad(lambda e: e * f(e), 0.0, 60 * t, limit=400, epsabs=1e-12, epsrel=1e-13)
    assert norm == pytest.approx(1.0, rel=1e-10)
    assert mean == pytest.approx(mean_e, rel=1e-10)


def test_beam_weights_sum_to_net_number_flux():
    # On a fine energy grid covering (0, inf) the weights sum to the net number
    # luminosities (n_e - n_x) and (n_ebar - n_xbar) over the reference
    # 1e51 erg/s / 11 MeV (reading C).
    w = W.single_angle_2f()
    w.update(n_energy=6000, e_min_mev=0.0, e_max_mev=600.0, lum_erg_s=[1e51, 2e51, 0.5e51, 1.5e51])
    run = O.Run(w)
    _, g, gb, _ = run.tables()
    lum = np.array(w["lum_erg_s"]) / 1e51
    n = lum * 11.0 / np.array(w["mean_e_mev"])
    assert g.sum() == pytest.approx(n[0] - n[2], rel=1e-7)
    assert gb.sum() == pytest.approx(n[1] - n[3], rel=1e-7)


def test_energy_bins_are_midpoints():
    w = W.single_angle_2f()
    run = O.Run(w)
    e, _, _, _ = run.tables()
    de = (w["e_max_mev"] - w["e_min_mev"]) / w["n_energy"]
    np.testing.assert_allclose(e, w["e_min_mev"] + (np.arange(w["n_energy"]) + 0.5) * de, rtol=0, atol=1e-12)
