"""Pins of the bulb geometry (eq 3.3, 3.14, 3.15, 3.17) in the oracle."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W


def _ma(na, r_nu=10.0):
    w = W.multi_angle_3f(2, na)
    w["r_nu_km"] = r_nu
    return O.Run(w)


def test_cosines_at_the_neutrinosphere_equal_the_emission_cosines():
    run = _ma(37)
    c, w = run.geometry(10.0)
    u = (np.arange(37) + 0.5) / 37
    np.testing.assert_allclose(c, u, rtol=3e-16)  # sqrt(fl(u^2)): one rounding
    np.testing.assert_allclose(w, np.full(37, 1 / 37), rtol=4e-16)


def test_cosines_near_the_neutrinosphere_keep_full_precision():
    # c^2 = 1 - (R/r)^2 (1 - u^2) = u^2 + 2 d/R - ... for r = R + d: compare
    # with the leading terms of the expansion at d = 1e-9 km, u = 1e-4.
    w = W.multi_angle_3f(2, 5000)
    run = O.Run(w)
    r = 10.0 + 1e-9
    c, _ = run.geometry(r)
    u = (np.arange(5000) + 0.5) / 5000
    eps = (r - 10.0) * (r + 10.0) / r ** 2   # exact to rounding for this r
    np.testing.assert_allclose(c, np.sqrt(u ** 2 + (1 - u ** 2) * eps), rtol=1e-15)
    assert c[0] ** 2 == pytest.approx(u[0] ** 2 + 2e-10, rel=1e-6)


@pytest.mark.parametrize("r", [10.5, 15.0, 40.0, 250.0])
def test_angle_weights_integrate_the_solid_angle_of_the_neutrinosphere(r):
    # sum_j w_j approximates int d cos(theta') over [sqrt(1 - (R/r)^2), 1],
    # i.e. 1 - sqrt(1 - (R/r)^2); the midpoint rule converges as N^-2.
    exact = 1 - math.sqrt(1 - (10.0 / r) ** 2)
    errs = []
    for na in (200, 400, 800):
        c, w = _ma(na).geometry(r)
        assert np.all(c > 0) and np.all(c <= 1)
        errs.append(abs(w.sum() - exact))
    assert errs[-1] < 1e-5 * exact
    if errs[0] > 1e-13:
        assert 3.0 < errs[0] / errs[1] < 5.0


@pytest.mark.parametrize("r", [12.0, 30.0, 100.0])
def test_radial_ray_kernel_reduces_to_the_single_angle_factor(r):
    # For a radial test ray (cos theta = 1), sum_j w_j (1 - c_j) approximates
    # int (1 - x) dx over [sqrt(1 - (R/r)^2), 1] = D(r/R) of eq 3.17.
    c, w = _ma(2000).geometry(r)
    d = O.dilution(r / 10.0)
    assert (w * (1 - c)).sum() == pytest.approx(d, rel=1e-5)


def test_single_angle_dilution_factor():
    assert O.dilution(1.0) == pytest.approx(0.5, abs=1e-15)
    for x in (50.0, 200.0):
        assert O.dilution(x) == pytest.approx(1 / (8 * x ** 4), rel=2 / x ** 2)
    # monotone decreasing
    xs = np.linspace(1.0, 30.0, 200)
    ds = np.array([O.dilution(x) for x in xs])
    assert np.all(np.diff(ds) < 0)


def test_single_angle_geometry_is_the_radial_ray():
    w = W.single_angle_2f()
    run = O.Run(w)
    c, d = run.geometry(25.0)
    assert c[0] == 1.0
    assert d[0] == pytest.approx(O.dilution(2.5), rel=1e-15)
