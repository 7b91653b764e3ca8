"""Closed-form pins of the oracle's Hamiltonian and integrators.

Vacuum oscillations (eq 3.5-3.6; three flavors with the PDG matrix), the
constant-density MSW solution (eq 3.7 with a constant potential), exact
propagation of a constant three-flavor Hamiltonian, and the reduction of
three flavors to two.  The expected values come from textbook formulas or a
dense eigendecomposition, never from the oracle itself.
"""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W


def _linear(w, **kw):
    """No self-interaction; matter potential constant (lambda_power 0) or off."""
    w = dict(w)
    w.update(mu0_km=0.0, lambda_power=0.0, lambda0_km=0.0)
    w.update(kw)
    return w


def _pmns(t12, t13, t23, d):
    c12, s12, c13, s13, c23, s23 = (math.cos(t12), math.sin(t12), math.cos(t13),
                                    math.sin(t13), math.cos(t23), math.sin(t23))
    r23 = np.array([[1, 0, 0], [0, c23, s23], [0, -s23, c23]], complex)
    u13 = np.array([[c13, 0, s13 * np.exp(-1j * d)], [0, 1, 0], [-s13 * np.exp(1j * d), 0, c13]])
    r12 = np.array([[c12, s12, 0], [-s12, c12, 0], [0, 0, 1]], complex)
    return r23 @ u13 @ r12


def test_vacuum_coefficient_matches_the_textbook_oscillation_phase():
    # Delta L / 2 = 1.26693 dm2[eV^2] L[km] / E[GeV]  =>  kappa / 2 = 1.26693e3 per MeV
    # (five printed digits: within half a unit of the last one).
    assert abs(O.vacuum_coefficient() / 2e3 - 1.26693) <= 0.5e-5


@pytest.mark.parametrize("species", [0, 1])
def test_two_flavor_single_angle_vacuum(species):
    w = _linear(W.single_angle_2f(), r_start_km=10.0, r_end_km=12.0, n_fixed_steps=20000)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    p = run.probabilities().reshape(2, -1)[species]
    e, _, _, _ = run.tables()
    delta = O.vacuum_coefficient() * w["dm2_ev2"] / e
    expect = 1 - math.sin(2 * w["theta"]) ** 2 * np.sin(delta * 2.0 / 2) ** 2
    np.testing.assert_allclose(p, expect, rtol=0, atol=1e-11)


def test_two_flavor_multi_angle_vacuum_uses_the_path_length():
    w = _linear(W.multi_angle_3f(16, 5), n_flavors=2, integrator=W.RK4_FIXED,
                r_start_km=11.0, r_end_km=13.0, n_fixed_steps=20000)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    p = run.probabilities().reshape(2, 5, 16)
    e, _, _, _ = run.tables()
    u = (np.arange(5) + 0.5) / 5
    R = w["r_nu_km"]
    L = np.sqrt(13.0 ** 2 - R ** 2 * (1 - u ** 2)) - np.sqrt(11.0 ** 2 - R ** 2 * (1 - u ** 2))
    delta = O.vacuum_coefficient() * w["dm2_ev2"] / e
    expect = 1 - math.sin(2 * w["theta"]) ** 2 * np.sin(np.outer(L, delta) / 2) ** 2
    np.testing.assert_allclose(p[0], expect, rtol=0, atol=1e-10)
    np.testing.assert_allclose(p[1], expect, rtol=0, atol=1e-10)


@pytest.mark.parametrize("lam", [1.5, -0.7])
def test_two_flavor_constant_density_msw(lam):
    w = _linear(W.single_angle_2f(), lambda0_km=lam, r_start_km=10.0, r_end_km=12.0,
                n_fixed_steps=20000, dm2_ev2=2.4e-3, theta=0.3)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    p = run.probabilities().reshape(2, -1)
    e, _, _, _ = run.tables()
    d = O.vacuum_coefficient() * w["dm2_ev2"] / e
    c2, s2 = math.cos(2 * w["theta"]), math.sin(2 * w["theta"])
    for s, a in ((0, lam), (1, -lam)):  # antineutrinos see -lambda (eq 3.4)
        dm = np.sqrt((d * c2 - a) ** 2 + (d * s2) ** 2)
        expect = 1 - (d * s2 / dm) ** 2 * np.sin(dm * 2.0 / 2) ** 2
        np.testing.assert_allclose(p[s], expect, rtol=0, atol=1e-10)


@pytest.mark.parametrize("delta_cp", [0.0, 1.1])
def test_three_flavor_vacuum_against_the_mass_basis_sum(delta_cp):
    w = _linear(W.multi_angle_3f(12, 0), integrator=W.RK4_FIXED, r_start_km=10.0,
                r_end_km=11.5, n_fixed_steps=20000, delta_cp=delta_cp, dm2_31_ev2=2.4e-3)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    psi = run.psi_complex().reshape(3, 2, -1)
    e, _, _, _ = run.tables()
    U = _pmns(w["theta12"], w["theta13"], w["theta23"], delta_cp)
    m = O.vacuum_coefficient() * np.array([0.0, w["dm2_21_ev2"], w["dm2_31_ev2"]])
    L = 1.5
    for s, Us in ((0, U), (1, U.conj())):  # antineutrinos: U -> U*
        ph = np.exp(-1j * np.outer(L / e, m))  # [k, i]
        amp = np.einsum("bi,ki,i->bk", Us, ph, Us[0].conj())  # <beta| ... |e>
        np.testing.assert_allclose(np.abs(psi[:, s, :]) ** 2, np.abs(amp) ** 2, rtol=0, atol=1e-10)


@pytest.mark.parametrize("lam", [3.0, -2.0])
def test_three_flavor_constant_matter_against_eigendecomposition(lam):
    w = _linear(W.multi_angle_3f(8, 0), integrator=W.RK4_FIXED, lambda0_km=lam,
                r_start_km=10.0, r_end_km=11.0, n_fixed_steps=20000, delta_cp=0.4)
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    psi = run.psi_complex().reshape(3, 2, -1)
    e, _, _, _ = run.tables()
    U = _pmns(w["theta12"], w["theta13"], w["theta23"], w["delta_cp"])
    m = O.vacuum_coefficient() * np.array([0.0, w["dm2_21_ev2"], w["dm2_31_ev2"]])
    for k, ek in enumerate(e):
        hv = U @ np.diag(m / ek) @ U.conj().T
        for s, H in ((0, hv + np.diag([lam, 0, 0])), (1, hv.conj() - np.diag([lam, 0, 0]))):
            ev, V = np.linalg.eigh(H)
            out = V @ (np.exp(-1j * ev * 1.0) * V.conj().T[:, 0])
            np.testing.assert_allclose(np.abs(psi[:, s, k]) ** 2, np.abs(out) ** 2, rtol=0, atol=1e-10)


def test_three_flavors_reduce_to_two_in_the_e_tau_sector():
    # theta12 = theta23 = 0 and dm2_21 = 0 decouple nu_mu; the e-tau block is
    # the two-flavor problem with (dm2_31, theta13), self-interaction included.
    base = W.single_angle_2f()
    base.update(r_start_km=50.0, r_end_km=150.0, integrator=W.RK_DP54, rtol=1e-11, dr_init_km=1e-3)
    w2 = dict(base, dm2_ev2=-2.4e-3, theta=0.15)
    w3 = dict(base, n_flavors=3, dm2_21_ev2=0.0, dm2_31_ev2=-2.4e-3, theta12=0.0, theta13=0.15,
              theta23=0.0, delta_cp=0.0)
    r2, r3 = O.Run(w2), O.Run(w3)
    assert r2.run_to_end() == O.DONE
    assert r3.run_to_end() == O.DONE
    p2, p3 = r2.probabilities(), r3.probabilities()
    psi3 = r3.psi_complex()
    assert np.abs(psi3[1]).max() == 0.0
    assert p2.min() < 0.5  # the window contains flavor conversion
    np.testing.assert_allclose(p3, p2, rtol=0, atol=1e-8)
