"""Pins of the oracle's exponential stepper (the paper's own scheme: exponential
steps of eq 3.10-3.12 inside the half/full-step loop with averaging and a
max-error control, Sections 4.2.3 and 5).

What fixes each part independently of the oracle's own code:
* the exponential: eq 3.11's printed closed form for two flavors, scipy's
  expm for three;
* exactness for an r-independent Hamiltonian (every exponential step is then
  the exact propagator): the textbook constant-density MSW formula, and a
  dense eigendecomposition for three flavors;
* the order of the scheme: convergence at second order on nonlinear cases
  against an independent integrator (the Dormand-Prince oracle at rtol 1e-13
  in the same lab frame);
* the compared pair: its difference shrinks as h^3 (both estimates second
  order), and the controller's h^(1/3) law then settles the error at
  safety^3.
"""

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def _herm(rng, n, scale):
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    h = (a + a.conj().T) / 2
    return h * (scale / np.linalg.norm(h, 2))


@pytest.mark.parametrize("scale", [1e-3, 0.3, 1.0, 20.0, 500.0])
def test_expm_matches_eq_3_11(scale):
    """Eq 3.11: for a traceless 2x2 Hamiltonian [[h11, h12], [h12*, -h11]],
    exp(-i H dl) = (1/lam) [[lam cos - i h11 sin, -i h12 sin],
                            [-i h12* sin, lam cos + i h11 sin]] (lam dl),
    lam = sqrt(h11^2 + |h12|^2) (eq 3.12)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        h = _herm(rng, 2, scale)
        h -= np.trace(h) / 2 * np.eye(2)
        dl = rng.uniform(0.1, 2.0)
        h11, h12 = h[0, 0].real, h[0, 1]
        lam = np.sqrt(h11**2 + abs(h12) ** 2)
        c, s = np.cos(lam * dl), np.sin(lam * dl)
        ref = np.array([[lam * c - 1j * h11 * s, -1j * h12 * s],
                        [-1j * np.conj(h12) * s, lam * c + 1j * h11 * s]]) / lam
        got = O.expm_herm(h, dl)
        assert np.abs(got - ref).max() < 1e-14 * max(1.0, scale * dl)


@pytest.mark.parametrize("scale", [1e-4, 0.5, 3.0, 100.0, 2000.0])
def test_expm_matches_library_3x3(scale):
    rng = np.random.default_rng(12)
    for _ in range(20):
        h = _herm(rng, 3, scale)  # not traceless: the definition holds for any Hermitian K
        t = rng.uniform(0.1, 1.5)
        ref = sl.expm(-1j * t * h)
        got = O.expm_herm(h, t)
        assert np.abs(got - ref).max() < 3e-15 * max(1.0, scale * t)
        assert np.abs(got @ got.conj().T - np.eye(3)).max() < 3e-15 * max(1.0, scale * t)


def test_expm_degenerate_spectra():
    for d in ([1.0, 1.0, -2.0], [0.7, -0.7, 0.0], [0.0, 0.0, 0.0]):
        h = np.diag(d).astype(complex)
        assert np.abs(O.expm_herm(h, 1.3) - np.diag(np.exp(-1.3j * np.array(d)))).max() < 1e-15


def _constant_case(n, r0=10.0, r1=60.0, h=0.7):
    """Single-angle run with mu0 = 0 and a constant matter potential: every
    exponential step is exact, whatever its size and whatever the controller
    does (the two estimates coincide, err = 0)."""
    w = W.exp_stepper_2f() if n == 2 else W.exp_stepper_3f(20, 0)
    w.update(n_energy=20, n_angle=0, mu0_km=0.0, lambda_power=0.0, lambda0_km=3.0,
             r_start_km=r0, r_end_km=r1, rtol=1e-9, dr_init_km=h, dr_max_km=h)
    R = O.Run(w)
    assert R.run_to_end() == O.DONE
    st = R.stats()
    assert st["r_km"] == r1 and st["rejected"] == 0 and R.last_error() < 1e-3
    return w, R


def test_constant_density_msw_two_flavors():
    """Textbook constant-density MSW: Delta_m = sqrt((Delta cos 2theta - lam)^2 +
    (Delta sin 2theta)^2), P_ee = 1 - sin^2 2theta_m sin^2(Delta_m L / 2) with
    Delta = kappa dm2 / E (its sign carries the hierarchy); antineutrinos lam -> -lam."""
    w, R = _constant_case(2)
    p = R.probabilities()
    e, _, _, _ = R.tables()
    ne, L = w["n_energy"], w["r_end_km"] - w["r_start_km"]
    delta = O.vacuum_coefficient() * w["dm2_ev2"] / e
    for s, sign in ((0, 1.0), (1, -1.0)):
        dc = delta * np.cos(2 * w["theta"]) - sign * w["lambda0_km"]
        ds = delta * np.sin(2 * w["theta"])
        dm = np.hypot(dc, ds)
        pee = 1 - (ds / dm) ** 2 * np.sin(dm * L / 2) ** 2
        np.testing.assert_allclose(p[s * ne:(s + 1) * ne], pee, rtol=0, atol=1e-12)


def test_constant_matter_three_flavors():
    """Three flavors in constant matter: psi(L) = V exp(-i Lambda L) V^dagger psi(0)
    from a dense Hermitian eigendecomposition of H = H_vac(E) + H_m (numpy eigh)."""
    w, R = _constant_case(3)
    p = R.probabilities()
    _, _, _, hv = R.tables()
    ne, L = w["n_energy"], w["r_end_km"] - w["r_start_km"]
    hm = np.diag([2.0 / 3.0, -1.0 / 3.0, -1.0 / 3.0]) * w["lambda0_km"]
    e1 = np.array([1.0, 0.0, 0.0])
    for s in (0, 1):
        for k in range(ne):
            h = hv[k] + hm if s == 0 else np.conj(hv[k]) - hm
            lam, v = np.linalg.eigh(h)
            psi = v @ (np.exp(-1j * lam * L) * (v.conj().T @ e1))
            assert abs(p[s * ne + k] - abs(psi[0]) ** 2) < 1e-12


def _fixed_step_errors(w, hs):
    ref = dict(w)
    ref.update(integrator=W.RK_DP54, rtol=1e-13, dr_init_km=1e-4)
    Rr = O.Run(ref)
    assert Rr.run_to_end() == O.DONE
    pref = Rr.probabilities()
    errs = []
    for h in hs:
        v = dict(w)
        v.update(rtol=1e30, dr_init_km=h, dr_max_km=h)  # every attempt accepted: fixed steps
        R = O.Run(v)
        assert R.run_to_end() == O.DONE
        errs.append(np.abs(R.probabilities() - pref).max())
    return errs


@pytest.mark.parametrize("n", [2, 3])
def test_second_order_convergence(n):
    """Nonlinear case (mu0 = 1e5 km^-1) from 100 km: halving the step divides
    the global error by 4.  A dropped average, a Hamiltonian taken at the wrong
    radius or from the wrong state would make it first order."""
    if n == 2:
        w = W.exp_stepper_2f()
        w.update(n_energy=30)
    else:
        w = W.exp_stepper_3f(8, 6)
    w.update(r_start_km=100.0, r_end_km=102.0)
    errs = _fixed_step_errors(w, (0.05, 0.025, 0.0125))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert 3.4 < ratios[0] < 4.6 and 3.6 < ratios[1] < 4.4, (errs, ratios)


def test_compared_pair_differs_at_third_order():
    """psi3 - psi7 = O(h^3): one attempt from the same state with h, h/2, h/4."""
    errs = []
    for h in (0.02, 0.01, 0.005):
        w = W.exp_stepper_2f()
        w.update(n_energy=30, r_start_km=100.0, r_end_km=110.0, rtol=1.0, dr_init_km=h, dr_max_km=h)
        R = O.Run(w)
        R.step_exp(1)
        errs.append(R.last_error())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(7.0 < q < 9.0 for q in ratios), (errs, ratios)


def test_controller_settles_at_safety_cubed():
    """With a third-order local error and the h^(1/3) controller, the scaled
    error of successive accepted attempts settles at safety^3 = 0.729."""
    w = W.exp_stepper_3f(12, 10)
    w.update(r_start_km=60.0, r_end_km=100.0, dr_init_km=1e-4)
    R = O.Run(w)
    tail = []
    for i in range(10):
        assert R.step_exp(1) == O.OK
        if i >= 4:
            tail.append(R.last_error())
    assert R.stats()["rejected"] == 0
    assert np.all(np.abs(np.array(tail) - 0.9**3) < 0.01), tail


def test_rejection_shrinks_the_step():
    w = W.exp_stepper_3f(12, 10)
    w.update(r_start_km=60.0, r_end_km=100.0, dr_init_km=0.5)
    R = O.Run(w)
    assert R.step_exp(1) == O.OK
    st = R.stats()
    assert st["rejected"] == 1 and st["accepted"] == 0 and st["r_km"] == 60.0
    assert R.last_error() > 1.0
    assert 0.5 * 0.2 <= st["dr_km"] < 0.5 * 0.9
    for _ in range(30):
        R.step_exp(1)
    assert R.stats()["accepted"] > 0


def test_norm_kept_on_tangential_trajectories_near_the_neutrinosphere():
    """Near R the cosine of the most tangential trajectories changes by orders
    of magnitude within a step; with the path length taken from the mean cosine
    of each evolution's two ends (Appendix A.4.3) the averaged estimates keep
    every beam normalised to the tolerance's order."""
    w = W.exp_stepper_3f(10, 400)
    w.update(dr_init_km=1e-5)
    R = O.Run(w)
    assert R.step_exp(6) == O.OK
    assert R.stats()["accepted"] >= 1
    psi = R.psi_complex()
    assert np.abs((np.abs(psi) ** 2).sum(axis=0) - 1.0).max() < 1e-8


def test_requires_the_lab_frame():
    w = W.exp_stepper_2f()
    w.update(frame=W.FRAME_COROTATING)
    R = O.Run(w)
    assert R.step_exp(1) == O.INVALID


def test_adaptive_run_agrees_with_dormand_prince():
    """At rtol 1e-9 the adaptive stepper stays within its truncation level of a
    tight Dormand-Prince solution of the same lab-frame equations."""
    w = W.exp_stepper_3f(10, 8)
    w.update(r_start_km=60.0, r_end_km=60.05)
    R = O.Run(w)
    assert R.run_to_end() == O.DONE
    ref = dict(w)
    ref.update(integrator=W.RK_DP54, rtol=1e-13, dr_init_km=1e-5)
    Rr = O.Run(ref)
    assert Rr.run_to_end() == O.DONE
    assert R.stats()["accepted"] > 20
    assert np.abs(R.probabilities() - Rr.probabilities()).max() < 1e-7
