"""Pins of the oracle's neutrino self-interaction (eq 3.8, 3.9, 3.13, 3.16).

The oracle evaluates H_nunu through two angle moments J0, J1 (the kernel
1 - cos(theta) cos(theta') factorises).  These tests recompute H_nunu as the
plain pairwise sum over every background beam, in the lab frame, on small
random states, and check the reduction of the four initial flavors to two
evolved species (reading N) against an explicit four-species integration.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W


def _lab_psi(run, psi_t, phase):
    """psi = exp(-i sigma Phi_j) psi~ for every beam (sigma = +1 nu, -1 nubar)."""
    n, ne, na = run.n, int(run.w["n_energy"]), run.na
    z = (psi_t[:, 0, :] + 1j * psi_t[:, 1, :]).reshape(n, 2, na, ne)
    sigma = np.array([1.0, -1.0])
    rot = np.exp(-1j * sigma[:, None, None] * phase[None, :, :])  # [s, j, a]
    return z * np.transpose(rot, (2, 0, 1))[:, :, :, None]


def _pairwise_hnunu(run, r, psi_lab):
    """H_nunu(i) = mu0 traceless( sum over beams b' of w_b' (1 - c_i c_b')
    [g rho_b' (nu) - gbar conj(rho_b') (nubar)] ), rho = 2 psi psi^dagger."""
    n, na = run.n, run.na
    _, g, gb, _ = run.tables()
    c, w = run.geometry(r)
    mu0 = run.w["mu0_km"]
    out = np.zeros((na, n, n), complex)
    for i in range(na):
        acc = np.zeros((n, n), complex)
        for j in range(na):
            kern = w[j] * (1 - c[i] * c[j]) if run.w["n_angle"] > 0 else w[0]
            for k in range(len(g)):
                v = psi_lab[:, 0, j, k]
                acc += kern * g[k] * 2 * np.outer(v, v.conj())
                v = psi_lab[:, 1, j, k]
                acc -= kern * gb[k] * np.conj(2 * np.outer(v, v.conj()))
        acc -= np.trace(acc) / n * np.eye(n)
        out[i] = mu0 * acc
    return out


@pytest.mark.parametrize("n,ne,na,r", [(3, 3, 4, 10.7), (2, 5, 3, 23.0), (3, 4, 0, 31.0), (2, 3, 0, 10.0)])
def test_collective_hamiltonian_equals_the_pairwise_sum(n, ne, na, r):
    w = W.multi_angle_3f(ne, na)
    w["n_flavors"] = n
    run = O.Run(w)
    psi = W.random_states(n, run.nb, seed=11 + n + na)
    phase = W.random_phases(n, run.na, seed=5 + ne)
    run.set_state(psi, phase, r)
    got = run.collective()
    expect = _pairwise_hnunu(run, r, _lab_psi(run, psi, phase))
    scale = np.abs(expect).max()
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-13 * scale)


def test_moments_are_hermitian_and_zero_phase_independent_on_the_diagonal():
    w = W.multi_angle_3f(5, 6)
    run = O.Run(w)
    psi = W.random_states(3, run.nb, seed=3)
    run.set_state(psi, W.random_phases(3, run.na, seed=4), 17.0)
    j0, j1 = run.moments()
    np.testing.assert_allclose(j0, j0.conj().T, atol=1e-15)
    np.testing.assert_allclose(j1, j1.conj().T, atol=1e-15)
    run.set_state(psi, np.zeros((run.na, 3)), 17.0)
    k0, k1 = run.moments()
    np.testing.assert_allclose(np.diag(j0), np.diag(k0), rtol=1e-14)
    np.testing.assert_allclose(np.diag(j1), np.diag(k1), rtol=1e-14)


def _explicit_four_species_rk4(w, nsteps):
    """Lab-frame RK4 of nu_e, nubar_e, nu_x, nubar_x beams (single angle, two
    flavors), with eq 3.8's sum over all four initial flavors and no reduction.
    Hamiltonians are made traceless (the trace only adds a common phase)."""
    run = O.Run(w)
    e, _, _, hv = run.tables()
    ne = len(e)
    de = (w["e_max_mev"] - w["e_min_mev"]) / ne
    f = np.empty((4, ne))
    for s in range(4):
        t = O.temperature(w["mean_e_mev"][s], w["eta"][s])
        f[s] = [O.spectrum(x, t, w["eta"][s]) for x in e]
    nrel = np.array(w["lum_erg_s"]) / 1e51 * 11.0 / np.array(w["mean_e_mev"])
    wt = nrel[:, None] * f * de  # [species, k]
    anti = np.array([False, True, False, True])
    psi = np.zeros((4, ne, 2), complex)
    psi[0, :, 0] = psi[1, :, 0] = 1.0   # born nu_e / nubar_e
    psi[2, :, 1] = psi[3, :, 1] = 1.0   # born nu_x / nubar_x

    def rhs(r, p):
        rho = 2 * np.einsum("ska,skb->skab", p, p.conj())
        acc = (wt[~anti, :, None, None] * rho[~anti]).sum((0, 1)) \
            - (wt[anti, :, None, None] * rho[anti].conj()).sum((0, 1))
        acc = acc - np.trace(acc) / 2 * np.eye(2)
        hnn = w["mu0_km"] * O.dilution(r / w["r_nu_km"]) * acc
        lam = w["lambda0_km"] * (w["lambda_rref_km"] / r) ** w["lambda_power"]
        hm = np.diag([lam / 2, -lam / 2])
        out = np.empty_like(p)
        for s in range(4):
            H = (hv.conj() - hm - hnn.conj()) if anti[s] else (hv + hm + hnn)
            out[s] = -1j * np.einsum("kab,kb->ka", H, p[s])
        return out

    r0, r1 = w["r_start_km"], w["r_end_km"]
    h = (r1 - r0) / nsteps
    for i in range(nsteps):
        r = r0 + i * h
        k1 = rhs(r, psi)
        k2 = rhs(r + h / 2, psi + h / 2 * k1)
        k3 = rhs(r + h / 2, psi + h / 2 * k2)
        k4 = rhs(r + h, psi + h * k3)
        psi = psi + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return np.abs(psi[:2, :, 0]) ** 2


def test_two_species_weights_reproduce_the_four_species_sum():
    w = W.single_angle_2f()
    w.update(n_energy=6, r_start_km=40.0, r_end_km=46.0, n_fixed_steps=6000,
             frame=W.FRAME_LAB, lum_erg_s=[1e51, 1.3e51, 0.8e51, 0.6e51])
    run = O.Run(w)
    assert run.step_rk4(w["n_fixed_steps"]) == O.OK
    p = run.probabilities().reshape(2, -1)
    expect = _explicit_four_species_rk4(w, w["n_fixed_steps"])
    assert np.abs(1 - expect).max() > 1e-4  # the window changes the flavor content
    np.testing.assert_allclose(p, expect, rtol=0, atol=1e-10)


def _exact_density_sums(w, psi):
    """Correctly rounded (math.fsum) energy sums of the single-angle density
    terms, formed with the same IEEE products as the oracle's sums: the
    pin of its compensated summation mode."""
    import math

    ref = O.Run(w)
    _, g, gb, _ = ref.tables()
    n, nb = psi.shape[0], psi.shape[2]
    ne = nb // 2
    ar, ai = psi[:, 0, :], psi[:, 1, :]
    out = np.empty((n, n), dtype=complex)
    for a in range(n):
        for c in range(n):
            re = ar[a] * ar[c] - ai[a] * (-ai[c])     # Re psi_a conj(psi_c), as c_mul forms it
            im = ar[a] * (-ai[c]) + ai[a] * ar[c]
            tre = np.concatenate([re[:ne] * g, re[ne:] * (-gb)])
            tim = np.concatenate([im[:ne] * g, (-im[ne:]) * (-gb)])
            out[a, c] = math.fsum(tre) + 1j * math.fsum(tim)
    return out


def test_compensated_sums_are_correctly_rounded_within_an_ulp():
    """Sum mode 1 (Neumaier) gives the single-angle J0 of random states (sums
    with heavy cancellation) within a couple of ulps of the correctly rounded
    sum, where the plain ascending sum (mode 0) is off by far more: the
    compensated mode, used to measure how much of a run's sensitivity is
    summation rounding, does what it claims."""
    w = dict(W.single_angle_2f(), n_flavors=3, n_energy=400)
    nb = 2 * 400
    psi = W.random_states(3, nb, seed=77)
    r = 13.5
    exact = _exact_density_sums(w, psi)
    ref = O.Run(w)
    ref.set_state(psi, None, r)
    _, wj = ref.geometry(r)
    target = 2.0 * exact * wj[0]
    errs = {}
    for mode in (0, 1, 3):
        o = O.Run(dict(w, sum_mode=mode))
        o.set_state(psi, None, r)
        j0, _ = o.moments()
        errs[mode] = np.abs(j0 - target)
    scale = np.abs(target).max()
    assert errs[1].max() <= 4 * np.finfo(float).eps * scale
    assert errs[3].max() <= 4 * np.finfo(float).eps * scale
    assert errs[0].max() > 10 * errs[1].max()
