"""Pins of the oracle's extended bulb model (eq 3.18: azimuth bins per emission
angle, kernel 1 - cos(gamma) with cos(gamma) = cos(theta) cos(theta') +
sin(theta) sin(theta') cos(phi - phi')).  The expected values come from the
bulb model (azimuthally symmetric states) and from the plain pairwise sum over
every background beam with the kernel computed from unit direction vectors,
never from the four-moment form itself (reading P: azimuth bins at the
midpoints of [0, 2 pi), sharing the emission-angle weight equally)."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05560_amd import workloads as W


def _ext(ne, na, np_, n=3, **kw):
    w = W.multi_angle_3f(ne, na)
    w.update(n_flavors=n, n_azimuth=np_, **kw)
    return w


def test_geometry_splits_the_emission_angle_weight_over_the_azimuth_bins():
    bulb = O.Run(W.multi_angle_3f(4, 6))
    ext = O.Run(_ext(4, 6, 5))
    assert ext.na == 30 and ext.nb == 2 * 4 * 30
    for r in (10.0, 10.3, 47.0):
        cb, wb = bulb.geometry(r)
        ce, we = ext.geometry(r)
        np.testing.assert_array_equal(ce, np.repeat(cb, 5))
        np.testing.assert_allclose(we * 5, np.repeat(wb, 5), rtol=1e-15)
    phi = ext.azimuth()
    np.testing.assert_allclose(phi, np.tile(2 * math.pi * (np.arange(5) + 0.5) / 5, 6), rtol=1e-15)


def test_single_angle_model_has_no_azimuth_bins():
    with pytest.raises(ValueError):
        O.Run(dict(W.single_angle_2f(), n_azimuth=4))


def _lab_psi(run, psi_t, phase):
    n, ne, na = run.n, int(run.w["n_energy"]), run.na
    z = (psi_t[:, 0, :] + 1j * psi_t[:, 1, :]).reshape(n, 2, na, ne)
    sigma = np.array([1.0, -1.0])
    rot = np.exp(-1j * sigma[:, None, None] * phase[None, :, :])  # [s, j, a]
    return z * np.transpose(rot, (2, 0, 1))[:, :, :, None]


def _pairwise(run, r, psi_lab):
    """H_nunu(i) = mu0 traceless( sum_b' w_b' (1 - n_i . n_b') [g rho (nu) - gbar conj(rho) (nubar)] )
    with n = (sin t cos p, sin t sin p, cos t) the unit direction of a trajectory."""
    n, na = run.n, run.na
    _, g, gb, _ = run.tables()
    c, w = run.geometry(r)
    phi = run.azimuth()
    s = np.sqrt(1 - c ** 2)
    dirs = np.stack([s * np.cos(phi), s * np.sin(phi), c], axis=1)
    mu0 = run.w["mu0_km"]
    out = np.zeros((na, n, n), complex)
    for i in range(na):
        acc = np.zeros((n, n), complex)
        for j in range(na):
            kern = w[j] * (1 - dirs[i] @ dirs[j])
            for k in range(len(g)):
                v = psi_lab[:, 0, j, k]
                acc += kern * g[k] * 2 * np.outer(v, v.conj())
                v = psi_lab[:, 1, j, k]
                acc -= kern * gb[k] * np.conj(2 * np.outer(v, v.conj()))
        acc -= np.trace(acc) / n * np.eye(n)
        out[i] = mu0 * acc
    return out


@pytest.mark.parametrize("n,ne,na,np_,r", [(3, 3, 3, 4, 10.7), (2, 4, 2, 5, 23.0), (3, 2, 4, 3, 10.0)])
def test_collective_hamiltonian_equals_the_pairwise_azimuth_sum(n, ne, na, np_, r):
    run = O.Run(_ext(ne, na, np_, n=n))
    psi = W.random_states(n, run.nb, seed=21 + n + np_)
    phase = W.random_phases(n, run.na, seed=8 + ne)
    run.set_state(psi, phase, r)
    got = run.collective()
    expect = _pairwise(run, r, _lab_psi(run, psi, phase))
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-13 * np.abs(expect).max())
    j2, j3 = run.moments_azimuth()
    assert np.abs(j2).max() > 1e-3 * np.abs(expect).max() / run.w["mu0_km"]   # the azimuth terms matter
    np.testing.assert_allclose(j2, j2.conj().T, atol=1e-15)
    np.testing.assert_allclose(j3, j3.conj().T, atol=1e-15)


def test_azimuthally_symmetric_states_evolve_as_the_bulb_model():
    ne, na, np_ = 6, 4, 3
    wb = dict(W.multi_angle_3f(ne, na), integrator=W.RK4_FIXED, r_start_km=20.0, r_end_km=20.0002, n_fixed_steps=40)
    we = dict(wb, n_azimuth=np_)
    bulb, ext = O.Run(wb), O.Run(we)
    psi = W.random_states(3, bulb.nb, seed=4)
    phase = W.random_phases(3, bulb.na, seed=6)
    # replicate every emission-angle trajectory over its azimuth bins
    pe = psi.reshape(3, 2, 2, na, 1, ne).repeat(np_, axis=4).reshape(3, 2, ext.nb)
    phe = phase.repeat(np_, axis=0)
    bulb.set_state(psi, phase, 20.0)
    ext.set_state(pe, phe, 20.0)
    j2, j3 = ext.moments_azimuth()
    j0, _ = ext.moments()
    assert np.abs(j2).max() <= 1e-14 * np.abs(j0).max() and np.abs(j3).max() <= 1e-14 * np.abs(j0).max()
    assert bulb.step_rk4(40) == O.OK and ext.step_rk4(40) == O.OK
    pb = bulb.probabilities().reshape(2, na, 1, ne).repeat(np_, axis=2)
    pe_ = ext.probabilities().reshape(2, na, np_, ne)
    np.testing.assert_allclose(pe_, pb, rtol=0, atol=1e-12)
