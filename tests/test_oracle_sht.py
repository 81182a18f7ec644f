"""Pins of the oracle transforms (Sec. III, Procedures 1-2) against facts
fixed by the paper and the mathematics."""

import math

import numpy as np
import pytest
import scipy.special as ss

from oracle import sht
from oracle.sampling import numerators_alternating
from tests import inputs


def _plan(L, s=0):
    return sht.Plan(L, s)


@pytest.mark.parametrize("L", [1, 2, 7, 32])
def test_exactly_L2_samples(L):
    """Eq. number_samples_sum: sum_k (2k+1) = L^2, and every ring k holds
    2k+1 equiangular longitudes starting at phi = 0."""
    ring, j, n = sht.ring_geometry(L)
    assert ring.size == L * L
    for k in range(L):
        assert np.count_nonzero(ring == k) == 2 * k + 1
    assert np.all(j[np.r_[0, np.cumsum(2 * np.arange(L) + 1)[:-1]]] == 0)


def test_Y00_constant():
    L = 12
    flm = np.zeros((1, L * L), complex)
    flm[0, 0] = 1.0
    f = sht.inverse(_plan(L), flm)
    np.testing.assert_allclose(f, 1 / math.sqrt(4 * math.pi), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("L", [3, 9, 16])
def test_inverse_equals_direct_sum_with_scipy_harmonics(L):
    """Eq. f_expansion_bandlimited summed term by term with scipy's Y_l^m."""
    p = _plan(L)
    flm = inputs.coeffs(L, 2, seed=7)
    ring, jj, nn = sht.ring_geometry(L)
    th = p.theta[ring]
    phi = 2 * math.pi * jj / nn
    ref = np.zeros((2, L * L), complex)
    ell, m, idx = sht.coeff_index(L)
    for i in idx:
        ref += flm[:, i:i + 1] * ss.sph_harm_y(ell[i], m[i], th, phi)[None, :]
    np.testing.assert_allclose(sht.inverse(p, flm), ref, rtol=1e-12, atol=1e-13)


def test_inverse_rings_matches_inverse():
    L = 20
    p = _plan(L)
    flm = inputs.coeffs(L, 3, seed=3)
    f = sht.inverse(p, flm)
    for k, v in sht.inverse_rings(p, flm, [0, 5, 19]).items():
        np.testing.assert_allclose(v, f[:, k * k:k * k + 2 * k + 1], rtol=1e-13, atol=1e-14)


def test_real_map_hermitian_symmetry():
    """Eq. yellm:conj: flm[l,-m] = (-1)^m conj(flm[l,m]) <=> real samples."""
    L = 14
    flm = inputs.coeffs(L, 1, seed=11)
    ell, m, idx = sht.coeff_index(L)
    for i in idx:
        if m[i] < 0:
            flm[0, i] = (-1.0) ** int(m[i]) * np.conj(flm[0, ell[i] ** 2 + ell[i] - m[i]])
        elif m[i] == 0:
            flm[0, i] = flm[0, i].real
    f = sht.inverse(_plan(L), flm)
    assert np.max(np.abs(f.imag)) < 1e-13 * np.max(np.abs(f.real))


@pytest.mark.parametrize("L", [2, 5, 12, 24])
def test_forward_equals_dense_solve(L):
    """Procedure 1 equals flm = Y^{-1} f with the dense L^2 x L^2 matrix."""
    p = _plan(L)
    f = inputs.samples_uniform(L, 2, seed=L)
    Y = sht.dense_Y(p)
    ref = np.linalg.solve(Y, f.T).T
    np.testing.assert_allclose(sht.forward(p, f), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("L,weighted", [(16, False), (64, False), (128, True)])
def test_round_trip_spectral_spatial_spectral(L, weighted):
    """Experiment 1 (Sec. IV-A): inverse then forward returns flm."""
    p = _plan(L)
    flm = inputs.coeffs(L, 2, seed=1, weighted=weighted)
    rec = sht.forward(p, sht.inverse(p, flm))
    assert sht.relmax(rec, flm) < 1e-12
    assert sht.e_max(rec, flm) < 1e-12 and sht.e_mean(rec, flm) < 1e-13


@pytest.mark.parametrize("L", [16, 48])
def test_round_trip_spatial_spectral_spatial(L):
    """Experiment 2 (Sec. IV-A): a random sample vector is band-limited on
    this scheme (L^2 samples = L^2 dof), so forward then inverse returns it."""
    p = _plan(L)
    f = inputs.samples_uniform(L, 2, seed=2)
    rec = sht.inverse(p, sht.forward(p, f))
    assert sht.relmax(rec, f) < 1e-12


def test_discrete_orthonormality():
    """forward of a sampled single harmonic is the unit coefficient vector."""
    L = 10
    p = _plan(L)
    for i in (0, 3, 17, 55, 99):
        e = np.zeros((1, L * L), complex)
        e[0, i] = 1.0
        rec = sht.forward(p, sht.inverse(p, e))
        np.testing.assert_allclose(rec, e, atol=1e-13)


@pytest.mark.parametrize("s", [0, 2, -2, 1])
def test_adjoint_dot_products(s):
    L = 10
    p = _plan(L, s)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, L * L)) + 1j * rng.standard_normal((2, L * L))
    y = inputs.coeffs(L, 2, seed=6, spin=s)
    a = np.vdot(sht.inverse(p, y), x)
    b = np.vdot(y, sht.inverse_adjoint(p, x))
    assert abs(a - b) <= 1e-13 * abs(a)
    c = np.vdot(sht.forward(p, x), y)
    d = np.vdot(x, sht.forward_adjoint(p, y))
    assert abs(c - d) <= 1e-12 * abs(c)


@pytest.mark.parametrize("L", [4, 9])
def test_adjoints_equal_dense_forms(L):
    p = _plan(L)
    Y = sht.dense_Y(p)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, L * L)) + 1j * rng.standard_normal((2, L * L))
    np.testing.assert_allclose(sht.inverse_adjoint(p, x), x @ Y.conj(), rtol=1e-12, atol=1e-13)
    Yinv_H = np.linalg.inv(Y).conj().T
    np.testing.assert_allclose(sht.forward_adjoint(p, x), x @ Yinv_H.T, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("s", [2, -2, 1])
def test_spin_inverse_dense_and_forward_small(s):
    """Spin (Sec. III-G): inverse against the dense spin matrix; forward
    against the dense least-squares solution at small L, where the order-wise
    elimination is still accurate."""
    L = 8
    p = _plan(L, s)
    flm = inputs.coeffs(L, 2, seed=4, spin=s)
    Y = sht.dense_Y(p)
    np.testing.assert_allclose(sht.inverse(p, flm), flm @ Y.T, rtol=1e-12, atol=1e-13)
    f = sht.inverse(p, flm)
    ell = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    cols = ell >= abs(s)
    ls = np.linalg.lstsq(Y[:, cols], f.T, rcond=None)[0].T
    fwd = sht.forward(p, f)
    np.testing.assert_allclose(fwd[:, cols], ls, rtol=0, atol=1e-8)
    np.testing.assert_allclose(fwd[:, cols], flm[:, cols], rtol=0, atol=1e-8)
    assert np.all(fwd[:, ~cols] == 0)


def test_alternating_placement_round_trip_small_L():
    L = 20
    p = sht.Plan(L, 0, numerators_alternating(L))
    flm = inputs.coeffs(L, 1, seed=9)
    assert sht.relmax(sht.forward(p, sht.inverse(p, flm)), flm) < 1e-11


def test_error_metrics_on_hand_example():
    a = np.array([1 + 1j, 2.0, 0.0, 4j])
    b = np.array([1.0, 2.0, 3.0, 4j])
    assert sht.e_max(a, b) == 3.0
    assert sht.e_mean(a, b) == 1.0
    assert math.isclose(sht.relmax(a, b), 3.0 / 4.0)


def test_planted_sign_error_is_caught():
    """A plausible mistake planted in a copy of the oracle's alias step
    (adding f~_m instead of subtracting it, Eq. signal_update) breaks the
    round trip, which the pins above check."""
    L = 8
    p = _plan(L)
    flm = inputs.coeffs(L, 1, seed=1)
    f = sht.inverse(p, flm)
    orig = np.ndarray.__isub__
    import oracle.sht as mod

    src_forward = mod.forward

    def bad_forward(plan, samples):
        work = np.asarray(samples, complex).copy()
        L_ = plan.L
        out = np.zeros_like(work)
        ring, jj, nn = sht.ring_geometry(L_)
        spectra = [None] * L_
        for am in range(L_ - 1, -1, -1):
            n = 2 * am + 1
            spectra[am] = np.fft.fft(work[:, am * am:am * am + n], axis=1) / n
            for m in ((am, -am) if am else (0,)):
                g = np.stack([spectra[k][:, m % (2 * k + 1)] for k in range(am, L_)], axis=1)
                fm = plan.solve(m, g)
                ell = np.arange(plan.l0(m), L_)
                out[:, ell * ell + ell + m] = fm
                if am > 0:
                    top = fm @ plan.table(m)[:am, :].T
                    ns = am * am
                    ph = np.exp(2j * math.pi * ((m * jj[:ns]) % nn[:ns]) / nn[:ns])
                    work[:, :ns] += top[:, ring[:ns]] * ph[None, :]  # planted: + instead of -
        return out

    assert sht.relmax(src_forward(p, f), flm) < 1e-13
    assert sht.relmax(bad_forward(p, f), flm) > 1e-3
    assert orig is np.ndarray.__isub__
