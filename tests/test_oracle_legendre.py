"""Pins of the oracle's Legendre / Wigner tables against facts fixed by the
mathematics and by independent libraries (Sec. III-F, Appendix A-B)."""

import math

import mpmath
import numpy as np
import pytest
import scipy.special as ss

from oracle import legendre as lg

RNG = np.random.default_rng(12345)
THETA = np.sort(RNG.uniform(0.02, math.pi - 0.02, 9))


def _tab(L, m, theta=THETA):
    return lg.scalar_table(L, m, np.cos(theta), np.sin(theta))


def test_closed_forms_low_degree():
    x, y = np.cos(THETA), np.sin(THETA)
    pi = math.pi
    ref = {
        (0, 0): np.full_like(x, 1 / math.sqrt(4 * pi)),
        (1, 0): math.sqrt(3 / (4 * pi)) * x,
        (1, 1): -math.sqrt(3 / (8 * pi)) * y,
        (2, 0): math.sqrt(5 / (16 * pi)) * (3 * x * x - 1),
        (2, 1): -math.sqrt(15 / (8 * pi)) * y * x,
        (2, 2): math.sqrt(15 / (32 * pi)) * y * y,
        (3, 3): -math.sqrt(35 / (64 * pi)) * y ** 3,
        (3, 0): math.sqrt(7 / (16 * pi)) * (5 * x ** 3 - 3 * x),
    }
    for (ell, m), val in ref.items():
        got = _tab(4, m)[ell - m]
        np.testing.assert_allclose(got, val, rtol=1e-14, atol=1e-15)
        # negative orders through Pt[l, -m] = (-1)^m Pt[l, m]
        np.testing.assert_allclose(_tab(4, -m)[ell - m], (-1) ** m * val, rtol=1e-14, atol=1e-15)


def test_against_scipy_sph_harm():
    L = 80
    for m in range(0, L, 7):
        T = _tab(L, m)
        for i, ell in enumerate(range(m, L)):
            ref = ss.sph_harm_y(ell, m, THETA, 0.0).real
            np.testing.assert_allclose(T[i], ref, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("ell,m,theta", [
    (10, 3, 0.4), (200, 57, 1.3), (700, 650, 1.9), (1023, 1000, 1.5707),
    (1023, 13, 0.0123), (2023, 560, 0.284), (2047, 1800, 1.4), (1500, 1499, 1.7), (1900, 300, 2.95),
])
def test_against_mpmath_ferrers(ell, m, theta):
    """High-precision reference, including seeds far below the FP64 range
    (at l=2023, m=560, theta=0.284 the seed Pt[m, m] is ~1e-309)."""
    mpmath.mp.dps = 40
    x = mpmath.cos(mpmath.mpf(theta))
    norm = mpmath.sqrt((2 * ell + 1) / (4 * mpmath.pi) * mpmath.factorial(ell - m) / mpmath.factorial(ell + m))
    ref = float(norm * mpmath.legenp(ell, m, x))
    got = lg.scalar_table(ell + 1, m, np.array([math.cos(theta)]), np.array([math.sin(theta)]))[ell - m, 0]
    assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-300) + 1e-280


def test_seed_underflow_recovers():
    v = lg.scalar_table(2024, 560, np.array([math.cos(0.284)]), np.array([math.sin(0.284)]))
    assert v[0, 0] == 0.0 or abs(v[0, 0]) < 1e-300  # seed below the FP64 range
    assert 1.0 < abs(v[-1, 0]) < 2.0


def test_addition_theorem():
    L = 96
    acc = np.zeros((L, THETA.size))
    for m in range(0, L):
        T = _tab(L, m)
        w = 1.0 if m == 0 else 2.0  # +-m contribute equally
        acc[m:] += w * T ** 2
    ell = np.arange(L)[:, None]
    np.testing.assert_allclose(acc, (2 * ell + 1) / (4 * math.pi) * np.ones_like(acc), rtol=1e-12)


def test_parity():
    L = 40
    for m in range(0, L, 3):
        a = _tab(L, m, THETA)
        b = _tab(L, m, math.pi - THETA)
        sign = np.array([(-1) ** (ell + m) for ell in range(m, L)])[:, None]
        np.testing.assert_allclose(b, sign * a, rtol=1e-12, atol=1e-14)


def test_gauss_legendre_orthonormality():
    L = 48
    x, w = np.polynomial.legendre.leggauss(L)
    th = np.arccos(x)
    for m in range(0, L, 5):
        T = lg.scalar_table(L, m, x, np.sin(th))
        gram = 2 * math.pi * (T * w[None, :]) @ T.T
        np.testing.assert_allclose(gram, np.eye(L - m), atol=2e-13)


# ---------------------------------------------------------------- spin ---

def test_spin_against_explicit_wigner_sum():
    tr = lg.trig_from_theta(THETA)
    for s in (-3, -2, -1, 0, 1, 2, 3):
        for m in range(-8, 9):
            T = lg.spin_table(13, m, s, tr)
            l0 = max(abs(m), abs(s))
            for i, ell in enumerate(range(l0, 13)):
                ref = (-1) ** s * math.sqrt((2 * ell + 1) / (4 * math.pi)) * lg.wigner_d_explicit(ell, m, -s, THETA)
                np.testing.assert_allclose(T[i], ref, rtol=1e-12, atol=5e-14)


def test_spin_zero_is_scalar():
    tr = lg.trig_from_theta(THETA)
    L = 60
    for m in range(-L + 1, L, 4):
        np.testing.assert_allclose(lg.spin_table(L, m, 0, tr), _tab(L, m), rtol=1e-12, atol=1e-14)


def test_spin_closed_forms():
    tr = lg.trig_from_theta(THETA)
    y = np.sin(THETA)
    # 1Y_1^0 = sqrt(3/(8 pi)) sin(theta); 2Y_2^0 = sqrt(15/(32 pi)) sin^2(theta)
    np.testing.assert_allclose(lg.spin_table(2, 0, 1, tr)[0], math.sqrt(3 / (8 * math.pi)) * y, rtol=1e-14)
    np.testing.assert_allclose(lg.spin_table(3, 0, 2, tr)[0], math.sqrt(15 / (32 * math.pi)) * y * y, rtol=1e-14)


def test_spin_conjugation_symmetry():
    """sY_{l,-m}(theta, 0) = (-1)^{m+s} (-s)Y_{l,m}(theta, 0)."""
    tr = lg.trig_from_theta(THETA)
    L = 30
    for s in (-2, 1, 2):
        for m in range(-L + 1, L, 3):
            a = lg.spin_table(L, -m, s, tr)
            b = lg.spin_table(L, m, -s, tr)
            np.testing.assert_allclose(a, (-1) ** (m + s) * b, rtol=1e-12, atol=1e-14)


def test_spin_orthonormality_gauss_legendre():
    L = 40
    x, w = np.polynomial.legendre.leggauss(L)
    tr = lg.trig_from_theta(np.arccos(x))
    for s in (2, -2):
        for m in (-30, -5, 0, 1, 17, 39):
            T = lg.spin_table(L, m, s, tr)
            gram = 2 * math.pi * (T * w[None, :]) @ T.T
            np.testing.assert_allclose(gram, np.eye(T.shape[0]), atol=2e-13)


def test_spin_high_degree_against_mpmath_jacobi():
    """d^l_{m,-s} through Jacobi polynomials at 40 digits, l up to 1000."""
    mpmath.mp.dps = 40
    for ell, m, s, theta in [(300, 7, 2, 0.8), (1000, -600, 2, 2.2), (999, 3, -2, 0.05)]:
        a, b = m, -s
        # for a-b >= 0 and a+b >= 0:
        # d^j_{ab} = (-1)^{a-b} sqrt((j+a)!(j-a)!/((j+b)!(j-b)!)) (sin t/2)^{a-b} (cos t/2)^{a+b}
        #            * P^{(a-b, a+b)}_{j-a}(cos t)
        # other cases are mapped there by the symmetries below.
        def d_mp(j, a, b, t):
            sgn = 1
            if a - b < 0:  # d^j_{ab} = (-1)^{a-b} d^j_{ba}
                sgn *= (-1) ** (a - b)
                a, b = b, a
            if a + b < 0:  # d^j_{ab} = (-1)^{a-b} d^j_{-a,-b}
                sgn *= (-1) ** (a - b)
                a, b = -a, -b
                if a - b < 0:
                    sgn *= (-1) ** (a - b)
                    a, b = b, a
            t = mpmath.mpf(t)
            f = mpmath.factorial
            pref = mpmath.sqrt(f(j + a) * f(j - a) / (f(j + b) * f(j - b)))
            sgn *= (-1) ** (a - b)
            return sgn * pref * mpmath.sin(t / 2) ** (a - b) * mpmath.cos(t / 2) ** (a + b) * \
                mpmath.jacobi(j - a, a - b, a + b, mpmath.cos(t))
        ref = float((-1) ** s * mpmath.sqrt((2 * ell + 1) / (4 * mpmath.pi)) * d_mp(ell, a, b, theta))
        got = lg.spin_table(ell + 1, m, s, lg.trig_from_theta(np.array([theta])))[-1, 0]
        assert abs(got - ref) <= 1e-10 * abs(ref) + 1e-280


# ------------------------------------------------- the printed formulas ---

def test_printed_recurrence_and_seed_disagree_with_definition():
    """Planted mistakes: the recurrence and seed exactly as typeset in
    Eq. three_term_recurrence / Eq. base_condition fail the closed forms that
    the corrected oracle passes, so the pins above would catch them."""
    th = 0.9
    x = math.cos(th)
    y00 = 1 / math.sqrt(4 * math.pi)
    y10 = math.sqrt(3 / (4 * math.pi)) * x
    y20 = math.sqrt(5 / (16 * math.pi)) * (3 * x * x - 1)
    ell, m = 1, 0
    lhs = math.sqrt(((ell + 1) ** 2 - m * m) * (2 * ell - 1) / (2 * ell + 1)) * y20
    rhs = math.sqrt((2 * ell + 3) * (2 * ell + 1)) * x * y10 - ell / (ell + 1) * math.sqrt(
        (ell * ell - m * m) * (2 * ell + 3) / (2 * ell + 1)) * y00
    assert abs(lhs - rhs) > 1e-2
    printed_seed_11 = -math.sqrt(math.factorial(2)) / 2 * math.sin(th)
    true_11 = -math.sqrt(3 / (8 * math.pi)) * math.sin(th)
    assert abs(printed_seed_11 / true_11 - 1 / math.sqrt(3 / (4 * math.pi))) < 1e-14
