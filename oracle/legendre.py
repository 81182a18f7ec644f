"""Scalar and spin-weighted associated Legendre tables in FP64 (oracle).

What is computed
----------------
Scalar (Sec. III-F, Appendix A, Eq. Sph_harmonics):
    Pt[l, m](theta) = Y_l^m(theta, 0)
                    = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!) P_l^m(cos theta),
with the Condon-Shortley phase inside P_l^m, for l = |m| .. L-1, and the
symmetry Pt[l, -m] = (-1)^m Pt[l, m] (Sec. III-F, from Eq. yellm:conj).

Spin (Sec. III-G, Appendix B):
    sPt[l, m](theta) = sY_l^m(theta, 0) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta)
with Wigner's small-d in the convention of Wigner's explicit sum, for
l = max(|m|, |s|) .. L-1.

Readings of the paper (the printed recursions are garbled)
----------------------------------------------------------
* The printed scalar three-term recurrence (Eq. three_term_recurrence) does
  not hold as typeset; this module uses the standard fully normalised
  recurrence in l
      sqrt((l+1)^2 - m^2) Pt[l+1] = sqrt((2l+1)(2l+3)) cos(theta) Pt[l]
                                    - sqrt((2l+3)(l^2 - m^2)/(2l-1)) Pt[l-1],
  which is what the printed equation is meant to be (same three terms, same
  direction of growth).
* The printed seed (Eq. base_condition) lacks the factor sqrt((2m+1)/(4 pi))
  that makes Pt[m, m] = Y_m^m(theta, 0); this module uses
      Pt[m, m] = (-1)^m sqrt((2m+1)/(4 pi)) sqrt((2m)!)/(2^m m!) sin^m(theta).
* The printed spin recurrence and seed (Appendix B) are garbled; this module
  follows the definition through Wigner d (Appendix B, first display): the
  standard upward recurrence of d^j_{ab} in j for fixed (a, b), started at
  j = max(|a|, |b|) from the single surviving term of Wigner's explicit sum.
* "Adaptive rescaling" (Sec. III-F, Sec. IV) is unspecified; here every value
  is carried as mantissa * 2**exponent with a per-theta exponent until it
  re-enters the FP64 range, so seeds far below 1e-308 still recur to O(1)
  values.

Pins: closed forms, scipy.special.sph_harm_y, mpmath's Ferrers functions at
high precision, the addition theorem, parity, Gauss-Legendre orthonormality,
and for spin the explicit Wigner sum (tests/test_oracle_legendre.py).
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "scalar_seed",
    "scalar_table",
    "spin_table",
    "wigner_d_explicit",
    "trig_from_theta",
]

_BIG = 2.0 ** 256
_SMALL = 2.0 ** -256


def trig_from_theta(theta):
    """cos/sin of theta and of theta/2 for arbitrary colatitudes in [0, pi]."""
    theta = np.asarray(theta, dtype=np.float64)
    return {
        "cos": np.cos(theta),
        "sin": np.sin(theta),
        "cos_half": np.cos(theta / 2),
        "sin_half": np.sin(theta / 2),
    }


# ---------------------------------------------------------------------------
# mantissa/exponent helpers: value = mant * 2**expo, |mant| in [0.5, 1) or 0
# ---------------------------------------------------------------------------

def _norm(mant, expo):
    m, e = np.frexp(mant)
    return m, expo + e.astype(np.int64)


def _int_me(c: int):
    """Exact positive Python integer -> (mantissa, exponent), correctly rounded."""
    nb = c.bit_length()
    shift = max(nb - 64, 0)
    top = c >> shift  # at most 64 bits; float() rounds it once
    m, e = math.frexp(float(top))
    return m, e + shift


def _sqrt_me(m: float, e: int):
    if e % 2:
        m, e = m * 2.0, e - 1
    return math.sqrt(m), e // 2


def _pow_me(x, p: int):
    """x**p for an array x >= 0 and integer p >= 0 by binary powering, kept in
    mantissa/exponent form so that no intermediate under- or overflows."""
    x = np.asarray(x, dtype=np.float64)
    rm = np.ones_like(x)
    re = np.zeros(x.shape, dtype=np.int64)
    bm, be = _norm(x.copy(), np.zeros(x.shape, dtype=np.int64))
    while p:
        if p & 1:
            rm, re = _norm(rm * bm, re + be)
        p >>= 1
        if p:
            bm, be = _norm(bm * bm, be + be)
    return rm, re


def _to_float(mant, expo):
    return np.ldexp(mant, np.clip(expo, -4000, 4000).astype(np.int32))


# ---------------------------------------------------------------------------
# scalar tables
# ---------------------------------------------------------------------------

def scalar_seed(m: int, sin_t):
    """Pt[|m|, |m|](theta) as (mantissa, exponent) arrays (m >= 0 branch).

    Closed form (corrected Eq. base_condition):
        (-1)^m sqrt((2m+1)/(4 pi)) * sqrt(C(2m, m) / 4^m) * sin^m(theta),
    using sqrt((2m)!)/(2^m m!) = sqrt(C(2m, m)/4^m) with the binomial taken
    exactly in integer arithmetic.
    """
    m = abs(int(m))
    cm, ce = _int_me(math.comb(2 * m, m))
    ce -= 2 * m
    cm, ce = _sqrt_me(cm, ce)
    sm, se = _pow_me(sin_t, m)
    mant = ((-1.0) ** m) * math.sqrt((2 * m + 1) / (4 * math.pi)) * cm * sm
    return _norm(mant, se + ce)


def scalar_table(L: int, m: int, cos_t, sin_t):
    """Array of shape (L - |m|, ntheta): row i holds Pt[|m| + i, m](theta)."""
    am = abs(int(m))
    cos_t = np.asarray(cos_t, dtype=np.float64)
    n = cos_t.size
    out = np.empty((L - am, n))
    if L <= am:
        return out
    p_cur, e = scalar_seed(am, sin_t)
    p_prev = np.zeros(n)
    out[0] = _to_float(p_cur, e)
    for i, ell in enumerate(range(am, L - 1)):
        den = (ell + 1) ** 2 - am * am
        a = math.sqrt((2 * ell + 1) * (2 * ell + 3) / den)
        b = 0.0 if ell == am else math.sqrt((2 * ell + 3) * (ell * ell - am * am) / ((2 * ell - 1) * den))
        p_next = a * cos_t * p_cur - b * p_prev
        p_prev, p_cur = p_cur, p_next
        big = np.maximum(np.abs(p_prev), np.abs(p_cur))
        hi = big > _BIG
        lo = (big < _SMALL) & (big > 0)
        if hi.any() or lo.any():
            scale = np.where(hi, 1.0 / _BIG, np.where(lo, _BIG, 1.0))
            p_prev = p_prev * scale
            p_cur = p_cur * scale
            e = e + np.where(hi, 256, np.where(lo, -256, 0))
        out[i + 1] = _to_float(p_cur, e)
    if m < 0 and am % 2:
        out = -out
    return out


# ---------------------------------------------------------------------------
# spin tables (Wigner d)
# ---------------------------------------------------------------------------

def _spin_seed(a: int, b: int, cos_h, sin_h):
    """d^j_{ab}(theta) at j = max(|a|, |b|): the single surviving term of
    Wigner's explicit sum, as (mantissa, exponent) arrays."""
    j = max(abs(a), abs(b))
    if abs(a) >= abs(b):
        k = b
        if a == j:
            sign, pc, ps = (-1) ** (j - b), j + b, j - b
        else:  # a == -j
            sign, pc, ps = 1, j - b, j + b
    else:
        k = a
        if b == j:
            sign, pc, ps = 1, j + a, j - a
        else:  # b == -j
            sign, pc, ps = (-1) ** (j + a), j - a, j + a
    cm, ce = _int_me(math.comb(2 * j, j + k))
    cm, ce = _sqrt_me(cm, ce)
    xm, xe = _pow_me(cos_h, pc)
    ym, ye = _pow_me(sin_h, ps)
    return _norm(sign * cm * xm * ym, ce + xe + ye)


def spin_table(L: int, m: int, s: int, trig):
    """Array of shape (L - l0, ntheta), l0 = max(|m|, |s|): row i holds
    sY_{l0+i}^m(theta, 0) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta)."""
    a, b = int(m), -int(s)
    l0 = max(abs(a), abs(b))
    cos_t = np.asarray(trig["cos"], dtype=np.float64)
    n = cos_t.size
    out = np.empty((max(L - l0, 0), n))
    if L <= l0:
        return out
    sgn_s = -1.0 if (s % 2) else 1.0
    d_cur, e = _spin_seed(a, b, trig["cos_half"], trig["sin_half"])
    d_prev = np.zeros(n)
    out[0] = sgn_s * math.sqrt((2 * l0 + 1) / (4 * math.pi)) * _to_float(d_cur, e)
    for i, j in enumerate(range(l0, L - 1)):
        if j == 0:  # a = b = 0: d^1_{00} = cos(theta)
            d_next = cos_t * d_cur
        else:
            c1 = (2 * j + 1) / (j * math.sqrt(((j + 1) ** 2 - a * a) * ((j + 1) ** 2 - b * b)))
            c2 = (j + 1) * math.sqrt((j * j - a * a) * (j * j - b * b)) / (
                j * math.sqrt(((j + 1) ** 2 - a * a) * ((j + 1) ** 2 - b * b)))
            d_next = c1 * (j * (j + 1) * cos_t - a * b) * d_cur - c2 * d_prev
        d_prev, d_cur = d_cur, d_next
        big = np.maximum(np.abs(d_prev), np.abs(d_cur))
        hi = big > _BIG
        lo = (big < _SMALL) & (big > 0)
        if hi.any() or lo.any():
            scale = np.where(hi, 1.0 / _BIG, np.where(lo, _BIG, 1.0))
            d_prev = d_prev * scale
            d_cur = d_cur * scale
            e = e + np.where(hi, 256, np.where(lo, -256, 0))
        ell = j + 1
        out[i + 1] = sgn_s * math.sqrt((2 * ell + 1) / (4 * math.pi)) * _to_float(d_cur, e)
    return out


def wigner_d_explicit(j: int, a: int, b: int, theta):
    """Wigner small-d d^j_{ab}(theta) from Wigner's explicit finite sum, with
    exact integer factorials.  Intended for small j only (a pin)."""
    theta = np.asarray(theta, dtype=np.float64)
    c = np.cos(theta / 2)
    s = np.sin(theta / 2)
    f = math.factorial
    pref = math.sqrt(f(j + a) * f(j - a) * f(j + b) * f(j - b))
    total = np.zeros_like(theta)
    for t in range(0, 2 * j + 1):
        if j + b - t < 0 or j - a - t < 0 or a - b + t < 0:
            continue
        den = f(j + b - t) * f(t) * f(a - b + t) * f(j - a - t)
        total = total + ((-1) ** (a - b + t)) * (pref / den) * c ** (2 * j + b - a - 2 * t) * s ** (a - b + 2 * t)
    return total
