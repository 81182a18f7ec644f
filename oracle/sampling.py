"""Colatitude placement of the L rings (oracle).

Sec. III-A: ring k (k = 0..L-1) sits at colatitude theta_k and carries 2k+1
equiangular longitudes phi_j = 2 pi j / (2k+1), j = 0..2k, so the scheme has
sum_k (2k+1) = L^2 samples (Eq. number_samples_sum).

Sec. III-D: every theta_k is drawn from the equiangular set
    Theta = { pi (2t+1) / (2L-1) : t = 0..L-1 }        (Eq. equiangular_set)
so a placement is a permutation of the odd numerators 1, 3, .., 2L-1 and is
stored exactly as integers n_k with theta_k = pi n_k / (2L-1).

Two orderings are given by the paper:
* the alternating vector of Eq. sampling_latitude,
* the condition-number-minimising greedy (Sec. III-D): fix theta_{L-1}
  farthest from the poles, then for m = L-2 down to 0 choose theta_m among the
  unused members of Theta to minimise the condition number of P_m, the matrix
  of Eq. Y_matrix built from rings m..L-1 and degrees m..L-1.

Readings: the condition number is the 2-norm one, sigma_max / sigma_min (the
paper's "largest over smallest eigenvalue" for a non-symmetric matrix);
candidates are the unused members of Theta; candidates whose condition number
lies within a relative 1e-12 of the minimum are tied and the smallest
numerator wins.  The 2 pi factor of P_m does not change its condition number
and is omitted.

Two evaluations of the same greedy are provided: "svd" forms every candidate
matrix and calls numpy's SVD-based cond (the literal reading, for small L);
"secular" uses the eigen-decomposition of B^T B of the fixed rows B and solves
the rank-one secular equation 1 + sum_i z_i^2/(d_i - lam) = 0 for the extreme
eigenvalues of B^T B + r r^T by bisection (same result, O(L^4) overall).
The two are pinned against each other in tests/test_oracle_sampling.py.
"""

from __future__ import annotations

import math

import numpy as np

from .legendre import scalar_table

__all__ = [
    "numerators_equiangular",
    "numerators_alternating",
    "numerators_greedy",
    "trig_from_numerators",
    "theta_from_numerators",
    "kappas",
]

TIE_RTOL = 1e-12


def numerators_equiangular(L: int) -> np.ndarray:
    """Odd numerators 1, 3, .., 2L-1 of the set Theta (Eq. equiangular_set)."""
    return 2 * np.arange(L, dtype=np.int64) + 1


def numerators_alternating(L: int) -> np.ndarray:
    """Eq. sampling_latitude: [pi, pi/(2L-1), pi(2L-3)/(2L-1), 3pi/(2L-1), ..]:
    even k take 2L-1-k (counting down from the south pole), odd k take k."""
    k = np.arange(L, dtype=np.int64)
    return np.where(k % 2 == 0, 2 * L - 1 - k, k)


def theta_from_numerators(L: int, num) -> np.ndarray:
    return math.pi * np.asarray(num, dtype=np.float64) / (2 * L - 1)


def trig_from_numerators(L: int, num):
    """cos/sin of theta_k = pi n_k/(2L-1) and of theta_k/2, evaluated through
    the complement pi - theta_k so that the south pole (n = 2L-1) gives
    sin = 0 and cos = -1 exactly."""
    D = 2 * L - 1
    num = np.asarray(num, dtype=np.int64)
    comp = (D - num).astype(np.float64) / D  # (pi - theta)/pi
    return {
        "cos": -np.cos(math.pi * comp),
        "sin": np.sin(math.pi * comp),
        "cos_half": np.sin(math.pi * comp / 2),
        "sin_half": np.cos(math.pi * comp / 2),
    }


def _order_rows(L, m, trig):
    """rows[i, :] = Pt[m..L-1, m] at the i-th colatitude."""
    return scalar_table(L, m, trig["cos"], trig["sin"]).T


def _kappa_svd(fixed, cand_rows):
    out = np.empty(cand_rows.shape[0])
    for i, r in enumerate(cand_rows):
        out[i] = np.linalg.cond(np.vstack([r[None, :], fixed]), 2)
    return out


def _kappa_secular(fixed, cand_rows):
    n = fixed.shape[1]
    if n == 1:  # no fixed rows: the 1x1 matrix [r]
        return np.where(cand_rows[:, 0] != 0, 1.0, np.inf)
    d, V = np.linalg.eigh(fixed.T @ fixed)  # ascending
    d[0] = 0.0  # B has n-1 rows: exactly one zero eigenvalue
    z2 = (cand_rows @ V) ** 2
    c = cand_rows.shape[0]

    def phi(lam):
        # a candidate row orthogonal to an eigenvector gives 0/0 terms: they
        # are exactly zero contributions
        with np.errstate(divide="ignore", invalid="ignore"):
            t = z2 / (d[None, :] - lam[:, None])
        return 1.0 + np.sum(np.where(z2 == 0.0, 0.0, t), axis=1)

    # smallest eigenvalue: unique root in (d[0], d[1]); geometric bisection
    hi = np.full(c, d[1])
    lo = np.full(c, d[1] * 2.0 ** -200)
    singular = phi(lo) >= 0.0
    for _ in range(280):
        mid = np.where(lo > 0, np.sqrt(lo * hi), 0.5 * (lo + hi))
        neg = phi(mid) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    lam_min = 0.5 * (lo + hi)
    # largest eigenvalue: unique root in (d[-1], d[-1] + |z|^2)
    lo = np.full(c, d[-1])
    hi = d[-1] + np.sum(z2, axis=1) * (1 + 1e-12) + 1e-300
    for _ in range(120):
        mid = 0.5 * (lo + hi)
        neg = phi(mid) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    lam_max = 0.5 * (lo + hi)
    kap = np.sqrt(lam_max / lam_min)
    kap[singular] = np.inf
    return kap


def numerators_greedy(L: int, method: str = "secular", return_kappa: bool = False):
    """Condition-number-minimising greedy placement (Sec. III-D)."""
    if method not in ("svd", "secular"):
        raise ValueError(method)
    allnum = numerators_equiangular(L)
    trig = trig_from_numerators(L, allnum)
    chosen = np.zeros(L, dtype=np.int64)
    kap_out = np.zeros(L)
    chosen[L - 1] = 2 * ((L - 1) // 2) + 1
    kap_out[L - 1] = 1.0
    used = np.zeros(L, dtype=bool)
    used[(chosen[L - 1] - 1) // 2] = True
    for m in range(L - 2, -1, -1):
        rows = _order_rows(L, m, trig)  # (L, n): one row per member of Theta
        fixed = rows[(chosen[m + 1:] - 1) // 2]
        cand = np.nonzero(~used)[0]  # ascending numerators
        cr = rows[cand]
        kap = _kappa_svd(fixed, cr) if method == "svd" else _kappa_secular(fixed, cr)
        kmin = np.min(kap)
        tied = np.nonzero(kap <= kmin * (1.0 + TIE_RTOL))[0]
        pick = cand[tied[0]]
        chosen[m] = allnum[pick]
        kap_out[m] = kap[tied[0]]
        used[pick] = True
    if return_kappa:
        return chosen, kap_out
    return chosen


def kappas(L: int, num) -> np.ndarray:
    """kappa_m = cond_2(P_m) for m = 0..L-1 for a given placement."""
    trig = trig_from_numerators(L, num)
    out = np.empty(L)
    for m in range(L):
        P = scalar_table(L, m, trig["cos"][m:], trig["sin"][m:]).T  # rows k >= m
        out[m] = np.linalg.cond(P, 2)
    return out
