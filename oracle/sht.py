"""Forward and inverse SHT on the L^2-sample scheme, their adjoints, and the
dense sampled-harmonic matrix (oracle, FP64, CPU).

Conventions (the paper fixes the geometry but not the array layout):
* coefficients: flm[b, l*l + l + m] for 0 <= l < L, |m| <= l (l-major);
* samples: f[b, k*k + j] is ring k (colatitude theta_k, Sec. III-A) at
  longitude phi_j = 2 pi j/(2k+1), j = 0..2k;
* spin s: coefficients with l < |s| do not exist and are held at zero.

Normalisation: the paper's G_m and P_m carry a common factor 2 pi
(Eq. gm_integral, Eq. Y_matrix) that cancels between the two directions.
This module works with G'_m = G_m/(2 pi) and P'_m = P_m/(2 pi), so that
    G'_m(theta_k) = (1/n_k) sum_j f(theta_k, phi_j) e^{-i m phi_j}
                  = sum_{l >= l0} flm[l, m] sPt[l, m](theta_k),
    A_m[k, i]     = sPt[l0 + i, m](theta_k),       l0 = max(|m|, |s|),
and P'_m is the block of rows k >= |m| of A_m.

What each function follows:
* inverse: Eq. f_inverse_SHT / Procedure 2 -- per order, G'_m on every ring
  from Eq. gm_integral, then f = sum_m G'_m(theta) e^{i m phi}, taken on each
  ring by folding order m into DFT bin (m mod n_k) and one inverse DFT.
* forward: block back-substitution in the sample domain.  The sampled
  harmonic matrix is block triangular in descending |m|: ring k only sees
  orders |m| <= k exactly, and orders above k alias into it.  So the orders
  are recovered from the highest down.  When order |m| is reached, ring |m|
  carries no higher order any more, its (2|m|+1)-point DFT is exact, and the
  rings above it were made clean earlier (reading of "(2m+1)-point FFT along
  each ring": every ring's own DFT, taken once it is clean).  Their bins
  m mod n_k give g'_{+-m} (Eq. gm_integral), the order-m system of Eq.
  gtof_inverse gives f_{+-m} (LU; least squares through the pseudo-inverse
  when |m| < |s|, where P'_m has L-|m| rows and L-|s| unknowns), and the
  order's field on the lower rings k < |m| (Eq. signal_subset) is
  subtracted from their samples (Eq. signal_update).
* inverse_adjoint / forward_adjoint: conjugate transposes with respect to the
  plain Euclidean inner products on C^{L^2} (the paper has no adjoints; the
  forward adjoint is the transpose of the Fourier-domain form of Procedure 1,
  which equals the spatial form in exact arithmetic).  Pinned by the dense
  matrices below and by dot-product tests.
* dense_Y: Y[(k, j), (l, m)] = sPt[l, m](theta_k) e^{i m phi_j} (tiny L).
* error metrics: Eqs. exp1:errors:max/mean and exp2:errors:max/mean.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .legendre import scalar_table, spin_table
from .sampling import numerators_alternating, numerators_greedy, trig_from_numerators

__all__ = [
    "Plan",
    "inverse",
    "forward",
    "inverse_adjoint",
    "forward_adjoint",
    "inverse_rings",
    "dense_Y",
    "coeff_index",
    "ring_geometry",
    "e_max",
    "e_mean",
    "relmax",
]


def coeff_index(L: int, s: int = 0):
    """(l, m, idx) arrays over all L^2 coefficients, idx = l*l + l + m."""
    ell = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    idx = np.arange(L * L)
    m = idx - ell * ell - ell
    return ell, m, idx


def ring_geometry(L: int):
    """(ring, j, n) arrays over all L^2 samples (ring-major layout)."""
    ring = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    j = np.arange(L * L) - ring * ring
    return ring, j, 2 * ring + 1


class Plan:
    """Geometry and per-order tables of one (L, spin) transform."""

    def __init__(self, L: int, spin: int = 0, numerators=None, placement: str = "greedy",
                 cache_bytes: float = 2e9):
        if L < 1:
            raise ValueError("L must be >= 1")
        if abs(spin) >= L:
            raise ValueError("|spin| must be < L")
        self.L = int(L)
        self.s = int(spin)
        if numerators is None:
            if placement == "greedy":
                numerators = numerators_greedy(L)
            elif placement == "alternating":
                numerators = numerators_alternating(L)
            else:
                raise ValueError(placement)
        self.num = np.asarray(numerators, dtype=np.int64)
        if sorted(self.num.tolist()) != list(range(1, 2 * L, 2)):
            raise ValueError("numerators must be a permutation of 1, 3, .., 2L-1")
        self.trig = trig_from_numerators(L, self.num)
        self.theta = math.pi * self.num / (2 * L - 1)
        entries = L * L * (L + 1) / 2 * (1 if spin == 0 else 2)
        self._cache = {} if entries * 8 * 1.7 <= cache_bytes else None
        self._solvers = {}

    def l0(self, m: int) -> int:
        return max(abs(m), abs(self.s))

    def orders(self):
        return range(-(self.L - 1), self.L)

    def table(self, m: int) -> np.ndarray:
        """A_m: shape (L, L - l0); A_m[k, i] = sPt[l0 + i, m](theta_k)."""
        key = m if self.s else abs(m)
        if self._cache is not None and key in self._cache:
            base = self._cache[key]
        else:
            if self.s == 0:
                base = scalar_table(self.L, abs(m), self.trig["cos"], self.trig["sin"]).T
            else:
                base = spin_table(self.L, m, self.s, self.trig).T
            if self._cache is not None:
                self._cache[key] = base
        if self.s == 0 and m < 0 and (abs(m) % 2):
            return -base
        return base

    def _solver(self, m: int):
        """Factorisation of P'_m (LU when square, pseudo-inverse otherwise)."""
        key = m if self.s else abs(m)
        if key in self._solvers:
            kind, fac = self._solvers[key]
        else:
            A = self.table(key)
            P = A[abs(key):, :]
            if P.shape[0] == P.shape[1]:
                kind, fac = "lu", sla.lu_factor(P)
            else:
                kind, fac = "pinv", np.linalg.pinv(P)
            if self._cache is not None:
                self._solvers[key] = (kind, fac)
        sign = -1.0 if (self.s == 0 and m < 0 and abs(m) % 2) else 1.0
        return kind, fac, sign

    def solve(self, m: int, g):
        """f_m = P'_m^{-1} g (rows of g are maps)."""
        kind, fac, sign = self._solver(m)
        if kind == "lu":
            return sign * sla.lu_solve(fac, g.T).T
        return sign * (g @ fac.T)

    def solve_adjoint(self, m: int, fbar):
        """gbar = P'_m^{-H} fbar (pseudo-inverse transpose when |m| < |s|)."""
        kind, fac, sign = self._solver(m)
        if kind == "lu":
            return sign * sla.lu_solve(fac, fbar.T, trans=1).T
        return sign * (fbar @ fac)


def _as_batch(x, L):
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[None, :]
    if x.shape[-1] != L * L:
        raise ValueError(f"expected last dimension L^2 = {L * L}")
    return x.astype(np.complex128)


def inverse(plan: Plan, flm) -> np.ndarray:
    """Samples f[b, k^2 + j] from coefficients (Procedure 2)."""
    L = plan.L
    flm = _as_batch(flm, L)
    B = flm.shape[0]
    G = np.zeros((L, 2 * L - 1, B), dtype=np.complex128)  # G'[k, m + L - 1, b]
    for m in plan.orders():
        l0 = plan.l0(m)
        ell = np.arange(l0, L)
        G[:, m + L - 1, :] = plan.table(m) @ flm[:, ell * ell + ell + m].T
    f = np.empty((B, L * L), dtype=np.complex128)
    ms = np.arange(-(L - 1), L)
    for k in range(L):
        n = 2 * k + 1
        H = np.zeros((n, B), dtype=np.complex128)
        np.add.at(H, ms % n, G[k])
        f[:, k * k:k * k + n] = n * np.fft.ifft(H.T, axis=1)
    return f


def inverse_rings(plan: Plan, flm, rings) -> dict:
    """Samples of the selected rings only, straight from Eq. f_inverse_SHT
    (tables evaluated at those colatitudes only); returns {k: (B, 2k+1)}."""
    L = plan.L
    flm = _as_batch(flm, L)
    rings = np.asarray(sorted(set(int(r) for r in rings)))
    sub = {key: val[rings] for key, val in plan.trig.items()}
    out = {}
    G = np.zeros((rings.size, 2 * L - 1, flm.shape[0]), dtype=np.complex128)
    for m in plan.orders():
        l0 = plan.l0(m)
        ell = np.arange(l0, L)
        if plan.s == 0:
            T = scalar_table(L, abs(m), sub["cos"], sub["sin"]).T
            if m < 0 and abs(m) % 2:
                T = -T
        else:
            T = spin_table(L, m, plan.s, sub).T
        G[:, m + L - 1, :] = T @ flm[:, ell * ell + ell + m].T
    ms = np.arange(-(L - 1), L)
    for i, k in enumerate(rings):
        n = 2 * k + 1
        H = np.zeros((n, flm.shape[0]), dtype=np.complex128)
        np.add.at(H, ms % n, G[i])
        out[int(k)] = n * np.fft.ifft(H.T, axis=1)
    return out


def _clean_ring_spectrum(work, k):
    """(1/n_k) DFT of ring k's samples (exact once no order above k remains)."""
    n = 2 * k + 1
    return np.fft.fft(work[:, k * k:k * k + n], axis=1) / n


def _order_field_on_lower_rings(plan: Plan, m: int, fm, geometry):
    """Samples of order m's part of the signal, sum_l f_lm Y_lm, on rings
    k < |m| (Eq. signal_subset), in ring-major order."""
    ring, jj, nn = geometry
    am = abs(m)
    ns = am * am
    g = fm @ plan.table(m)[:am, :].T  # G'_m(theta_k), k < |m|
    phase = np.exp(2j * math.pi * ((m * jj[:ns]) % nn[:ns]) / nn[:ns])
    return g[:, ring[:ns]] * phase[None, :]


def forward(plan: Plan, f) -> np.ndarray:
    """Coefficients from samples by sample-domain block back-substitution in
    descending |m| (Eqs. gm_integral, gtof_inverse, signal_subset and
    signal_update; see the module docstring)."""
    L = plan.L
    work = _as_batch(f, L).copy()
    B = work.shape[0]
    flm = np.zeros((B, L * L), dtype=np.complex128)
    geometry = ring_geometry(L)
    spectra = {}
    for am in range(L - 1, -1, -1):
        spectra[am] = _clean_ring_spectrum(work, am)
        for m in sorted({am, -am}, reverse=True):
            g = np.stack([spectra[k][:, m % (2 * k + 1)] for k in range(am, L)], axis=1)
            fm = plan.solve(m, g)
            ell = np.arange(plan.l0(m), L)
            flm[:, ell * ell + ell + m] = fm
            if am > 0:
                work[:, :am * am] -= _order_field_on_lower_rings(plan, m, fm, geometry)
    return flm


def inverse_adjoint(plan: Plan, fbar) -> np.ndarray:
    """Y^H fbar: per-ring unnormalised analysis DFT, unfold, A_m^T."""
    L = plan.L
    fbar = _as_batch(fbar, L)
    B = fbar.shape[0]
    D = [np.fft.fft(fbar[:, k * k:k * k + 2 * k + 1], axis=1) for k in range(L)]
    out = np.zeros((B, L * L), dtype=np.complex128)
    for m in plan.orders():
        l0 = plan.l0(m)
        ell = np.arange(l0, L)
        Gm = np.stack([D[k][:, m % (2 * k + 1)] for k in range(L)], axis=1)  # (B, L)
        out[:, ell * ell + ell + m] = Gm @ plan.table(m)
    return out


def forward_adjoint(plan: Plan, ybar) -> np.ndarray:
    """forward^H ybar: the transpose of the Fourier-domain form of Procedure 1
    (ascending |m|), followed by the adjoint of the normalised ring DFT."""
    L = plan.L
    ybar = _as_batch(ybar, L)
    B = ybar.shape[0]
    Hbar = [np.zeros((B, 2 * k + 1), dtype=np.complex128) for k in range(L)]
    for am in range(L):
        for m in ((am, -am) if am else (0,)):
            l0 = plan.l0(m)
            ell = np.arange(l0, L)
            fbar_m = ybar[:, ell * ell + ell + m].copy()
            A = plan.table(m)
            if am > 0:
                u = np.stack([Hbar[k][:, m % (2 * k + 1)] for k in range(am)], axis=1)
                fbar_m -= u @ A[:am, :]
            gbar = plan.solve_adjoint(m, fbar_m)  # (B, L - am)
            for i, k in enumerate(range(am, L)):
                Hbar[k][:, m % (2 * k + 1)] = gbar[:, i]
    out = np.empty((B, L * L), dtype=np.complex128)
    for k in range(L):
        out[:, k * k:k * k + 2 * k + 1] = np.fft.ifft(Hbar[k], axis=1)
    return out


def dense_Y(plan: Plan) -> np.ndarray:
    """Dense L^2 x L^2 sampled-harmonic matrix (columns l < |s| are zero)."""
    L = plan.L
    ring, jj, nn = ring_geometry(L)
    phi = 2 * math.pi * jj / nn
    Y = np.zeros((L * L, L * L), dtype=np.complex128)
    for m in plan.orders():
        l0 = plan.l0(m)
        A = plan.table(m)  # (L, L - l0)
        for i, ell in enumerate(range(l0, L)):
            Y[:, ell * ell + ell + m] = A[ring, i] * np.exp(1j * m * phi)
    return Y


def e_max(a, b) -> float:
    """Eqs. exp1:errors:max / exp2:errors:max: max |a - b|."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def e_mean(a, b) -> float:
    """Eqs. exp1:errors:mean / exp2:errors:mean: mean |a - b| over the L^2 entries."""
    d = np.abs(np.asarray(a) - np.asarray(b))
    return float(np.mean(d))


def relmax(a, b) -> float:
    """max |a - b| / max |b| (per call, over all entries)."""
    b = np.asarray(b)
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(np.asarray(a) - b))) / (den if den > 0 else 1.0)
