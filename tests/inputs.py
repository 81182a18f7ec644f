"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and bench.py.  Holds no arithmetic of the transform itself: only random
draws, the (1+l)^-1 weighting of the workloads, and index bookkeeping.

Recipes (numpy.random.default_rng, PCG64):
* coefficients: standard_normal((B, L*L, 2)) -> re + i im, in the l-major
  order idx = l*l + l + m; optionally divided by (1 + l); entries with
  l < |s| set to zero for spin s.
* samples: uniform(-1, 1) real and imaginary parts, shape (B, L*L).
* batched uneven workload: Ls = rng.choice([64,128,256,512], n), then
  spins = rng.choice([0, 2, -2], n), then one coefficient draw per map in
  map order, all from the same generator.
"""

import numpy as np


def degree_of_index(L):
    return np.repeat(np.arange(L), 2 * np.arange(L) + 1)


def coeffs(L, B=1, seed=0, weighted=False, spin=0, rng=None):
    rng = np.random.default_rng(seed) if rng is None else rng
    x = rng.standard_normal((B, L * L, 2))
    flm = x[..., 0] + 1j * x[..., 1]
    ell = degree_of_index(L)
    if weighted:
        flm = flm / (1.0 + ell)[None, :]
    if spin:
        flm[:, ell < abs(spin)] = 0.0
    return flm


def samples_uniform(L, B=1, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (B, L * L)) + 1j * rng.uniform(-1, 1, (B, L * L))


def uneven_batch(n=64, seed=2, Ls=(64, 128, 256, 512), spins=(0, 2, -2)):
    rng = np.random.default_rng(seed)
    Lsel = rng.choice(np.asarray(Ls), n)
    ssel = rng.choice(np.asarray(spins), n)
    maps = [coeffs(int(L), 1, spin=int(s), rng=rng)[0] for L, s in zip(Lsel, ssel)]
    return [int(v) for v in Lsel], [int(v) for v in ssel], maps
