"""Write oracle values at the headline band-limit L = 1024 for the GPU parity
tests, which cannot run the FP64 oracle's forward there (minutes per map on
the host).  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_parity_L1024.py

Files (one value per line, "idx re im" with 17 significant digits, after
'#' header lines that give the recipe and max |value| over the whole
output, the denominator of the relative error):
* forward_L1024_seed5.txt: forward (Procedure 1, the oracle's sample-domain
  block back-substitution) of the samples f = inverse(flm) of map 0 of the
  headline input, flm ~ (N(0,1) + i N(0,1)) (1+l)^-1 from seed 5
  (Eq. f_inverse_SHT gives f; the test recomputes f with the oracle's
  inverse on the host, which takes seconds);
* iadj_L1024_seed3.txt: inverse adjoint Y^H x of x ~ N(0,1) + i N(0,1)
  samples, seed 3 (the adjoint the L = 1024, batch 8 differentiation
  workload back-propagates through);
* fadj_L1024_seed3.txt: forward adjoint Y^{-H} y of y ~ (N(0,1) + i N(0,1))
  (1+l)^-1 coefficients, seed 3 (after the draw of x).
Stored entries: every coefficient with l < 8, plus 1024 indices drawn with
numpy.random.default_rng(1024).choice(L*L, 1024, replace=False) (sorted);
for the inverse adjoint the same indices address coefficients, for the
forward adjoint they address samples.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import sht  # noqa: E402
from tests import inputs  # noqa: E402

L = 1024


def golden_theta(L):
    return [int(x) for x in open(os.path.join(HERE, f"theta_greedy_L{L}.txt")) if not x.startswith("#")]


def indices():
    rng = np.random.default_rng(1024)
    pick = rng.choice(L * L, 1024, replace=False)
    return np.unique(np.concatenate([np.arange(64), pick]))


def write(name, header, values, idx):
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        for line in header:
            fh.write(f"# {line}\n")
        fh.write(f"# max_abs {np.max(np.abs(values)):.17e}\n")
        for i in idx:
            v = values[i]
            fh.write(f"{int(i)} {v.real:.17e} {v.imag:.17e}\n")
    print("wrote", path, flush=True)


def main():
    op = sht.Plan(L, 0, numerators=golden_theta(L))
    idx = indices()
    t0 = time.time()
    flm = inputs.coeffs(L, 1, seed=5, weighted=True)
    f = sht.inverse(op, flm)
    g = sht.forward(op, f)[0]
    write("forward_L1024_seed5.txt",
          ["oracle forward of oracle inverse(flm), flm = inputs.coeffs(1024, 1, seed=5, weighted=True)",
           f"round trip max|g - flm|/max|flm| = {sht.relmax(g, flm[0]):.3e}"], g, idx)
    print(f"forward done in {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, L * L)) + 1j * rng.standard_normal((1, L * L))
    y = inputs.coeffs(L, 1, weighted=True, rng=rng)
    write("iadj_L1024_seed3.txt",
          ["oracle inverse_adjoint(x), x = N(0,1) + i N(0,1) samples from default_rng(3)"],
          sht.inverse_adjoint(op, x)[0], idx)
    write("fadj_L1024_seed3.txt",
          ["oracle forward_adjoint(y), y = inputs.coeffs(1024, 1, weighted=True) drawn after x from default_rng(3)"],
          sht.forward_adjoint(op, y)[0], idx)
    print(f"all done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
