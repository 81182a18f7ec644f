"""Write oracle samples of the inverse at L = 2048 on selected rings for the
GPU parity tests (the oracle's per-ring evaluation takes minutes per ring
set at this band-limit).  Calls only oracle/ and the seeded generators.

    python tests/golden/make_parity_L2048.py

Input: map 0 of flm = inputs.coeffs(2048, 2, seed=4, weighted=True,
spin=s), i.e. (N(0,1) + i N(0,1)) (1+l)^-1 zeroed for l < |s|, for s = 0
and s = 2, on the greedy placement of tests/golden/theta_greedy_L2048.txt.
Rings (Eq. f_inverse_SHT evaluated ring by ring, oracle.sht.inverse_rings):
* the ring whose colatitude numerator is nearest 370 (theta ~ 0.284, where
  the Legendre seeds of orders m ~ 560 fall far below the FP64 range and the
  recursion must rescale, Sec. III-F);
* the ring nearest the north pole (numerator 1) and ring 0 at the south
  pole (theta = pi);
* the equator ring (numerator 2047): every 8th sample.
Files inverse_L2048_s{s}_seed4.txt: '#' header lines (recipe, max |f| over
the stored rings), then "ring j re im" per stored sample.
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

L = 2048


def golden_theta():
    return np.asarray([int(x) for x in open(os.path.join(HERE, f"theta_greedy_L{L}.txt")) if not x.startswith("#")])


def rings(num):
    return [int(np.argmin(np.abs(num - 370))), int(np.argmin(num)), 0, int(np.argmin(np.abs(num - 2047)))]


def main(spins):
    num = golden_theta()
    rs = rings(num)
    for s in spins:
        t0 = time.time()
        op = sht.Plan(L, s, numerators=num)
        flm = inputs.coeffs(L, 2, seed=4, weighted=True, spin=s)[:1]
        out = sht.inverse_rings(op, flm, rs)
        den = max(np.max(np.abs(v)) for v in out.values())
        path = os.path.join(HERE, f"inverse_L2048_s{s}_seed4.txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle inverse_rings, map 0 of inputs.coeffs(2048, 2, seed=4, weighted=True, spin={s})\n")
            fh.write(f"# rings {' '.join(str(r) for r in rs)} (numerators {' '.join(str(int(num[r])) for r in rs)})\n")
            fh.write(f"# max_abs {den:.17e}\n")
            for r in rs:
                step = 8 if r == rs[-1] else 1
                for j in range(0, 2 * r + 1, step):
                    v = out[r][0, j]
                    fh.write(f"{r} {j} {v.real:.17e} {v.imag:.17e}\n")
        print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0, 2])
