"""Write the oracle's greedy colatitude placements (Sec. III-D) as integer
numerator files tests/golden/theta_greedy_L{L}.txt (theta_k = pi n_k/(2L-1)).

Calls only oracle/.  Usage: python tests/golden/make_theta.py 32 64 128 ...
Each file holds one numerator per line, ring k on line k, followed by a
comment line with the maximum condition number of the placement.
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sampling import numerators_greedy  # noqa: E402


def main(argv):
    for L in [int(a) for a in argv]:
        t0 = time.time()
        num, kap = numerators_greedy(L, method="secular", return_kappa=True)
        path = os.path.join(HERE, f"theta_greedy_L{L}.txt")
        with open(path, "w") as fh:
            fh.write("\n".join(str(int(n)) for n in num) + "\n")
            fh.write(f"# max_kappa {kap.max():.6e}\n")
        print(f"L={L} max_kappa={kap.max():.4g} seconds={time.time() - t0:.1f}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
