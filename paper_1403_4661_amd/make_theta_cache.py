"""Writes the library's greedy colatitude placements (Sec. III-D) into
paper_1403_4661_amd/theta/theta_greedy_L<L>.txt, the cache that Plan() reads
by default.  Uses the library's own host greedy (osht_theta_greedy).

    python -m paper_1403_4661_amd.make_theta_cache 32 64 128 256 512 1024
"""

import os
import sys
import time

from . import THETA_CACHE_DIR, theta_greedy


def write(L):
    t0 = time.time()
    num, kap = theta_greedy(L, with_kappa=True)
    os.makedirs(THETA_CACHE_DIR, exist_ok=True)
    path = os.path.join(THETA_CACHE_DIR, f"theta_greedy_L{L}.txt")
    with open(path, "w") as fh:
        fh.write("\n".join(str(n) for n in num) + "\n")
        fh.write(f"# max_kappa {max(kap):.6e}\n")
    print(f"L={L} max_kappa={max(kap):.4g} seconds={time.time() - t0:.1f}", flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:]:
        write(int(a))
