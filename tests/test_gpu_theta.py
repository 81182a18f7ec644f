"""Greedy placement computed on the device (Sec. III-D): osht_theta_greedy_device.

- For small L it equals the oracle's greedy (oracle.sampling), and for
  L = 32 ... 512 the golden placements, integer for integer (the golden files
  were written by the oracle and pinned there).
- Its cond_2(P_m) values agree with the host greedy's to 1e-9 relative (the
  two reduce S = B^T B to tridiagonal form by different Householder codes, so
  only rounding differs).
"""

import os

import numpy as np
import pytest

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="device greedy switched off: one run faulted the GPU (L = 5) with no cause found yet; "
                            "the entry point returns OSHT_ENOTSUP"),
]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(L):
    return [int(x) for x in open(os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")) if not x.startswith("#")]


@pytest.mark.parametrize("L", [1, 2, 5, 9, 16, 31])
def test_device_greedy_matches_oracle(L):
    from oracle.sampling import numerators_greedy
    from paper_1403_4661_amd import theta_greedy
    assert theta_greedy(L, device=True) == numerators_greedy(L).tolist()


@pytest.mark.parametrize("L", [32, 64, 128, 256, 512])
def test_device_greedy_matches_golden(L):
    from paper_1403_4661_amd import theta_greedy
    assert theta_greedy(L, device=True) == _golden(L)


def test_device_kappa_matches_host():
    from paper_1403_4661_amd import theta_greedy
    L = 96
    num_h, kap_h = theta_greedy(L, with_kappa=True)
    num_d, kap_d = theta_greedy(L, with_kappa=True, device=True)
    assert num_d == num_h
    kh, kd = np.array(kap_h), np.array(kap_d)
    assert np.all(np.isfinite(kd))
    assert np.max(np.abs(kd - kh) / kh) < 1e-9


def test_device_greedy_rejects_bad_arguments():
    import ctypes
    from paper_1403_4661_amd import lib
    assert lib().osht_theta_greedy_device(0, (ctypes.c_int32 * 1)(), None) == -1
    assert lib().osht_theta_greedy_device(4, None, None) == -1
