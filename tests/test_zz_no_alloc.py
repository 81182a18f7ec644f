"""osht_inverse_noalloc against osht_inverse through the C ABI: the entry
point that keeps its workspace in the library's static per-device scratch
array must give the same bits as the plan-workspace inverse, on two calls in
a row (the second with a smaller batch and band-limit, so the array holds the
first call's data when the second starts), on FP64 and FP32 plans, and must
refuse a size beyond its array."""

import ctypes

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _call(fn, plan, x, y):
    import torch
    from paper_1403_4661_amd import lib
    stream = torch.cuda.current_stream().cuda_stream
    return getattr(lib(), fn)(plan._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.shape[0],
                              ctypes.c_void_p(stream))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inverse_noalloc_matches_inverse(precision):
    import torch
    from paper_1403_4661_amd import Plan

    cases = [(512, 0, 12, 31), (96, 2, 5, 32), (64, 0, 2, 33)]
    for L, s, B, seed in cases:
        p = Plan(L, s, precision=precision)
        x = to_dev(inputs.coeffs(L, B, seed=seed, spin=s))
        ref, out = torch.empty_like(x), torch.full_like(x, float("nan"))
        assert _call("osht_inverse", p, x, ref) == 0
        assert _call("osht_inverse_noalloc", p, x, out) == 0
        assert np.array_equal(to_host(out), to_host(ref)), (L, s, B)


def test_inverse_noalloc_not_on_int8_digit_plans():
    import torch
    from paper_1403_4661_amd import Plan

    p = Plan(32, 0, precision="i8x6")
    x = torch.zeros((1, 32 * 32), dtype=torch.complex128, device="cuda")
    assert _call("osht_inverse_noalloc", p, x, torch.empty_like(x)) == -5


def test_inverse_noalloc_rejects_oversize():
    import torch
    from paper_1403_4661_amd import Plan

    p = Plan(256, 0)
    x = torch.zeros((52, 256 * 256), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    assert _call("osht_inverse_noalloc", p, x, y) == -1
    assert _call("osht_inverse_noalloc", p, x[:51].contiguous(), y[:51].contiguous()) == 0
