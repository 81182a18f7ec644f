"""Parity at the headline size, in the launch configuration bench.py times.

Workload: spin 0, L = 1024, batch 16, flm ~ (N(0,1) + i N(0,1)) (1+l)^-1 from
seed 5 (the bench's input), one call per direction on the default plan
(greedy placement, b = 48 forward blocks, dense in-block alias solve).

- Inverse, every precision: rings 0, 1, 511, 512 and 1023 of maps 0 and 15
  against the oracle's ring-by-ring evaluation of the inverse definition
  (each ring on its own, from the per-order tables at that colatitude).
- Forward against the oracle: map 0's samples are replaced by the oracle's
  own inverse of map 0 (computed on the host, seconds), the batch of 16 is
  transformed, and map 0's coefficients are compared with the oracle's
  forward of the same samples at 1088 stored entries (every l < 8 plus 1024
  seeded indices; tests/golden/forward_L1024_seed5.txt, written by
  tests/golden/make_parity_L1024.py, which calls only the oracle).  Relative
  to max |flm| over the whole output: FP64 <= 1e-11, FP32 modes <= 1e-6.
- Forward, every map: the forward of band-limited samples returns their
  coefficients (a property that holds at any size).  The samples come from
  the FP64 plan's inverse, itself pinned to the oracle above; the expected
  value is the input flm.  FP64: <= 1e-11 (the method's FP64 floor for this
  input is ~1.6e-12).  FP32 modes: <= 1e-6.
"""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import oracle_plan, read_golden_values, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

L, B, SEED = 1024, 16, 5
RINGS = [0, 1, 511, 512, 1023]
MAPS = [0, 15]
PRECISIONS = ["fp64", "fp32", "fp32-fwd", "i8x6", "i8x8", "fwd32"]
TOL = {"fp64": 1e-11, "fp32": 1e-6, "fp32-fwd": 1e-6, "i8x6": 1e-6, "i8x8": 1e-11, "fwd32": 1e-6}
# the inverse alone: the int8 digit splits are finer than FP32; fwd32 runs
# the FP64 inverse
TOL_INV = dict(TOL, i8x6=1e-8, fwd32=1e-11)

_cache = {}


def flm_host():
    if "flm" not in _cache:
        _cache["flm"] = inputs.coeffs(L, B, seed=SEED, weighted=True)
    return _cache["flm"]


def plan(precision):
    from paper_1403_4661_amd import Plan
    key = ("plan", precision)
    if key not in _cache:
        _cache[key] = Plan(L, 0, precision=precision)
    return _cache[key]


def oracle_rings():
    if "rings" not in _cache:
        from oracle import sht
        _cache["rings"] = sht.inverse_rings(oracle_plan(L), flm_host()[MAPS], RINGS)
    return _cache["rings"]


def fp64_samples():
    """The FP64 plan's inverse of the headline input, on the device."""
    if "f64" not in _cache:
        _cache["f64"] = plan("fp64").inverse(to_dev(flm_host()))
    return _cache["f64"]


@pytest.fixture(scope="module", autouse=True)
def _teardown():
    yield
    _cache.clear()
    import torch
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_headline_inverse_sampled_rings(precision):
    f = to_host(fp64_samples()) if precision == "fp64" else to_host(plan(precision).inverse(to_dev(flm_host())))
    ref = oracle_rings()
    err = 0.0
    for k, v in ref.items():
        got = f[MAPS, k * k:k * k + 2 * k + 1]
        err = max(err, relmax(got, v))
    assert err < TOL_INV[precision], err


def oracle_map0_samples():
    """The oracle's inverse of map 0 (the input of the stored oracle forward)."""
    if "f0" not in _cache:
        from oracle import sht
        _cache["f0"] = sht.inverse(oracle_plan(L), flm_host()[:1])
    return _cache["f0"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_headline_forward_vs_oracle_map0(precision):
    import torch
    head, rows = read_golden_values("forward_L1024_seed5.txt")
    idx = np.asarray([int(r[0]) for r in rows])
    ref = np.asarray([float(r[1]) + 1j * float(r[2]) for r in rows])
    f = fp64_samples().clone()
    f[0] = torch.as_tensor(oracle_map0_samples()[0]).to(f.device)
    g = to_host(plan(precision).forward(f))
    err = np.max(np.abs(g[0, idx] - ref)) / head["max_abs"]
    assert err < TOL[precision], err


@pytest.mark.parametrize("precision", PRECISIONS)
def test_headline_forward_returns_coefficients(precision):
    g = to_host(plan(precision).forward(fp64_samples()))
    assert relmax(g, flm_host()) < TOL[precision]


def test_headline_repeat_calls_bitwise():
    """Two calls on the same input give the same bits (fixed reduction orders)."""
    p = plan("fp32-fwd")
    f = fp64_samples()
    a, b = to_host(p.forward(f)), to_host(p.forward(f))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fwd32", "i8x6"])
def test_headline_round_trip_gate(precision):
    """Inverse then forward on one plan returns the headline input to
    <= 1e-6 (the gate bench.py applies to its headline path): the forward's
    FP32 coefficient rows alone stay well inside it."""
    back = to_host(plan(precision).forward(plan(precision).inverse(to_dev(flm_host()))))
    assert relmax(back, flm_host()) < 1e-6
