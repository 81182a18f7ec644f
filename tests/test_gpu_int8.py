"""The inverse apply on int8 digit splits (OSHT_PREC_I8X6 / _I8X8): A_m and
the coefficients are written as 6 or 8 signed 7-bit digits under
power-of-two scales, the digit products are accumulated exactly by the int8
matrix cores, and the scaled sums are added in FP64.

Against the FP64 oracle, element by element (relative to max |f| of the
call): 6 digits <= 1e-8 (the split's error falls about 2^7 per digit; CPU
emulation gives 2e-10 at L = 256), 8 digits <= 1e-11 (the FP64 bar).  The
forward of an I8X6 plan runs the FP32_FWD forward (<= 1e-6), of an I8X8 plan
the FP64 one (<= 1e-11); the inverse adjoint reads FP64 A_m (<= 1e-12).
Shapes: tiny and ragged band-limits (tails of the 64-row, 64-column and
64-deep tiles), batches that leave the column tile partly empty, spin +-2
and -1 (both signs of m in their own slots), and bit-for-bit repeatability.
"""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import oracle_plan, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_INV = {"i8x6": 1e-8, "i8x8": 1e-11}
TOL_FWD = {"i8x6": 1e-6, "i8x8": 1e-11}
_plans, _oplans = {}, {}


def plan(L, s, precision):
    from paper_1403_4661_amd import Plan
    key = (L, s, precision)
    if key not in _plans:
        _plans[key] = Plan(L, s, precision=precision, force_spin_forward=s != 0)
    return _plans[key]


def oplan(L, s=0):
    if (L, s) not in _oplans:
        _oplans[(L, s)] = oracle_plan(L, s)
    return _oplans[(L, s)]


CASES = [(1, 1, 0, False, 1), (2, 2, 0, False, 2), (33, 3, 0, False, 3), (65, 2, 0, False, 4),
         (100, 17, 0, True, 5), (130, 5, 0, True, 6), (16, 2, 2, False, 7), (21, 1, -1, False, 8),
         (40, 3, -2, True, 9)]


@pytest.mark.parametrize("precision", ["i8x6", "i8x8"])
@pytest.mark.parametrize("L,B,s,weighted,seed", CASES)
def test_int8_inverse_matches_oracle(L, B, s, weighted, seed, precision):
    from oracle import sht
    flm = inputs.coeffs(L, B, seed=seed, weighted=weighted, spin=s)
    got = to_host(plan(L, s, precision).inverse(to_dev(flm)))
    assert relmax(got, sht.inverse(oplan(L, s), flm)) < TOL_INV[precision]


@pytest.mark.parametrize("precision", ["i8x6", "i8x8"])
@pytest.mark.parametrize("L,B,weighted,seed", [(33, 3, False, 3), (100, 17, True, 5)])
def test_int8_plan_forward_and_adjoint(L, B, weighted, seed, precision):
    from oracle import sht
    op = oplan(L)
    flm = inputs.coeffs(L, B, seed=seed, weighted=weighted)
    f = sht.inverse(op, flm)
    p = plan(L, 0, precision)
    assert relmax(to_host(p.forward(to_dev(f))), sht.forward(op, f)) < TOL_FWD[precision]
    assert relmax(to_host(p.inverse_adjoint(to_dev(f))), sht.inverse_adjoint(op, f)) < 1e-12


def test_int8_inverse_repeatable_and_zero_maps():
    """Fixed reduction order: repeated calls agree bit for bit; an all-zero
    map (exponent of an empty column) gives exact zeros beside a nonzero map."""
    import torch
    p = plan(65, 0, "i8x6")
    flm = inputs.coeffs(65, 3, seed=11)
    flm[1] = 0.0
    x = to_dev(flm)
    a, b = to_host(p.inverse(x)), to_host(p.inverse(x))
    assert np.array_equal(a, b)
    assert np.all(a[1] == 0.0)
    assert relmax(a[[0, 2]], __import__("oracle").sht.inverse(oplan(65), flm[[0, 2]])) < TOL_INV["i8x6"]


@pytest.mark.parametrize("L,B,seed", [(256, 4, 12), (1024, 2, 13)])
def test_int8_zero_steps_skip_bit_identical(L, B, seed, monkeypatch):
    """The digit rows are the rings sorted by sin(theta), and each 64-row
    tile starts its k loop at its first k-step holding a nonzero digit.  The
    steps it skips hold zero digits only, so the result equals that of the
    full k loop bit for bit (OSHT_OZ_KSKIP=0 builds a plan without the
    skip)."""
    from paper_1403_4661_amd import Plan
    x = to_dev(inputs.coeffs(L, B, seed=seed, weighted=True))
    p = Plan(L, 0, precision="i8x6")
    a = to_host(p.inverse(x))
    del p
    monkeypatch.setenv("OSHT_OZ_KSKIP", "0")
    q = Plan(L, 0, precision="i8x6")
    b = to_host(q.inverse(x))
    del q
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["i8x6", "fp64"])
def test_ring_cut_changes_only_rounding(precision, monkeypatch):
    """Orders whose Legendre values on a ring all lie below 2^-80 are left out
    of that ring's fold (and, on int8 plans, of the apply's row tiles).  What
    they would add is below FP64 resolution: the inverse agrees with a plan
    that keeps every order (OSHT_RING_CUT=0) to rounding, relative to max |f|."""
    from paper_1403_4661_amd import Plan
    L, B = 1024, 2
    x = to_dev(inputs.coeffs(L, B, seed=14, weighted=True))
    p = Plan(L, 0, precision=precision)
    a = to_host(p.inverse(x))
    del p
    monkeypatch.setenv("OSHT_RING_CUT", "0")
    q = Plan(L, 0, precision=precision)
    b = to_host(q.inverse(x))
    del q
    assert relmax(a, b) < 1e-14


def test_int8_round_trip_headline_size():
    """L = 1024, batch 16, headline input: inverse then forward on one I8X6
    plan returns the coefficients to <= 1e-6 (the FP32 inverse alone gives
    ~2.6e-5: the forward amplifies an inverse error ~250 times at this L)."""
    L, B = 1024, 16
    p = plan(L, 0, "i8x6")
    flm = inputs.coeffs(L, B, seed=5, weighted=True)
    back = to_host(p.forward(p.inverse(to_dev(flm))))
    assert relmax(back, flm) < 1e-6
    del _plans[(L, 0, "i8x6")]


def teardown_module(module):
    _plans.clear()
