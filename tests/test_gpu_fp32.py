"""GPU parity of the FP32 precision modes against the FP64 oracle.

OSHT_PREC_FP32 ("fp32") applies A_m (inverse and its adjoint) with FP32
matrices on FP32 matrix cores (16-term FP32 slices summed in FP64);
OSHT_PREC_FP32_FWD ("fp32-fwd") also the forward's coefficient rows
P_m^{-1}.  The alias rows of Q_m, which feed the descending-order chain of
Procedure 1, the ring DFTs and all buffers stay FP64.  Tolerance: 1e-6 max
relative error, the bar for the mixed-precision path (an FP32 rounding of
6e-8 per matrix entry and per right-hand-side entry, amplified by the
conditioning of P_m)."""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import oracle_plan, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-6
_plans = {}


def plan32(L, s=0, precision="fp32"):
    from paper_1403_4661_amd import Plan
    if (L, s, precision) not in _plans:
        _plans[(L, s, precision)] = Plan(L, s, precision=precision)
    return _plans[(L, s, precision)]


_oplans = {}


def oplan(L, s=0):
    if (L, s) not in _oplans:
        _oplans[(L, s)] = oracle_plan(L, s)
    return _oplans[(L, s)]


def test_fp32_plan_memory_and_flags():
    from paper_1403_4661_amd import Plan
    p64, p32, p32f = Plan(64), plan32(64), plan32(64, 0, "fp32-fwd")
    assert p32.info()["flags"] & 0xF == 1 and p32f.info()["flags"] & 0xF == 2
    assert p32.info()["device_bytes"] < p64.info()["device_bytes"]
    # A_m moves to FP32; Q_m is held in FP32 and (for its alias rows) FP64
    assert p32.info()["device_bytes"] <= p64.info()["device_bytes"]


@pytest.mark.parametrize("L,B,s,weighted,seed", [(33, 3, 0, False, 3), (100, 17, 0, True, 5), (16, 2, 2, False, 6),
                                                 (21, 1, -1, False, 8)])
def test_fp32_inverse(L, B, s, weighted, seed):
    from oracle import sht
    flm = inputs.coeffs(L, B, seed=seed, weighted=weighted, spin=s)
    got = to_host(plan32(L, s).inverse(to_dev(flm)))
    assert relmax(got, sht.inverse(oplan(L, s), flm)) < TOL


@pytest.mark.parametrize("precision", ["fp32", "fp32-fwd"])
@pytest.mark.parametrize("L,B,weighted,seed", [(33, 3, False, 3), (100, 17, True, 5), (256, 2, True, 1)])
def test_fp32_forward(L, B, weighted, seed, precision):
    from oracle import sht
    op = oplan(L)
    flm = inputs.coeffs(L, B, seed=seed, weighted=weighted)
    f = sht.inverse(op, flm)
    got = to_host(plan32(L, 0, precision).forward(to_dev(f)))
    assert relmax(got, sht.forward(op, f)) < TOL
    assert relmax(got, flm) < TOL


@pytest.mark.parametrize("L,B", [(32, 2), (33, 3)])
def test_fp32_adjoints(L, B):
    from oracle import sht
    rng = np.random.default_rng(L)
    x = rng.standard_normal((B, L * L)) + 1j * rng.standard_normal((B, L * L))
    y = inputs.coeffs(L, B, seed=L)
    p = plan32(L)
    assert relmax(to_host(p.inverse_adjoint(to_dev(x))), sht.inverse_adjoint(oplan(L), x)) < TOL
    # the forward adjoint reads the FP64 copy of Q_m
    assert relmax(to_host(p.forward_adjoint(to_dev(y))), sht.forward_adjoint(oplan(L), y)) < 1e-10


@pytest.mark.parametrize("L,b", [(33, 1), (70, 7)])
def test_fp32_forward_block_sizes(L, b, monkeypatch):
    from oracle import sht
    from paper_1403_4661_amd import Plan
    monkeypatch.setenv("OSHT_FWD_BLOCK", str(b))
    p = Plan(L, 0, precision="fp32-fwd")
    flm = inputs.coeffs(L, 2, seed=L + b)
    f = sht.inverse(oplan(L), flm)
    got = to_host(p.forward(to_dev(f)))
    assert relmax(got, sht.forward(oplan(L), f)) < TOL
