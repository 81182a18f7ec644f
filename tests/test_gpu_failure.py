"""Failure detection on the device path.

* Singular placements: the alternating placement (Eq. sampling_latitude) makes
  some P_m numerically singular from L = 128 up (cond ~1e18 at L = 256), so
  plan creation must fail with OSHT_ESINGULAR instead of producing a plan;
  below that it converges (the paper's "order 10^2" conditioning at L ~ 47).
* Unstable spin forward (Sec. III-G; the order-by-order chain amplifies
  rounding for spin +-2 beyond L ~ 9): the plan-time FP64 self-check
  forward(inverse(a)) - a flags it, and forward-direction calls are refused
  (OSHT_ENOTSUP) unless the plan forces them.
* Non-finite outputs: OSHT_CHECK_FINITE plans record NaN / Inf outputs in a
  sticky status, also through the batch scheduler.
* Batch-size changes: descriptor tables kept per batch size give the same
  results as a fresh plan when sizes alternate, including past the table
  cache's capacity.
"""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

ESINGULAR, ENOTSUP, ENONFINITE, OK = -4, -5, -7, 0


@pytest.mark.parametrize("L", [128, 256])
def test_alternating_placement_is_rejected_as_singular(L):
    from paper_1403_4661_amd import OshtError, Plan
    with pytest.raises(OshtError) as e:
        Plan(L, 0, placement="alternating")
    assert e.value.code == ESINGULAR


def test_alternating_placement_small_L_converges():
    from paper_1403_4661_amd import Plan
    p = Plan(47, 0, placement="alternating")
    info = p.info()
    assert info["max_inv_residual"] <= 1e-10
    # the paper quotes cond(P_m) "of the order 10^2" at L ~ 47 for this placement
    assert 1e2 <= info["max_kappa"] < 1e4
    flm = inputs.coeffs(47, 1, seed=3)
    assert relmax(to_host(p.forward(p.inverse(to_dev(flm)))), flm) < 1e-9


@pytest.mark.parametrize("L", [32, 256])
def test_spin0_self_check_is_at_rounding_level(L):
    from paper_1403_4661_amd import Plan
    info = Plan(L, 0).info()
    assert info["fwd_unstable"] == 0
    assert info["fwd_check_err"] < 1e-12


@pytest.mark.parametrize("s", [2, -2])
def test_spin_forward_stable_at_small_L(s):
    from paper_1403_4661_amd import Plan
    p = Plan(8, s)
    info = p.info()
    assert info["fwd_unstable"] == 0 and info["fwd_check_err"] < 1e-8
    flm = inputs.coeffs(8, 2, seed=5, spin=s)
    assert relmax(to_host(p.forward(p.inverse(to_dev(flm)))), flm) < 1e-8


@pytest.mark.parametrize("s", [2, -2])
def test_spin_forward_unstable_is_refused(s):
    import torch
    from paper_1403_4661_amd import OshtError, Plan, batch_run

    L = 16
    p = Plan(L, s)
    info = p.info()
    assert info["fwd_unstable"] == 1 and info["fwd_check_err"] > 1e-8
    flm = to_dev(inputs.coeffs(L, 2, seed=6, spin=s))
    f = p.inverse(flm)  # the inverse is unaffected
    for call in (p.forward, p.forward_adjoint):
        with pytest.raises(OshtError) as e:
            call(f)
        assert e.value.code == ENOTSUP
    out = torch.empty_like(f)
    with pytest.raises(OshtError) as e:
        batch_run([(p, "forward", f, out)])
    assert e.value.code == ENOTSUP
    # forcing runs the chain; its error is the method's, of the size the
    # self-check reported
    q = Plan(L, s, force_spin_forward=True)
    assert q.info()["fwd_unstable"] == 1
    back = to_host(q.forward(q.inverse(flm)))
    assert np.all(np.isfinite(back))
    assert relmax(back, to_host(flm)) > 1e-8


def test_check_finite_records_nan_and_inf():
    import torch
    from paper_1403_4661_amd import Plan, batch_run

    L = 32
    p = Plan(L, 0, check_finite=True)
    flm = to_dev(inputs.coeffs(L, 2, seed=1))
    f = p.inverse(flm)
    assert p.status() == OK
    bad = flm.clone()
    bad[1, 17] = complex(float("nan"), 0.0)
    p.inverse(bad)
    assert p.status() == ENONFINITE
    assert p.status() == OK  # cleared by the read
    fs = f.clone()
    fs[0, 5] = complex(0.0, float("inf"))
    p.forward(fs)
    assert p.status() == ENONFINITE
    out = torch.empty_like(f)
    batch_run([(p, "inverse", bad, out)])
    assert p.status() == ENONFINITE
    batch_run([(p, "inverse", flm, out)])
    assert p.status() == OK
    # without the flag the status stays OK
    q = Plan(L, 0)
    q.inverse(bad)
    assert q.status() == OK


def test_alternating_batch_sizes_match_fresh_plan():
    """Batch sizes 1, 3, 1, 3, then ten distinct sizes (past the table
    cache's capacity), then 3 again: every result equals the one of a plan
    that only ever saw that batch size."""
    from paper_1403_4661_amd import Plan

    L = 40
    p = Plan(L, 0)
    sizes = [1, 3, 1, 3] + list(range(2, 12)) + [3]
    for i, B in enumerate(sizes):
        flm = inputs.coeffs(L, B, seed=100 + i)
        x = to_dev(flm)
        ref_plan = Plan(L, 0)
        fi, ri = p.inverse(x), ref_plan.inverse(x)
        assert np.array_equal(to_host(fi), to_host(ri)), B
        assert np.array_equal(to_host(p.forward(fi)), to_host(ref_plan.forward(ri))), B
