"""Differentiation through the hand-written adjoints (torch.autograd.Function).

Workload: spin 0, L = 1024, batch 8; flm and t_lm ~ N(0,1)(1+l)^-1 drawn from
seed 3 (flm first), target = inverse(t_lm);
loss = sum over maps and samples of |inverse(flm) - target|^2.
The gradient convention for a real loss of complex inputs is
dloss/dRe + i dloss/dIm (torch's), which for f = Y flm is 2 Y^H (f - target).
Central finite differences with h = 1e-6 on the real and imaginary parts of
32 entries (rng.choice after the draws) check it; the loss is quadratic, so
the differences are exact up to rounding.  The adjoint kernels themselves are
compared with the oracle's adjoints at L = 128, where the oracle is quick, and
at L = 1024 on one map against oracle values stored at 1088 entries
(tests/golden/iadj_L1024_seed3.txt, fadj_L1024_seed3.txt, written by
tests/golden/make_parity_L1024.py from the oracle alone)."""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import oracle_plan, read_golden_values, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def _loss_diff(plan, xp, xm, target):
    """loss(xp) - loss(xm), summed term by term so that the O(1) parts of
    the two losses cancel before the sum."""
    fp, fm = plan.inverse(xp), plan.inverse(xm)
    return float(((fp - target).abs() ** 2 - (fm - target).abs() ** 2).sum())


def test_inverse_autograd_matches_finite_differences_L1024():
    import torch
    from paper_1403_4661_amd import InverseSHT, Plan

    L, B = 1024, 8
    rng = np.random.default_rng(3)
    flm_h = inputs.coeffs(L, B, weighted=True, rng=rng)
    t_h = inputs.coeffs(L, B, weighted=True, rng=rng)
    idx = rng.choice(B * L * L, 32, replace=False)
    plan = Plan(L, 0)
    target = plan.inverse(to_dev(t_h))
    flm = to_dev(flm_h).requires_grad_(True)
    f = InverseSHT.apply(plan, flm)
    loss = ((f - target).abs() ** 2).sum()
    loss.backward()
    grad = flm.grad.detach().reshape(-1).cpu().numpy()
    h = 1e-6
    base = to_dev(flm_h).reshape(-1)
    fd = np.zeros(len(idx), complex)
    for n, i in enumerate(idx):
        for part, unit in ((0, 1.0), (1, 1j)):
            xp, xm = base.clone(), base.clone()
            xp[i] += h * unit
            xm[i] -= h * unit
            d = _loss_diff(plan, xp.reshape(B, -1), xm.reshape(B, -1), target) / (2 * h)
            fd[n] += d if part == 0 else 1j * d
    g = grad[idx]
    scale = np.max(np.abs(g))
    assert scale > 0
    assert np.max(np.abs(fd - g)) / scale < 1e-5
    # the analytic form: 2 Y^H (f - target)
    ref = 2 * to_host(plan.inverse_adjoint((f.detach() - target).contiguous())).reshape(-1)
    assert np.max(np.abs(ref[idx] - g)) <= 1e-12 * scale


def test_forward_autograd_matches_adjoint():
    import torch
    from paper_1403_4661_amd import ForwardSHT, Plan
    from oracle import sht

    L, B = 64, 2
    plan = Plan(L, 0)
    rng = np.random.default_rng(4)
    f = to_dev(inputs.samples_uniform(L, B, seed=4)).requires_grad_(True)
    w = to_dev(rng.standard_normal((B, L * L)) + 1j * rng.standard_normal((B, L * L)))
    out = ForwardSHT.apply(plan, f)
    loss = (out * w.conj()).real.sum()  # Re<w, F f>: gradient is F^H w
    loss.backward()
    ref = sht.forward_adjoint(oracle_plan(L), to_host(w))
    assert relmax(f.grad.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("s", [0, 2])
def test_adjoints_vs_oracle_L128(s):
    from oracle import sht
    from paper_1403_4661_amd import Plan

    L, B = 128, 2
    plan = Plan(L, s)
    rng = np.random.default_rng(128 + s)
    x = rng.standard_normal((B, L * L)) + 1j * rng.standard_normal((B, L * L))
    op = oracle_plan(L, s)
    assert relmax(to_host(plan.inverse_adjoint(to_dev(x))), sht.inverse_adjoint(op, x)) < 1e-11
    if s == 0:
        y = inputs.coeffs(L, B, seed=7)
        assert relmax(to_host(plan.forward_adjoint(to_dev(y))), sht.forward_adjoint(op, y)) < 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_adjoints_vs_oracle_L1024(precision, tol):
    """Both adjoints at the differentiation workload's band-limit, one map:
    inverse adjoint of N(0,1) samples and forward adjoint of (1+l)^-1
    weighted coefficients (seed 3), against the stored oracle values.  The
    FP32 plan's inverse adjoint reads FP32 A_m; its forward adjoint is FP64."""
    from paper_1403_4661_amd import Plan

    L = 1024
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, L * L)) + 1j * rng.standard_normal((1, L * L))
    y = inputs.coeffs(L, 1, weighted=True, rng=rng)
    plan = Plan(L, 0, precision=precision)
    for name, fn, arg, t in (("iadj_L1024_seed3.txt", plan.inverse_adjoint, x, tol),
                             ("fadj_L1024_seed3.txt", plan.forward_adjoint, y, 1e-11)):
        head, rows = read_golden_values(name)
        idx = np.asarray([int(r[0]) for r in rows])
        ref = np.asarray([float(r[1]) + 1j * float(r[2]) for r in rows])
        got = to_host(fn(to_dev(arg)))[0]
        err = np.max(np.abs(got[idx] - ref)) / head["max_abs"]
        assert err < t, (name, err)
