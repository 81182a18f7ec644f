"""GPU parity: every transform of the HIP library against the FP64 oracle,
element by element, through the C ABI (via the thin Python binding)."""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import golden_theta, oracle_plan, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

_plans = {}


def gpu_plan(L, s=0, placement="greedy"):
    """Spin plans force their forward: these tests compare the kernels with
    the oracle running the same order-by-order chain, also where the
    plan-time self-check marks the chain unstable (tests/test_gpu_failure.py
    covers that gate)."""
    from paper_1403_4661_amd import Plan
    key = (L, s, placement)
    if key not in _plans:
        _plans[key] = Plan(L, s, placement=placement, force_spin_forward=s != 0)
    return _plans[key]


_oplans = {}


def oplan(L, s=0, placement="greedy"):
    key = (L, s, placement)
    if key not in _oplans:
        _oplans[key] = oracle_plan(L, s, placement)
    return _oplans[key]


def test_plan_basics_L32():
    p = gpu_plan(32)
    info = p.info()
    assert info["L"] == 32 and info["nsamples"] == 32 * 32 and info["ncoeffs"] == 32 * 32
    assert info["max_inv_residual"] < 1e-12
    assert info["fwd_unstable"] == 0 and info["fwd_check_err"] < 1e-13
    assert p.theta_numerators() == golden_theta(32).tolist()


# (L, B, spin, weighted, seed): config 1 first, then ragged tiles and edges
CASES = [
    (32, 1, 0, False, 0),
    (1, 1, 0, False, 1),
    (2, 2, 0, False, 2),
    (33, 3, 0, False, 3),
    (65, 2, 0, False, 4),
    (100, 17, 0, True, 5),
    (16, 2, 2, False, 6),
    (16, 2, -2, False, 7),
    (21, 1, 1, False, 8),
]


@pytest.mark.parametrize("L,B,s,weighted,seed", CASES)
def test_inverse_matches_oracle(L, B, s, weighted, seed):
    flm = inputs.coeffs(L, B, seed=seed, weighted=weighted, spin=s)
    ref = __import__("oracle").sht.inverse(oplan(L, s), flm)
    got = to_host(gpu_plan(L, s).inverse(to_dev(flm)))
    assert relmax(got, ref) < 1e-12


@pytest.mark.parametrize("L,B,s,weighted,seed", [c for c in CASES if c[2] == 0])
def test_forward_matches_oracle(L, B, s, weighted, seed):
    from oracle import sht
    op = oplan(L, s)
    f = sht.inverse(op, inputs.coeffs(L, B, seed=seed, weighted=weighted))
    ref = sht.forward(op, f)
    got = to_host(gpu_plan(L, s).forward(to_dev(f)))
    assert relmax(got, ref) < 1e-11


@pytest.mark.parametrize("L", [16, 33])
def test_forward_random_samples_matches_oracle(L):
    """Experiment 2 input: random samples are band-limited on this scheme."""
    from oracle import sht
    f = inputs.samples_uniform(L, 2, seed=L)
    ref = sht.forward(oplan(L), f)
    got = to_host(gpu_plan(L).forward(to_dev(f)))
    assert relmax(got, ref) < 1e-11


@pytest.mark.parametrize("s", [2, -2, 1])
def test_spin_forward_small_L(s):
    """Spin forward (Sec. III-G) at L = 6, where the order-wise elimination is
    still accurate.  At larger L it is unstable on this scheme in FP64, in the
    oracle and on the GPU alike: its error grows by orders of magnitude per
    few degrees, and plans refuse the spin forward once their self-check
    fails."""
    from oracle import sht
    L = 6
    flm = inputs.coeffs(L, 2, seed=11, spin=s)
    f = sht.inverse(oplan(L, s), flm)
    ref = sht.forward(oplan(L, s), f)
    got = to_host(gpu_plan(L, s).forward(to_dev(f)))
    assert relmax(got, ref) < 1e-10
    assert relmax(got, flm) < 1e-9


@pytest.mark.parametrize("L,B,s", [(32, 2, 0), (33, 3, 0), (17, 2, 2), (12, 1, -1)])
def test_adjoints_match_oracle(L, B, s):
    from oracle import sht
    rng = np.random.default_rng(L + 100 * abs(s) + (s < 0))
    x = rng.standard_normal((B, L * L)) + 1j * rng.standard_normal((B, L * L))
    y = inputs.coeffs(L, B, seed=L, spin=s)
    p = gpu_plan(L, s)
    ia = to_host(p.inverse_adjoint(to_dev(x)))
    assert relmax(ia, sht.inverse_adjoint(oplan(L, s), x)) < 1e-12
    if s == 0 or L <= 12:
        fa = to_host(p.forward_adjoint(to_dev(y)))
        assert relmax(fa, sht.forward_adjoint(oplan(L, s), y)) < 1e-10
    # dot-product identities on the GPU results themselves
    inv_y = to_host(p.inverse(to_dev(y)))
    assert abs(np.vdot(inv_y, x) - np.vdot(y, ia)) <= 1e-12 * abs(np.vdot(inv_y, x))


def test_config2_L512_forward_inverse():
    """L = 512, batch 1, flm ~ N(0,1)(1+l)^-1 (seed 1): both directions."""
    from oracle import sht
    L = 512
    flm = inputs.coeffs(L, 1, seed=1, weighted=True)
    op = oplan(L)
    f_ref = sht.inverse(op, flm)
    p = gpu_plan(L)
    f = to_host(p.inverse(to_dev(flm)))
    assert relmax(f, f_ref) < 1e-12
    flm_gpu = to_host(p.forward(to_dev(f_ref)))
    assert relmax(flm_gpu, sht.forward(op, f_ref)) < 1e-11
    assert relmax(flm_gpu, flm) < 1e-11


def test_deterministic_bitwise():
    L, B = 40, 3
    p = gpu_plan(L)
    x = to_dev(inputs.coeffs(L, B, seed=9))
    a, b = to_host(p.inverse(x)), to_host(p.inverse(x))
    assert np.array_equal(a, b)
    fa, fb = to_host(p.forward(to_dev(a))), to_host(p.forward(to_dev(a)))
    assert np.array_equal(fa, fb)


def test_bad_arguments_rejected():
    import torch
    from paper_1403_4661_amd import OshtError
    p = gpu_plan(8)
    x = torch.zeros((2, 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(OshtError):
        p.inverse(x, out=x)  # aliasing
    with pytest.raises(TypeError):
        p.inverse(x.to(torch.complex64))
    with pytest.raises(ValueError):
        p.inverse(torch.zeros((2, 63), dtype=torch.complex128, device="cuda"))


def test_alternating_placement_L20():
    from oracle import sht
    L = 20
    flm = inputs.coeffs(L, 1, seed=12)
    op = oplan(L, 0, "alternating")
    p = gpu_plan(L, 0, "alternating")
    assert p.theta_numerators() == op.num.tolist()
    f = sht.inverse(op, flm)
    assert relmax(to_host(p.inverse(to_dev(flm))), f) < 1e-12
    assert relmax(to_host(p.forward(to_dev(f))), sht.forward(op, f)) < 1e-10


@pytest.mark.parametrize("L,s,b", [(33, 0, 1), (70, 0, 7), (70, 0, 64), (100, 0, 16), (47, 0, 47), (8, 2, 3),
                                   (9, -1, 4)])
def test_forward_block_sizes(L, s, b, monkeypatch):
    """The blocked sweep (b levels per block, alias rows inside a block solved
    as a small triangular system) equals the oracle for every block size."""
    from oracle import sht
    from paper_1403_4661_amd import Plan
    monkeypatch.setenv("OSHT_FWD_BLOCK", str(b))
    p = Plan(L, s, force_spin_forward=s != 0)
    flm = inputs.coeffs(L, 2, seed=L + b, spin=s)
    f = sht.inverse(oplan(L, s), flm)
    ref = sht.forward(oplan(L, s), f)
    got = to_host(p.forward(to_dev(f)))
    tol = 1e-11 if s == 0 else 1e-8  # spin: alias-chain error growth (the method's, not the kernels')
    assert relmax(got, ref) < tol
    # the forward adjoint runs the same blocks in ascending order
    y = inputs.coeffs(L, 2, seed=L + b + 1, spin=s)
    fa = to_host(p.forward_adjoint(to_dev(y)))
    assert relmax(fa, sht.forward_adjoint(oplan(L, s), y)) < (1e-10 if s == 0 else 1e-7)


@pytest.mark.parametrize("dense", [1, 0])
@pytest.mark.parametrize("L,s,b,B", [(70, 0, 16, 3), (100, 0, 32, 2), (130, 0, 48, 5), (9, -1, 4, 2), (8, 2, 3, 1)])
def test_forward_delta_paths(L, s, b, B, dense, monkeypatch):
    """The in-block alias system solved through the precomputed (I + W)^-1
    (one FP64 matrix-core product per block) or by level-wise substitution:
    both equal the oracle, and repeated calls agree bit for bit."""
    from oracle import sht
    from paper_1403_4661_amd import Plan
    monkeypatch.setenv("OSHT_FWD_BLOCK", str(b))
    monkeypatch.setenv("OSHT_DELTA_DENSE", str(dense))
    p = Plan(L, s, force_spin_forward=s != 0)
    flm = inputs.coeffs(L, B, seed=L + 3 * b, spin=s)
    f = sht.inverse(oplan(L, s), flm)
    ref = sht.forward(oplan(L, s), f)
    tol = 1e-11 if s == 0 else 1e-8
    fd = to_dev(f)
    outs = [p.forward(fd) for _ in range(2)]
    assert relmax(to_host(outs[0]), ref) < tol
    assert bool((outs[0] == outs[1]).all())


def test_autotuned_plan_matches_oracle_and_caches_choice(tmp_path):
    """OSHT_TUNE: the forward block shape and the applies' stream shapes are
    timed on the device and cached; a second plan reads the cached choice;
    results stay at oracle parity, and every stream shape gives the same
    bits as the default one."""
    import shutil
    from oracle import sht
    from paper_1403_4661_amd import THETA_CACHE_DIR, Plan
    L = 64
    shutil.copy(f"{THETA_CACHE_DIR}/theta_greedy_L{L}.txt", tmp_path)
    p = Plan(L, 0, theta_cache_dir=str(tmp_path), tune=True)
    files = [f for f in tmp_path.iterdir() if f.name.startswith("tune_fwd_")]
    assert len(files) == 1
    b, cpw, fv, iv = (int(x) for x in files[0].read_text().split()[:4])
    assert 1 <= b <= L and cpw in (1, 2, 4) and fv in (0, 1, 2) and iv in (0, 1, 2)
    p2 = Plan(L, 0, theta_cache_dir=str(tmp_path), tune=True)
    flm = inputs.coeffs(L, 3, seed=21)
    f = sht.inverse(oplan(L), flm)
    ref = sht.forward(oplan(L), f)
    for q in (p, p2):
        assert relmax(to_host(q.forward(to_dev(f))), ref) < 1e-11
    # the stream shapes sum k in the same order: the inverse is bit-identical
    # to an untuned plan's (the forward may differ in rounding if b differs)
    p0 = Plan(L, 0, theta_cache_dir=str(tmp_path))
    x = to_dev(flm)
    assert bool((p.inverse(x) == p0.inverse(x)).all())


@pytest.mark.parametrize("precision", ["fp64", "fwd32", "fp32"])
@pytest.mark.parametrize("var", ["1,1", "2,2"])
def test_apply_stream_shapes_bit_identical(monkeypatch, precision, var):
    """The alternative stream shapes of the applies (k depth 16 in 3 stages,
    k depth 32 in 2) sum k in the default shape's order, so a plan forced to
    them gives the same bits in both directions (L = 100: ragged row, column
    and k tiles; batch 5)."""
    from paper_1403_4661_amd import Plan
    L, B = 100, 5
    flm = to_dev(inputs.coeffs(L, B, seed=41, weighted=True))
    p0 = Plan(L, 0, precision=precision)
    monkeypatch.setenv("OSHT_GEMM_VAR", var)
    p1 = Plan(L, 0, precision=precision)
    f0, f1 = p0.inverse(flm), p1.inverse(flm)
    assert bool((f0 == f1).all())
    assert bool((p0.forward(f0) == p1.forward(f0)).all())
