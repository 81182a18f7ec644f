"""Pins of the oracle's colatitude placements (Sec. III-D)."""

import math
import os

import numpy as np
import pytest

from oracle import sampling as smp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(L):
    path = os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")
    vals = [int(x) for x in open(path) if x.strip() and not x.startswith("#")]
    return np.asarray(vals)


def test_equiangular_set_contains_pole_not_zero():
    L = 9
    th = smp.theta_from_numerators(L, smp.numerators_equiangular(L))
    assert th.size == L
    assert math.isclose(th[-1], math.pi) and th.min() > 0
    np.testing.assert_allclose(np.diff(th), 2 * math.pi / (2 * L - 1))


@pytest.mark.parametrize("L", [2, 3, 8, 12, 13, 47])
def test_alternating_vector_as_printed(L):
    """Eq. sampling_latitude: [pi, pi/(2L-1), pi(2L-3)/(2L-1), 3pi/(2L-1), ...,
    pi(2 floor((L-1)/2) + 1)/(2L-1)]."""
    n = smp.numerators_alternating(L)
    D = 2 * L - 1
    assert n[0] == D
    if L > 1:
        assert n[1] == 1
    if L > 2:
        assert n[2] == D - 2
    if L > 3:
        assert n[3] == 3
    assert n[-1] == 2 * ((L - 1) // 2) + 1
    assert sorted(n.tolist()) == list(range(1, D + 1, 2))


def test_trig_exact_at_pole():
    t = smp.trig_from_numerators(5, [9])
    assert t["sin"][0] == 0.0 and t["cos"][0] == -1.0 and t["cos_half"][0] == 0.0 and t["sin_half"][0] == 1.0


@pytest.mark.parametrize("L", [2, 3, 5, 8, 16, 24, 40])
def test_greedy_svd_equals_secular(L):
    a, ka = smp.numerators_greedy(L, "svd", return_kappa=True)
    b, kb = smp.numerators_greedy(L, "secular", return_kappa=True)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(ka, kb, rtol=1e-9)


@pytest.mark.parametrize("L", [8, 20, 33])
def test_greedy_choices_are_minimal(L):
    """Re-check every greedy choice independently: among the members of Theta
    unused at step m, the chosen one minimises cond_2(P_m) (dense SVD)."""
    from oracle.legendre import scalar_table
    num = smp.numerators_greedy(L)
    assert num[-1] == 2 * ((L - 1) // 2) + 1          # farthest from the poles
    assert num[0] == 2 * L - 1                        # the pole is left for m = 0
    allnum = smp.numerators_equiangular(L)
    for m in range(L - 2, -1, -1):
        unused = [c for c in allnum if c not in set(num[m + 1:].tolist())]
        best = None
        for c in unused:
            rows = np.concatenate([[c], num[m + 1:]])
            tr = smp.trig_from_numerators(L, rows)
            P = scalar_table(L, m, tr["cos"], tr["sin"]).T
            k = np.linalg.cond(P)
            if best is None or k < best[0] * (1 - 1e-9):
                best = (k, c)
        assert best[1] == num[m]


def test_alternating_condition_number_order_1e2_at_L47():
    """Sec. IV-E: with the alternating vector at L ~ 47 the largest kappa_m is
    'of the order 10^2'."""
    k = smp.kappas(47, smp.numerators_alternating(47))
    assert 1e2 <= k.max() < 1e3


def test_greedy_far_better_conditioned_than_alternating_at_L64():
    """Figs. 3-4 (Sec. III-D): the greedy placement has a much smaller max kappa."""
    ka = smp.kappas(64, smp.numerators_alternating(64)).max()
    kg = smp.kappas(64, smp.numerators_greedy(64)).max()
    assert kg < 20 and ka > 100 * kg


@pytest.mark.parametrize("L", [32, 64, 128])
def test_golden_files_reproduce(L):
    np.testing.assert_array_equal(_read_golden(L), smp.numerators_greedy(L))


@pytest.mark.parametrize("L", [32, 64, 128, 256, 512, 1024])
def test_golden_files_are_valid_placements(L):
    path = os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    n = _read_golden(L)
    assert sorted(n.tolist()) == list(range(1, 2 * L, 2))
    assert n[0] == 2 * L - 1 and n[-1] == 2 * ((L - 1) // 2) + 1
