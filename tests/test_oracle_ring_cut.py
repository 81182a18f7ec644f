"""The ring cut, checked on the oracle.

On a ring near a pole the normalised Legendre values P_l^m(theta_k) decay
exponentially once |m| exceeds about l sin(theta_k) (Sec. III-F).  The GPU
path leaves out of each ring's fold (and of the forward's gathers) every
order whose values on that ring all lie below 2^-80: such an order adds less
than 2^-80 sum_l |f_lm| to the ring's samples.  Here the oracle's own tables
are masked the same way, row by row: the inverse changes only at FP64
rounding, while a sizeable share of rows is dropped (8% of the (order, ring)
rows at L = 64, 14% at 128; 28% at 1024 on the GPU plan).
"""

import numpy as np
import pytest

from oracle import sht
from tests import inputs


class _CutPlan:
    """An oracle plan whose tables A_m have the rows (rings) with every
    |value| < 2^-80 set to zero."""

    def __init__(self, plan):
        self._plan = plan
        self.rows = 0
        self.dropped = 0

    def __getattr__(self, name):
        return getattr(self._plan, name)

    def table(self, m):
        A = np.array(self._plan.table(m), copy=True)
        neg = np.max(np.abs(A), axis=1) < 2.0 ** -80
        self.rows += A.shape[0]
        self.dropped += int(neg.sum())
        A[neg, :] = 0.0
        return A


@pytest.mark.parametrize("L,seed,share", [(64, 21, 0.05), (128, 22, 0.10)])
def test_ring_cut_changes_inverse_only_at_rounding(L, seed, share):
    op = sht.Plan(L)
    flm = inputs.coeffs(L, 2, seed=seed, weighted=True)
    full = sht.inverse(op, flm)
    cp = _CutPlan(op)
    cut = sht.inverse(cp, flm)
    assert cp.dropped > share * cp.rows
    assert np.max(np.abs(cut - full)) / np.max(np.abs(full)) < 1e-15


def test_ring_cut_rows_are_a_polar_suffix_of_orders():
    """On each ring the dropped orders are the largest ones: once an order
    is below the bound on a ring, every larger order is too, so a per-ring
    cut |m| < cut_k describes the dropped set exactly (L = 64)."""
    L = 64
    op = sht.Plan(L)
    neg = np.zeros((L, L), dtype=bool)  # [ring, |m|]
    for am in range(L):
        A = op.table(am)
        neg[:, am] = np.max(np.abs(A), axis=1) < 2.0 ** -80
    for k in range(L):
        row = neg[k]
        if row.any():
            first = int(np.argmax(row))
            assert row[first:].all(), f"ring {k}: order {first} dropped but a larger one kept"
