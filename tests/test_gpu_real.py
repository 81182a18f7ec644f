"""Real maps (spin 0): two real maps per complex transform.

- forward_real of real samples (U[-1, 1], the paper's Experiment 2 input;
  every real sample vector is band-limited on this scheme) equals the
  oracle's forward of the same samples, and has the conjugation symmetry
  f_{l,-m} = (-1)^m conj(f_lm);
- inverse_real of arbitrary complex coefficients equals the real part of the
  oracle's inverse;
- odd and even batches (the last map of an odd batch travels alone);
- at the headline size (L = 1024, 32 real maps = 16 complex transforms),
  inverse_real then forward_real returns coefficients with the symmetry
  (the property the forward has at any size; input seed 5 weighted
  (1+l)^-1 and symmetrised).
"""

import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import oracle_plan, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

_plans = {}


def plan(L, precision="fp64"):
    from paper_1403_4661_amd import Plan
    if (L, precision) not in _plans:
        _plans[(L, precision)] = Plan(L, 0, precision=precision)
    return _plans[(L, precision)]


def real_samples(L, B, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (B, L * L))


def reflect(flm, L):
    """R(x)_lm = (-1)^m conj(x_{l,-m})."""
    out = np.empty_like(flm)
    for l in range(L):
        m = np.arange(-l, l + 1)
        out[:, l * l + l + m] = ((-1.0) ** np.abs(m)) * np.conj(flm[:, l * l + l - m])
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32-fwd"])
@pytest.mark.parametrize("L,B", [(1, 1), (2, 2), (16, 3), (33, 4), (64, 5)])
def test_forward_real_matches_oracle(L, B, precision):
    import torch
    from oracle import sht
    f = real_samples(L, B, seed=L + B)
    ref = sht.forward(oracle_plan(L), f.astype(np.complex128))
    got = to_host(plan(L, precision).forward_real(torch.as_tensor(f).cuda()))
    tol = 1e-11 if precision == "fp64" else 1e-6
    assert relmax(got, ref) < tol
    assert relmax(reflect(got, L), got) < (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("L,B", [(1, 1), (16, 2), (33, 3), (64, 5)])
def test_inverse_real_is_real_part_of_oracle_inverse(L, B, precision):
    from oracle import sht
    flm = inputs.coeffs(L, B, seed=2 * L + B)  # no symmetry: the real part is returned
    ref = sht.inverse(oracle_plan(L), flm).real
    got = to_host(plan(L, precision).inverse_real(to_dev(flm)))
    assert got.dtype == np.float64
    assert relmax(got, ref) < (1e-12 if precision == "fp64" else 1e-6)


def test_real_bad_arguments():
    import torch
    from paper_1403_4661_amd import Plan
    p = plan(8)
    with pytest.raises(TypeError):
        p.forward_real(torch.zeros((2, 64), dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        Plan(8, 2).inverse_real(torch.zeros((1, 64), dtype=torch.complex128, device="cuda"))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32-fwd", 1e-6)])
def test_real_round_trip_headline_size(precision, tol):
    """L = 1024, 32 real maps: the FP64 plan's inverse_real of symmetric
    coefficients, then forward_real on the given plan, returns them."""
    L, B = 1024, 32
    flm = inputs.coeffs(L, B, seed=5, weighted=True)
    flm = 0.5 * (flm + reflect(flm, L))
    f = plan(L, "fp64").inverse_real(to_dev(flm))
    back = to_host(plan(L, precision).forward_real(f))
    assert relmax(back, flm) < tol
    del f
    _plans.clear()
