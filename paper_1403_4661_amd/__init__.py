"""MI355X implementation of the forward and inverse spherical harmonic
transforms on the optimal-dimensionality L^2-sample scheme of Khalid, Kennedy
& McEwen (IEEE TSP 2014).

A thin binding over the C ABI of include/osht.h (libosht.so, built in-tree):
it checks shapes, dtypes and devices of torch tensors and passes their device
pointers and the current HIP stream; every step of every transform runs in
the library's HIP kernels.  PyTorch supplies device memory and streams only.

    plan = Plan(L=1024, spin=0)
    f   = plan.inverse(flm)        # flm: complex128 cuda tensor (B, L*L)
    flm = plan.forward(f)
    InverseSHT.apply(plan, flm)    # differentiable (hand-written adjoints)

Layouts: coefficients flm[b, l*l + l + m]; samples f[b, k*k + j] for ring k
(colatitude theta_k = pi n_k/(2L-1)), longitude phi_j = 2 pi j/(2k+1).
"""

import ctypes
import os

from . import _lib
from ._lib import OshtError, lib  # noqa: F401

__all__ = ["Plan", "InverseSHT", "ForwardSHT", "theta_greedy", "theta_alternating", "lib", "OshtError",
           "THETA_CACHE_DIR"]

THETA_CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "theta")


def theta_greedy(L, with_kappa=False):
    """Greedy colatitude numerators n_k (host computation in the library)."""
    num = (ctypes.c_int32 * L)()
    kap = (ctypes.c_double * L)()
    _lib.check(lib().osht_theta_greedy(L, num, kap))
    out = [int(v) for v in num]
    return (out, [float(v) for v in kap]) if with_kappa else out


def theta_alternating(L):
    num = (ctypes.c_int32 * L)()
    _lib.check(lib().osht_theta_alternating(L, num))
    return [int(v) for v in num]


class Plan:
    """A transform plan for band-limit L and spin s on the current device."""

    def __init__(self, L, spin=0, placement="greedy", precision="fp64", theta_cache_dir=THETA_CACHE_DIR,
                 device=None):
        """precision: "fp64" (FP64 throughout) or "fp32" (order-wise applies on
        FP32-stored matrices with FP32 matrix cores; everything else FP64)."""
        import torch

        if placement not in ("greedy", "alternating"):
            raise ValueError("placement must be 'greedy' or 'alternating'")
        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        flags = (_lib.OSHT_PREC_FP64 if precision == "fp64" else _lib.OSHT_PREC_FP32) | (
            _lib.OSHT_THETA_GREEDY if placement == "greedy" else _lib.OSHT_THETA_ALTERNATING)
        self.L, self.spin, self.precision = int(L), int(spin), precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = ctypes.c_void_p()
        d = theta_cache_dir.encode() if theta_cache_dir else None
        with torch.cuda.device(self.device):
            _lib.check(lib().osht_plan_create(self.L, self.spin, flags, d, ctypes.byref(self._h)))

    # -- queries ------------------------------------------------------------
    def info(self):
        info = _lib.OshtInfo()
        _lib.check(lib().osht_plan_info(self._h, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in info._fields_ if f != "reserved"}

    def theta_numerators(self):
        num = (ctypes.c_int32 * self.L)()
        _lib.check(lib().osht_plan_theta(self._h, num))
        return [int(v) for v in num]

    def set_profiling(self, enable=True):
        """Event timing of the library's named kernel launches (resets counters)."""
        _lib.check(lib().osht_plan_set_profiling(self._h, 1 if enable else 0))

    def kernel_time(self, name):
        """(launches, total milliseconds) of a named kernel since profiling was enabled."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _lib.check(lib().osht_plan_kernel_time(self._h, name.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    # -- transforms ---------------------------------------------------------
    def _run(self, fn, x, out=None):
        import torch

        if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128:
            raise TypeError("expected a complex128 torch tensor")
        if x.device != self.device:
            raise ValueError(f"tensor on {x.device}, plan on {self.device}")
        squeeze = x.dim() == 1
        xb = x.reshape(1, -1) if squeeze else x
        if xb.dim() != 2 or xb.shape[1] != self.L * self.L:
            raise ValueError(f"expected shape (B, {self.L * self.L})")
        xb = xb.contiguous()
        y = torch.empty_like(xb) if out is None else out
        if y.shape != xb.shape or y.dtype != torch.complex128 or not y.is_contiguous() or y.device != self.device:
            raise ValueError("bad output tensor")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(getattr(lib(), fn)(self._h, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      xb.shape[0], ctypes.c_void_p(stream)))
        return y.reshape(-1) if squeeze else y

    def inverse(self, flm, out=None):
        """Samples from coefficients (Procedure 2)."""
        return self._run("osht_inverse", flm, out)

    def forward(self, f, out=None):
        """Coefficients from samples (Procedure 1)."""
        return self._run("osht_forward", f, out)

    def inverse_adjoint(self, fbar, out=None):
        return self._run("osht_inverse_adjoint", fbar, out)

    def forward_adjoint(self, flmbar, out=None):
        return self._run("osht_forward_adjoint", flmbar, out)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().osht_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class InverseSHT(torch.autograd.Function):
        """f = inverse(flm); gradient flm_bar = inverse^H f_bar (the
        conjugate-transpose convention of torch for C-linear maps)."""

        @staticmethod
        def forward(ctx, plan, flm):
            ctx.plan = plan
            return plan.inverse(flm)

        @staticmethod
        def backward(ctx, grad_f):
            return None, ctx.plan.inverse_adjoint(grad_f.contiguous())

    class ForwardSHT(torch.autograd.Function):
        """flm = forward(f); gradient f_bar = forward^H flm_bar."""

        @staticmethod
        def forward(ctx, plan, f):
            ctx.plan = plan
            return plan.forward(f)

        @staticmethod
        def backward(ctx, grad_flm):
            return None, ctx.plan.forward_adjoint(grad_flm.contiguous())

    return InverseSHT, ForwardSHT


def __getattr__(name):
    if name in ("InverseSHT", "ForwardSHT"):
        inv, fwd = _autograd()
        globals()["InverseSHT"], globals()["ForwardSHT"] = inv, fwd
        return globals()[name]
    raise AttributeError(name)
