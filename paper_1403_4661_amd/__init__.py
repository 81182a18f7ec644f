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
           "THETA_CACHE_DIR", "batch_run", "BatchGraph"]

THETA_CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "theta")


def theta_greedy(L, with_kappa=False, device=False):
    """Greedy colatitude numerators n_k, computed by the library on the host
    or (device=True) on the current GPU."""
    num = (ctypes.c_int32 * L)()
    kap = (ctypes.c_double * L)()
    fn = lib().osht_theta_greedy_device if device else lib().osht_theta_greedy
    _lib.check(fn(L, num, kap))
    out = [int(v) for v in num]
    return (out, [float(v) for v in kap]) if with_kappa else out


def theta_alternating(L):
    num = (ctypes.c_int32 * L)()
    _lib.check(lib().osht_theta_alternating(L, num))
    return [int(v) for v in num]


class Plan:
    """A transform plan for band-limit L and spin s on the current device."""

    def __init__(self, L, spin=0, placement="greedy", precision="fp64", theta_cache_dir=THETA_CACHE_DIR,
                 device=None, tune=False, force_spin_forward=False, check_finite=False):
        """precision: "fp64" (FP64 throughout), "fp32" (inverse and its
        adjoint on FP32 A_m with FP32 matrix cores; the forward sweep, DFTs
        and buffers FP64), "fp32-fwd" (also the forward's P_m^{-1} rows in
        FP32; its alias rows stay FP64), "i8x6" (the inverse apply as exact
        int8 matrix-core products of 6-digit splits, ~2e-10; the forward as
        "fp32-fwd"), "i8x8" (8 digits, FP64 grade; the forward FP64) or
        "fwd32" (the inverse FP64, the forward as "fp32-fwd").
        tune: time the forward sweep's block shapes on this device and keep
        the fastest (cached in theta_cache_dir).
        force_spin_forward: run the forward of a spin != 0 plan even when the
        plan-time self-check marks it unstable (info()["fwd_unstable"]);
        otherwise forward() and forward_adjoint() raise OshtError (ENOTSUP).
        check_finite: every transform scans its output for NaN / Inf; read
        the sticky result with status()."""
        import torch

        if placement not in ("greedy", "alternating"):
            raise ValueError("placement must be 'greedy' or 'alternating'")
        prec = {"fp64": _lib.OSHT_PREC_FP64, "fp32": _lib.OSHT_PREC_FP32, "fp32-fwd": _lib.OSHT_PREC_FP32_FWD,
                "i8x6": _lib.OSHT_PREC_I8X6, "i8x8": _lib.OSHT_PREC_I8X8, "fwd32": _lib.OSHT_PREC_FWD32}
        if precision not in prec:
            raise ValueError("precision must be 'fp64', 'fp32', 'fp32-fwd', 'i8x6', 'i8x8' or 'fwd32'")
        flags = prec[precision] | (
            _lib.OSHT_THETA_GREEDY if placement == "greedy" else _lib.OSHT_THETA_ALTERNATING) | (
            _lib.OSHT_TUNE if tune else 0) | (
            _lib.OSHT_SPIN_FWD_FORCE if force_spin_forward else 0) | (
            _lib.OSHT_CHECK_FINITE if check_finite else 0)
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
        return {f: getattr(info, f) for f, _ in info._fields_}

    def status(self):
        """Sticky output status (check_finite plans): OSHT_OK, or
        OSHT_ENONFINITE when an output since the last call held NaN / Inf.
        Waits for the device; clears the record."""
        st = ctypes.c_int32()
        _lib.check(lib().osht_plan_status(self._h, ctypes.byref(st)))
        return int(st.value)

    def theta_numerators(self):
        num = (ctypes.c_int32 * self.L)()
        _lib.check(lib().osht_plan_theta(self._h, num))
        return [int(v) for v in num]

    def set_profiling(self, enable=True, only=None):
        """Event timing of the library's named kernel launches (resets
        counters); `only` restricts timing to one kernel name."""
        _lib.check(lib().osht_plan_set_profiling(self._h, 1 if enable else 0, only.encode() if only else None))

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

    def _run_real(self, fn, x, in_dtype, out_dtype, out=None):
        import torch

        if not isinstance(x, torch.Tensor) or x.dtype != in_dtype:
            raise TypeError(f"expected a {in_dtype} torch tensor")
        if x.device != self.device:
            raise ValueError(f"tensor on {x.device}, plan on {self.device}")
        if self.spin != 0:
            raise ValueError("real-map transforms are defined for spin 0 only")
        squeeze = x.dim() == 1
        xb = x.reshape(1, -1) if squeeze else x
        if xb.dim() != 2 or xb.shape[1] != self.L * self.L:
            raise ValueError(f"expected shape (B, {self.L * self.L})")
        xb = xb.contiguous()
        y = torch.empty(xb.shape, dtype=out_dtype, device=self.device) if out is None else out
        if y.shape != xb.shape or y.dtype != out_dtype or not y.is_contiguous() or y.device != self.device:
            raise ValueError("bad output tensor")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(getattr(lib(), fn)(self._h, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      xb.shape[0], ctypes.c_void_p(stream)))
        return y.reshape(-1) if squeeze else y

    def forward_real(self, f, out=None):
        """Coefficients (complex128, full layout) of real maps (float64
        samples); two maps per complex transform.  Spin 0."""
        import torch
        return self._run_real("osht_forward_real", f, torch.float64, torch.complex128, out)

    def inverse_real(self, flm, out=None):
        """Real samples (float64): the real part of the inverse, exact for
        coefficients with f_{l,-m} = (-1)^m conj(f_lm).  Spin 0."""
        import torch
        return self._run_real("osht_inverse_real", flm, torch.complex128, torch.float64, out)

    def inverse(self, flm, out=None):
        """Samples from coefficients (Procedure 2)."""
        return self._run("osht_inverse", flm, out)

    def inverse_noalloc(self, flm, out=None):
        """As inverse(), on the library's static scratch array instead of the
        plan's workspace (no device allocation inside the call; pass `out`
        to avoid torch's allocation as well)."""
        return self._run("osht_inverse_noalloc", flm, out)

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


class BatchGraph:
    """A HIP graph captured by batch_run (freed with the object)."""

    def __init__(self):
        self._h = ctypes.c_void_p()

    def close(self):
        if self._h.value:
            lib().osht_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run(jobs, graph=None):
    """Runs jobs = [(plan, direction, in_tensor, out_tensor), ...] as one
    unit on the current stream (direction: "inverse", "forward",
    "inverse_adjoint", "forward_adjoint").  With graph (a BatchGraph) the
    jobs are captured into a HIP graph on first use and the graph is
    replayed while the job list is unchanged."""
    import torch

    arr = (_lib.OshtJob * len(jobs))()
    keep = []
    for i, (plan, direction, x, y) in enumerate(jobs):
        for t in (x, y):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_contiguous():
                raise TypeError("batch jobs take contiguous complex128 tensors")
            if t.device != plan.device:
                raise ValueError("tensor and plan on different devices")
        n = plan.L * plan.L
        if x.numel() % n or x.numel() != y.numel():
            raise ValueError(f"job {i}: expected matching (B, {n}) tensors")
        arr[i] = _lib.OshtJob(plan._h.value, _lib.OSHT_DIR[direction], 0, x.data_ptr(), y.data_ptr(), x.numel() // n)
        keep.append((x, y))
    stream = torch.cuda.current_stream().cuda_stream
    gp = ctypes.byref(graph._h) if graph is not None else None
    _lib.check(lib().osht_batch_run(arr, len(jobs), ctypes.c_void_p(stream), gp))
    return graph


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
