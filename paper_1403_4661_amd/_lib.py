"""ctypes loader for libosht.so (the C ABI of include/osht.h).

The library is built in-tree by paper_1403_4661_amd.build; importing this
module never builds or falls back to anything else: a missing library is an
ImportError-like failure at first use.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libosht.so")

OSHT_OK = 0
OSHT_EINVAL = -1
OSHT_ENOMEM = -2
OSHT_EHIP = -3
OSHT_ESINGULAR = -4
OSHT_ENOTSUP = -5
OSHT_EIO = -6
OSHT_ENONFINITE = -7

OSHT_PREC_FP64 = 0x0
OSHT_PREC_FP32 = 0x1
OSHT_PREC_FP32_FWD = 0x2
OSHT_PREC_I8X6 = 0x3
OSHT_PREC_I8X8 = 0x4
OSHT_PREC_FWD32 = 0x5
OSHT_THETA_GREEDY = 0x00
OSHT_THETA_ALTERNATING = 0x10
OSHT_TUNE = 0x100
OSHT_SPIN_FWD_FORCE = 0x200
OSHT_CHECK_FINITE = 0x400

EXPORTED = (
    "osht_theta_greedy",
    "osht_theta_greedy_device",
    "osht_theta_alternating",
    "osht_plan_create",
    "osht_plan_destroy",
    "osht_plan_info",
    "osht_plan_theta",
    "osht_inverse",
    "osht_forward",
    "osht_inverse_adjoint",
    "osht_forward_adjoint",
    "osht_forward_real",
    "osht_inverse_real",
    "osht_strerror",
    "osht_last_error_message",
    "osht_plan_set_profiling",
    "osht_plan_kernel_time",
    "osht_batch_run",
    "osht_graph_destroy",
    "osht_plan_status",
    "osht_inverse_noalloc",
)


class OshtInfo(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("spin", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("fwd_unstable", ctypes.c_int32),
        ("nsamples", ctypes.c_int64),
        ("ncoeffs", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("max_kappa", ctypes.c_double),
        ("max_inv_residual", ctypes.c_double),
        ("fwd_check_err", ctypes.c_double),
    ]


class OshtJob(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("direction", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("inp", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("batch", ctypes.c_int64),
    ]


OSHT_DIR = {"inverse": 0, "forward": 1, "inverse_adjoint": 2, "forward_adjoint": 3}


class OshtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"osht error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (loaded once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1403_4661_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes libosht bind to that single runtime, so torch's device
    # pointers and stream handles are valid inside the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    L.osht_theta_greedy.argtypes = [ctypes.c_int, i32p, dp]
    L.osht_theta_greedy_device.argtypes = [ctypes.c_int, i32p, dp]
    L.osht_theta_alternating.argtypes = [ctypes.c_int, i32p]
    L.osht_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_char_p,
                                   ctypes.POINTER(vp)]
    L.osht_plan_destroy.argtypes = [vp]
    L.osht_plan_info.argtypes = [vp, ctypes.POINTER(OshtInfo)]
    L.osht_plan_theta.argtypes = [vp, i32p]
    for name in ("osht_inverse", "osht_forward", "osht_inverse_adjoint", "osht_forward_adjoint", "osht_forward_real",
                 "osht_inverse_real", "osht_inverse_noalloc"):
        fn = getattr(L, name)
        fn.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        fn.restype = ctypes.c_int
    L.osht_batch_run.argtypes = [ctypes.POINTER(OshtJob), ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.osht_graph_destroy.argtypes = [vp]
    L.osht_plan_status.argtypes = [vp, i32p]
    L.osht_plan_set_profiling.argtypes = [vp, ctypes.c_int, ctypes.c_char_p]
    L.osht_plan_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
    L.osht_strerror.argtypes = [ctypes.c_int]
    L.osht_strerror.restype = ctypes.c_char_p
    L.osht_last_error_message.argtypes = []
    L.osht_last_error_message.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("osht_strerror", "osht_last_error_message"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc):
    if rc != OSHT_OK:
        L = lib()
        detail = L.osht_last_error_message().decode(errors="replace")
        raise OshtError(rc, f"{L.osht_strerror(rc).decode()}: {detail}")
