"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, rejects bad arguments before touching a GPU, and its host
placement greedy reproduces the oracle's placements exactly."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osht.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _lib():
    from paper_1403_4661_amd import lib
    return lib()


def _golden(L):
    return [int(x) for x in open(os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")) if not x.startswith("#")]


def test_header_symbols_exported():
    decl = set(re.findall(r"\b(osht_[a-z_]+)\s*\(", open(HEADER).read()))
    assert {"osht_plan_create", "osht_forward", "osht_inverse"} <= decl
    L = _lib()
    for name in sorted(decl):
        assert hasattr(L, name), name


def test_strerror_and_codes():
    L = _lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.osht_strerror(code) and L.osht_strerror(code) != b"unknown error"
    assert L.osht_strerror(-99) == b"unknown error"


@pytest.mark.parametrize("L,spin,flags", [(0, 0, 0), (-3, 0, 0), (5000, 0, 0), (8, 8, 0), (8, -9, 0),
                                          (8, 0, 0x800), (8, 0, 0x20), (8, 0, 0x1000)])
def test_plan_create_rejects_bad_arguments(L, spin, flags):
    lib = _lib()
    h = ctypes.c_void_p()
    rc = lib.osht_plan_create(L, spin, flags, None, ctypes.byref(h))
    assert rc in (-1, -5) and not h.value


def test_plan_create_rejects_unsupported_precision():
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.osht_plan_create(8, 0, 0x6, None, ctypes.byref(h)) == -5


def test_transforms_reject_null_plan_and_pointers():
    lib = _lib()
    for fn in ("osht_inverse", "osht_forward", "osht_inverse_adjoint", "osht_forward_adjoint"):
        assert getattr(lib, fn)(None, ctypes.c_void_p(16), ctypes.c_void_p(4096), 1, None) == -1
    assert lib.osht_plan_destroy(None) == 0
    assert lib.osht_plan_info(None, None) == -1
    st = ctypes.c_int32(5)
    assert lib.osht_plan_status(None, ctypes.byref(st)) == -1


def test_theta_rejects_bad_arguments():
    lib = _lib()
    assert lib.osht_theta_greedy(0, (ctypes.c_int32 * 1)(), None) == -1
    assert lib.osht_theta_greedy(4, None, None) == -1


@pytest.mark.parametrize("L", [1, 2, 3, 12, 47])
def test_alternating_matches_oracle(L):
    from paper_1403_4661_amd import theta_alternating
    from oracle.sampling import numerators_alternating
    assert theta_alternating(L) == numerators_alternating(L).tolist()


@pytest.mark.parametrize("L", [2, 5, 9, 16, 31])
def test_greedy_small_matches_oracle(L):
    from paper_1403_4661_amd import theta_greedy
    from oracle.sampling import numerators_greedy
    assert theta_greedy(L) == numerators_greedy(L).tolist()


@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_greedy_matches_golden(L):
    from paper_1403_4661_amd import theta_greedy
    assert theta_greedy(L) == _golden(L)


@pytest.mark.parametrize("L", [32, 64, 128, 256, 512, 1024, 2048])
def test_shipped_placement_cache_matches_golden(L):
    """The placements shipped with the package (written by the library's own
    greedy) equal the oracle's, integer for integer."""
    from paper_1403_4661_amd import THETA_CACHE_DIR
    mine = os.path.join(THETA_CACHE_DIR, f"theta_greedy_L{L}.txt")
    gold = os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")
    if not (os.path.exists(mine) and os.path.exists(gold)):
        pytest.skip("placement not generated for this L")
    a = [int(x) for x in open(mine) if not x.startswith("#")]
    assert a == _golden(L)


def test_single_hip_runtime_in_process():
    """Loading the library after torch must not map a second HIP runtime."""
    import subprocess
    import sys
    code = ("import paper_1403_4661_amd as P; P.lib(); "
            "m = open('/proc/self/maps').read(); "
            "print(len(set(l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l)))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, check=True)
    assert out.stdout.strip() == "1"


def test_device_greedy_is_switched_off():
    """osht_theta_greedy_device reports OSHT_ENOTSUP (switched off) after
    checking its arguments, without touching a device."""
    lib = _lib()
    assert lib.osht_theta_greedy_device(0, (ctypes.c_int32 * 1)(), None) == -1
    assert lib.osht_theta_greedy_device(8, (ctypes.c_int32 * 8)(), None) == -5
