"""The C ABI library loads, exports every function include/cholgrad.h declares, and rejects bad
arguments on the host before touching a GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cholgrad.h")
LIB = os.path.join(ROOT, "paper_1602_07527_amd", "libcholgrad.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcholgrad.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("chol_factor", "chol_rev", "chol_fwd", "chol_factor_ex", "chol_rev_ex", "chol_fwd_ex",
                 "chol_workspace_bytes", "chol_workspace_bytes_ex",
                 "chol_status_string", "chol_version"):
        assert want in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def _lib():
    from paper_1602_07527_amd import load_library
    return load_library()


def test_host_only_queries():
    lib = _lib()
    assert lib.chol_version() == 100
    assert lib.chol_status_string(0) == b"success"
    assert lib.chol_workspace_bytes(1, 0, 0, 0) == 0
    assert lib.chol_workspace_bytes(1, 0, 1000, 0) > 0
    assert lib.chol_workspace_bytes(1, 0, 1000, 40) == 0     # nb not a multiple of 16
    assert lib.chol_workspace_bytes(1, 0, 1000, 272) == 0    # nb above 256
    assert lib.chol_workspace_bytes(1, 0, 1000, 48) > 0
    assert lib.chol_workspace_bytes(1, 0, 1000, 256) > lib.chol_workspace_bytes(1, 0, 1000, 128)
    assert lib.chol_workspace_bytes(1, 0, 1000, 0) == lib.chol_workspace_bytes(1, 0, 1000, 256)  # holds any automatic width
    assert lib.chol_workspace_bytes(1, 9, 1000, 0) == 0      # unknown precision


def test_invalid_arguments_rejected_on_host():
    lib = _lib()
    fake = ctypes.c_void_p(4096)        # never dereferenced: validation fails first
    ws = ctypes.c_void_p(1 << 20)
    big = 1 << 40
    assert lib.chol_rev(7, 10, fake, 10, fake, 10, 0, 0, ws, big, None) == -1
    assert lib.chol_rev(0, -1, fake, 10, fake, 10, 0, 0, ws, big, None) == -2
    assert lib.chol_rev(0, 10, None, 10, fake, 10, 0, 0, ws, big, None) == -3
    assert lib.chol_rev(0, 10, fake, 9, fake, 10, 0, 0, ws, big, None) == -4
    assert lib.chol_rev(0, 10, fake, 10, ctypes.c_void_p(4097), 10, 0, 0, ws, big, None) == -5
    assert lib.chol_rev(0, 10, fake, 10, fake, 3, 0, 0, ws, big, None) == -6
    assert lib.chol_rev(0, 10, fake, 10, fake, 10, 5, 0, ws, big, None) == -7
    assert lib.chol_rev(0, 10, fake, 10, fake, 10, 0, 200, ws, big, None) == -8
    assert lib.chol_rev(0, 10, fake, 10, fake, 10, 0, 0, ws, 16, None) == -102
    assert lib.chol_rev(0, 10, fake, 10, fake, 10, 0, 0, ctypes.c_void_p((1 << 20) + 8), big, None) == -102
    assert lib.chol_rev(0, 0, None, 0, None, 0, 0, 0, None, 0, None) == 0   # n == 0 is a no-op
    assert lib.chol_fwd(0, 10, fake, 10, fake, 10, 33, ws, big, None) == -7
    assert lib.chol_fwd(0, 10, fake, 10, fake, 10, 0, None, big, None) == -102
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 0, 3, 0, ws, big, None) == -9      # diag variant
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 0, -1, 0, ws, big, None) == -9
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 0, 2, 0, ws, 16, None) == -102
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 256, 2, 0, ws, big, None) == -103  # Level-2, nb > 128
    assert lib.chol_fwd_ex(0, 10, fake, 10, fake, 10, 160, 2, 0, ws, big, None) == -103
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 0, 0, 2, ws, big, None) == -10     # layout
    assert lib.chol_rev_ex(0, 10, fake, 10, fake, 10, 0, 0, 0, 1, ws, 16, None) == -102
    assert lib.chol_rev_ex(0, 10, fake, 9, fake, 10, 0, 0, 0, 1, ws, big, None) == -4
    assert lib.chol_fwd_ex(0, 10, fake, 10, fake, 10, 0, 3, 0, ws, big, None) == -8
    assert lib.chol_fwd_ex(0, 10, fake, 10, fake, 10, 0, 1, 0, None, big, None) == -102
    assert lib.chol_fwd_ex(0, 10, fake, 10, fake, 10, 0, 0, 7, ws, big, None) == -9
    assert lib.chol_fwd_ex(0, 10, fake, 10, fake, 10, 33, 0, 1, ws, big, None) == -7
    assert lib.chol_factor_ex(0, 10, fake, 10, 0, 2, fake, ws, big, None) == -6               # layout
    assert lib.chol_factor_ex(0, 10, fake, 10, 0, 1, None, ws, big, None) == -7
    assert lib.chol_factor_ex(0, 10, fake, 5, 0, 1, fake, ws, big, None) == -4
    assert lib.chol_factor_ex(0, 10, fake, 10, 0, 1, fake, ws, 16, None) == -102
    assert lib.chol_factor_ex(0, 0, None, 0, 0, 1, None, None, 0, None) == 0
    # column-major rev / fwd need n*n more doubles for the transposed copy of L
    ext = lib.chol_workspace_bytes_ex
    assert ext(1, 0, 1000, 0, 0) == lib.chol_workspace_bytes(1, 0, 1000, 0)
    assert ext(1, 0, 1000, 0, 1) == lib.chol_workspace_bytes(1, 0, 1000, 0) + 8 * 1000 * 1000
    assert ext(2, 0, 1000, 0, 1) == lib.chol_workspace_bytes(2, 0, 1000, 0) + 8 * 1000 * 1000
    assert ext(0, 0, 1000, 0, 1) == lib.chol_workspace_bytes(0, 0, 1000, 0)
    assert ext(1, 0, 1000, 0, 5) == 0 and ext(1, 0, 0, 0, 1) == 0
    assert lib.chol_factor(0, 10, fake, 10, 0, None, ws, big, None) == -6
    assert lib.chol_factor(0, 10, fake, 5, 0, fake, ws, big, None) == -4
    assert lib.chol_factor(0, 0, None, 0, 0, None, None, 0, None) == 0


def test_precision_modes_on_host():
    """The reduced-precision trailing modes (FP32 and split-bf16) exist only for the single-matrix
    calls; the batched calls refuse them as unsupported before any launch."""
    lib = _lib()
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    big = 1 << 40
    assert lib.chol_workspace_bytes(1, 2, 1000, 0) == lib.chol_workspace_bytes(1, 0, 1000, 0) > 0
    assert lib.chol_workspace_bytes(1, 3, 1000, 0) == lib.chol_workspace_bytes(1, 0, 1000, 0)
    assert lib.chol_workspace_bytes(1, 6, 1000, 0) == 0       # no mode 6
    assert lib.chol_batched_workspace_bytes(2, 1, 4) == 0
    assert lib.chol_batched_workspace_bytes(1, 1, 512) > lib.chol_batched_workspace_bytes(0, 1, 512) > 0
    assert lib.chol_factor_batched(2, 1, None, None, None, 4, None, None, 0, None) == -103
    assert lib.chol_factor_batched(3, 1, None, None, None, 4, None, None, 0, None) == -103
    assert lib.chol_batched_workspace_bytes(3, 1, 4) == 0
    assert lib.chol_factor_batched(7, 1, None, None, None, 4, None, None, 0, None) == -1


def test_noalloc_entry_rejects_on_host():
    """chol_rev_noalloc validates every argument, then its size limits (n <= 4096, nb <= 128),
    before it touches a device."""
    lib = _lib()
    fake = ctypes.c_void_p(4096)
    f = lib.chol_rev_noalloc
    assert f(7, 10, fake, 10, fake, 10, 0, 0, None) == -1
    assert f(0, -1, fake, 10, fake, 10, 0, 0, None) == -2
    assert f(0, 10, None, 10, fake, 10, 0, 0, None) == -3
    assert f(0, 10, fake, 9, fake, 10, 0, 0, None) == -4
    assert f(0, 10, fake, 10, fake, 3, 0, 0, None) == -6
    assert f(0, 10, fake, 10, fake, 10, 2, 0, None) == -7
    assert f(0, 10, fake, 10, fake, 10, 0, 40, None) == -8
    assert f(0, 10, fake, 10, fake, 10, 0, 144, None) == -8      # valid for chol_rev, above 128 here
    assert f(0, 4097, fake, 4097, fake, 4097, 0, 0, None) == -104
    assert f(1, 10, fake, 10, fake, 10, 0, 0, None) == -103
    assert f(0, 0, None, 0, None, 0, 0, 0, None) == 0
    assert lib.chol_status_string(-104).startswith(b"problem larger")


def test_storage_and_split_modes_on_host():
    """CHOL_PREC_F64_TRAIL_BF16X6 (4) and the FP32-storage single-matrix modes (1 and
    CHOL_PREC_F32_TRAIL_BF16X3 = 5): the FP32-storage workspace adds n*n doubles per matrix
    argument (one for the factor, two for rev / fwd) to the FP64 sweep's; the batched calls refuse
    the split and FP32-trailing modes as unsupported."""
    lib = _lib()
    n = 1000
    copy = 8 * n * n
    for op, copies in ((0, 1), (1, 2), (2, 2)):
        f64 = lib.chol_workspace_bytes(op, 0, n, 0)
        assert lib.chol_workspace_bytes(op, 4, n, 0) == f64
        assert lib.chol_workspace_bytes(op, 1, n, 0) == f64 + copies * copy
        assert lib.chol_workspace_bytes(op, 5, n, 0) == f64 + copies * copy
        assert lib.chol_workspace_bytes_ex(op, 1, n, 0, 1) == f64 + copies * copy   # no transposed copy of L
    for prec in (2, 3, 4, 5):
        assert lib.chol_batched_workspace_bytes(prec, 4, 100) == 0
        assert lib.chol_factor_batched(prec, 1, None, None, None, 4, None, None, 0, None) == -103
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    big = 1 << 40
    assert lib.chol_rev(1, 10, ctypes.c_void_p(4098), 10, fake, 10, 0, 0, ws, big, None) == -3   # float alignment
    assert lib.chol_rev(1, 10, fake, 10, fake, 10, 0, 0, ws, 16, None) == -102
    assert lib.chol_rev_ex(5, 10, fake, 10, fake, 10, 0, 256, 2, 0, ws, big, None) == -103        # Level-2, nb > 128
    assert lib.chol_factor(1, 10, fake, 10, 0, None, ws, big, None) == -6
    assert lib.chol_fwd_ex(1, 10, fake, 10, fake, 10, 0, 0, 3, ws, big, None) == -9
    assert lib.chol_rev_noalloc(1, 10, fake, 10, fake, 10, 0, 0, None) == -103
