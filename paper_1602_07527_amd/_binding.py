"""ctypes binding of libcholgrad (argument marshalling only: every step runs in the HIP kernels).

Tensors are torch CUDA (ROCm) tensors used as device memory; calls are enqueued on torch's current
stream of the tensors' device.  Errors from the C ABI raise CholError.  There is no CPU path: if
the library is not built, every entry point raises.
"""
import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcholgrad.so")

PREC_F64 = 0
PREC_F32 = 1
PREC_F64_TRAIL_F32 = 2
PREC_F64_TRAIL_BF16X3 = 3
PREC_F64_TRAIL_BF16X6 = 4
PREC_F32_TRAIL_BF16X3 = 5
# Precision modes of the single-matrix calls: FP64 storage, or FP32 storage ('f32*', float32
# tensors, computed on FP64 copies inside the library).
_PRECS = {"f64": PREC_F64, "f64_trail_f32": PREC_F64_TRAIL_F32, "f64_trail_bf16x3": PREC_F64_TRAIL_BF16X3,
          "f64_trail_bf16x6": PREC_F64_TRAIL_BF16X6, "f32": PREC_F32, "f32_trail_bf16x3": PREC_F32_TRAIL_BF16X3}


def _storage(precision):
    """Tensor dtype of a single-matrix precision mode."""
    return (torch.float32,) if str(precision).startswith("f32") else (torch.float64,)
SBAR_SYM, SBAR_TRIL = 0, 1
OP_FACTOR, OP_REV, OP_FWD = 0, 1, 2
_FORMS = {"sym": SBAR_SYM, "tril": SBAR_TRIL}
DIAG_AUTO, DIAG_SYMBOLIC, DIAG_LEVEL2 = 0, 1, 2
_DIAGS = {"auto": DIAG_AUTO, "symbolic": DIAG_SYMBOLIC, "level2": DIAG_LEVEL2}
LAYOUT_ROW_MAJOR, LAYOUT_COL_MAJOR = 0, 1
_LAYOUTS = {"row": LAYOUT_ROW_MAJOR, "col": LAYOUT_COL_MAJOR}
_OPS = {"factor": OP_FACTOR, "rev": OP_REV, "fwd": OP_FWD}

_lib = None


def _pick(table, key, what):
    """table[key], or a ValueError naming the accepted values."""
    try:
        return table[key]
    except (KeyError, TypeError):
        raise ValueError(f"unknown {what} {key!r}; expected one of {sorted(table)}") from None


class CholError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def load_library():
    """Load libcholgrad.so from the package folder (raises ImportError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
                          "g.build()'` from the repository root")
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, i32, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.chol_workspace_bytes.argtypes = [i32, i32, i64, i32]
    lib.chol_workspace_bytes.restype = sz
    lib.chol_workspace_bytes_ex.argtypes = [i32, i32, i64, i32, i32]
    lib.chol_workspace_bytes_ex.restype = sz
    lib.chol_factor.argtypes = [i32, i64, vp, i64, i32, vp, vp, sz, vp]
    lib.chol_factor.restype = i32
    lib.chol_factor_ex.argtypes = [i32, i64, vp, i64, i32, i32, vp, vp, sz, vp]
    lib.chol_factor_ex.restype = i32
    lib.chol_rev.argtypes = [i32, i64, vp, i64, vp, i64, i32, i32, vp, sz, vp]
    lib.chol_rev_ex.argtypes = [i32, i64, vp, i64, vp, i64, i32, i32, i32, i32, vp, sz, vp]
    lib.chol_rev.restype = i32
    lib.chol_rev_noalloc.argtypes = [i32, i64, vp, i64, vp, i64, i32, i32, vp]
    lib.chol_rev_noalloc.restype = i32
    lib.chol_fwd.argtypes = [i32, i64, vp, i64, vp, i64, i32, vp, sz, vp]
    lib.chol_fwd_ex.argtypes = [i32, i64, vp, i64, vp, i64, i32, i32, i32, vp, sz, vp]
    lib.chol_fwd.restype = i32
    lib.chol_factor_fwd.argtypes = [i32, i64, vp, i64, vp, i64, i32, vp, vp, sz, vp]
    lib.chol_factor_fwd.restype = i32
    lib.chol_status_string.argtypes = [i32]
    lib.chol_status_string.restype = ctypes.c_char_p
    lib.chol_version.argtypes = []
    lib.chol_version.restype = i32
    lib.chol_batched_workspace_bytes.argtypes = [i32, i32, i64]
    lib.chol_batched_workspace_bytes.restype = sz
    lib.chol_factor_batched.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp, sz, vp]
    lib.chol_factor_batched.restype = i32
    lib.chol_rev_batched.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, i32, vp, sz, vp]
    lib.chol_rev_batched.restype = i32
    lib.chol_fwd_batched.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, vp, sz, vp]
    lib.chol_fwd_batched.restype = i32
    lib.chol_factor_rev_batched.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, i32, vp, vp, sz, vp]
    lib.chol_factor_rev_batched.restype = i32
    lib.chol_gp_nll_batched.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp, vp, sz, vp]
    lib.chol_gp_nll_batched.restype = i32
    lib.chol_profile_begin.argtypes = [i32]
    lib.chol_profile_begin.restype = i32
    lib.chol_profile_end.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.chol_profile_end.restype = i32
    _lib = lib
    return lib


def _check(fn, status):
    if status != 0:
        lib = load_library()
        raise CholError(fn, status, lib.chol_status_string(status).decode())


def _square(name, t, dtypes=(torch.float64,), layout="row"):
    """n of a square matrix tensor in the given storage: 'row' (unit column stride) or 'col'
    (column-major, unit row stride, e.g. `x.T.contiguous().T`)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must be {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square 2-D, got {tuple(t.shape)}")
    n = t.shape[0]
    if layout == "col":
        if n > 0 and (t.stride(0) != 1 or t.stride(1) < n):
            raise ValueError(f"{name} must be column-major with unit row stride for layout='col'")
    elif n > 0 and (t.stride(1) != 1 or t.stride(0) < n):
        raise ValueError(f"{name} must be row-major with unit column stride")
    return n


def _ld(t, layout="row"):
    """Leading dimension of a matrix tensor in its storage layout (1 for an empty matrix)."""
    if t.shape[0] == 0:
        return 1
    return t.stride(1) if layout == "col" else t.stride(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_bytes(op, n, nb=0, precision="f64", layout="row"):
    """Device workspace bytes for op in {'factor', 'rev', 'fwd'} at size n and block size nb, for
    matrices stored in `layout` ('row' or 'col')."""
    op_code, prec = _pick(_OPS, op, "op"), _pick(_PRECS, precision, "precision")
    lay = _pick(_LAYOUTS, layout, "layout")
    return int(load_library().chol_workspace_bytes_ex(op_code, prec, int(n), int(nb), lay))


def _workspace(op, n, nb, device, workspace, precision="f64", layout="row"):
    need = workspace_bytes(op, n, nb, precision, layout)
    if workspace is None:
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if workspace.device != device or workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace must hold {need} bytes on {device}")
    return workspace


def chol_factor(A, nb=0, workspace=None, info=None, precision="f64", layout="row"):
    """In place: tril(A) = Sigma -> tril(A) = L, strict upper set to 0.  Returns (A, info) where
    info is a device int32 tensor (0, or the 1-based column of the first non-positive pivot).
    precision: 'f64', 'f64_trail_f32' (trailing updates on FP32 MFMA) or 'f64_trail_bf16x3'
    (trailing updates as split-bfloat16 products).  layout: 'row', or 'col' for column-major
    (LAPACK) storage of A."""
    lib = load_library()
    prec, lay = _pick(_PRECS, precision, "precision"), _pick(_LAYOUTS, layout, "layout")
    n = _square("A", A, _storage(precision), layout)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    ws = _workspace("factor", n, nb, A.device, workspace, precision, layout)
    with torch.cuda.device(A.device):
        _check("chol_factor", lib.chol_factor_ex(prec, n, A.data_ptr(), _ld(A, layout), nb, lay,
                                                 info.data_ptr(), ws.data_ptr(), ws.numel(),
                                                 _stream(A.device)))
    return A, info


def chol_rev(L, A, form="sym", nb=0, workspace=None, precision="f64", diag="auto", layout="row"):
    """In place: tril(A) = L-bar -> A = Sigma-bar in the chosen form ('sym' or 'tril').
    diag: diagonal-block variant, 'auto', 'symbolic' or 'level2' (CHOL_DIAG_*); layout: 'row', or
    'col' for column-major (LAPACK) storage of L and A."""
    lib = load_library()
    prec, fm, dv = _pick(_PRECS, precision, "precision"), _pick(_FORMS, form, "form"), _pick(_DIAGS, diag, "diag")
    lay = _pick(_LAYOUTS, layout, "layout")
    n = _square("L", L, _storage(precision), layout)
    if _square("A", A, _storage(precision), layout) != n or A.device != L.device:
        raise ValueError("L and A must have the same size and device")
    ws = _workspace("rev", n, nb, A.device, workspace, precision, layout)
    with torch.cuda.device(A.device):
        _check("chol_rev", lib.chol_rev_ex(prec, n, L.data_ptr(), _ld(L, layout), A.data_ptr(), _ld(A, layout),
                                           fm, nb, dv, lay, ws.data_ptr(), ws.numel(), _stream(A.device)))
    return A


def chol_rev_noalloc(L, A, form="sym", nb=0, precision="f64"):
    """chol_rev without a workspace: the library's static device scratch (n <= 4096, nb <= 128;
    symbolic diagonal blocks; row-major).  Calls overlapping on one device race (see the header)."""
    lib = load_library()
    prec, fm = _pick(_PRECS, precision, "precision"), _pick(_FORMS, form, "form")
    n = _square("L", L)
    if _square("A", A) != n or A.device != L.device:
        raise ValueError("L and A must have the same size and device")
    with torch.cuda.device(A.device):
        _check("chol_rev_noalloc", lib.chol_rev_noalloc(prec, n, L.data_ptr(), _ld(L), A.data_ptr(), _ld(A), fm,
                                                        nb, _stream(A.device)))
    return A


def chol_fwd(L, A, nb=0, workspace=None, precision="f64", diag="auto", layout="row"):
    """In place: tril(A) = tril(Sigma-dot) -> tril(A) = L-dot, strict upper set to 0.
    diag: diagonal-block variant, 'auto', 'symbolic' or 'level2' (CHOL_DIAG_*); layout: 'row', or
    'col' for column-major (LAPACK) storage of L and A."""
    lib = load_library()
    prec, dv = _pick(_PRECS, precision, "precision"), _pick(_DIAGS, diag, "diag")
    lay = _pick(_LAYOUTS, layout, "layout")
    n = _square("L", L, _storage(precision), layout)
    if _square("A", A, _storage(precision), layout) != n or A.device != L.device:
        raise ValueError("L and A must have the same size and device")
    ws = _workspace("fwd", n, nb, A.device, workspace, precision, layout)
    with torch.cuda.device(A.device):
        _check("chol_fwd", lib.chol_fwd_ex(prec, n, L.data_ptr(), _ld(L, layout), A.data_ptr(), _ld(A, layout),
                                           nb, dv, lay, ws.data_ptr(), ws.numel(), _stream(A.device)))
    return A


def chol_factor_fwd(A, D, nb=0, workspace=None, info=None, precision="f64"):
    """In place, one sweep: tril(A) = Sigma -> L and tril(D) = tril(Sigma-dot) -> L-dot (strict
    upper triangles set to 0).  Returns (A, D, info)."""
    lib = load_library()
    prec = _pick(_PRECS, precision, "precision")
    n = _square("A", A, _storage(precision))
    if _square("D", D, _storage(precision)) != n or D.device != A.device:
        raise ValueError("A and D must have the same size and device")
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    ws = _workspace("fwd", n, nb, A.device, workspace, precision)
    with torch.cuda.device(A.device):
        _check("chol_factor_fwd", lib.chol_factor_fwd(prec, n, A.data_ptr(), A.stride(0) if n else 1,
                                                      D.data_ptr(), D.stride(0) if n else 1, nb, info.data_ptr(),
                                                      ws.data_ptr(), ws.numel(), _stream(A.device)))
    return A, D, info


def profile_begin(max_launches=1 << 16):
    """Start bracketing every sweep's panel-contraction launch with HIP events."""
    _check("chol_profile_begin", load_library().chol_profile_begin(int(max_launches)))


def profile_end():
    """Stop and return {'rev'|'factor'|'fwd': (kernel_ms, flops, algorithmic_bytes, launches)}."""
    ms = (ctypes.c_double * 3)()
    fl = (ctypes.c_double * 3)()
    by = (ctypes.c_double * 3)()
    nl = (ctypes.c_int64 * 3)()
    _check("chol_profile_end", load_library().chol_profile_end(ms, fl, by, nl))
    return {k: (ms[i], fl[i], by[i], int(nl[i])) for i, k in enumerate(("rev", "factor", "fwd"))}


# ------------------------------------------------------------------------------------------------
# Batched forms (one call over many problems: step-synchronous grouped launches, or one
# persistent launch for the forward sweep)

BATCH_NMAX = 512


_BATCH_PREC = {torch.float64: PREC_F64, torch.float32: PREC_F32}


class Batch:
    """Device-side description of a list of square matrices (sizes, pointers, leading dimensions),
    built once and reusable across calls on the same tensors.  All matrices share one dtype:
    float64 (FP64) or float32 (FP32 storage, computed in FP64 inside the library)."""

    def __init__(self, mats):
        if len(mats) == 0:
            raise ValueError("empty batch")
        dev = mats[0].device
        self.dtype = mats[0].dtype
        if self.dtype not in _BATCH_PREC:
            raise TypeError(f"batched calls take float64 or float32 matrices, got {self.dtype}")
        self.prec = _BATCH_PREC[self.dtype]
        sizes, ptrs, lds = [], [], []
        for t in mats:
            if t.device != dev:
                raise ValueError("all matrices of a batch must be on one device")
            n = _square("batch matrix", t, (self.dtype,))
            sizes.append(n)
            ptrs.append(t.data_ptr())
            lds.append(t.stride(0) if n else 1)
        self.device = dev
        self.mats = list(mats)
        self.sizes = sizes
        self.n_max = max(sizes)
        if self.n_max > BATCH_NMAX:
            raise ValueError(f"batched calls support n <= {BATCH_NMAX}")
        self.n = torch.tensor(sizes, dtype=torch.int64).to(dev)
        self.ptr = torch.tensor(ptrs, dtype=torch.int64).to(dev)
        self.ld = torch.tensor(lds, dtype=torch.int64).to(dev)

    def __len__(self):
        return len(self.sizes)


class Vecs:
    """Device-side pointer table of a list of vectors (one per matrix of a Batch), built once and
    reusable across calls on the same tensors, as Batch is for the matrices."""

    def __init__(self, vecs):
        if len(vecs) == 0:
            raise ValueError("empty vector list")
        self.device, self.dtype = vecs[0].device, vecs[0].dtype
        for v in vecs:
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == self.dtype and v.is_contiguous()
                    and v.dim() == 1 and v.device == self.device):
                raise ValueError("vectors must be contiguous 1-D device tensors of one dtype and device")
        self.vecs = list(vecs)
        self.sizes = [int(v.numel()) for v in vecs]
        self.ptr = torch.tensor([v.data_ptr() for v in vecs], dtype=torch.int64).to(self.device)

    def __len__(self):
        return len(self.sizes)


def _vec_ptrs(vecs, sizes, dev, dtype):
    if not isinstance(vecs, Vecs):
        vecs = Vecs(list(vecs)) if len(vecs) else None
    if vecs is None or vecs.sizes != list(sizes) or vecs.device != dev or vecs.dtype != dtype:
        raise ValueError(f"vectors must be contiguous {dtype} device tensors matching the sizes")
    return vecs.ptr


def batched_workspace_bytes(batch, n_max, prec=PREC_F64):
    return int(load_library().chol_batched_workspace_bytes(int(prec), int(batch), int(n_max)))


def _batch_ws(batch, n_max, device, workspace, prec=PREC_F64):
    need = batched_workspace_bytes(batch, n_max, prec)
    if workspace is None:
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace must hold {need} bytes")
    return workspace


def _as_batch(x):
    return x if isinstance(x, Batch) else Batch(x)


def chol_factor_batched(A, info=None, workspace=None):
    """In place on every matrix: tril = Sigma -> L (strict upper 0).  Returns the device int32
    info array (0, LAPACK-style pivot index, or -1 for an invalid entry)."""
    lib = load_library()
    A = _as_batch(A)
    if info is None:
        info = torch.empty(len(A), dtype=torch.int32, device=A.device)
    ws = _batch_ws(len(A), A.n_max, A.device, workspace, A.prec)
    with torch.cuda.device(A.device):
        _check("chol_factor_batched", lib.chol_factor_batched(
            A.prec, len(A), A.n.data_ptr(), A.ptr.data_ptr(), A.ld.data_ptr(), A.n_max, info.data_ptr(),
            ws.data_ptr(), ws.numel(), _stream(A.device)))
    return info


def chol_rev_batched(L, A, form="sym", workspace=None):
    """In place on every A[b]: tril = L-bar -> Sigma-bar (form 'sym' or 'tril')."""
    lib = load_library()
    L, A = _as_batch(L), _as_batch(A)
    if L.sizes != A.sizes or L.dtype != A.dtype or L.device != A.device:
        raise ValueError("L and A batches must have the same sizes, dtype and device")
    ws = _batch_ws(len(A), A.n_max, A.device, workspace, A.prec)
    with torch.cuda.device(A.device):
        _check("chol_rev_batched", lib.chol_rev_batched(
            A.prec, len(A), A.n.data_ptr(), L.ptr.data_ptr(), L.ld.data_ptr(), A.ptr.data_ptr(),
            A.ld.data_ptr(), A.n_max, _pick(_FORMS, form, "form"), ws.data_ptr(), ws.numel(), _stream(A.device)))
    return A.mats


def chol_fwd_batched(L, A, workspace=None):
    """In place on every A[b]: tril = tril(Sigma-dot) -> L-dot (strict upper 0)."""
    lib = load_library()
    L, A = _as_batch(L), _as_batch(A)
    if L.sizes != A.sizes or L.dtype != A.dtype or L.device != A.device:
        raise ValueError("L and A batches must have the same sizes, dtype and device")
    ws = _batch_ws(len(A), A.n_max, A.device, workspace, A.prec)
    with torch.cuda.device(A.device):
        _check("chol_fwd_batched", lib.chol_fwd_batched(
            A.prec, len(A), A.n.data_ptr(), L.ptr.data_ptr(), L.ld.data_ptr(), A.ptr.data_ptr(),
            A.ld.data_ptr(), A.n_max, ws.data_ptr(), ws.numel(), _stream(A.device)))
    return A.mats


def chol_factor_rev_batched(A, G, form="sym", info=None, workspace=None):
    """Per problem b, in one launch: A[b] (Sigma -> L, kept) then G[b] (L-bar -> Sigma-bar in the
    chosen form, on that L).  Returns the device int32 info array."""
    lib = load_library()
    A, G = _as_batch(A), _as_batch(G)
    if A.sizes != G.sizes or A.dtype != G.dtype or A.device != G.device:
        raise ValueError("A and G batches must have the same sizes, dtype and device")
    if info is None:
        info = torch.empty(len(A), dtype=torch.int32, device=A.device)
    ws = _batch_ws(len(A), A.n_max, A.device, workspace, A.prec)
    with torch.cuda.device(A.device):
        _check("chol_factor_rev_batched", lib.chol_factor_rev_batched(
            A.prec, len(A), A.n.data_ptr(), A.ptr.data_ptr(), A.ld.data_ptr(), G.ptr.data_ptr(),
            G.ld.data_ptr(), A.n_max, _pick(_FORMS, form, "form"), info.data_ptr(), ws.data_ptr(), ws.numel(),
            _stream(A.device)))
    return info


def chol_gp_nll_batched(A, y, G, f=None, info=None, workspace=None):
    """Per problem b, in one launch: A[b] (Sigma -> L), f[b] = sum log L_ii + |L^-1 y_b|^2 / 2 and
    G[b] = df_b/dSigma_b (symmetric).  y is a list of vectors or a prebuilt Vecs.  Returns
    (f, info) device tensors."""
    lib = load_library()
    A, G = _as_batch(A), _as_batch(G)
    if A.sizes != G.sizes or A.dtype != G.dtype or A.device != G.device:
        raise ValueError("A and G batches must have the same sizes, dtype and device")
    yp = _vec_ptrs(y, A.sizes, A.device, A.dtype)
    if f is None:
        f = torch.empty(len(A), dtype=A.dtype, device=A.device)
    elif f.dtype != A.dtype or f.numel() < len(A) or not f.is_contiguous() or f.device != A.device:
        raise ValueError(f"f must be a contiguous {A.dtype} device tensor with one entry per problem")
    if info is None:
        info = torch.empty(len(A), dtype=torch.int32, device=A.device)
    ws = _batch_ws(len(A), A.n_max, A.device, workspace, A.prec)
    with torch.cuda.device(A.device):
        _check("chol_gp_nll_batched", lib.chol_gp_nll_batched(
            A.prec, len(A), A.n.data_ptr(), A.ptr.data_ptr(), A.ld.data_ptr(), yp.data_ptr(),
            G.ptr.data_ptr(), G.ld.data_ptr(), f.data_ptr(), A.n_max, info.data_ptr(), ws.data_ptr(),
            ws.numel(), _stream(A.device)))
    return f, info
