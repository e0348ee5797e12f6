"""ctypes binding of ``libata.so`` (argument marshalling only).

The functions named like the C entry points (``ata_create``, ``ata_gram``,
``ata_gram_batched``, ``ata_destroy``, ``ata_set_option``, ``ata_get_report``,
``ata_plan_query``) take plain integers for device pointers and streams and
return what the C call returns, raising ``AtaError`` on a non-OK status.
``gram`` is the torch convenience wrapper: it allocates the packed output
tensor on the input's device and calls ``ata_gram`` on the current stream.

There is no fallback: if the library is missing, or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libata.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ata.h")

F64, F32, F32_BF16X3, F32_FP8E4M3 = 0, 1, 2, 3
DTYPE_NAMES = {"f64": F64, "f32": F32, "bf16x3": F32_BF16X3, "fp8": F32_FP8E4M3}

OPT_LEAF_CUTOFF, OPT_MAX_STRASSEN_DEPTH, OPT_SPREAD_TAU = 0, 1, 2
OPT_RESIDUAL, OPT_WORKSPACE_LIMIT, OPT_RESIDUAL_SEED, OPT_PROFILE = 3, 4, 5, 6
OPT_LEAF_TILE, OPT_BATCH_GRAPH, OPT_BATCH_PERSISTENT = 7, 8, 9
OPT_XCD_CHUNK, OPT_TILE_BAND, OPT_SPLIT_TARGET, OPT_BATCH_USE_TABLE = 10, 11, 12, 13
OPT_EQUILIBRATE = 14
OPT_LEAF_PERSISTENT = 15
OPT_FUSE_PRESUM = 16
OPT_STRASSEN_FORM = 17
OPT_BALANCE_TAIL = 18
OPT_BOUNDED_WORKSPACE = 19
OPT_OVERLAP = 20
OPT_FUSE_COMBINE = 21

STATUS = {0: "ATA_OK", 1: "ATA_ERR_INVALID_VALUE", 2: "ATA_ERR_NOT_SUPPORTED",
          3: "ATA_ERR_OUT_OF_MEMORY", 4: "ATA_ERR_HIP", 5: "ATA_ERR_INTERNAL"}


class AtaError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class Report(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("strassen_levels", ctypes.c_int32),
                ("leaf_cutoff", ctypes.c_int64), ("ata_nodes", ctypes.c_int64),
                ("syrk_leaves", ctypes.c_int64), ("gemm_leaves", ctypes.c_int64),
                ("strassen_nodes", ctypes.c_int64), ("multiplications", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("kernel_launches", ctypes.c_int64),
                ("flagged_nodes", ctypes.c_int64), ("residual", ctypes.c_double),
                ("profiled_calls", ctypes.c_int64), ("phase_ms", ctypes.c_double * 5),
                ("leaf_tile", ctypes.c_int32), ("leaf_persistent", ctypes.c_int32),
                ("tail_split_leaves", ctypes.c_int32), ("tail_split_chunks", ctypes.c_int32),
                ("overlapped", ctypes.c_int32), ("leaf_rounds", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        return d


class TuneEntry(ctypes.Structure):
    _fields_ = [("leaf_cutoff", ctypes.c_int64), ("max_depth", ctypes.c_int32),
                ("leaf_tile", ctypes.c_int32), ("ms", ctypes.c_double)]


class Leaf(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("contraction", ctypes.c_int64), ("out_row0", ctypes.c_int64),
                ("out_col0", ctypes.c_int64), ("ksplit", ctypes.c_int32), ("pad_", ctypes.c_int32)]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libata.so (raises if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    L.ata_create.argtypes = [ctypes.POINTER(vp)]
    L.ata_destroy.argtypes = [vp]
    L.ata_gram.argtypes = [vp, vp, i64, i64, i64, st, vp, vp]
    L.ata_gram_noalloc.argtypes = [vp, vp, i64, i64, i64, st, vp, vp]
    L.ata_gram_batched.argtypes = [vp, i64, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                   ctypes.POINTER(i64), ctypes.POINTER(i64), st,
                                   ctypes.POINTER(vp), vp]
    L.ata_set_option.argtypes = [vp, st, ctypes.c_double]
    L.ata_get_report.argtypes = [vp, ctypes.POINTER(Report)]
    L.ata_plan_query.argtypes = [i64, i64, st, i64, i32, ctypes.POINTER(Report),
                                 ctypes.POINTER(Leaf), i64, ctypes.POINTER(i64)]
    L.ata_check_columns.argtypes = [vp, vp, i64, i64, i64, st, vp, ctypes.POINTER(i64), i64,
                                    ctypes.POINTER(ctypes.c_double), vp]
    L.ata_residual.argtypes = [vp, vp, i64, i64, i64, st, vp, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_double), vp]
    L.ata_autotune.argtypes = [vp, vp, i64, i64, i64, st, vp, vp, ctypes.POINTER(TuneEntry)]
    L.ata_gemm_tn.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, st, vp, i64, vp]
    L.ata_gram_scaled.argtypes = [vp, vp, i64, i64, i64, st, ctypes.c_double, ctypes.c_double, vp, vp]
    L.ata_gram_aat.argtypes = [vp, vp, i64, i64, i64, st, vp, vp]
    L.ata_unpack.argtypes = [vp, vp, i64, st, vp, i64, vp]
    L.ata_autotune_batched.argtypes = [vp, i64, vp, vp, vp, vp, st, vp, vp, ctypes.POINTER(TuneEntry)]
    L.ata_tune_save.argtypes = [vp, ctypes.c_char_p]
    L.ata_tune_load.argtypes = [vp, ctypes.c_char_p]
    L.ata_get_spread.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64, ctypes.POINTER(i64),
                                 ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_uint8), i64,
                                 ctypes.POINTER(i64)]
    L.ata_status_string.argtypes = [st]
    L.ata_status_string.restype = ctypes.c_char_p
    for name in ("ata_create", "ata_destroy", "ata_gram", "ata_gram_noalloc", "ata_gram_batched", "ata_set_option",
                 "ata_get_report", "ata_plan_query", "ata_residual", "ata_check_columns", "ata_autotune",
                 "ata_autotune_batched",
                 "ata_gemm_tn", "ata_gram_scaled", "ata_gram_aat", "ata_unpack",
                 "ata_tune_save", "ata_tune_load", "ata_get_spread"):
        getattr(L, name).restype = st
    _LIB = L
    return L


def header_symbols() -> list:
    """Entry points declared in include/ata.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|ata_status_t)\s+(ata_\w+)\s*\(", text, re.M)))


def _check(status: int, where: str) -> None:
    if status != 0:
        raise AtaError(status, where)


# ----------------------------------------------------------- C-ABI mirrors
def ata_create() -> int:
    h = ctypes.c_void_p()
    _check(lib().ata_create(ctypes.byref(h)), "ata_create")
    return h.value


def ata_destroy(h: int) -> None:
    _check(lib().ata_destroy(h), "ata_destroy")


def ata_gram(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, stream: int = 0) -> None:
    _check(lib().ata_gram(h, A, m, n, lda, dtype, C, stream), "ata_gram")


def ata_gram_noalloc(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, stream: int = 0) -> None:
    _check(lib().ata_gram_noalloc(h, A, m, n, lda, dtype, C, stream), "ata_gram_noalloc")


NOALLOC_SCRATCH_BYTES = 256 << 20      # ATA_NOALLOC_SCRATCH_BYTES


def batch_arrays(A_ptrs, ms, ns, ldas, C_ptrs):
    """ctypes arrays for ata_gram_batched, built once and reusable across calls."""
    b = len(A_ptrs)
    arr_p = ctypes.c_void_p * b
    arr_i = ctypes.c_int64 * b
    return arr_p(*A_ptrs), arr_i(*ms), arr_i(*ns), arr_i(*ldas), arr_p(*C_ptrs)


def ata_gram_batched(h: int, A_ptrs, ms, ns, ldas, dtype: int, C_ptrs, stream: int = 0) -> None:
    arrs = (A_ptrs, ms, ns, ldas, C_ptrs)
    if not isinstance(A_ptrs, ctypes.Array):
        arrs = batch_arrays(A_ptrs, ms, ns, ldas, C_ptrs)
    _check(lib().ata_gram_batched(h, len(arrs[0]), arrs[0], arrs[1], arrs[2], arrs[3], dtype, arrs[4],
                                  stream), "ata_gram_batched")


def ata_gemm_tn(h: int, A: int, B: int, m: int, n: int, k: int, lda: int, ldb: int, dtype: int,
                C: int, ldc: int, stream: int = 0) -> None:
    _check(lib().ata_gemm_tn(h, A, B, m, n, k, lda, ldb, dtype, C, ldc, stream), "ata_gemm_tn")


def ata_gram_scaled(h: int, A: int, m: int, n: int, lda: int, dtype: int, alpha: float, beta: float,
                    C: int, stream: int = 0) -> None:
    _check(lib().ata_gram_scaled(h, A, m, n, lda, dtype, alpha, beta, C, stream), "ata_gram_scaled")


def ata_gram_aat(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, stream: int = 0) -> None:
    _check(lib().ata_gram_aat(h, A, m, n, lda, dtype, C, stream), "ata_gram_aat")


def ata_unpack(h: int, Cp: int, n: int, dtype: int, F: int, ldf: int, stream: int = 0) -> None:
    _check(lib().ata_unpack(h, Cp, n, dtype, F, ldf, stream), "ata_unpack")


def ata_set_option(h: int, key: int, value: float) -> None:
    _check(lib().ata_set_option(h, key, float(value)), "ata_set_option")


def ata_get_report(h: int) -> dict:
    r = Report()
    _check(lib().ata_get_report(h, ctypes.byref(r)), "ata_get_report")
    return r.as_dict()


def ata_get_spread(h: int, n: int):
    """(nu, [(c0, w, flag), ...]) of the last ata_gram call's spread check:
    nu as a list of n floats, then every AtA node in the recursion's pre-order."""
    count = ctypes.c_int64()
    _check(lib().ata_get_spread(h, None, 0, None, None, None, 0, ctypes.byref(count)), "ata_get_spread")
    k = count.value
    nu = (ctypes.c_double * max(n, 1))()
    c0 = (ctypes.c_int64 * max(k, 1))()
    w = (ctypes.c_int64 * max(k, 1))()
    fl = (ctypes.c_uint8 * max(k, 1))()
    _check(lib().ata_get_spread(h, nu, n, c0, w, fl, k, ctypes.byref(count)), "ata_get_spread")
    return list(nu)[:n], [(c0[i], w[i], fl[i]) for i in range(k)]


def ata_plan_query(m: int, n: int, dtype: int, leaf_cutoff: int = 0, max_depth: int = -1):
    """(report dict, list of leaf dicts) of the plan; host only."""
    info = Report()
    count = ctypes.c_int64()
    _check(lib().ata_plan_query(m, n, dtype, leaf_cutoff, max_depth, ctypes.byref(info), None, 0,
                                ctypes.byref(count)), "ata_plan_query")
    leaves = (Leaf * max(count.value, 1))()
    _check(lib().ata_plan_query(m, n, dtype, leaf_cutoff, max_depth, None, leaves, count.value,
                                ctypes.byref(count)), "ata_plan_query")
    out = [{k: getattr(leaves[i], k) for k, _ in Leaf._fields_} for i in range(count.value)]
    return info.as_dict(), out


def ata_residual(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, seed: int,
                 stream: int = 0) -> float:
    r = ctypes.c_double()
    _check(lib().ata_residual(h, A, m, n, lda, dtype, C, seed, ctypes.byref(r), stream),
           "ata_residual")
    return r.value


def ata_check_columns(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, cols,
                      stream: int = 0) -> float:
    """FP64 sampled-column check on the GPU: ||C_S - (A^T A)_S||_F / ||(A^T A)_S||_F."""
    arr = (ctypes.c_int64 * max(len(cols), 1))(*[int(c) for c in cols])
    r = ctypes.c_double()
    _check(lib().ata_check_columns(h, A, m, n, lda, dtype, C, arr, len(cols), ctypes.byref(r), stream),
           "ata_check_columns")
    return r.value


def ata_autotune(h: int, A: int, m: int, n: int, lda: int, dtype: int, C: int, stream: int = 0) -> dict:
    e = TuneEntry()
    _check(lib().ata_autotune(h, A, m, n, lda, dtype, C, stream, ctypes.byref(e)), "ata_autotune")
    return {k: getattr(e, k) for k, _ in TuneEntry._fields_}


def ata_autotune_batched(h: int, A_ptrs, ms, ns, ldas, dtype: int, C_ptrs, stream: int = 0) -> dict:
    arrs = (A_ptrs, ms, ns, ldas, C_ptrs)
    if not isinstance(A_ptrs, ctypes.Array):
        arrs = batch_arrays(A_ptrs, ms, ns, ldas, C_ptrs)
    e = TuneEntry()
    _check(lib().ata_autotune_batched(h, len(arrs[0]), arrs[0], arrs[1], arrs[2], arrs[3], dtype, arrs[4],
                                      stream, ctypes.byref(e)), "ata_autotune_batched")
    return {k: getattr(e, k) for k, _ in TuneEntry._fields_}


def ata_tune_save(h: int, path: str) -> None:
    _check(lib().ata_tune_save(h, path.encode()), "ata_tune_save")


def ata_tune_load(h: int, path: str) -> None:
    _check(lib().ata_tune_load(h, path.encode()), "ata_tune_load")


def status_string(s: int) -> str:
    return lib().ata_status_string(s).decode()


# ------------------------------------------------------------ torch wrapper
class Handle:
    """Owns one ata handle; options are set by keyword."""

    def __init__(self, **options):
        self.h = ata_create()
        for k, v in options.items():
            self.set(k, v)

    def set(self, name: str, value) -> None:
        key = {"leaf_cutoff": OPT_LEAF_CUTOFF, "max_depth": OPT_MAX_STRASSEN_DEPTH,
               "spread_tau": OPT_SPREAD_TAU, "residual": OPT_RESIDUAL,
               "workspace_limit": OPT_WORKSPACE_LIMIT, "residual_seed": OPT_RESIDUAL_SEED,
               "profile": OPT_PROFILE, "leaf_tile": OPT_LEAF_TILE,
               "batch_graph": OPT_BATCH_GRAPH, "batch_persistent": OPT_BATCH_PERSISTENT,
               "xcd_chunk": OPT_XCD_CHUNK, "tile_band": OPT_TILE_BAND,
               "split_target": OPT_SPLIT_TARGET, "batch_use_table": OPT_BATCH_USE_TABLE,
               "equilibrate": OPT_EQUILIBRATE, "leaf_persistent": OPT_LEAF_PERSISTENT,
               "fuse_presum": OPT_FUSE_PRESUM, "strassen_form": OPT_STRASSEN_FORM,
               "balance_tail": OPT_BALANCE_TAIL, "bounded_workspace": OPT_BOUNDED_WORKSPACE,
               "overlap": OPT_OVERLAP, "fuse_combine": OPT_FUSE_COMBINE}[name]
        ata_set_option(self.h, key, value)

    def report(self) -> dict:
        return ata_get_report(self.h)

    def spread(self, n: int):
        """Column norms and per-node spread flags of the last ata_gram call."""
        return ata_get_spread(self.h, n)

    def autotune(self, A, dtype=None) -> dict:
        """Tune the plan for A's shape bucket (A's contents are only read)."""
        import torch
        mode = _mode_of(A, dtype)
        m, n = A.shape
        lda = max(A.stride(0) if m > 1 else n, n, 1)
        C = torch.empty(n * (n + 1) // 2, dtype=A.dtype, device=A.device)
        stream = torch.cuda.current_stream(A.device).cuda_stream
        return ata_autotune(self.h, A.data_ptr(), m, n, lda, mode, C.data_ptr(), stream)

    def tune_save(self, path: str) -> None:
        ata_tune_save(self.h, path)

    def tune_load(self, path: str) -> None:
        ata_tune_load(self.h, path)

    def close(self) -> None:
        if self.h:
            ata_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mode_of(A, dtype):
    import torch
    if dtype is None:
        return F64 if A.dtype == torch.float64 else F32
    return DTYPE_NAMES[dtype] if isinstance(dtype, str) else int(dtype)


_DEFAULT = {}


TUNE_TABLE = os.path.join(HERE, "tune_table.json")


def default_handle(device_index: int) -> Handle:
    """One long-lived handle per device (keeps its plan cache and workspace),
    with the packaged autotune table loaded when it exists."""
    if device_index not in _DEFAULT:
        h = Handle()
        if os.path.exists(TUNE_TABLE):
            h.tune_load(TUNE_TABLE)
        _DEFAULT[device_index] = h
    return _DEFAULT[device_index]


def gemm_tn(A, B, dtype=None, handle: Handle | None = None, out=None):
    """Dense C = A^T B (n x k) of 2-D CUDA tensors with contiguous rows."""
    import torch
    mode = _mode_of(A, dtype)
    want = torch.float64 if mode == F64 else torch.float32
    for X in (A, B):
        if X.dim() != 2 or not X.is_cuda or X.dtype != want:
            raise ValueError(f"need 2-D {want} tensors on a GPU")
        if X.shape[0] > 1 and X.shape[1] > 0 and X.stride(1) != 1:
            raise ValueError("rows must be contiguous")
    m, n = A.shape
    if B.shape[0] != m:
        raise ValueError("A and B need the same number of rows")
    k = B.shape[1]
    C = out if out is not None else torch.empty((n, k), dtype=want, device=A.device)
    h = handle or default_handle(A.device.index or 0)
    lda = max(A.stride(0) if m > 1 else n, n, 1)
    ldb = max(B.stride(0) if m > 1 else k, k, 1)
    ldc = max(C.stride(0) if n > 1 else k, k, 1)
    stream = torch.cuda.current_stream(A.device).cuda_stream
    ata_gemm_tn(h.h, A.data_ptr(), B.data_ptr(), m, n, k, lda, ldb, mode, C.data_ptr(), ldc, stream)
    return C


def gram_batched(As, dtype=None, handle: Handle | None = None, outs=None):
    """Packed lower triangles of A_i^T A_i for a list of 2-D CUDA tensors (one call)."""
    import torch
    if not As:
        return []
    mode = _mode_of(As[0], dtype)
    want = torch.float64 if mode == F64 else torch.float32
    ms, ns, ldas, aps, cps, res = [], [], [], [], [], []
    for i, A in enumerate(As):
        if A.dim() != 2 or not A.is_cuda or A.dtype != want:
            raise ValueError(f"member {i}: need a 2-D {want} tensor on a GPU")
        m, n = A.shape
        if n > 0 and m > 1 and A.stride(1) != 1:
            raise ValueError(f"member {i}: rows must be contiguous")
        lda = max(A.stride(0) if m > 1 else n, n, 1)
        C = outs[i] if outs is not None else torch.empty(n * (n + 1) // 2, dtype=want, device=A.device)
        ms.append(m); ns.append(n); ldas.append(lda); aps.append(A.data_ptr()); cps.append(C.data_ptr())
        res.append(C)
    h = handle or default_handle(As[0].device.index or 0)
    stream = torch.cuda.current_stream(As[0].device).cuda_stream
    ata_gram_batched(h.h, aps, ms, ns, ldas, mode, cps, stream)
    return res


def gram(A, dtype=None, handle: Handle | None = None, out=None):
    """Packed lower triangle of A^T A for a 2-D CUDA tensor A (row-major rows)."""
    import torch
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D tensor on a GPU")
    mode = _mode_of(A, dtype)
    want = torch.float64 if mode == F64 else torch.float32
    if A.dtype != want:
        raise TypeError(f"mode {mode} needs a {want} input")
    m, n = A.shape
    if n > 0 and m > 1 and A.stride(1) != 1:
        raise ValueError("A's rows must be contiguous (stride(1) == 1)")
    lda = A.stride(0) if m > 1 else max(n, 1)
    lda = max(lda, n, 1)
    if out is None:
        out = torch.empty(n * (n + 1) // 2, dtype=want, device=A.device)
    h = handle or default_handle(A.device.index or 0)
    stream = torch.cuda.current_stream(A.device).cuda_stream
    ata_gram(h.h, A.data_ptr(), m, n, lda, mode, out.data_ptr(), stream)
    return out
