"""Python binding of libmm's C ABI (include/mm.h).

Argument marshalling only: torch tensors become raw device pointers, leading
dimensions and a hipStream_t; every step of every product runs in the HIP
kernels of libmm.so.  There is no CPU fallback: without the built library or a
GPU every call raises.

torch is imported before libmm.so is loaded so that the library binds to the
HIP runtime torch already mapped (both carry the soname libamdhip64.so.7), so
torch's pointers and streams are valid inside the library.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_OK, MM_E_INVAL, MM_E_NOMEM, MM_E_DEVICE, MM_E_BUSY, MM_E_UNSUPPORTED, MM_E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6
MM_F64, MM_F32, MM_SPLIT_BF16_3, MM_SPLIT_BF16_6 = 0, 1, 2, 3
METHODS = {"f64": MM_F64, "f32": MM_F32, "split3": MM_SPLIT_BF16_3, "split6": MM_SPLIT_BF16_6}

_lib = None


class MMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status}: {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("device", ctypes.c_int32),
                ("dry_run_tflops", ctypes.c_double), ("dry_run_fail_id", ctypes.c_uint64),
                ("variants", ctypes.c_int32 * 4), ("variants_large", ctypes.c_int32 * 4),
                ("large_mn", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("useful_flop", ctypes.c_double), ("first_arrival_s", ctypes.c_double),
                ("last_done_s", ctypes.c_double), ("tflops", ctypes.c_double),
                ("peak_bytes", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("mean_batch", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# (name, restype, argtypes) of every export declared in include/mm.h
_i64, _i32, _p, _d, _sz, _u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t, ctypes.c_uint64
_st = ctypes.c_int
EXPORTS = [
    ("mm_version", ctypes.c_char_p, []),
    ("mm_status_string", ctypes.c_char_p, [_st]),
    ("mm_last_error", ctypes.c_char_p, []),
    ("mm_init", _st, [ctypes.c_int]),
    ("mm_gemm_f64", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("mm_gemm_f32", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p]),
    ("mm_split_bf16", _st, [_i64, _i64, _p, _i64, _i32, _i32, _p, _i64, _p]),
    ("mm_split_workspace_bytes", _sz, [_i64, _i64, _i64, _i32]),
    ("mm_gemm_split_bf16", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i32, _i32, _p, _sz, _p]),
    ("mm_strassen_workspace_bytes", _sz, [_i64, _i64, _i64]),
    ("mm_gemm_strassen_f64", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _sz, _p]),
    ("mm_gemm_ex_workspace_bytes", _sz, [_st, _st, _st, _i64, _i64, _i64]),
    ("mm_gemm_ex", _st, [_st, _st, _st, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _sz, _p]),
    ("mm_residual_workspace_bytes", _sz, [_i64, _i64, _i64]),
    ("mm_residual_f64", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i32, _i32, _p, _p, _p, _sz, _p]),
    ("mm_residual_noalloc_max_bytes", _sz, []),
    ("mm_residual_f64_noalloc", _st, [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i32, _i32, _p, _p, _p]),
    ("mm_gemm_grouped", _st, [ctypes.POINTER(Problem), _i32, _st, ctypes.POINTER(_p), _p]),
    ("mm_grouped_plan_destroy", _st, [_p]),
    ("mm_grouped_plan_launch", _st, [_p, _p]),
    ("mm_grouped_plan_info", _st, [_p, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                                   ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("mm_gemm_grouped_config", _st, [ctypes.POINTER(Problem), _i32, _st, _i32, _i32, ctypes.POINTER(_p), _p]),
    ("mm_grouped_autotune", _st, [ctypes.POINTER(Problem), _i32, _st, _i32, _i32, ctypes.POINTER(_i32),
                                  ctypes.POINTER(_i32), ctypes.POINTER(_d), _p]),
    ("mm_grouped_pair_count", _i32, [_st]),
    ("mm_grouped_pair_info", _st, [_st, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("mm_variant_count", _i32, [_st]),
    ("mm_variant_info", _st, [_st, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    ("mm_select_variant", _i32, [_st, _i64, _i64, _i64]),
    ("mm_gemm_variant", _st, [_st, _i32, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _sz, _p]),
    ("mm_autotune", _st, [_st, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i32, _i32,
                          ctypes.POINTER(_i32), ctypes.POINTER(_d), _p]),
    ("mm_autotune_save", _st, [ctypes.c_char_p]),
    ("mm_autotune_load", _st, [ctypes.c_char_p]),
    ("mm_autotune_clear", _st, []),
    ("mm_serve_create", _st, [ctypes.POINTER(ServeConfig), ctypes.POINTER(_p)]),
    ("mm_serve_submit", _st, [_p, ctypes.POINTER(Problem), _st, _d, ctypes.POINTER(_u64)]),
    ("mm_serve_wait", _st, [_p, _u64, _i64, ctypes.POINTER(_st), ctypes.POINTER(_d)]),
    ("mm_serve_clock", _d, [_p]),
    ("mm_serve_stats", _st, [_p, ctypes.POINTER(ServeStats)]),
    ("mm_serve_destroy", _st, [_p]),
]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmm.so (after torch) and declare every export."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- binds libmm to torch's HIP runtime

    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or python -m paper_2408_15384_amd.build")
    lib = ctypes.CDLL(path)
    for name, res, args in EXPORTS:
        fn = getattr(lib, name)  # AttributeError: the library lacks a declared export
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def lib() -> ctypes.CDLL:
    return load_library()


def check(status: int) -> None:
    if status != MM_OK:
        raise MMError(status, lib().mm_last_error().decode())


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ld(t, name) -> int:
    """Leading dimension of a 2-D GPU tensor used as a row-major matrix."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    return row_major_ld(t, name)


def row_major_ld(t, name="X") -> int:
    """Leading dimension (elements between row starts) of a 2-D tensor whose
    rows are contiguous and do not overlap; ValueError otherwise."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.numel() == 0:
        return max(int(t.shape[1]), 1)
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major (unit column stride)")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        # rows overlap (e.g. an expanded or broadcast view): passing the row
        # length as the leading dimension would make the kernels read or write
        # past the tensor's storage
        raise ValueError(f"{name} is not a row-major matrix: row stride {t.stride(0)} < {t.shape[1]} columns")
    if t.shape[0] == 1:
        return max(int(t.shape[1]), 1)
    return int(t.stride(0))


def _shapes(A, B):
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError(f"inner dimensions differ: {tuple(A.shape)} x {tuple(B.shape)}")
    return int(M), int(N), int(K)


def gemm_f64(A, B, C=None, stream=None):
    """C = A.B in binary64 on the FP64 matrix cores (mm_gemm_f64)."""
    import torch
    M, N, K = _shapes(A, B)
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("gemm_f64 needs float64 operands")
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    check(lib().mm_gemm_f64(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                            C.data_ptr(), _ld(C, "C"), _stream(stream)))
    return C


def gemm_f32(A, B, C=None, stream=None):
    """C = A.B in FP32 on the FP32 matrix cores (mm_gemm_f32)."""
    import torch
    M, N, K = _shapes(A, B)
    if A.dtype != torch.float32 or B.dtype != torch.float32:
        raise TypeError("gemm_f32 needs float32 operands")
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    check(lib().mm_gemm_f32(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                            C.data_ptr(), _ld(C, "C"), _stream(stream)))
    return C


def split_bf16(X, nplanes: int, transpose: bool = False, out=None, stream=None):
    """bfloat16 planes of FP32 X (mm_split_bf16), returned as int16 bit patterns
    of shape (nplanes, rows, cols) or (nplanes, cols, rows) if transposed."""
    import torch
    rows, cols = X.shape
    shape = (nplanes, cols, rows) if transpose else (nplanes, rows, cols)
    if out is None:
        out = torch.empty(shape, dtype=torch.int16, device=X.device)
    check(lib().mm_split_bf16(rows, cols, X.data_ptr(), _ld(X, "X"), nplanes, int(bool(transpose)),
                              out.data_ptr(), rows * cols, _stream(stream)))
    return out


def split_workspace_bytes(M: int, N: int, K: int, nprod: int) -> int:
    return int(lib().mm_split_workspace_bytes(M, N, K, nprod))


def gemm_split_bf16(A, B, nprod: int = 6, C=None, out_dtype=None, workspace=None, stream=None):
    """C = A.B for FP32 operands by the split method (mm_gemm_split_bf16)."""
    import torch
    M, N, K = _shapes(A, B)
    if A.dtype != torch.float32 or B.dtype != torch.float32:
        raise TypeError("gemm_split_bf16 needs float32 operands")
    if C is None:
        C = torch.empty((M, N), dtype=out_dtype or torch.float32, device=A.device)
    if C.dtype not in (torch.float32, torch.float64):
        raise TypeError("C must be float32 or float64")
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    check(lib().mm_gemm_split_bf16(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                   C.data_ptr(), _ld(C, "C"), int(C.dtype == torch.float64), nprod,
                                   ws_ptr or None, ws_bytes, _stream(stream)))
    return C


def gemm_strassen_f64(A, B, C=None, workspace=None, stream=None):
    """C = A.B in binary64 by one Strassen-Winograd level (mm_gemm_strassen_f64)."""
    import torch
    M, N, K = _shapes(A, B)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device=A.device)
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    check(lib().mm_gemm_strassen_f64(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                                     C.data_ptr(), _ld(C, "C"), ws_ptr or None, ws_bytes, _stream(stream)))
    return C


def gemm_ex(method, A, B, opa: str = "N", opb: str = "N", C=None, workspace=None, stream=None):
    """C = op(A).op(B) with op 'N' (as stored) or 'T' (transposed), mm_gemm_ex.
    A and B are the stored (row-major) tensors."""
    import torch
    m = METHODS.get(method, method)
    ta, tb = int(opa.upper() == "T"), int(opb.upper() == "T")
    M, K = (A.shape[1], A.shape[0]) if ta else (A.shape[0], A.shape[1])
    K2, N = (B.shape[1], B.shape[0]) if tb else (B.shape[0], B.shape[1])
    if K != K2:
        raise ValueError("inner dimensions differ")
    M, N, K = int(M), int(N), int(K)
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64 if m == MM_F64 else torch.float32, device=A.device)
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    check(lib().mm_gemm_ex(m, ta, tb, M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"),
                           C.data_ptr(), _ld(C, "C"), ws_ptr or None, ws_bytes, _stream(stream)))
    return C


def gemm_colmajor_f64(A_cm, B_cm, M: int, N: int, K: int, C_cm=None, stream=None):
    """Column-major (Fortran-order) binary64 C = A.B on flat device buffers of
    M*K, K*N and M*N elements: computed as the row-major C^T = B^T.A^T."""
    import torch
    if C_cm is None:
        C_cm = torch.empty(M * N, dtype=torch.float64, device=A_cm.device)
    gemm_f64(B_cm.view(N, K), A_cm.view(K, M), C_cm.view(N, M), stream=stream)
    return C_cm


def _residual_args(A, B, C, x, out):
    import torch
    M, N, K = _shapes(A, B)
    if tuple(C.shape) != (M, N):
        raise ValueError("C shape")
    code = {torch.float64: 0, torch.float32: 1}
    if A.dtype != B.dtype or A.dtype not in code or C.dtype not in code:
        raise TypeError("A, B must share float64/float32; C float64/float32")
    if x.dtype != torch.float64 or x.numel() != N:
        raise ValueError("x must be float64 of length N")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=A.device)
    return (M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"), C.data_ptr(), _ld(C, "C"),
            code[A.dtype], code[C.dtype], x.data_ptr(), out.data_ptr()), out


def residual_f64(A, B, C, x, out=None, workspace=None, stream=None):
    """Device tensor [||C.x - A.(B.x)||^2, ||A.(B.x)||^2] in binary64 (mm_residual_f64)."""
    args, out = _residual_args(A, B, C, x, out)
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    check(lib().mm_residual_f64(*args, ws_ptr or None, ws_bytes, _stream(stream)))
    return out


def residual_f64_noalloc(A, B, C, x, out=None, stream=None):
    """mm_residual_f64_noalloc: the same probe with the library's fixed scratch
    (no device allocation by the library; `out` is allocated here if None)."""
    args, out = _residual_args(A, B, C, x, out)
    check(lib().mm_residual_f64_noalloc(*args, _stream(stream)))
    return out


def variant_count(method) -> int:
    return int(lib().mm_variant_count(METHODS.get(method, method)))


def variant_info(method, variant: int):
    bm, bn, bk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().mm_variant_info(METHODS.get(method, method), variant, ctypes.byref(bm), ctypes.byref(bn),
                                ctypes.byref(bk)))
    return bm.value, bn.value, bk.value


PAIR_BASE = 64   # MM_PAIR_BASE: grouped variant id of size-class pair 0


def grouped_pair_count(method) -> int:
    return int(lib().mm_grouped_pair_count(METHODS.get(method, method)))


def grouped_pair_info(method, pair: int):
    """(small variant, large variant, pct) of size-class pair `pair`; its
    grouped variant id is PAIR_BASE + pair."""
    s, l, pct = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().mm_grouped_pair_info(METHODS.get(method, method), pair, ctypes.byref(s), ctypes.byref(l),
                                     ctypes.byref(pct)))
    return s.value, l.value, pct.value


def select_variant(method, M, N, K) -> int:
    return int(lib().mm_select_variant(METHODS.get(method, method), M, N, K))


def gemm_variant(method, variant: int, A, B, C, workspace=None, stream=None):
    M, N, K = _shapes(A, B)
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    check(lib().mm_gemm_variant(METHODS.get(method, method), variant, M, N, K, A.data_ptr(), _ld(A, "A"),
                                B.data_ptr(), _ld(B, "B"), C.data_ptr(), _ld(C, "C"), ws_ptr or None, ws_bytes,
                                _stream(stream)))
    return C


def autotune(method, A, B, C, warmup: int = 2, reps: int = 5, stream=None):
    """Time every variant on these operands; returns (variant, median ms)."""
    M, N, K = _shapes(A, B)
    v, ms = ctypes.c_int32(), ctypes.c_double()
    check(lib().mm_autotune(METHODS.get(method, method), M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(),
                            _ld(B, "B"), C.data_ptr(), _ld(C, "C"), warmup, reps, ctypes.byref(v),
                            ctypes.byref(ms), _stream(stream)))
    return v.value, ms.value


def autotune_save(path: str) -> None:
    check(lib().mm_autotune_save(path.encode()))


def autotune_load(path: str) -> None:
    check(lib().mm_autotune_load(path.encode()))


def autotune_clear() -> None:
    check(lib().mm_autotune_clear())


def _problems(As: Sequence, Bs: Sequence, Cs: Sequence):
    n = len(As)
    arr = (Problem * max(n, 1))()
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        M, N, K = _shapes(A, B)
        arr[i] = Problem(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"), C.data_ptr(), _ld(C, "C"))
    return arr, n


class GroupedPlan:
    """Owns an mm_grouped_plan (tile map, descriptors, captured graph).
    variant/schedule None: the autotuned (or default) choice."""

    def __init__(self, method, variant=None, schedule=None):
        self.method = METHODS.get(method, method)
        self.variant, self.schedule = variant, schedule
        self.handle = ctypes.c_void_p(None)

    def run(self, As, Bs, Cs, stream=None):
        arr, n = _problems(As, Bs, Cs)
        if self.variant is None:
            check(lib().mm_gemm_grouped(arr, n, self.method, ctypes.byref(self.handle), _stream(stream)))
        else:
            check(lib().mm_gemm_grouped_config(arr, n, self.method, self.variant, self.schedule or 0,
                                               ctypes.byref(self.handle), _stream(stream)))
        return Cs

    def replay(self, stream=None):
        """Replay the captured graph with the operands of the last run."""
        check(lib().mm_grouped_plan_launch(self.handle, _stream(stream)))

    def info(self):
        v, s, t, grid, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().mm_grouped_plan_info(self.handle, ctypes.byref(v), ctypes.byref(s), ctypes.byref(t),
                                         ctypes.byref(grid), ctypes.byref(g)))
        return {"variant": v.value, "schedule": s.value, "tiles": t.value, "grid": grid.value, "graph": bool(g.value)}

    def close(self):
        if self.handle:
            check(lib().mm_grouped_plan_destroy(self.handle))
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_grouped(method, As, Bs, Cs, variant=None, schedule=0, stream=None):
    """One grouped launch without a plan (plan_inout = NULL)."""
    arr, n = _problems(As, Bs, Cs)
    if variant is None:
        check(lib().mm_gemm_grouped(arr, n, METHODS.get(method, method), None, _stream(stream)))
    else:
        check(lib().mm_gemm_grouped_config(arr, n, METHODS.get(method, method), variant, schedule, None,
                                           _stream(stream)))
    return Cs


def grouped_autotune(method, As, Bs, Cs, warmup: int = 1, reps: int = 5, stream=None):
    """Time every (variant, schedule) on this batch; returns (variant, schedule, ms)."""
    arr, n = _problems(As, Bs, Cs)
    v, sch, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    check(lib().mm_grouped_autotune(arr, n, METHODS.get(method, method), warmup, reps, ctypes.byref(v),
                                    ctypes.byref(sch), ctypes.byref(ms), _stream(stream)))
    return v.value, sch.value, ms.value


class Server:
    """A continuous-batching request loop (mm_serve_*)."""

    def __init__(self, budget_bytes: int, slots: int = 4, max_batch: int = 64, queue_capacity: int = 1 << 16,
                 device: int = 0, dry_run_tflops: float = 0.0, dry_run_fail_id: int = 0, variants=None,
                 variants_large=None, large_mn: int = 0):
        v = (ctypes.c_int32 * 4)(*(variants if variants is not None else (-1, -1, -1, -1)))
        vl = (ctypes.c_int32 * 4)(*(variants_large if variants_large is not None else (-1, -1, -1, -1)))
        cfg = ServeConfig(budget_bytes, slots, max_batch, queue_capacity, device, dry_run_tflops, dry_run_fail_id,
                          v, vl, large_mn)
        self.handle = ctypes.c_void_p(None)
        check(lib().mm_serve_create(ctypes.byref(cfg), ctypes.byref(self.handle)))

    def clock(self) -> float:
        return float(lib().mm_serve_clock(self.handle))

    def submit(self, A, B, C, method, arrival_s: float = -1.0) -> int:
        M, N, K = _shapes(A, B)
        p = Problem(M, N, K, A.data_ptr(), _ld(A, "A"), B.data_ptr(), _ld(B, "B"), C.data_ptr(), _ld(C, "C"))
        rid = ctypes.c_uint64()
        check(lib().mm_serve_submit(self.handle, ctypes.byref(p), METHODS.get(method, method), arrival_s,
                                    ctypes.byref(rid)))
        return rid.value

    def submit_raw(self, prob: Problem, method: int, arrival_s: float = -1.0) -> int:
        rid = ctypes.c_uint64()
        check(lib().mm_serve_submit(self.handle, ctypes.byref(prob), method, arrival_s, ctypes.byref(rid)))
        return rid.value

    def wait(self, rid: int, timeout_us: int = -1):
        st, lat = ctypes.c_int(), ctypes.c_double()
        check(lib().mm_serve_wait(self.handle, rid, timeout_us, ctypes.byref(st), ctypes.byref(lat)))
        return st.value, lat.value

    def stats(self) -> dict:
        s = ServeStats()
        check(lib().mm_serve_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self.handle:
            check(lib().mm_serve_destroy(self.handle))
            self.handle = ctypes.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
