"""CPU oracle for the dense product C = A.B and the methods built on it.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (no kernels, headers, helpers or tables) and never
imports it.

Contents, each citing what it follows:

* ``gemm`` / ``gemm_entries`` -- the textbook product of section III (the
  displayed sum over k of A[i][k]*B[k][j]) as the paper's plain triple loop
  (section VI), in binary64, k ascending, no fused multiply-add; written in C
  (``gemm_ref.c``, which walks the loops in i, k, j order without changing
  any entry's operations) and called through ctypes.
* ``bf16_round`` / ``split_planes`` / ``split_product`` -- the split-precision
  form: an FP32 matrix is written as a sum of bfloat16 planes (round to
  nearest even at each step), the product is approximated by the sum of a
  fixed subset of plane-by-plane products.  The paper does not define this
  form; the reading used (2 planes with 3 products, 3 planes with 6 products)
  is listed with the other readings in the design notes.  Every plane value
  and every plane product is exact in binary64, so ``split_product`` is the
  method's exact value up to binary64 rounding of the k-sums.
* ``freivalds`` -- the residual probe r = C.x - A.(B.x) for a given vector x,
  built only from ``gemm`` with N = 1.
* ``abs_product`` / ``elementwise_bound`` -- |A||B| and the per-entry error
  bound 4*K*u*(|A||B|)_ij used by the parity tests; ``normwise_rel`` -- the
  normwise relative error ||C - R||_F / ||R||_F.
* ``strassen`` / ``strassen_product_bound`` -- one level of the Strassen-
  Winograd scheme (cited in the literature review) and the per-entry bound
  between two evaluations of it, carried through its sums.

Pins (tests/test_oracle_pins.py): exact rational brute force, identity and
zero products, the rank-1 closed form, integer products against exact integer
arithmetic, K = 1 outer products, transposition symmetry, and a library
cross-check; for the split form, agreement of ``bf16_round`` with a library
bfloat16 cast, exact 3-plane reconstruction and the 9-product identity;
hand-worked values of ``normwise_rel``; for the Strassen bound, a worst-case
second evaluation that stays within it and reaches it, and the exact rational
evaluation of the scheme.  tests/test_oracle_mutations.py plants slips in
private copies of the C loop and of the Strassen bound and checks that the
pins reject each.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gemm_ref.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Flags are part of the oracle's definition: no contraction into FMA, no
# fast-math reassociation.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile gemm_ref.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.orc_gemm.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
        lib.orc_gemm.restype = None
        lib.orc_gemm_entries.argtypes = [i64, p, i64, p, i64, i64, p, p, p]
        lib.orc_gemm_entries.restype = None
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def _as_f64(x) -> np.ndarray:
    x = np.asarray(x)
    return np.ascontiguousarray(x, dtype=np.float64)


def gemm(A, B) -> np.ndarray:
    """C = A.B in binary64 by the definition (inputs widened exactly to binary64)."""
    A = _as_f64(A)
    B = _as_f64(B)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} x {B.shape}")
    M, K = A.shape
    N = B.shape[1]
    C = np.empty((M, N), dtype=np.float64)
    if M and N:
        _load().orc_gemm(M, N, K, A.ctypes.data, max(K, 1), B.ctypes.data, max(N, 1),
                         C.ctypes.data, max(N, 1))
    return C


def gemm_entries(A, B, rows, cols) -> np.ndarray:
    """Entries C[rows[t], cols[t]] of A.B, each by the definition."""
    A = _as_f64(A)
    B = _as_f64(B)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    M, K = A.shape
    N = B.shape[1]
    if B.shape[0] != K or rows.shape != cols.shape:
        raise ValueError("shape mismatch")
    if rows.size and (rows.min() < 0 or rows.max() >= M or cols.min() < 0 or cols.max() >= N):
        raise IndexError("entry outside the product")
    out = np.empty(rows.shape, dtype=np.float64)
    if rows.size:
        _load().orc_gemm_entries(K, A.ctypes.data, max(K, 1), B.ctypes.data, max(N, 1),
                                 rows.size, rows.ctypes.data, cols.ctypes.data, out.ctypes.data)
    return out


def abs_product(A, B) -> np.ndarray:
    """(|A||B|) in binary64, the scale of the per-entry error bound."""
    return gemm(np.abs(_as_f64(A)), np.abs(_as_f64(B)))


# Unit roundoff of the accumulation format.
U_F64 = 2.0 ** -53
U_F32 = 2.0 ** -24


def elementwise_bound(absAB: np.ndarray, K: int, u: float) -> np.ndarray:
    """|C - C_ref|_ij <= 4*K*u*(|A||B|)_ij, the stated parity bound."""
    return 4.0 * max(int(K), 1) * u * absAB


# ---------------------------------------------------------------------------
# Split-precision form.
# ---------------------------------------------------------------------------

def bf16_round(x) -> np.ndarray:
    """Round FP32 values to bfloat16 (8 significant bits) with round to nearest,
    ties to even, returned as FP32.  Bit method: add 0x7FFF plus the lowest kept
    bit, then clear the 16 dropped bits.  NaN is kept as a quiet NaN."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = rounded.view(np.float32).copy()
    nan = np.isnan(x)
    if nan.any():
        out[nan] = np.float32("nan")
    return out


def split_planes(x, nplanes: int):
    """Write FP32 x as bfloat16 planes: plane_0 = bf16(x); each next plane is
    bf16 of what the previous planes leave over, the leftover being formed in
    FP32 (exact, since it is a difference of nearby FP32 values)."""
    if nplanes not in (1, 2, 3):
        raise ValueError("nplanes must be 1, 2 or 3")
    rest = np.ascontiguousarray(x, dtype=np.float32)
    planes = []
    for _ in range(nplanes):
        p = bf16_round(rest)
        planes.append(p)
        rest = (rest - p).astype(np.float32)
    return planes


# Plane-pair products summed by each method: (plane of A, plane of B).
SPLIT_TERMS = {
    3: (2, ((0, 0), (0, 1), (1, 0))),
    6: (3, ((0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0))),
    9: (3, tuple((p, q) for p in range(3) for q in range(3))),
}


def split_product(A, B, nprod: int) -> np.ndarray:
    """Value of the split method: sum over its plane pairs (p, q) of
    plane_p(A) . plane_q(B), every product and the sum in binary64."""
    if nprod not in SPLIT_TERMS:
        raise ValueError("nprod must be 3, 6 or 9")
    nplanes, terms = SPLIT_TERMS[nprod]
    PA = split_planes(A, nplanes)
    PB = split_planes(B, nplanes)
    C = np.zeros((np.shape(A)[0], np.shape(B)[1]), dtype=np.float64)
    for p, q in terms:
        C = C + gemm(PA[p], PB[q])
    return C


# ---------------------------------------------------------------------------
# Residual probe.
# ---------------------------------------------------------------------------

def freivalds(A, B, C, x):
    """Return (||C.x - A.(B.x)||_2^2, ||A.(B.x)||_2^2) in binary64 for the
    probe vector x (length N), every product by the definition."""
    x = _as_f64(x).reshape(-1, 1)
    y = gemm(B, x)
    z = gemm(A, y)
    w = gemm(C, x)
    r = (w - z).ravel()
    z = z.ravel()
    return float(np.dot(r, r)), float(np.dot(z, z))


def normwise_rel(C, R) -> float:
    """||C - R||_F / ||R||_F in binary64."""
    C = _as_f64(C)
    R = _as_f64(R)
    d = np.linalg.norm((C - R).ravel())
    n = np.linalg.norm(R.ravel())
    return float(d / n) if n else float(d)


# ---------------------------------------------------------------------------
# One level of Strassen's scheme in Winograd's form (the sub-cubic family the
# paper cites in its literature review).  With A, B split in 2 x 2 quadrants
# (M, N, K even):
#   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2
#   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21
#   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
#   P5 = S1 T1,  P6 = S2 T2,   P7 = S3 T3
#   U1 = P1 + P2, U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5,
#   U5 = U4 + P3, U6 = U3 - P4, U7 = U3 + P5
#   C11 = U1, C12 = U5, C21 = U6, C22 = U7
# Every sum is one binary64 rounding in this order; the seven products are the
# definitional loop (``gemm``).
# ---------------------------------------------------------------------------

def strassen_parts(A, B):
    """The operands of the seven products, in order P1..P7, as (X, Y) pairs."""
    A = _as_f64(A)
    B = _as_f64(B)
    M, K = A.shape
    N = B.shape[1]
    if M % 2 or N % 2 or K % 2:
        raise ValueError("one Strassen level needs even M, N, K")
    m, k, n = M // 2, K // 2, N // 2
    A11, A12, A21, A22 = A[:m, :k], A[:m, k:], A[m:, :k], A[m:, k:]
    B11, B12, B21, B22 = B[:k, :n], B[:k, n:], B[k:, :n], B[k:, n:]
    S1 = A21 + A22
    S2 = S1 - A11
    S3 = A11 - A21
    S4 = A12 - S2
    T1 = B12 - B11
    T2 = B22 - T1
    T3 = B22 - B12
    T4 = T2 - B21
    return [(A11, B11), (A12, B21), (S4, B22), (A22, T4), (S1, T1), (S2, T2), (S3, T3)]


def strassen_combine(P):
    """C from the seven products P1..P7 (Winograd's U-sequence)."""
    P1, P2, P3, P4, P5, P6, P7 = P
    U1 = P1 + P2
    U2 = P1 + P6
    U3 = U2 + P7
    U4 = U2 + P5
    U5 = U4 + P3
    U6 = U3 - P4
    U7 = U3 + P5
    return np.block([[U1, U5], [U6, U7]])


def strassen(A, B):
    """One Strassen-Winograd level with every product by ``gemm``."""
    return strassen_combine([gemm(X, Y) for X, Y in strassen_parts(A, B)])


def strassen_product_bound(A, B):
    """Per-entry bound on the difference between two evaluations of the
    scheme that form the S and T sums identically (one binary64 rounding
    each, in the order above) and whose seven products differ by at most the
    stated parity bound e_P = 4*k*u*(|X||Y|) (k the inner size K/2).

    The bound is carried through the U-sequence.  For one sum U = X +- Y with
    inputs that differ by at most e_X and e_Y, rounding to nearest gives
    fl(v) = v/(1 + d) with |d| <= u, so each side's rounding error is at most
    u times its own computed |U|; the other side's |U| is at most |U_ref| +
    e_U.  Hence
        e_U <= e_X + e_Y + u*|U_ref| + u*(|U_ref| + e_U),
        e_U <= (e_X + e_Y + 2*u*|U_ref|) / (1 - u),
    with U_ref this oracle's own computed sums.  The four quadrants take the
    bound of the U that forms them (C11 = U1, C12 = U5, C21 = U6, C22 = U7)."""
    parts = strassen_parts(A, B)
    k = parts[0][0].shape[1]
    e = [elementwise_bound(gemm(np.abs(X), np.abs(Y)), k, U_F64) for X, Y in parts]
    P = [gemm(X, Y) for X, Y in parts]
    P1, P2, P3, P4, P5, P6, P7 = P
    e1, e2, e3, e4, e5, e6, e7 = e

    def carry(ex, ey, U):
        return (ex + ey + 2.0 * U_F64 * np.abs(U)) / (1.0 - U_F64)

    U1 = P1 + P2
    U2 = P1 + P6
    U3 = U2 + P7
    U4 = U2 + P5
    U5 = U4 + P3
    U6 = U3 - P4
    U7 = U3 + P5
    f1 = carry(e1, e2, U1)
    f2 = carry(e1, e6, U2)
    f3 = carry(f2, e7, U3)
    f4 = carry(f2, e5, U4)
    f5 = carry(f4, e3, U5)
    f6 = carry(f3, e4, U6)
    f7 = carry(f3, e5, U7)
    return np.block([[f1, f5], [f6, f7]])
