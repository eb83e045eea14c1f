"""Plants plausible slips in a private copy of the oracle's C source (on the
CPU only) and checks that the pins reject every mutant: the pins are strong
enough to notice a dropped term, a wrong index, a sign slip or a transposed
operand."""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "gemm_ref.c")

MUTANTS = {
    "dropped_last_term": ("for (int64_t k = 0; k < K; ++k) {", "for (int64_t k = 0; k + 1 < K; ++k) {"),
    "transposed_B": ("c[j] = c[j] + a * b[j];", "c[j] = c[j] + a * B[j * ldb + k];"),
    "sign_slip": ("c[j] = c[j] + a * b[j];", "c[j] = c[j] - a * b[j];"),
    "wrong_ld": ("const double a = A[i * lda + k];\n            const double *restrict b = B + k * ldb;",
                 "const double a = A[i * K + k];\n            const double *restrict b = B + k * N;"),
    "row_col_swap": ("c[j]", "C[j * ldc + i]"),
    "fma_contracted": ("-ffp-contract=off", "-ffp-contract=fast"),
}


def _build_mutant(tmp_path, name):
    src = open(SRC).read()
    flags = list(oracle.CFLAGS)
    old, new = MUTANTS[name]
    if old.startswith("-ffp"):
        flags = [new if f == old else f for f in flags] + ["-march=native"]
    else:
        assert old in src, name
        src = src.replace(old, new)
    path = tmp_path / f"{name}.c"
    path.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", *flags, str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.orc_gemm.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
    return lib


def _gemm(lib, A, B, ld_pad=0):
    M, K = A.shape
    N = B.shape[1]
    Ap = np.zeros((M, K + ld_pad)); Ap[:, :K] = A
    Bp = np.zeros((K, N + ld_pad)); Bp[:, :N] = B
    # room for a mutant that writes C transposed
    C = np.zeros((max(M, N), N + ld_pad + max(M, N)))
    lib.orc_gemm(M, N, K, Ap.ctypes.data, K + ld_pad, Bp.ctypes.data, N + ld_pad, C.ctypes.data, N + ld_pad)
    return C.ravel()[: M * (N + ld_pad)].reshape(M, N + ld_pad)[:, :N]


def _pins_hold(lib):
    """A compact replay of the pins: rational brute force with every rounding,
    integer exactness with padded leading dimensions, identity."""
    rng = np.random.default_rng(0)
    for (M, N, K) in [(2, 3, 4), (4, 3, 2), (5, 5, 5)]:
        A = rng.standard_normal((M, K))
        B = rng.standard_normal((K, N))
        C = _gemm(lib, A, B)
        for i in range(M):
            for j in range(N):
                s = Fraction(0)
                for k in range(K):
                    s = Fraction(float(s + Fraction(float(Fraction(A[i, k]) * Fraction(B[k, j])))))
                if float(s) != C[i, j]:
                    return False
    A = rng.integers(-8, 9, (6, 7)).astype(float)
    B = rng.integers(-8, 9, (7, 5)).astype(float)
    if not np.array_equal(_gemm(lib, A, B, ld_pad=3), (A.astype(int) @ B.astype(int)).astype(float)):
        return False
    return np.array_equal(_gemm(lib, A, np.eye(7)), A)


def test_unmutated_source_passes(tmp_path):
    so = tmp_path / "libok.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, SRC, "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.orc_gemm.argtypes = [i64, i64, i64, p, i64, p, i64, p, i64]
    assert _pins_hold(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    if name == "fma_contracted":
        # only meaningful where the host compiler can form an FMA
        out = subprocess.run(["gcc", "-march=native", "-dM", "-E", "-x", "c", "/dev/null"],
                             capture_output=True, text=True).stdout
        if "__FMA__" not in out:
            pytest.skip("host has no FMA")
    assert not _pins_hold(_build_mutant(tmp_path, name))


# Slips in a private copy of the Strassen bound's source: each must let the
# worst-case second evaluation of the scheme (every product at the edge of its
# parity bound) fall outside the mutated bound.
BOUND_MUTANTS = {
    "dropped_P2_term": ("f1 = carry(e1, e2, U1)", "f1 = carry(e1, 0 * e2, U1)"),
    "dropped_P3_term": ("f5 = carry(f4, e3, U5)", "f5 = carry(f4, 0 * e3, U5)"),
    "dropped_P4_term": ("f6 = carry(f3, e4, U6)", "f6 = carry(f3, 0 * e4, U6)"),
    "skipped_P7_on_C21": ("f6 = carry(f3, e4, U6)", "f6 = carry(f2, e4, U6)"),
    "no_sum_rounding": ("2.0 * U_F64 * np.abs(U)", "0.0 * np.abs(U)"),
    "one_side_rounding": ("2.0 * U_F64 * np.abs(U)", "1.0 * U_F64 * np.abs(U)"),
    "halved_product_bound": ("e = [elementwise_bound(", "e = [0.5 * elementwise_bound("),
}


@pytest.mark.parametrize("name", sorted(BOUND_MUTANTS))
def test_strassen_bound_mutant_is_caught(name):
    import inspect

    from paper_2408_15384_amd import inputs as I
    from test_oracle_pins import STRASSEN_BOUND_SHAPES, _worst_case_second_evaluation

    src = inspect.getsource(oracle.strassen_product_bound)
    old, new = BOUND_MUTANTS[name]
    assert old in src, name
    ns = dict(vars(oracle))
    exec(src.replace(old, new), ns)
    mutant = ns["strassen_product_bound"]
    for (M, N, K) in STRASSEN_BOUND_SHAPES:
        A, B = I.pair("uniform_f64", M, N, K, seed=K)
        Q, P = _worst_case_second_evaluation(A, B)
        assert np.all(np.abs(Q - P) <= oracle.strassen_product_bound(A, B))
        assert np.any(np.abs(Q - P) > mutant(A, B)), (name, (M, N, K))
