"""Pins of the CPU oracle against facts that do not come from the oracle:
exact rational arithmetic, closed forms, exact integer arithmetic, a hand
worked example and a library routine.  Each plausible slip in the oracle (a
dropped term, a wrong index or sign, a transposed operand, a lost leading
dimension) fails at least one of these."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2408_15384_amd import inputs as I

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gamma(K):
    return K * U / (1 - K * U)


def _exact(A, B):
    M, K = A.shape
    N = B.shape[1]
    return [[sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K)) for j in range(N)]
            for i in range(M)]


def _sequential(A, B):
    """Each rounding of the k-ascending sum modelled exactly: s <- fl(s + fl(a*b))."""
    M, K = A.shape
    N = B.shape[1]
    out = np.empty((M, N))
    for i in range(M):
        for j in range(N):
            s = Fraction(0)
            for k in range(K):
                p = float(Fraction(float(A[i, k])) * Fraction(float(B[k, j])))
                s = Fraction(float(s + Fraction(p)))
            out[i, j] = float(s)
    return out


SHAPES = [(1, 1, 1), (2, 3, 4), (4, 3, 2), (5, 1, 6), (1, 6, 5), (6, 6, 6), (3, 5, 1), (2, 2, 7)]


@pytest.mark.parametrize("shape", SHAPES)
def test_rational_bruteforce(shape):
    M, N, K = shape
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal((M, K)) * np.exp2(rng.integers(-20, 20, (M, K)))
    B = rng.standard_normal((K, N)) * np.exp2(rng.integers(-20, 20, (K, N)))
    C = oracle.gemm(A, B)
    ex = _exact(A, B)
    absAB = oracle.abs_product(A, B)
    for i in range(M):
        for j in range(N):
            err = abs(Fraction(float(C[i, j])) - ex[i][j])
            assert err <= Fraction(gamma(K)) * Fraction(float(absAB[i, j])) * (1 + Fraction(1, 10 ** 6))
    # every rounding reproduced: the oracle is the k-ascending sum, no FMA
    assert np.array_equal(C, _sequential(A, B))


def test_textbook_example():
    rows = {}
    with open(os.path.join(GOLDEN, "textbook_2x3x2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, r, c, *vals = line.split()
            rows[name] = np.array([float(v) for v in vals]).reshape(int(r), int(c))
    assert np.array_equal(oracle.gemm(rows["A"], rows["B"]), rows["C"])


@pytest.mark.parametrize("M,N,K", [(7, 5, 9), (33, 17, 65)])
def test_identity_and_zero(M, N, K):
    rng = np.random.default_rng(1)
    A = rng.random((M, K)) * 2 - 1
    B = rng.random((K, N)) * 2 - 1
    assert np.array_equal(oracle.gemm(A, np.eye(K)), A)
    assert np.array_equal(oracle.gemm(np.eye(M), A), A)
    assert np.array_equal(oracle.gemm(np.eye(K), B), B)
    assert not oracle.gemm(A, np.zeros((K, N))).any()
    assert not oracle.gemm(np.zeros((M, K)), B).any()


@pytest.mark.parametrize("M,N,K", [(9, 11, 13), (64, 48, 1000)])
def test_rank1_closed_form_exact(M, N, K):
    """(u v^T)(w x^T) = (v.w) u x^T, exact for small integers."""
    rng = np.random.default_rng(2)
    u = rng.integers(-8, 9, M).astype(float)
    v = rng.integers(-8, 9, K).astype(float)
    w = rng.integers(-8, 9, K).astype(float)
    x = rng.integers(-8, 9, N).astype(float)
    C = oracle.gemm(np.outer(u, v), np.outer(w, x))
    vw = int(np.dot(v.astype(np.int64), w.astype(np.int64)))
    assert np.array_equal(C, float(vw) * np.outer(u, x))


def test_rank1_closed_form_float():
    M, N, K = 12, 10, 300
    rng = np.random.default_rng(3)
    u, v, w, x = (rng.random(n) * 2 - 1 for n in (M, K, K, N))
    C = oracle.gemm(np.outer(u, v), np.outer(w, x))
    vw = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(v, w))
    ref = np.array([[float(vw * Fraction(float(a)) * Fraction(float(b))) for b in x] for a in u])
    absref = np.abs(ref)
    bound = 3 * gamma(K + 2) * float(sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(v, w))) \
        * np.outer(np.abs(u), np.abs(x))
    assert np.all(np.abs(C - ref) <= bound + 0 * absref)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (31, 17, 129), (200, 150, 300)])
def test_integer_inputs_exact(M, N, K):
    A, B = I.pair("int_f64", M, N, K, seed=M)
    C = oracle.gemm(A, B)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(C, ref.astype(np.float64))


def test_k1_outer_product_single_rounding():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((37, 1))
    b = rng.standard_normal((1, 23))
    assert np.array_equal(oracle.gemm(a, b), a * b)


def test_transpose_symmetry_bitwise():
    rng = np.random.default_rng(5)
    A = rng.random((19, 27)) * 2 - 1
    B = rng.random((27, 14)) * 2 - 1
    assert np.array_equal(oracle.gemm(B.T, A.T), oracle.gemm(A, B).T)


def test_library_crosscheck():
    A, B = I.pair("uniform_f64", 200, 150, 300, seed=6)
    C = oracle.gemm(A, B)
    bound = 2 * gamma(300) * oracle.abs_product(A, B)
    assert np.all(np.abs(C - A @ B) <= bound)


def test_entries_match_full_product():
    A, B = I.pair("uniform_f64", 40, 30, 50, seed=7)
    C = oracle.gemm(A, B)
    rng = np.random.default_rng(8)
    r = rng.integers(0, 40, 100)
    c = rng.integers(0, 30, 100)
    assert np.array_equal(oracle.gemm_entries(A, B, r, c), C[r, c])
    with pytest.raises(IndexError):
        oracle.gemm_entries(A, B, [40], [0])


def test_thread_count_does_not_change_bits():
    A, B = I.pair("uniform_f64", 130, 70, 90, seed=9)
    n0 = oracle.get_threads()
    try:
        oracle.set_threads(1)
        C1 = oracle.gemm(A, B)
        oracle.set_threads(max(2, os.cpu_count() or 2))
        C8 = oracle.gemm(A, B)
    finally:
        oracle.set_threads(n0)
    assert np.array_equal(C1, C8)


def test_empty_shapes():
    assert oracle.gemm(np.zeros((0, 3)), np.zeros((3, 4))).shape == (0, 4)
    assert not oracle.gemm(np.ones((3, 0)), np.ones((0, 4))).any()


# ----------------------------------------------------------------- split form

def test_bf16_round_matches_library_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(10)
    x = np.concatenate([
        (rng.standard_normal(20000) * np.exp2(rng.integers(-60, 60, 20000))).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.3895314e38, -3.3895314e38], np.float32),
    ])
    # exact ties: a bf16 value plus half of its last place, odd and even kept bit
    base = (rng.integers(0x3F80, 0x4080, 2000).astype(np.uint32) << 16)
    ties = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("kind", ["uniform_f32", "m2e_f32"])
def test_three_planes_reconstruct_exactly(kind):
    A, _ = I.pair(kind, 300, 1, 200, seed=11)
    h, m, lo = oracle.split_planes(A, 3)
    for p in (h, m, lo):
        assert np.array_equal(oracle.bf16_round(p), p)
    assert np.array_equal(h.astype(np.float64) + m.astype(np.float64) + lo.astype(np.float64),
                          A.astype(np.float64))


def test_two_planes_residual_bound():
    A, _ = I.pair("uniform_f32", 400, 1, 300, seed=12)
    h, lo = oracle.split_planes(A, 2)
    resid = np.abs(A.astype(np.float64) - h.astype(np.float64) - lo.astype(np.float64))
    assert np.all(resid <= 2.0 ** -16 * np.abs(A.astype(np.float64)))
    assert resid.max() > 0  # two planes do not hold every FP32 value


def test_nine_products_equal_the_product():
    A, B = I.pair("uniform_f32", 40, 30, 64, seed=13)
    C9 = oracle.split_product(A, B, 9)
    C = oracle.gemm(A, B)
    bound = 12 * gamma(64) * oracle.abs_product(A, B)
    assert np.all(np.abs(C9 - C) <= bound)


def test_split3_integer_inputs_exact():
    A, B = I.pair("int_f32", 50, 40, 70, seed=14)
    assert np.array_equal(oracle.split_product(A, B, 3), oracle.gemm(A, B))
    assert np.array_equal(oracle.split_product(A, B, 6), oracle.gemm(A, B))


def test_split_error_bands():
    """Design error of each split method against the exact product."""
    A, B = I.pair("uniform_f32", 128, 128, 512, seed=15)
    R = oracle.gemm(A, B)
    e3 = oracle.normwise_rel(oracle.split_product(A, B, 3), R)
    e6 = oracle.normwise_rel(oracle.split_product(A, B, 6), R)
    assert 1e-6 < e3 < 1e-5       # two planes hold ~17 bits: not FP32 accurate
    assert e6 < 1e-7              # the 6-product form meets the 1e-6 target by design


# ------------------------------------------------------------- residual probe

def test_freivalds_exact_product_zero_and_planted_error():
    A, B = I.pair("int_f64", 30, 20, 25, seed=16)
    C = oracle.gemm(A, B)
    x = I.integer(I.rng_for(17), (20,))
    r2, z2 = oracle.freivalds(A, B, C, x)
    assert r2 == 0.0 and z2 > 0
    C2 = C.copy()
    C2[3, 7] += 5.0
    r2, _ = oracle.freivalds(A, B, C2, x)
    assert r2 == (5.0 * x[7]) ** 2


# ------------------------------------------------------------- Strassen level

def test_strassen_exact_on_integers():
    """The scheme is algebraically the product: exact whenever every
    intermediate is representable."""
    for (M, N, K) in [(2, 2, 2), (6, 4, 10), (64, 48, 32)]:
        A, B = I.pair("int_f64", M, N, K, seed=M + K)
        assert np.array_equal(oracle.strassen(A, B), oracle.gemm(A, B))


def test_strassen_each_formula_matters():
    """Dropping or flipping any one term of the scheme breaks exactness: the
    integer pin sees every formula."""
    A, B = I.pair("int_f64", 8, 8, 8, seed=21)
    R = oracle.gemm(A, B)
    P = [oracle.gemm(X, Y) for X, Y in oracle.strassen_parts(A, B)]
    for i in range(7):
        Q = list(P)
        Q[i] = -Q[i]
        assert not np.array_equal(oracle.strassen_combine(Q), R)


def test_strassen_float_close_to_product():
    A, B = I.pair("uniform_f64", 96, 80, 128, seed=22)
    # normwise: a few multiples of the conventional K*u growth
    assert oracle.normwise_rel(oracle.strassen(A, B), oracle.gemm(A, B)) < 20 * 128 * oracle.U_F64


def _push(P, e, sign):
    """The binary64 values farthest from P in direction `sign` that differ
    from P by at most e, exactly (checked in rational arithmetic)."""
    Q = (P + sign * e).ravel()
    Pf, ef = P.ravel(), e.ravel()
    for t in range(Q.size):
        while abs(Fraction(float(Q[t])) - Fraction(float(Pf[t]))) > Fraction(float(ef[t])):
            Q[t] = np.nextafter(Q[t], Pf[t])
    return Q.reshape(P.shape)


def _worst_case_second_evaluation(A, B):
    """Another evaluation of the scheme whose seven products each sit at the
    edge of the per-product parity bound 4*k*u*(|X||Y|), with the signs that
    make every quadrant's deviations add up (P4 enters C21 negated), and whose
    S, T and U sums are rounded as the oracle rounds them."""
    parts = oracle.strassen_parts(A, B)
    k = A.shape[1] // 2
    P = [oracle.gemm(X, Y) for X, Y in parts]
    e = [oracle.elementwise_bound(oracle.gemm(np.abs(X), np.abs(Y)), k, oracle.U_F64) for X, Y in parts]
    signs = [1, 1, 1, -1, 1, 1, 1]
    Q = [_push(p, ee, sg) for p, ee, sg in zip(P, e, signs)]
    return oracle.strassen_combine(Q), oracle.strassen_combine(P)


# (64, 64, 2) and (66, 98, 34) have inner sizes k = 1 and 17, where the
# roundings of the U-sums are not small against the product bounds.
STRASSEN_BOUND_SHAPES = [(64, 64, 2), (66, 98, 34), (40, 56, 128)]


@pytest.mark.parametrize("shape", STRASSEN_BOUND_SHAPES)
def test_strassen_bound_holds_and_is_tight_at_the_worst_case(shape):
    M, N, K = shape
    A, B = I.pair("uniform_f64", M, N, K, seed=K)
    Q, P = _worst_case_second_evaluation(A, B)
    D = np.abs(Q - P)
    bound = oracle.strassen_product_bound(A, B)
    assert np.all(D <= bound)
    # tight: in every quadrant some entry reaches 80% of the bound (over 99%
    # once k >= 17); tests/test_oracle_mutations.py shows that a bound missing
    # any one term falls below this worst case
    m, n = M // 2, N // 2
    for qi in (slice(0, m), slice(m, M)):
        for qj in (slice(0, n), slice(n, N)):
            assert (D[qi, qj] / bound[qi, qj]).max() >= 0.8


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 6, 4), (6, 4, 8)])
def test_strassen_bound_against_the_exact_scheme(shape):
    """Exact rational evaluation of the scheme (products and sums without
    rounding) is another evaluation whose products lie within gamma_k of the
    oracle's, inside the parity bound: the oracle's scheme must stay within
    the carried bound of it."""
    M, N, K = shape
    rng = np.random.default_rng(M * 100 + N * 10 + K)
    A = rng.standard_normal((M, K)) * np.exp2(rng.integers(-6, 6, (M, K)))
    B = rng.standard_normal((K, N)) * np.exp2(rng.integers(-6, 6, (K, N)))
    S = oracle.strassen(A, B)
    bound = oracle.strassen_product_bound(A, B)
    parts = oracle.strassen_parts(A, B)
    m, n = M // 2, N // 2

    def mat(X, Y):
        return [[sum((Fraction(float(X[i, t])) * Fraction(float(Y[t, j])) for t in range(X.shape[1])), Fraction(0))
                 for j in range(Y.shape[1])] for i in range(X.shape[0])]

    P1, P2, P3, P4, P5, P6, P7 = [mat(X, Y) for X, Y in parts]
    for i in range(m):
        for j in range(n):
            u2 = P1[i][j] + P6[i][j]
            u3 = u2 + P7[i][j]
            exact = {(0, 0): P1[i][j] + P2[i][j], (0, 1): u2 + P5[i][j] + P3[i][j],
                     (1, 0): u3 - P4[i][j], (1, 1): u3 + P5[i][j]}
            for (qi, qj), v in exact.items():
                r, c = qi * m + i, qj * n + j
                assert abs(Fraction(float(S[r, c])) - v) <= Fraction(float(bound[r, c]))


def test_strassen_rejects_odd():
    with pytest.raises(ValueError):
        oracle.strassen(np.ones((3, 2)), np.ones((2, 2)))


# ------------------------------------------------------------ normwise error

def test_normwise_rel_hand_worked():
    """||C - R||_F / ||R||_F on hand-worked cases; each catches a different
    slip (wrong norm, computed value in the denominator, missing square root)."""
    R = np.ones((2, 2))
    C = R.copy()
    C[0, 0] += 0.5
    # ||C - R||_F = 0.5 and ||R||_F = 2: 0.25 (the max norm would give 0.5,
    # ||C||_F in the denominator 0.218..., squared norms 0.0625)
    assert oracle.normwise_rel(C, R) == 0.25
    C[1, 1] -= 0.5
    # two entries off by 0.5: sqrt(0.5) / 2 (the max norm would give 0.5 / 1)
    assert oracle.normwise_rel(C, R) == pytest.approx(0.35355339059327373, rel=1e-15)
    # the reference, not the computed value, is the scale: |(0, 4)| / |(3, 4)| = 4/5
    assert oracle.normwise_rel(np.array([[3.0, 0.0]]), np.array([[3.0, 4.0]])) == 0.8
    # float32 results are widened exactly before the difference is formed
    R32 = np.array([[1.0, 0.0]])
    C32 = np.array([[1.0 + 2.0 ** -23, 0.0]], dtype=np.float32)
    assert oracle.normwise_rel(C32, R32) == 2.0 ** -23
