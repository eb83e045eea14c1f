"""GPU parity of the single-problem entry points against the CPU oracle, on
seeded inputs, through the C ABI (ctypes binding).  Bar: bit-exact on
integer-valued inputs; otherwise |C - C_ref|_ij <= 4*K*u*(|A||B|)_ij with u the
unit roundoff of the accumulation format; for the split form also the
normwise error against the exact product."""
import numpy as np
import pytest

import oracle
from paper_2408_15384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mm():
    from paper_2408_15384_amd import api
    api.load_library()
    assert api.lib().mm_init(0) == 0, api.lib().mm_last_error()
    return api


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_within_bound(C, A, B, u):
    A64, B64 = np.asarray(A, np.float64), np.asarray(B, np.float64)
    R = oracle.gemm(A64, B64)
    bound = oracle.elementwise_bound(oracle.abs_product(A64, B64), A64.shape[1], u)
    err = np.abs(np.asarray(C, np.float64) - R)
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} entries outside the bound; worst ratio {(err / np.maximum(bound, 1e-300)).max()}"
    return R


RAGGED = [(1, 1, 1), (2, 3, 5), (15, 17, 31), (33, 63, 65), (127, 129, 255), (257, 130, 100), (300, 200, 513),
          (64, 64, 64), (128, 256, 16)]


@pytest.mark.parametrize("shape", RAGGED)
def test_f64_ragged_uniform(mm, shape):
    M, N, K = shape
    A, B = I.pair("uniform_f64", M, N, K, seed=M * 7 + N)
    C = host(mm.gemm_f64(dev(A), dev(B)))
    assert_within_bound(C, A, B, oracle.U_F64)


def test_f64_config_256_seed0(mm):
    A, B = I.pair("uniform_f64", 256, 256, 256, seed=0)
    C = host(mm.gemm_f64(dev(A), dev(B)))
    assert_within_bound(C, A, B, oracle.U_F64)


@pytest.mark.parametrize("n", [256, 1024])
def test_f64_integer_bit_exact(mm, n):
    A, B = I.pair("int_f64", n, n, n, seed=0)
    C = host(mm.gemm_f64(dev(A), dev(B)))
    assert np.array_equal(C, oracle.gemm(A, B))


@pytest.mark.parametrize("method", ["f64", "f32"])
def test_every_variant_ragged(mm, method):
    M, N, K = 300, 270, 333
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    A, B = I.pair(kind, M, N, K, seed=3)
    dA, dB = dev(A), dev(B)
    u = oracle.U_F64 if method == "f64" else oracle.U_F32
    outs = []
    for v in range(mm.variant_count(method)):
        C = torch.full((M, N), float("nan"), dtype=dA.dtype, device="cuda")
        mm.gemm_variant(method, v, dA, dB, C)
        Ch = host(C)
        assert_within_bound(Ch, A, B, u)
        outs.append(Ch)


@pytest.mark.parametrize("method", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(300, 272, 320), (129, 136, 64), (64, 8, 32), (513, 260, 96)])
def test_direct_tile_shapes(mm, method, shape):
    """Shapes the direct-to-LDS tiles take (K a multiple of 32, N of the
    vector): edge rows and columns clamped, every variant the same bound."""
    M, N, K = shape
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    A, B = I.pair(kind, M, N, K, seed=N)
    dA, dB = dev(A), dev(B)
    u = oracle.U_F64 if method == "f64" else oracle.U_F32
    for v in range(mm.variant_count(method)):
        C = torch.full((M, N), float("nan"), dtype=dA.dtype, device="cuda")
        mm.gemm_variant(method, v, dA, dB, C)
        assert_within_bound(host(C), A, B, u)
    Ai, Bi = I.pair("int_f64" if method == "f64" else "int_f32", M, N, K, seed=N + 1)
    for v in range(mm.variant_count(method)):
        C = torch.empty((M, N), dtype=dA.dtype, device="cuda")
        mm.gemm_variant(method, v, dev(Ai), dev(Bi), C)
        assert np.array_equal(host(C).astype(np.float64), oracle.gemm(Ai, Bi)), f"variant {v}"


def _padded_view(X, ld, fill=float("nan"), tight=False, offset=0):
    """X (host) as a device view with leading dimension ld in a buffer whose
    padding holds `fill`, starting `offset` elements into it; tight: the
    buffer ends at X's last element."""
    rows, cols = X.shape
    size = offset + ((rows - 1) * ld + cols if tight else rows * ld + 64)
    buf = torch.full((size,), fill, dtype=torch.float64 if X.dtype == np.float64 else torch.float32, device="cuda")
    v = torch.as_strided(buf, (rows, cols), (ld, 1), offset)
    v.copy_(torch.from_numpy(np.ascontiguousarray(X)).cuda())
    return v


@pytest.mark.parametrize("method", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(257, 131, 45), (64, 5, 17), (300, 130, 1), (70, 67, 49), (33, 4, 250)])
def test_direct_tile_any_k_and_n(mm, method, shape):
    """The direct-to-LDS tiles on K not a multiple of their K step and N not a
    multiple of the vector: operands are views with vector-aligned leading
    dimensions whose padding holds NaN (A's columns past K must be cleared
    before they meet B's zero rows), B's buffer ending at its last element (no
    load may reach past it).  Every variant within the bound of the oracle;
    integer inputs bit-exact."""
    M, N, K = shape
    elem = 8 if method == "f64" else 4
    vec = 16 // elem
    lda = (K + vec - 1) // vec * vec + vec
    ldb = (N + vec - 1) // vec * vec + vec
    u = oracle.U_F64 if method == "f64" else oracle.U_F32
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    for k2, (A, B) in ((kind, I.pair(kind, M, N, K, seed=M + K)),
                       ("int", I.pair("int_f64" if method == "f64" else "int_f32", M, N, K, seed=M + K + 1))):
        dA, dB = _padded_view(A, lda), _padded_view(B, ldb, tight=True)
        for v in range(mm.variant_count(method)):
            C = torch.full((M, N), float("nan"), dtype=dA.dtype, device="cuda")
            mm.gemm_variant(method, v, dA, dB, C)
            got = host(C).astype(np.float64)
            if k2 == "int":
                assert np.array_equal(got, oracle.gemm(A, B)), f"variant {v}"
            else:
                assert_within_bound(got, A, B, u)


@pytest.mark.parametrize("method", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(257, 131, 45), (70, 67, 49), (300, 260, 64), (33, 8, 250)])
def test_direct_tile_any_leading_dimension(mm, method, shape):
    """The direct-to-LDS tiles on leading dimensions that are not multiples of
    the 16-byte vector and on bases one element past a 16-byte boundary: a
    row then starts mid-vector, and its last chunk runs into the next row's
    first elements (NaN padding here) -- past N they meet only columns that
    are not stored, past K the cleared slots.  Every variant within the bound
    of the oracle; integer inputs bit-exact."""
    M, N, K = shape
    u = oracle.U_F64 if method == "f64" else oracle.U_F32
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    lda, ldb = K + 1, N + 3
    for k2, (A, B) in ((kind, I.pair(kind, M, N, K, seed=M + N)),
                       ("int", I.pair("int_f64" if method == "f64" else "int_f32", M, N, K, seed=M + N + 1))):
        dA, dB = _padded_view(A, lda, offset=1), _padded_view(B, ldb, tight=True, offset=1)
        for v in range(mm.variant_count(method)):
            C = torch.full((M, N), float("nan"), dtype=dA.dtype, device="cuda")
            mm.gemm_variant(method, v, dA, dB, C)
            got = host(C).astype(np.float64)
            if k2 == "int":
                assert np.array_equal(got, oracle.gemm(A, B)), f"variant {v}"
            else:
                assert_within_bound(got, A, B, u)


def _span_limit_ld(rows_before_last, extra, elem):
    """Largest leading dimension (a multiple of the 16-byte vector) whose
    slice span (rows_before_last * ld + extra) * elem stays below 2^31 - 1."""
    vec = 16 // elem
    ld = ((2 ** 31 - 1) // elem - extra) // rows_before_last
    ld -= ld % vec
    while (rows_before_last * ld + extra) * elem >= 2 ** 31 - 1:
        ld -= vec
    return ld


@pytest.mark.parametrize("method,variant", [("f64", 12), ("f32", 11)])
def test_direct_tile_huge_leading_dimensions(mm, method, variant):
    """The direct tiles address a K slice through one buffer resource per
    operand with 32-bit lane offsets.  A leading dimension at the largest
    value whose slice still fits (offsets near 2^31) takes the direct path;
    one vector more takes the register tile.  Both match the oracle."""
    bm, bn, bk = mm.variant_info(method, variant)
    dt = torch.float64 if method == "f64" else torch.float32
    elem = 8 if method == "f64" else 4
    M, N, K = bm + 44, bn + 8, 2 * bk
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    A, B = I.pair(kind, M, N, K, seed=M + N)
    u = oracle.U_F64 if method == "f64" else oracle.U_F32
    vec = 16 // elem
    lda_in = _span_limit_ld(bm - 1, bk, elem)
    ldb_in = _span_limit_ld(bk - 1, bn, elem)
    for lda, ldb in ((lda_in, N), (lda_in + vec, N), (K, ldb_in), (K, ldb_in + vec)):
        Ab = torch.empty((M, lda), dtype=dt, device="cuda")
        Bb = torch.empty((K, ldb), dtype=dt, device="cuda")
        Ab[:, :K] = dev(A)
        Bb[:, :N] = dev(B)
        C = torch.full((M, N), float("nan"), dtype=dt, device="cuda")
        mm.gemm_variant(method, variant, Ab[:, :K], Bb[:, :N], C)
        assert_within_bound(host(C), A, B, u)
        del Ab, Bb, C
        torch.cuda.empty_cache()


def test_f64_leading_dims_and_misaligned(mm):
    M, N, K = 70, 45, 37
    A, B = I.pair("uniform_f64", M, N, K, seed=4)
    # padded leading dimensions (odd, so 16-byte vector loads are not allowed)
    Ab = torch.zeros((M, K + 3), dtype=torch.float64, device="cuda")
    Bb = torch.zeros((K, N + 5), dtype=torch.float64, device="cuda")
    Cb = torch.full((M, N + 7), -7.0, dtype=torch.float64, device="cuda")
    Ab[:, :K] = dev(A)
    Bb[:, :N] = dev(B)
    mm.gemm_f64(Ab[:, :K], Bb[:, :N], Cb[:, :N])
    Ch = host(Cb)
    assert_within_bound(Ch[:, :N], A, B, oracle.U_F64)
    assert np.all(Ch[:, N:] == -7.0), "wrote outside C"
    # misaligned base pointer (offset by one element)
    flat = torch.zeros(M * K + 1, dtype=torch.float64, device="cuda")
    flat[1:] = dev(A).reshape(-1)
    Ch = host(mm.gemm_f64(flat[1:].view(M, K), dev(B)))
    assert_within_bound(Ch, A, B, oracle.U_F64)


def test_degenerate_sizes(mm):
    A = torch.ones((5, 0), dtype=torch.float64, device="cuda")
    B = torch.ones((0, 4), dtype=torch.float64, device="cuda")
    C = torch.full((5, 4), 3.0, dtype=torch.float64, device="cuda")
    mm.gemm_f64(A, B, C)
    assert not host(C).any()            # K == 0 is the empty sum
    E = mm.gemm_f64(torch.ones((0, 3), dtype=torch.float64, device="cuda"),
                    torch.ones((3, 4), dtype=torch.float64, device="cuda"))
    assert E.shape == (0, 4)
    C32 = torch.full((5, 4), 3.0, dtype=torch.float32, device="cuda")
    mm.gemm_f32(A.float(), B.float(), C32)
    assert not host(C32).any()


def test_invalid_arguments_rejected(mm):
    lib = mm.lib()
    A = torch.ones((4, 4), dtype=torch.float64, device="cuda")
    p = A.data_ptr()
    assert lib.mm_gemm_f64(-1, 4, 4, p, 4, p, 4, p, 4, None) == mm.MM_E_INVAL
    assert lib.mm_gemm_f64(4, 4, 4, p, 3, p, 4, p + 4096, 4, None) == mm.MM_E_INVAL      # lda < K
    assert lib.mm_gemm_f64(4, 4, 4, p, 4, p, 4, p, 4, None) == mm.MM_E_INVAL            # C overlaps A
    assert lib.mm_gemm_f64(4, 4, 4, None, 4, p, 4, p + 4096, 4, None) == mm.MM_E_INVAL  # NULL A
    assert lib.mm_gemm_split_bf16(4, 4, 4, p, 4, p, 4, p + 4096, 4, 0, 5, None, 0, None) == mm.MM_E_INVAL
    assert b"nprod" in lib.mm_last_error()


@pytest.mark.parametrize("shape", RAGGED)
def test_f32_ragged_uniform(mm, shape):
    M, N, K = shape
    A, B = I.pair("uniform_f32", M, N, K, seed=M * 5 + K)
    C = host(mm.gemm_f32(dev(A), dev(B)))
    assert_within_bound(C, A, B, oracle.U_F32)


def test_f32_integer_bit_exact(mm):
    A, B = I.pair("int_f32", 512, 384, 640, seed=0)
    C = host(mm.gemm_f32(dev(A), dev(B)))
    assert np.array_equal(C.astype(np.float64), oracle.gemm(A, B))


# ------------------------------------------------------------------ split form

@pytest.mark.parametrize("nplanes", [1, 2, 3])
@pytest.mark.parametrize("transpose", [False, True])
def test_split_planes_bit_exact(mm, nplanes, transpose):
    X = I.uniform_f32(I.rng_for(20), (67, 131)) * np.float32(3.7)
    P = host(mm.split_bf16(dev(X), nplanes, transpose=transpose))
    ref = oracle.split_planes(X, nplanes)
    for p in range(nplanes):
        r = (ref[p].view(np.uint32) >> 16).astype(np.uint16)
        if transpose:
            r = r.T
        assert np.array_equal(P[p].view(np.uint16), r), f"plane {p}"


@pytest.mark.parametrize("nprod", [3, 6])
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 65), (129, 127, 255), (256, 256, 256), (70, 300, 40)])
def test_split_matches_emulation(mm, nprod, shape):
    M, N, K = shape
    A, B = I.pair("uniform_f32", M, N, K, seed=K)
    C = host(mm.gemm_split_bf16(dev(A), dev(B), nprod=nprod, out_dtype=torch.float64))
    E = oracle.split_product(A, B, nprod)
    bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32)
    assert np.all(np.abs(C - E) <= bound)


@pytest.mark.parametrize("kind", ["uniform_f32", "m2e_f32"])
def test_split_normwise_error(mm, kind):
    n = 512
    A, B = I.pair(kind, n, n, n, seed=0)
    R = oracle.gemm(A, B)
    e6 = oracle.normwise_rel(host(mm.gemm_split_bf16(dev(A), dev(B), nprod=6, out_dtype=torch.float64)), R)
    e3 = oracle.normwise_rel(host(mm.gemm_split_bf16(dev(A), dev(B), nprod=3, out_dtype=torch.float64)), R)
    assert e6 <= 1e-6
    if kind == "uniform_f32":
        assert 1e-6 < e3 < 1e-5   # the 3-product form is not FP32-accurate on zero-mean data
    else:
        assert e3 <= 3e-6   # all-positive data: about 1e-6 at n = 512, falling as 1/sqrt(K)


def test_split_integer_bit_exact(mm):
    A, B = I.pair("int_f32", 200, 300, 400, seed=1)
    R = oracle.gemm(A, B)
    for nprod in (3, 6):
        C = host(mm.gemm_split_bf16(dev(A), dev(B), nprod=nprod))
        assert np.array_equal(C.astype(np.float64), R)


def test_split_explicit_workspace_and_variants(mm):
    M, N, K = 200, 190, 180
    A, B = I.pair("uniform_f32", M, N, K, seed=2)
    dA, dB = dev(A), dev(B)
    E = oracle.split_product(A, B, 6)
    bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(E)
    ws = torch.empty(mm.split_workspace_bytes(M, N, K, 6), dtype=torch.uint8, device="cuda")
    C = host(mm.gemm_split_bf16(dA, dB, nprod=6, workspace=ws))
    assert np.all(np.abs(C - E) <= bound)
    for v in range(mm.variant_count("split6")):
        C = torch.empty((M, N), dtype=torch.float32, device="cuda")
        mm.gemm_variant("split6", v, dA, dB, C)
        assert np.all(np.abs(host(C) - E) <= bound)


@pytest.mark.parametrize("nprod", [3, 6])
@pytest.mark.parametrize("shape", [(300, 270, 333), (64, 64, 32), (129, 7, 70), (1, 1, 1), (33, 65, 1000)])
def test_split_variants_bit_identical(mm, nprod, shape):
    """Every split variant -- planes read by registers or by direct loads, or
    the fused tile that splits the FP32 operands itself -- sums the same plane
    products in the same order, so all results are equal bit for bit."""
    M, N, K = shape
    method = f"split{nprod}"
    A, B = I.pair("uniform_f32", M, N, K, seed=M + N)
    dA, dB = dev(A), dev(B)
    # the same operands behind a misaligned base and padded leading dimensions;
    # NaN padding: a tile's last K step reads A's row past K and must clear it
    pa = torch.full((M, K + 3), float("nan"), dtype=torch.float32, device="cuda")
    pb = torch.full((K, N + 5), float("nan"), dtype=torch.float32, device="cuda")
    pa[:, 1:K + 1] = dA
    pb[:, 2:N + 2] = dB
    vA, vB = pa[:, 1:K + 1], pb[:, 2:N + 2]
    ref = None
    for v in range(mm.variant_count(method)):
        for a, b in ((dA, dB), (vA, vB)):
            C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
            mm.gemm_variant(method, v, a, b, C)
            Ch = host(C)
            if ref is None:
                ref = Ch
            assert np.array_equal(Ch, ref), f"variant {v} {mm.variant_info(method, v)}"
    E = oracle.split_product(A, B, nprod)
    bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(E)
    assert np.all(np.abs(ref - E) <= bound)


# ------------------------------------------------------------------ residual

def test_split_at_the_k_limit_bit_exact(mm):
    """Split products at the largest K the split methods take (2^26 - 32):
    the direct tiles' lane offsets over 16 plane rows reach ~2^31 bytes.
    Integer-valued operands with a sparse A keep every partial sum exact in
    FP32, so every variant must equal the oracle bit for bit."""
    K = (1 << 26) - 32
    M, N = 16, 16
    rng = np.random.default_rng(26)
    nnz = 4096
    cols = np.sort(np.concatenate([rng.choice(K - 64, size=(M, nnz - 64)), np.tile(np.arange(K - 64, K), (M, 1))], axis=1), axis=1)
    vals = rng.integers(-8, 9, size=cols.shape).astype(np.float32)
    A = torch.zeros((M, K), dtype=torch.float32, device="cuda")
    rows = np.repeat(np.arange(M), cols.shape[1])
    A.index_put_((torch.from_numpy(rows).cuda(), torch.from_numpy(cols.reshape(-1)).cuda()),
                 torch.from_numpy(vals.reshape(-1)).cuda(), accumulate=True)
    kk = torch.arange(K, device="cuda", dtype=torch.int64).view(K, 1)
    jj = torch.arange(N, device="cuda", dtype=torch.int64).view(1, N)
    B = (((kk * 7 + jj * 3) % 17) - 8).to(torch.float32)          # integers in [-8, 8]
    R = oracle.gemm(host(A).astype(np.float64), host(B).astype(np.float64))
    assert np.abs(R).max() < 2 ** 24                                # every partial sum exact in FP32
    ws = torch.empty(mm.split_workspace_bytes(M, N, K, 6), dtype=torch.uint8, device="cuda")
    for method in ("split3", "split6"):
        # the default choice, and the 64x64 and 256x128 direct-ring variants
        for v in (None, 8, 14):
            C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
            if v is None:
                mm.gemm_split_bf16(A, B, 3 if method == "split3" else 6, C=C, workspace=ws)
            else:
                mm.gemm_variant(method, v, A, B, C, workspace=ws)
            assert np.array_equal(host(C).astype(np.float64), R), f"{method} variant {v}"


def test_residual_exact_and_planted(mm):
    M, N, K = 90, 70, 110
    A, B = I.pair("int_f64", M, N, K, seed=5)
    C = oracle.gemm(A, B)
    x = I.integer(I.rng_for(6), (N,))
    r2, z2 = host(mm.residual_f64(dev(A), dev(B), dev(C), dev(x)))
    o_r2, o_z2 = oracle.freivalds(A, B, C, x)
    assert r2 == 0.0 and o_r2 == 0.0 and z2 == o_z2
    C2 = C.copy()
    C2[11, 13] += 3.0
    r2, _ = host(mm.residual_f64(dev(A), dev(B), dev(C2), dev(x)))
    assert r2 == (3.0 * x[13]) ** 2


def test_residual_float_inputs(mm):
    M, N, K = 300, 257, 129
    A, B = I.pair("uniform_f32", M, N, K, seed=7)
    x = I.probe_vector(N)
    dA, dB = dev(A), dev(B)
    C = mm.gemm_split_bf16(dA, dB, nprod=6)
    r2, z2 = host(mm.residual_f64(dA, dB, C, dev(x)))
    o_r2, o_z2 = oracle.freivalds(A, B, host(C), x)
    assert abs(z2 - o_z2) <= 1e-12 * o_z2
    assert abs(np.sqrt(r2) - np.sqrt(o_r2)) <= 1e-9 * np.sqrt(o_z2)
    assert np.sqrt(r2 / z2) < 1e-6


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512, 1024])
def test_f64_paper_sizes_box_muller(mm, n):
    """The paper's sizes with its N(0,1) Box-Muller inputs."""
    A, B = I.pair("normal_f64", n, n, n, seed=n)
    C = host(mm.gemm_f64(dev(A), dev(B)))
    assert_within_bound(C, A, B, oracle.U_F64)


# ------------------------------------------------------------------ full size

@pytest.mark.parametrize("n", [4096, 8192])
@pytest.mark.parametrize("kind", ["uniform_f64", "int_f64"])
def test_f64_full_size_sampled(mm, kind, n):
    A, B = I.pair(kind, n, n, n, seed=0)
    C = host(mm.gemm_f64(dev(A), dev(B)))
    rng = np.random.default_rng(99)
    rows = np.concatenate([rng.integers(0, n, 1500), [0, n - 1, n - 1, 0]])
    cols = np.concatenate([rng.integers(0, n, 1500), [0, n - 1, 0, n - 1]])
    ref = oracle.gemm_entries(A, B, rows, cols)
    got = C[rows, cols]
    if kind == "int_f64":
        assert np.array_equal(got, ref)
    else:
        absref = oracle.gemm_entries(np.abs(A), np.abs(B), rows, cols)
        assert np.all(np.abs(got - ref) <= 4 * n * oracle.U_F64 * absref)


@pytest.mark.parametrize("kind", ["uniform_f32", "m2e_f32"])
def test_f32_and_split_8192_rows(mm, kind):
    """Precision configuration at full size, default variants: three whole rows
    of the FP32 and split products against the oracle -- per entry against the
    split emulation, normwise against the exact product (<= 1e-6 where the
    method reaches it: 3 planes always, 2 planes on the positive m*2^e set)."""
    n = 8192
    A, B = I.pair(kind, n, n, n, seed=0)
    dA, dB = dev(A), dev(B)
    rows = [0, 4095, n - 1]
    Ar = A[rows]
    R = oracle.gemm(Ar, B)
    absR = oracle.abs_product(Ar, B)
    C32 = host(mm.gemm_f32(dA, dB))[rows]
    assert np.all(np.abs(C32 - R) <= oracle.elementwise_bound(absR, n, oracle.U_F32))
    for nprod in (3, 6):
        C = host(mm.gemm_split_bf16(dA, dB, nprod=nprod))[rows].astype(np.float64)
        E = oracle.split_product(Ar, B, nprod)
        assert np.all(np.abs(C - E) <= oracle.elementwise_bound(absR, n, oracle.U_F32) + 2.0 ** -24 * np.abs(E))
        err = oracle.normwise_rel(C, R)
        if nprod == 6 or kind == "m2e_f32":
            assert err <= 1e-6, (nprod, kind, err)
        else:
            assert err <= 1e-5, (nprod, kind, err)


def test_peak_probe_runs(mm):
    """The measurement aids (MFMA-only throughput, matrix/vector overlap)
    launch for every dtype and role and write their output (they compute no
    product, so only completion is checked)."""
    import ctypes
    from paper_2408_15384_amd import build as B
    lib = ctypes.CDLL(B.PEAK_LIB)
    fn = lib.mm_peak_mfma
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    out = torch.full((4 * 256,), float("nan"), dtype=torch.float32, device="cuda")
    for dtype in (0, 1, 2):
        for chains in (8, 16, 32):
            out.fill_(float("nan"))
            assert fn(dtype, chains, 4, 16, out.data_ptr(), torch.cuda.current_stream().cuda_stream) == 0
            torch.cuda.synchronize()
            assert torch.isfinite(out).all()
    ov = lib.mm_peak_overlap
    ov.restype = ctypes.c_int32
    ov.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    out = torch.full((4 * 512,), float("nan"), dtype=torch.float32, device="cuda")
    for role in (0, 1, 2):
        out.fill_(float("nan"))
        assert ov(role, 4, 16, out.data_ptr(), torch.cuda.current_stream().cuda_stream) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
