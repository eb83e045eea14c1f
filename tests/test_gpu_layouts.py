"""Transposed and column-major operands (mm_gemm_ex) on the GPU: the result
must be bit-identical to the row-major product on explicitly transposed
inputs, and within the oracle's per-entry bound."""
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


KIND = {"f64": "uniform_f64", "f32": "uniform_f32", "split3": "uniform_f32", "split6": "uniform_f32"}


def nn(mm, method, A, B):
    if method == "f64":
        return mm.gemm_f64(A, B)
    if method == "f32":
        return mm.gemm_f32(A, B)
    return mm.gemm_split_bf16(A, B, nprod=int(method[-1]))


@pytest.mark.parametrize("method", ["f64", "f32", "split3", "split6"])
@pytest.mark.parametrize("ops", ["NN", "NT", "TN", "TT"])
@pytest.mark.parametrize("shape", [(70, 45, 37), (129, 257, 100)])
def test_transposed_operands(mm, method, ops, shape):
    M, N, K = shape
    Aop, Bop = I.pair(KIND[method], M, N, K, seed=M + N)
    As = np.ascontiguousarray(Aop.T) if ops[0] == "T" else Aop
    Bs = np.ascontiguousarray(Bop.T) if ops[1] == "T" else Bop
    C = mm.gemm_ex(method, torch.from_numpy(As).cuda(), torch.from_numpy(Bs).cuda(), ops[0], ops[1])
    ref = nn(mm, method, torch.from_numpy(Aop).cuda(), torch.from_numpy(Bop).cuda())
    torch.cuda.synchronize()
    Ch = C.cpu().numpy()
    assert np.array_equal(Ch, ref.cpu().numpy())
    if method.startswith("split"):
        R = oracle.split_product(Aop, Bop, int(method[-1]))
        bound = oracle.elementwise_bound(oracle.abs_product(Aop, Bop), K, oracle.U_F32) + 2.0 ** -24 * np.abs(R)
    else:
        R = oracle.gemm(Aop, Bop)
        bound = oracle.elementwise_bound(oracle.abs_product(Aop, Bop), K, oracle.U_F64 if method == "f64" else oracle.U_F32)
    assert np.all(np.abs(Ch.astype(np.float64) - R) <= bound)


def test_transposed_with_leading_dims_and_workspace(mm):
    M, N, K = 33, 65, 47
    Aop, Bop = I.pair("uniform_f64", M, N, K, seed=3)
    Ast = torch.zeros((K, M + 5), dtype=torch.float64, device="cuda")   # A stored transposed, padded rows
    Bst = torch.zeros((N, K + 3), dtype=torch.float64, device="cuda")   # B stored transposed, padded rows
    Ast[:, :M] = torch.from_numpy(np.ascontiguousarray(Aop.T)).cuda()
    Bst[:, :K] = torch.from_numpy(np.ascontiguousarray(Bop.T)).cuda()
    ws = torch.empty(mm.lib().mm_gemm_ex_workspace_bytes(0, 1, 1, M, N, K), dtype=torch.uint8, device="cuda")
    C = mm.gemm_ex("f64", Ast[:, :M], Bst[:, :K], "T", "T", workspace=ws)
    torch.cuda.synchronize()
    R = oracle.gemm(Aop, Bop)
    bound = oracle.elementwise_bound(oracle.abs_product(Aop, Bop), K, oracle.U_F64)
    assert np.all(np.abs(C.cpu().numpy() - R) <= bound)
    with pytest.raises(mm.MMError):
        mm.gemm_ex("f64", Ast[:, :M], Bst[:, :K], "T", "T", workspace=ws[:16])


def test_column_major_product(mm):
    M, N, K = 40, 30, 50
    A, B = I.pair("int_f64", M, N, K, seed=4)
    A_cm = torch.from_numpy(np.asfortranarray(A).ravel(order="K")).cuda()
    B_cm = torch.from_numpy(np.asfortranarray(B).ravel(order="K")).cuda()
    C_cm = mm.gemm_colmajor_f64(A_cm, B_cm, M, N, K)
    torch.cuda.synchronize()
    C = C_cm.cpu().numpy().reshape(N, M).T      # column-major buffer read back
    assert np.array_equal(C, oracle.gemm(A, B))


# ------------------------------------------------------------ command line

@pytest.mark.parametrize("argv", [
    ["96", "80", "72"],
    ["64", "48", "80", "--method", "split6", "--inputs", "normal", "--trans-b"],
    ["64", "48", "80", "--method", "f32", "--trans-a", "--trans-b"],
    ["96", "64", "128", "--method", "strassen", "--inputs", "int"],
])
def test_cli_runs_on_gpu(argv):
    from paper_2408_15384_amd import cli
    a = cli.parse(argv + ["--reps", "3", "--warmup", "1"])
    res = cli.run(a)
    assert res["median_s"] > 0 and res["min_s"] <= res["median_s"]
    tol = 1e-5 if a.method in ("f32", "split6") else 1e-13
    assert res["freivalds_rel_residual"] < tol


def test_row_shard_equals_rows_of_whole_product(mm):
    # one GPU's share of a row-sharded product: the same rows, bit for bit
    n, m = 1536, 192
    A, B = I.pair("uniform_f64", n, n, n, seed=31)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for v in range(mm.variant_count("f64")):
        Cf = torch.empty((n, n), dtype=torch.float64, device="cuda")
        mm.gemm_variant("f64", v, dA, dB, Cf)
        for r0 in (0, 5 * m):
            Cs = torch.empty((m, n), dtype=torch.float64, device="cuda")
            mm.gemm_variant("f64", v, dA[r0:r0 + m], dB, Cs)
            torch.cuda.synchronize()
            assert torch.equal(Cs, Cf[r0:r0 + m]), f"variant {v} rows {r0}.."
