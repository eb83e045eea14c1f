"""One Strassen-Winograd level on the GPU against the oracle's evaluation of
the same scheme (per-entry bound carried through the sums), the plain
product (normwise) and exact integer arithmetic."""
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


def run(mm, A, B):
    C = mm.gemm_strassen_f64(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    return C.cpu().numpy()


@pytest.mark.parametrize("shape", [(2, 2, 2), (64, 64, 64), (130, 258, 96), (512, 384, 640)])
def test_strassen_integer_exact(mm, shape):
    M, N, K = shape
    A, B = I.pair("int_f64", M, N, K, seed=M)
    assert np.array_equal(run(mm, A, B), oracle.gemm(A, B))


@pytest.mark.parametrize("shape", [(66, 98, 34), (256, 256, 256), (300, 200, 512)])
def test_strassen_matches_oracle_scheme(mm, shape):
    M, N, K = shape
    A, B = I.pair("uniform_f64", M, N, K, seed=K)
    C = run(mm, A, B)
    assert np.all(np.abs(C - oracle.strassen(A, B)) <= oracle.strassen_product_bound(A, B))
    assert oracle.normwise_rel(C, oracle.gemm(A, B)) < 20 * K * oracle.U_F64


def test_strassen_odd_and_degenerate(mm):
    with pytest.raises(mm.MMError) as e:
        run(mm, np.ones((3, 4)), np.ones((4, 6)))
    assert e.value.status == mm.MM_E_UNSUPPORTED
    A = torch.ones((4, 0), dtype=torch.float64, device="cuda")
    B = torch.ones((0, 6), dtype=torch.float64, device="cuda")
    C = torch.full((4, 6), 2.0, dtype=torch.float64, device="cuda")
    mm.gemm_strassen_f64(A, B, C)
    torch.cuda.synchronize()
    assert not C.cpu().numpy().any()


@pytest.mark.parametrize("kind", ["int_f64", "uniform_f64"])
def test_strassen_8192_sampled(mm, kind):
    n = 8192
    A, B = I.pair(kind, n, n, n, seed=0)
    C = run(mm, A, B)
    rng = np.random.default_rng(5)
    rows, cols = rng.integers(0, n, 1000), rng.integers(0, n, 1000)
    ref = oracle.gemm_entries(A, B, rows, cols)
    if kind == "int_f64":
        assert np.array_equal(C[rows, cols], ref)
    else:
        absref = oracle.gemm_entries(np.abs(A), np.abs(B), rows, cols)
        assert np.all(np.abs(C[rows, cols] - ref) <= 64 * n * oracle.U_F64 * absref)
