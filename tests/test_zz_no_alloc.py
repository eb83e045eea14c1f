"""The no-allocation residual entry point (mm_residual_f64_noalloc) against
mm_residual_f64 through the C ABI: the same kernels on the same inputs, so the
two results must be equal bit for bit.  Two calls in a row on the fixed
scratch, the second with a smaller input, each against the allocating entry
point; sizes beyond the fixed scratch are refused."""
import ctypes

import numpy as np
import pytest

from paper_2408_15384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mm():
    from paper_2408_15384_amd import api
    api.load_library()
    assert api.lib().mm_init(0) == 0, api.lib().mm_last_error()
    return api


def product(mm, kind, M, N, K, seed):
    A, B = I.pair(kind, M, N, K, seed=seed)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = mm.gemm_f64(dA, dB) if A.dtype == np.float64 else mm.gemm_f32(dA, dB)
    x = torch.from_numpy(I.probe_vector(N, seed=seed)).cuda()
    return dA, dB, C, x


@pytest.mark.parametrize("kind", ["uniform_f64", "uniform_f32"])
def test_noalloc_equals_allocating_entry(mm, kind):
    big = (2000, 1500, 3000)
    small = (100, 64, 50)
    for i, (M, N, K) in enumerate((big, small)):
        dA, dB, C, x = product(mm, kind, M, N, K, seed=40 + i)
        if i == 1:
            # a planted error: the probe must see it in both entry points
            C[7, 5] += 0.25
        ref = mm.residual_f64(dA, dB, C, x)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        mm.residual_f64_noalloc(dA, dB, C, x, out=out)
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert np.array_equal(r, o), (M, N, K, r, o)
        assert o[1] > 0
        if i == 1:
            assert o[0] > 0.25 ** 2 * float(x[5]) ** 2 * 0.99


def test_noalloc_limit(mm):
    lib = mm.lib()
    cap = int(lib.mm_residual_noalloc_max_bytes())
    assert cap == 2 << 20
    # K + 2M + 512 doubles must fit: the largest K for M = 1 fits, one more does not
    M, N = 1, 8
    K_fit = cap // 8 - 2 * M - 512
    for K, ok in ((K_fit, True), (K_fit + 1, False)):
        A = torch.zeros((M, K), dtype=torch.float64, device="cuda")
        B = torch.zeros((K, N), dtype=torch.float64, device="cuda")
        C = torch.zeros((M, N), dtype=torch.float64, device="cuda")
        x = torch.ones(N, dtype=torch.float64, device="cuda")
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        st = lib.mm_residual_f64_noalloc(M, N, K, A.data_ptr(), K, B.data_ptr(), N, C.data_ptr(), N, 0, 0,
                                         x.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        if ok:
            assert st == 0, lib.mm_last_error()
            assert out.cpu().numpy().tolist() == [0.0, 0.0]
        else:
            assert st == -1 and b"scratch" in lib.mm_last_error()
            assert np.isnan(out.cpu().numpy()).all()   # nothing was enqueued
