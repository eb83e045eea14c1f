"""Tile-covering parity at the full sizes, in the launch configurations the
benchmark times.

Single products at M = N = K = 8192 (binary64 on uniform and integer-valued
inputs, FP32, and both split forms on the two FP32 input sets): one whole row
of C from every band of BM rows of the default variant's workgroup tile (at a
seeded position inside the band) plus the last row, so every workgroup tile of
the launch has checked entries -- all BN-wide column tiles of each band lie on
that row.  Bar: bit-exact on integers; |C - C_ref| <= 4*K*u*(|A||B|) per entry
for binary64 and FP32 (section III sum in the oracle); the split forms per
entry against the oracle's plane emulation, within the FP32 accumulation bound
plus the final rounding of the stored FP32 value.

The 512-problem batch (dimensions log-uniform on [32, 1024], seed 0) at the
autotuned (variant, schedule) of each FP32-input method, replayed from its
plan's graph: every entry of every problem against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2408_15384_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_FULL = 8192


@pytest.fixture(scope="module")
def mm():
    from paper_2408_15384_amd import api
    api.load_library()
    assert api.lib().mm_init(0) == 0, api.lib().mm_last_error()
    return api


def band_rows(n, bm, seed):
    """One row per band of bm rows, at a seeded offset inside the band, and
    the last row."""
    rng = np.random.default_rng(seed)
    bands = (n + bm - 1) // bm
    rows = [min(b * bm + int(rng.integers(0, bm)), n - 1) for b in range(bands)]
    return sorted(set(rows + [n - 1]))


def tile_hits(rows, bm):
    return {r // bm for r in rows}


@pytest.mark.parametrize("kind", ["uniform_f64", "int_f64"])
def test_f64_8192_every_tile(mm, kind):
    n = N_FULL
    v = mm.select_variant("f64", n, n, n)
    bm, bn, _ = mm.variant_info("f64", v)
    rows = band_rows(n, bm, seed=11)
    assert tile_hits(rows, bm) == set(range((n + bm - 1) // bm))
    A, B = I.pair(kind, n, n, n, seed=0)
    C = mm.gemm_f64(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    got = C[rows].cpu().numpy()
    del C
    R = oracle.gemm(A[rows], B)
    if kind == "int_f64":
        assert np.array_equal(got, R)
    else:
        bound = oracle.elementwise_bound(oracle.abs_product(A[rows], B), n, oracle.U_F64)
        bad = np.abs(got - R) > bound
        assert not bad.any(), f"variant {v}: {bad.sum()} entries outside the bound"


@pytest.mark.parametrize("kind", ["uniform_f32", "m2e_f32"])
def test_f32_and_split_8192_every_tile(mm, kind):
    n = N_FULL
    A, B = I.pair(kind, n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    # FP32
    v = mm.select_variant("f32", n, n, n)
    bm, _, _ = mm.variant_info("f32", v)
    rows = band_rows(n, bm, seed=12)
    assert tile_hits(rows, bm) == set(range((n + bm - 1) // bm))
    mm.gemm_f32(dA, dB, C)
    torch.cuda.synchronize()
    got = C[rows].cpu().numpy().astype(np.float64)
    R = oracle.gemm(A[rows], B)
    absR = oracle.abs_product(A[rows], B)
    assert np.all(np.abs(got - R) <= oracle.elementwise_bound(absR, n, oracle.U_F32)), f"fp32 variant {v}"
    # split forms: per entry against the plane emulation
    ws = torch.empty(mm.split_workspace_bytes(n, n, n, 6), dtype=torch.uint8, device="cuda")
    for nprod, method in ((3, "split3"), (6, "split6")):
        v = mm.select_variant(method, n, n, n)
        bm, _, _ = mm.variant_info(method, v)
        rows = band_rows(n, bm, seed=13 + nprod)
        assert tile_hits(rows, bm) == set(range((n + bm - 1) // bm))
        C.fill_(float("nan"))
        mm.gemm_split_bf16(dA, dB, nprod, C=C, workspace=ws)
        torch.cuda.synchronize()
        got = C[rows].cpu().numpy().astype(np.float64)
        E = oracle.split_product(A[rows], B, nprod)
        absR = oracle.abs_product(A[rows], B)
        bound = oracle.elementwise_bound(absR, n, oracle.U_F32) + 2.0 ** -24 * np.abs(E)
        bad = np.abs(got - E) > bound
        assert not bad.any(), f"{method} variant {v}: {bad.sum()} entries outside the bound"


@pytest.mark.parametrize("method", ["f32", "split3", "split6"])
def test_grouped_batch_autotuned_every_entry(mm, method):
    shapes = [tuple(int(v) for v in s) for s in I.grouped_shapes(512, 32, 1024, seed=0)]
    hostA, hostB, As, Bs, Cs = [], [], [], [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B = I.pair("uniform_f32", M, N, K, seed=(0, i))
        hostA.append(A)
        hostB.append(B)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.empty((M, N), dtype=torch.float32, device="cuda"))
    try:
        v, s, _ = mm.grouped_autotune(method, As, Bs, Cs, warmup=1, reps=2)
        plan = mm.GroupedPlan(method)
        plan.run(As, Bs, Cs)
        info = plan.info()
        assert (info["variant"], info["schedule"]) == (v, s)
        for C in Cs:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        plan.close()
    finally:
        mm.autotune_clear()
    nprod = {"f32": 0, "split3": 3, "split6": 6}[method]
    for i, (M, N, K) in enumerate(shapes):
        got = Cs[i].cpu().numpy().astype(np.float64)
        A, B = hostA[i], hostB[i]
        absR = oracle.abs_product(A, B)
        if nprod == 0:
            ref = oracle.gemm(A, B)
            bound = oracle.elementwise_bound(absR, K, oracle.U_F32)
        else:
            ref = oracle.split_product(A, B, nprod)
            bound = oracle.elementwise_bound(absR, K, oracle.U_F32) + 2.0 ** -24 * np.abs(ref)
        bad = np.abs(got - ref) > bound
        assert not bad.any(), f"{method} (variant {v}, schedule {s}) problem {i} {M}x{N}x{K}: {bad.sum()} entries"
