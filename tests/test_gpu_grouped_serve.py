"""GPU parity of the grouped launch, its graph-replayed plans, the autotuner
and the serving loop, through the C ABI.  A grouped or served result must be
bit-identical to the single-problem kernel with the same tile variant, and
within the per-entry bound of the oracle."""
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
DT = {"f64": torch.float64, "f32": torch.float32, "split3": torch.float32, "split6": torch.float32}


def make_batch(method, shapes, seed):
    As, Bs, Cs, hostAB = [], [], [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B = I.pair(KIND[method], M, N, K, seed=(seed, i))
        hostAB.append((A, B))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.full((M, N), float("nan"), dtype=DT[method], device="cuda"))
    return As, Bs, Cs, hostAB


def ragged_shapes(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    dims = I.log_uniform_dims(rng, 3 * n, lo, hi).reshape(n, 3)
    shapes = [tuple(int(x) for x in d) for d in dims]
    shapes[3] = (shapes[3][0], shapes[3][1], 0)      # K == 0: C := 0
    shapes[5] = (0, shapes[5][1], shapes[5][2])      # empty
    shapes[7] = (1, 1, 1)
    return shapes


def singles(mm, method, variant, As, Bs):
    out = []
    for A, B in zip(As, Bs):
        C = torch.full((A.shape[0], B.shape[1]), float("nan"), dtype=DT[method], device="cuda")
        mm.gemm_variant(method, variant, A, B, C)
        out.append(C)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in out]


def check_oracle(method, hostAB, Cs, idx):
    for i in idx:
        A, B = hostAB[i]
        C = Cs[i].cpu().numpy() if hasattr(Cs[i], "cpu") else Cs[i]
        if C.size == 0:
            continue
        K = A.shape[1]
        if method in ("split3", "split6"):
            R = oracle.split_product(A, B, int(method[-1]))
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(R)
        else:
            R = oracle.gemm(A, B)
            u = oracle.U_F64 if method == "f64" else oracle.U_F32
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, u)
        assert np.all(np.abs(C - R) <= bound), f"problem {i} shape {A.shape}x{B.shape}"


@pytest.mark.parametrize("method", ["f64", "f32", "split3", "split6"])
def test_grouped_equals_single_every_schedule(mm, method):
    shapes = ragged_shapes(40, 1, 300, seed=1)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=2)
    variant = 1
    ref = singles(mm, method, variant, As, Bs)
    for schedule in (0, 1, 2, 3):
        for C in Cs:
            C.fill_(float("nan"))
        mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
        torch.cuda.synchronize()
        for i, C in enumerate(Cs):
            assert np.array_equal(C.cpu().numpy(), ref[i], equal_nan=False), f"schedule {schedule} problem {i}"
    check_oracle(method, hostAB, Cs, range(len(shapes)))


@pytest.mark.parametrize("method", ["f32", "split6"])
def test_grouped_more_problems_than_the_staged_table(mm, method):
    """1100 problems: past the 1024 prefix sums a persistent workgroup stages
    in LDS, so the owner search reads global memory; every schedule still
    equals the single-problem kernel (a 64x64 variant for the split form)."""
    shapes = ragged_shapes(1100, 1, 48, seed=31)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=32)
    # split: a plane-reading variant and a ring-fused one (streamed form)
    for variant in ([1] if method == "f32" else [8, ring_variants(mm, method)[0]]):
        ref = singles(mm, method, variant, As, Bs)
        for schedule in (0, 1, 2, 3):
            for C in Cs:
                C.fill_(float("nan"))
            mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"variant {variant} schedule {schedule} problem {i}"
    check_oracle(method, hostAB, Cs, range(0, len(shapes), 50))


def ring_variants(mm, method):
    """The ring-fused split variants (buffer loads, pairwise planes): those with a
    streamed persistent form."""
    return [v for v in range(mm.variant_count(method)) if mm.variant_info(method, v)[2] == 32 and v >= 15]


@pytest.mark.parametrize("method", ["split3", "split6"])
def test_grouped_streamed_every_schedule(mm, method):
    """Ring-fused variants under every schedule (0 and 1: the streamed
    persistent form with a fixed stride; 2: with per-XCD tickets; 3: one
    workgroup per tile), on a ragged batch with a K == 0 problem, an empty one
    and a 1x1x1 one: each equals the single-problem kernel bit for bit.  Then
    a batch with one problem whose leading dimension is too large for the
    ring's 31-bit lane offsets, which runs the plain persistent form."""
    shapes = ragged_shapes(40, 1, 300, seed=41)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=42)
    for variant in ring_variants(mm, method):
        ref = singles(mm, method, variant, As, Bs)
        for schedule in (0, 1, 2, 3):
            for C in Cs:
                C.fill_(float("nan"))
            mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"variant {variant} schedule {schedule} problem {i}"
    check_oracle(method, hostAB, Cs, range(len(shapes)))
    # one operand view with lda = 2^23 + 2^18 floats (two rows of a 35 MB
    # buffer): 63 rows of it span more than 2^31 bytes
    lda = (1 << 23) + (1 << 18)
    big = torch.zeros(lda + 40, dtype=torch.float32, device="cuda")
    A0 = torch.as_strided(big, (2, 40), (lda, 1))
    A0.copy_(torch.from_numpy(I.pair("uniform_f32", 2, 30, 40, seed=43)[0]).cuda())
    B0 = torch.from_numpy(I.pair("uniform_f32", 2, 30, 40, seed=43)[1]).cuda()
    As2, Bs2 = [A0, *As[:6]], [B0, *Bs[:6]]
    Cs2 = [torch.full((a.shape[0], b.shape[1]), float("nan"), dtype=torch.float32, device="cuda") for a, b in zip(As2, Bs2)]
    variant = ring_variants(mm, method)[0]
    ref = singles(mm, method, variant, As2, Bs2)
    for schedule in (1, 2):
        for C in Cs2:
            C.fill_(float("nan"))
        mm.gemm_grouped(method, As2, Bs2, Cs2, variant=variant, schedule=schedule)
        torch.cuda.synchronize()
        for i, C in enumerate(Cs2):
            assert np.array_equal(C.cpu().numpy(), ref[i]), f"large lda, schedule {schedule} problem {i}"


@pytest.mark.parametrize("method", ["split3", "split6"])
def test_grouped_every_split_variant(mm, method):
    # plane-reading and fused variants alike: grouped == single, bit for bit
    shapes = ragged_shapes(24, 1, 300, seed=21)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=22)
    for variant in range(mm.variant_count(method)):
        ref = singles(mm, method, variant, As, Bs)
        for schedule in (2, 3):
            for C in Cs:
                C.fill_(float("nan"))
            mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"variant {variant} schedule {schedule} problem {i}"
    check_oracle(method, hostAB, Cs, range(len(shapes)))


@pytest.mark.parametrize("method", ["f64", "f32"])
def test_grouped_every_dense_variant(mm, method):
    """Every dense tile variant (4-wave and 16-wave workgroups, register-staged
    and direct rings of 2-4 buffers, K steps of 16 and 32) in the persistent
    form with a work counter and with one workgroup per tile, on a ragged
    batch: grouped == single, bit for bit."""
    shapes = ragged_shapes(24, 1, 300, seed=61)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=62)
    for variant in range(mm.variant_count(method)):
        ref = singles(mm, method, variant, As, Bs)
        for schedule in (2, 3):
            for C in Cs:
                C.fill_(float("nan"))
            mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"variant {variant} schedule {schedule} problem {i}"
    check_oracle(method, hostAB, Cs, range(len(shapes)))


def pair_member(mm, method, pair, M, N, K):
    """The variant size-class pair `pair` runs an M x N x K problem on: the
    small one when its tiles execute at most pct % of the large one's padded
    work (rows, columns and K rounded up to the tile), else the large one."""
    small, large, pct = mm.grouped_pair_info(method, pair)

    def work(v):
        bm, bn, bk = mm.variant_info(method, v)
        return -(-M // bm) * bm * (-(-N // bn) * bn) * (-(-max(K, 1) // bk) * bk)
    return small if work(small) * 100 <= pct * work(large) else large


@pytest.mark.parametrize("method", ["f64", "f32", "split3", "split6"])
def test_grouped_size_class_pairs(mm, method):
    """Every size-class pair under every schedule, on a ragged batch (K == 0,
    an empty problem, 1x1x1) whose problems fall to both members: each problem
    equals, bit for bit, the single-problem kernel of the member the pair's
    rule picks for its shape; then a plan of the pair replayed with eager work
    in between."""
    shapes = ragged_shapes(40, 1, 300, seed=51)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=52)
    for pair in range(mm.grouped_pair_count(method)):
        small, large, _ = mm.grouped_pair_info(method, pair)
        ref = {v: singles(mm, method, v, As, Bs) for v in (small, large)}
        member = [pair_member(mm, method, pair, *sh) for sh in shapes]
        assert small in member and large in member
        for schedule in (0, 1, 2, 3):
            for C in Cs:
                C.fill_(float("nan"))
            mm.gemm_grouped(method, As, Bs, Cs, variant=mm.PAIR_BASE + pair, schedule=schedule)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[member[i]][i]), \
                    f"pair {pair} schedule {schedule} problem {i} shape {shapes[i]}"
    check_oracle(method, hostAB, Cs, range(len(shapes)))
    pair = mm.grouped_pair_count(method) - 1
    member = [pair_member(mm, method, pair, *sh) for sh in shapes]
    ref = {v: singles(mm, method, v, As, Bs) for v in set(member)}
    plan = mm.GroupedPlan(method, variant=mm.PAIR_BASE + pair, schedule=3)
    try:
        plan.run(As, Bs, Cs)
        assert plan.info()["graph"] and plan.info()["variant"] == mm.PAIR_BASE + pair
        for rep in range(3):
            for C in Cs:
                C.fill_(float("nan"))
            junk = torch.randn(256, 256, device="cuda").sum()
            torch.cuda.synchronize()
            plan.replay()
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[member[i]][i]), f"replay {rep} problem {i}"
            del junk
    finally:
        torch.cuda.synchronize()
        plan.close()


@pytest.mark.parametrize("method", ["f64", "split6"])
def test_plan_graph_replay(mm, method):
    shapes = ragged_shapes(24, 8, 260, seed=3)
    As, Bs, Cs, hostAB = make_batch(method, shapes, seed=4)
    plan = mm.GroupedPlan(method)
    try:
        plan.run(As, Bs, Cs)
        info = plan.info()
        assert info["graph"] and info["tiles"] > 0
        ref = singles(mm, method, info["variant"], As, Bs)
        for rep in range(4):
            for C in Cs:
                C.fill_(float("nan"))
            # eager work and a synchronisation between replays
            junk = torch.randn(512, 512, device="cuda").sum()
            torch.cuda.synchronize()
            plan.run(As, Bs, Cs)
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"replay {rep} problem {i}"
        # new operands at new addresses, same shapes: descriptors refreshed
        As2, Bs2, Cs2, hostAB2 = make_batch(method, shapes, seed=5)
        plan.run(As2, Bs2, Cs2)
        torch.cuda.synchronize()
        ref2 = singles(mm, method, info["variant"], As2, Bs2)
        for i, C in enumerate(Cs2):
            assert np.array_equal(C.cpu().numpy(), ref2[i])
        check_oracle(method, hostAB2, Cs2, range(0, len(shapes), 3))
        # other shapes: refused
        with pytest.raises(mm.MMError):
            plan.run(As[:-1], Bs[:-1], Cs[:-1])
    finally:
        torch.cuda.synchronize()
        plan.close()
    del junk


@pytest.mark.parametrize("method,variant", [("f32", 1), ("split3", 8)])
@pytest.mark.parametrize("schedule", [0, 2, 3])
def test_plan_replay_every_schedule(mm, method, variant, schedule):
    """A plan's graph holds [split pass ->] counter reset -> grouped product;
    replayed several times with eager work and synchronisation in between,
    every replay equals the single-problem kernel (schedule 2 depends on the
    in-graph reset of its work counter; variant 8 reads planes, so the split
    pass is in the graph too)."""
    shapes = ragged_shapes(30, 4, 200, seed=41)
    As, Bs, Cs, _ = make_batch(method, shapes, seed=42)
    ref = singles(mm, method, variant, As, Bs)
    plan = mm.GroupedPlan(method, variant=variant, schedule=schedule)
    try:
        plan.run(As, Bs, Cs)
        assert plan.info()["graph"] and plan.info()["schedule"] == schedule
        for rep in range(4):
            for C in Cs:
                C.fill_(float("nan"))
            junk = torch.randn(256, 256, device="cuda").sum()
            torch.cuda.synchronize()
            plan.replay()
            torch.cuda.synchronize()
            for i, C in enumerate(Cs):
                assert np.array_equal(C.cpu().numpy(), ref[i]), f"replay {rep} problem {i}"
            del junk
    finally:
        torch.cuda.synchronize()
        plan.close()


def test_grouped_config4_shapes_sampled(mm):
    shapes = [tuple(int(x) for x in s) for s in I.grouped_shapes(512, 32, 1024, seed=0)]
    As, Bs, Cs, hostAB = make_batch("f32", shapes, seed=0)
    plan = mm.GroupedPlan("split6")
    try:
        plan.run(As, Bs, Cs)
        torch.cuda.synchronize()
        check_oracle("split6", hostAB, Cs, range(0, 512, 37))
        v = plan.info()["variant"]
        idx = list(range(0, 512, 17))
        ref = singles(mm, "split6", v, [As[i] for i in idx], [Bs[i] for i in idx])
        for j, i in enumerate(idx):
            assert np.array_equal(Cs[i].cpu().numpy(), ref[j])
    finally:
        torch.cuda.synchronize()
        plan.close()


def test_autotuners(mm, tmp_path):
    A, B = I.pair("uniform_f64", 512, 512, 512, seed=8)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((512, 512), dtype=torch.float64, device="cuda")
    mm.autotune_clear()
    v, ms = mm.autotune("f64", dA, dB, C, warmup=1, reps=3)
    assert 0 <= v < mm.variant_count("f64") and ms > 0
    assert mm.select_variant("f64", 512, 512, 512) == v
    path = str(tmp_path / "tune.json")
    mm.autotune_save(path)
    mm.autotune_clear()
    mm.autotune_load(path)
    assert mm.select_variant("f64", 512, 512, 512) == v
    C2 = mm.gemm_f64(dA, dB)
    torch.cuda.synchronize()
    assert np.array_equal(C2.cpu().numpy(), singles(mm, "f64", v, [dA], [dB])[0])
    shapes = ragged_shapes(16, 16, 200, seed=9)
    As, Bs, Cs, hostAB = make_batch("f32", shapes, seed=9)
    gv, gs, gms = mm.grouped_autotune("f32", As, Bs, Cs, warmup=1, reps=2)
    assert (0 <= gv < mm.variant_count("f32") or 0 <= gv - mm.PAIR_BASE < mm.grouped_pair_count("f32")) \
        and gs in (0, 1, 2, 3) and gms > 0
    plan = mm.GroupedPlan("f32")
    plan.run(As, Bs, Cs)
    torch.cuda.synchronize()
    assert plan.info()["variant"] == gv
    plan.close()
    check_oracle("f32", hostAB, Cs, range(len(shapes)))
    mm.autotune_clear()


# ------------------------------------------------------------------ serving

METHOD_ID = {"f64": 0, "f32": 1, "split3": 2, "split6": 3}


def serve_all(mm, reqs, budget, slots, max_batch, one_at_a_time=False, **server_kw):
    # the results start as NaN, written on torch's stream; the server's slot
    # streams do not wait for it, so the fills finish before any submission
    outs = [torch.full((A.shape[0], B.shape[1]), float("nan"), dtype=DT[method], device="cuda")
            for method, A, B in reqs]
    torch.cuda.synchronize()
    with mm.Server(budget_bytes=budget, slots=slots, max_batch=max_batch, **server_kw) as srv:
        ids = []
        for (method, A, B), C in zip(reqs, outs):
            rid = srv.submit(A, B, C, METHOD_ID[method])
            if one_at_a_time:
                st, _ = srv.wait(rid)
                assert st == 0
            else:
                ids.append(rid)
        for rid in ids:
            st, lat = srv.wait(rid)
            assert st == 0 and lat > 0
        stats = srv.stats()
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in outs], stats


def test_serving_alone_equals_mix(mm):
    rng = np.random.default_rng(11)
    methods = ["f64", "split6", "f32", "split3"]
    reqs, hostAB = [], []
    for i in range(32):
        m = methods[i % 4]
        M, N, K = (int(x) for x in I.log_uniform_dims(rng, 3, 16, 700))
        A, B = I.pair(KIND[m], M, N, K, seed=(12, i))
        hostAB.append((m, A, B))
        reqs.append((m, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
    alone, _ = serve_all(mm, reqs, budget=1 << 34, slots=1, max_batch=1, one_at_a_time=True)
    mix, st = serve_all(mm, reqs, budget=1 << 34, slots=4, max_batch=16)
    assert st["completed"] == 32 and st["failed"] == 0
    for i in range(32):
        assert np.array_equal(alone[i], mix[i]), f"request {i}"
    for i, (m, A, B) in enumerate(hostAB):
        check_oracle(m, [(A, B)], [mix[i]], [0])
    # a tight budget forces queueing; results unchanged
    tight, st2 = serve_all(mm, reqs, budget=3 * 700 * 700 * 8 * 3, slots=4, max_batch=16)
    assert st2["peak_bytes"] <= 3 * 700 * 700 * 8 * 3
    for i in range(32):
        assert np.array_equal(tight[i], mix[i])


def test_serving_stats(mm):
    reqs = []
    for i in range(20):
        A, B = I.pair("uniform_f64", 256, 256, 256, seed=(13, i))
        reqs.append(("f64", torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
    _, st = serve_all(mm, reqs, budget=1 << 32, slots=2, max_batch=8)
    assert st["completed"] == 20
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["useful_flop"] == 20 * 2 * 256 ** 3
    assert st["tflops"] > 0 and st["launches"] >= 1


def test_serving_large_class_and_workspace_growth(mm):
    """Requests of the large class (M*N >= 1024^2) with plane-reading split
    tiles: each slot's split workspace grows several times while earlier
    launches still run (outgrown buffers are kept, not freed).  Results equal
    the same requests served one at a time and stay within the oracle bound."""
    shapes = [(300, 200, 96), (1024, 1024, 64), (1040, 1100, 160), (200, 300, 500), (1100, 1030, 384),
              (1200, 1024, 640), (700, 90, 33), (1030, 1200, 1000)]
    methods = ["split6", "split3", "f64", "split6", "split3", "split6", "f64", "split6"]
    reqs, hostAB = [], []
    for i, ((M, N, K), m) in enumerate(zip(shapes, methods)):
        A, B = I.pair(KIND[m], M, N, K, seed=(14, i))
        hostAB.append((m, A, B))
        reqs.append((m, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
    # large class: the 128x128 register tile for binary64, plane-reading 256x128 split tiles
    kw = dict(variants=[-1, -1, -1, -1], variants_large=[0, -1, 14, 9], large_mn=1024 * 1024)
    alone, _ = serve_all(mm, reqs, budget=1 << 34, slots=1, max_batch=1, one_at_a_time=True, **kw)
    mix, st = serve_all(mm, reqs, budget=1 << 34, slots=2, max_batch=4, **kw)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for i in range(len(reqs)):
        assert np.array_equal(alone[i], mix[i]), f"request {i}"
    for i, (m, A, B) in enumerate(hostAB):
        check_oracle(m, [(A, B)], [mix[i]], [0])

