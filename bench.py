#!/usr/bin/env python3
"""Benchmark of the dense product C = A.B on one MI355X.

Headline (the JSON line's `value`): binary64 GEMM throughput at M = N = K = 8192
(entries uniform on [-1, 1), seed 0), in TFLOP/s = 2N^3 / time, inputs resident
in HBM before the timed region.  A step is one C = A.B through the C ABI.
Protocol: W untimed warm-up steps, then K timed steps between device
synchronisations (15 by default, the repetition count of the paper's
experiments); each launch is also bracketed by HIP events on its stream, whose
mean is the kernel duration used for the roofline.

Also reported in the same line (context, not the headline):
  * cpu_baseline: the CPU oracle timed on a bounded sample of the same product
    (the first rows of C), on all host cores, and the sample's error;
  * precision: plain FP32 versus the split-bfloat16 forms at N = 8192 on two
    input sets, each with its error against the binary64 oracle (sampled rows)
    and its binary64 residual probe;
  * grouped: 512 FP32 problems with dimensions log-uniform on [32, 1024], one
    graph-replayed launch (tile variant and schedule autotuned), plain FP32
    versus split, with the residual probe of every result and the oracle's
    error on a sample;
  * serving: Poisson arrivals of GEMM requests (dimensions log-uniform on
    [64, 4096], half binary64, half FP32-accurate split), operands resident on
    the device, a 64 GiB admission budget; p50/p99 latency and throughput,
    the residual probe of every result;

  * peak: the MFMA-only throughput of each dtype on this GPU (the ceiling);
  * strassen: one Strassen-Winograd level on the binary64 product at 8192;
  * shard: one GPU's share (1024 rows) of a row-sharded 8192 product;
  * layouts: transposed operands (NN, NT, TN, TT) at 8192;
  * paper sizes: the paper's experiment (Box-Muller inputs, 32..1024), GPU
    against the oracle on one and on all host cores, and the oracle's thread
    scaling (1, 2, 4, 8, 16 threads) at 1024.

Usage: python bench.py [--gpus 1] [--steps 15] [--warmup 3]
                       [--sections peak,precision,grouped,serving,strassen,shard,layouts,paper|none]
                       [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2408_15384_amd import inputs as I  # noqa: E402

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}   # dense TFLOP/s, MI355X datasheet
HBM_TBS = 8.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemm_f64_8192.txt")
# What the headline kernel is compiled from: the tile bodies and the kernel
# wrapper, plus (added in kernel_source_hash) the compile flags and the
# variant's own entry of the binary64 table.
KERNEL_SOURCES = ["paper_2408_15384_amd/csrc/gemm_tile.h", "paper_2408_15384_amd/csrc/gptr.h",
                  "paper_2408_15384_amd/csrc/gemm_mfma.hip"]
VARIANTS_FILE = "paper_2408_15384_amd/csrc/variants.h"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def f64_variant_entry(variant: int) -> str:
    """The X(variant, ...) entry of the binary64 variant table."""
    import re
    text = open(os.path.join(ROOT, VARIANTS_FILE)).read()
    table = text[text.index("#define MM_F64_VARIANTS"):text.index("#define MM_F32_VARIANTS")]
    m = re.search(r"X\(\s*%d\s*,[^)]*\)" % variant, table)
    return m.group(0) if m else ""


def _code_only(text: str) -> str:
    """Source text without // comments and blank lines (a comment edit does not
    change the compiled kernel)."""
    import re
    lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line)


def kernel_source_hash(variant: int = 4) -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            h.update(_code_only(f.read()).encode())
    from paper_2408_15384_amd import build as B
    h.update(repr([B.ARCH, *B.COMMON[:-2], *B.DEVICE_FLAGS]).encode())   # flags, less the include path
    h.update(f64_variant_entry(variant).encode())
    return h.hexdigest()[:16]


def read_traffic(variant):
    """HBM bytes per launch of the headline kernel from the committed rocprofv3
    counter summary, or None when it is missing, was taken on other sources or
    on another tile variant."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_hash(variant):
        return None
    if vals.get("tile_variant") != str(variant):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(torch, fn, steps, warmup):
    """Wall time per step over `steps` and the mean HIP-event duration of each launch."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ev = [e0.elapsed_time(e1) for e0, e1 in evs]
    return wall * 1e3, float(np.mean(ev)), float(np.median(ev)), float(np.min(ev))


def cpu_baseline(A, B, C_gpu, target_s=12.0):
    """Oracle on the first rows of the same product, on all host cores."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    n = B.shape[1]
    K = A.shape[1]
    rows = max(cores, 4)
    t0 = time.perf_counter()
    oracle.gemm(A[:rows], B)
    dt = time.perf_counter() - t0
    rows = int(min(A.shape[0], max(rows, rows * target_s / max(dt, 1e-3))))
    rows = max(cores, (rows // cores) * cores)
    t0 = time.perf_counter()
    R = oracle.gemm(A[:rows], B)
    dt = time.perf_counter() - t0
    flop = 2.0 * rows * n * K
    # error of the GPU rows against the oracle rows: normwise, and per entry
    # against 4*K*u*(|A||B|) on a column subsample
    G = C_gpu[:rows]
    cols = np.arange(0, n, max(1, n // 256))
    rr, cc = np.meshgrid(np.arange(rows), cols, indexing="ij")
    absab = oracle.gemm_entries(np.abs(A[:rows]), np.abs(B), rr.ravel(), cc.ravel()).reshape(rr.shape)
    ratio = float((np.abs(G[:, cols] - R[:, cols]) / np.maximum(4 * K * oracle.U_F64 * absab, 1e-300)).max())
    return {
        "value": flop / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of C for M=N=K={n} binary64 (the plain loop, walked i-k-j, OpenMP over rows), "
                  f"{flop:.3g} FLOP in {dt:.1f} s",
        "gflops": flop / dt / 1e9,
        "cpu_model": _cpu_model(),
        "sample_normwise_err": float(np.linalg.norm(G - R) / np.linalg.norm(R)),
        "sample_max_err_over_bound": ratio,
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sampled_rows_error(A, B, C, rows=4, method="exact"):
    import oracle
    R = oracle.gemm(A[:rows].astype(np.float64), B.astype(np.float64))
    return float(np.linalg.norm(C[:rows].astype(np.float64) - R) / np.linalg.norm(R))


def precision_section(torch, mm, n, steps, warmup):
    out = {}
    x = torch.from_numpy(I.probe_vector(n)).cuda()
    for kind in ("uniform_f32", "m2e_f32"):
        A, B = I.pair(kind, n, n, n, seed=0)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        C = torch.empty((n, n), dtype=torch.float32, device="cuda")
        ws = torch.empty(mm.split_workspace_bytes(n, n, n, 6), dtype=torch.uint8, device="cuda")
        res = {}
        for name, fn, peak, mult in (
                ("fp32", lambda: mm.gemm_f32(dA, dB, C), PEAK["f32"], 1),
                ("split3", lambda: mm.gemm_split_bf16(dA, dB, 3, C=C, workspace=ws), PEAK["bf16"], 3),
                ("split6", lambda: mm.gemm_split_bf16(dA, dB, 6, C=C, workspace=ws), PEAK["bf16"], 6)):
            wall, ev, med, mn = timed_steps(torch, fn, max(3, steps // 3), warmup)
            r2z2 = mm.residual_f64(dA, dB, C, x).cpu().numpy()
            Ch = C.cpu().numpy()
            tf = 2.0 * n ** 3 / (ev * 1e-3) / 1e12
            res[name] = {"ms": ev, "tflops_useful": tf,
                         "mfma_frac": tf * mult / peak,
                         "normwise_err_vs_oracle_rows0_3": sampled_rows_error(A, B, Ch),
                         "freivalds_rel_residual": float(np.sqrt(r2z2[0] / r2z2[1]))}
            log(f"  precision {kind} {name}: {ev:.3f} ms {tf:.1f} TFLOP/s err {res[name]['normwise_err_vs_oracle_rows0_3']:.2e}")
        res["split6_beats_fp32"] = res["split6"]["ms"] < res["fp32"]["ms"]
        out[kind] = res
        del dA, dB, C, ws
        torch.cuda.empty_cache()
    return out


def sizes_section(torch, mm, sizes=((1024, 30), (4096, 10))):
    """The plain binary64 product at the other sizes of the headline's
    configuration (N = 1024 and 4096; 8192 is the headline): HIP-event
    throughput on uniform [-1, 1) inputs, each result checked against the
    oracle on its first rows (normwise and per entry within the bound), and
    the integer-valued inputs (uniform integers in [-8, 8]) bit-exact against
    the oracle -- the whole product at 1024, 64 rows spread over the tile rows
    at 4096."""
    import oracle
    out = {}
    for n, steps in sizes:
        A, B = I.pair("uniform_f64", n, n, n, seed=0)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        C = torch.empty((n, n), dtype=torch.float64, device="cuda")
        wall, ev, med, mn = timed_steps(torch, lambda: mm.gemm_f64(dA, dB, C), steps, 3)
        tf = 2.0 * n ** 3 / (ev * 1e-3) / 1e12
        Ch = C.cpu().numpy()
        R = oracle.gemm(A[:4], B)
        bound = oracle.elementwise_bound(oracle.abs_product(A[:4], B), n, oracle.U_F64)
        res = {"ms": ev, "tflops": tf, "frac_of_peak": tf / PEAK["f64"],
               "variant": mm.select_variant("f64", n, n, n),
               "normwise_err_vs_oracle_rows0_3": float(np.linalg.norm(Ch[:4] - R) / np.linalg.norm(R)),
               "within_bound_rows0_3": bool(np.all(np.abs(Ch[:4] - R) <= bound))}
        Ai, Bi = I.pair("int_f64", n, n, n, seed=1)
        dAi, dBi = torch.from_numpy(Ai).cuda(), torch.from_numpy(Bi).cuda()
        mm.gemm_f64(dAi, dBi, C)
        Ci = C.cpu().numpy()
        if n <= 1024:
            rows = np.arange(n)
        else:
            rows = np.unique(np.linspace(0, n - 1, 64).astype(np.int64))
        res["int_bit_exact_rows"] = int(len(rows))
        res["int_bit_exact"] = bool(np.array_equal(Ci[rows], oracle.gemm(Ai[rows], Bi)))
        out[str(n)] = res
        log(f"  binary64 {n}: {ev:.3f} ms {tf:.1f} TFLOP/s ({tf / PEAK['f64']:.1%}), integer inputs bit-exact on "
            f"{len(rows)} rows: {res['int_bit_exact']}")
        del dA, dB, dAi, dBi, C
        torch.cuda.empty_cache()
    return out


def grouped_section(torch, mm, reps=10):
    shapes = [tuple(int(v) for v in s) for s in I.grouped_shapes(512, 32, 1024, seed=0)]
    As, Bs, Cs = [], [], []
    flop = 0.0
    roof_s = 0.0
    for i, (M, N, K) in enumerate(shapes):
        A, B = I.pair("uniform_f32", M, N, K, seed=(0, i))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.empty((M, N), dtype=torch.float32, device="cuda"))
        flop += 2.0 * M * N * K
    out = {"problems": 512, "flop": flop}
    import oracle
    x_all = torch.from_numpy(I.probe_vector(1024)).cuda()
    rws = torch.empty(mm.lib().mm_residual_workspace_bytes(1024, 1024, 1024), dtype=torch.uint8, device="cuda")
    sample = sorted(np.random.default_rng(4).choice(len(shapes), size=8, replace=False).tolist())
    for method, peak, mult in (("f32", PEAK["f32"], 1), ("split6", PEAK["bf16"], 6), ("split3", PEAK["bf16"], 3)):
        roof = 0.0
        for (M, N, K) in shapes:
            bytes_ = 4.0 * (M * K + K * N + M * N)
            roof += max(2.0 * M * N * K * mult / (peak * 1e12), bytes_ / (HBM_TBS * 1e12))
        v, s, _ = mm.grouped_autotune(method, As, Bs, Cs, warmup=1, reps=3)
        plan = mm.GroupedPlan(method)
        plan.run(As, Bs, Cs)
        wall, ev, med, mn = timed_steps(torch, plan.replay, reps, 2)
        # one-shot launch with the same configuration, the problem array marshalled once
        arr, cnt = mm._problems(As, Bs, Cs)
        mid = mm.METHODS[method]
        eager = timed_steps(torch, lambda: mm.check(mm.lib().mm_gemm_grouped_config(
            arr, cnt, mid, v, s, None, mm._stream(None))), reps, 2)
        info = plan.info()
        plan.close()
        torch.cuda.synchronize()
        # binary64 residual probe of every result, and the oracle's normwise
        # error on a seeded sample of the problems
        r2z2 = torch.empty((len(shapes), 2), dtype=torch.float64, device="cuda")
        for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
            mm.residual_f64(A, B, C, x_all[:B.shape[1]], out=r2z2[i], workspace=rws)
        rr = r2z2.cpu().numpy()
        rel = np.sqrt(rr[:, 0] / np.maximum(rr[:, 1], 1e-300))
        errs = []
        for i in sample:
            M, N, K = shapes[i]
            A, B = I.pair("uniform_f32", M, N, K, seed=(0, i))
            errs.append(oracle.normwise_rel(Cs[i].cpu().numpy().astype(np.float64), oracle.gemm(A, B)))
        out[method] = {"variant": v, "schedule": s, "tiles": info["tiles"], "grid": info["grid"],
                       "graph_ms": ev, "eager_ms": eager[1],
                       "tflops_useful": flop / (ev * 1e-3) / 1e12, "roofline_ms": roof * 1e3,
                       "frac_of_roofline": roof * 1e3 / ev,
                       "freivalds_rel_residual_all": {"median": float(np.median(rel)), "max": float(rel.max())},
                       "normwise_err_vs_oracle_sample": {"problems": len(errs), "max": float(max(errs))}}
        log(f"  grouped {method}: {ev:.3f} ms graph, {eager[1]:.3f} ms eager, {out[method]['tflops_useful']:.1f} TFLOP/s, "
            f"residual max {rel.max():.2e}, sampled error max {max(errs):.2e}")
    return out


class ServingWorkload:
    """Request stream of the serving configuration with resident operands: every
    request's A and B are views into seeded 4096 x 4096 operand banks (binary64
    for FP64 requests, FP32 for split ones) at seeded offsets (columns in whole
    32-byte units, so each view starts aligned like an allocation of its own);
    C is per request."""

    def __init__(self, torch, mm, count=10000, rate=20000.0, seed=0):
        self.count, self.rate = count, rate
        self.t_arr, self.dims, self.is_f64 = I.serving_requests(count, rate, 64, 4096, 0.5, seed=seed)
        rng = I.rng_for(1)
        self.bank64 = [I.uniform_f64(rng, (4096, 4096)) for _ in range(2)]
        self.bank32 = [I.uniform_f32(rng, (4096, 4096)) for _ in range(2)]
        self.d64 = [torch.from_numpy(b).cuda() for b in self.bank64]
        self.d32 = [torch.from_numpy(b).cuda() for b in self.bank32]
        offs = np.random.default_rng(2).integers(0, 1 << 30, size=(count, 4))
        c64 = int(sum(int(d[0]) * int(d[1]) for d, f in zip(self.dims, self.is_f64) if f))
        c32 = int(sum(int(d[0]) * int(d[1]) for d, f in zip(self.dims, self.is_f64) if not f))
        self.out64 = torch.empty(max(c64, 1), dtype=torch.float64, device="cuda")
        self.out32 = torch.empty(max(c32, 1), dtype=torch.float32, device="cuda")
        self.reqs = []
        p64 = p32 = 0
        for i in range(count):
            M, N, K = (int(v) for v in self.dims[i])
            # column offsets in whole 32-byte units: each request's operands
            # start aligned, as separate allocations would
            ra, ca = offs[i, 0] % (4097 - M), (offs[i, 1] % (4097 - K)) // 4 * 4
            rb, cb = offs[i, 2] % (4097 - K), (offs[i, 3] % (4097 - N)) // 4 * 4
            if self.is_f64[i]:
                A, B = self.d64[0][ra:ra + M, ca:ca + K], self.d64[1][rb:rb + K, cb:cb + N]
                C = self.out64[p64:p64 + M * N].view(M, N)
                p64 += M * N
                method = mm.MM_F64
            else:
                A, B = self.d32[0][ra:ra + M, ca:ca + K], self.d32[1][rb:rb + K, cb:cb + N]
                C = self.out32[p32:p32 + M * N].view(M, N)
                p32 += M * N
                method = mm.MM_SPLIT_BF16_6
            prob = mm.Problem(M, N, K, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), C.data_ptr(), N)
            self.reqs.append((prob, method, (ra, ca, rb, cb), C, A, B))
        torch.cuda.synchronize()

    LARGE_MN = 1024 * 1024

    def tune(self, mm, sample=48):
        """Grouped autotuner on a sample batch of each (method, size class) of the
        requests; returns (variants, variants_large)."""
        out = ([-1, -1, -1, -1], [-1, -1, -1, -1])
        for method in (mm.MM_F64, mm.MM_SPLIT_BF16_6):
            for large in (False, True):
                idx = [i for i in range(self.count) if self.reqs[i][1] == method and
                       (self.reqs[i][0].M * self.reqs[i][0].N >= self.LARGE_MN) == large][:sample]
                As = [self.reqs[i][4] for i in idx]
                Bs = [self.reqs[i][5] for i in idx]
                Cs = [self.reqs[i][3] for i in idx]
                v, sch, ms = mm.grouped_autotune(method, As, Bs, Cs, warmup=1, reps=3)
                if v >= mm.PAIR_BASE:
                    # the server runs one tile variant per (method, size class):
                    # of a size-class pair the tuner chose, the faster member
                    members = mm.grouped_pair_info(method, v - mm.PAIR_BASE)[:2]
                    v = min(members, key=lambda m: self._grouped_ms(mm, method, m, As, Bs, Cs))
                out[int(large)][method] = v
        return out

    @staticmethod
    def _grouped_ms(mm, method, variant, As, Bs, Cs, reps=5):
        import torch
        plan = mm.GroupedPlan(method, variant=variant, schedule=3)
        try:
            plan.run(As, Bs, Cs)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                plan.replay()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / reps
        finally:
            torch.cuda.synchronize()
            plan.close()


def serving_section(torch, mm, wl=None, slots=8, max_batch=64, budget=64 << 30, variants=None, check=16,
                    rate=None, probe=True):
    """One serving run of the workload's request stream.  `rate` replays the
    same requests with their arrival times scaled to that rate (default: the
    workload's own).  `check` requests are checked against the oracle: a
    seeded sample of the smaller ones entry by entry, plus the largest
    binary64 and the largest split request of the large class (M*N >= 1024^2)
    on seeded rows, all columns."""
    import oracle
    if wl is None:
        wl = ServingWorkload(torch, mm)
    if variants is None:
        variants = wl.tune(mm)
    small_v, large_v = variants
    count = wl.count
    rate = float(rate or wl.rate)
    t_arr = wl.t_arr * (wl.rate / rate)
    kw = dict(budget_bytes=budget, slots=slots, max_batch=max_batch, variants=small_v, variants_large=large_v,
              large_mn=wl.LARGE_MN)
    srv = mm.Server(**kw)
    try:
        # warm the kernels once outside the measured stream of requests
        for prob, method, *_ in wl.reqs[:8]:
            srv.wait(srv.submit_raw(prob, method))
        srv.close()
        srv = mm.Server(**kw)
        start = srv.clock() + 0.05
        ids = []
        for i, (prob, method, *_) in enumerate(wl.reqs):
            due = start + float(t_arr[i])
            while srv.clock() < due:
                pass
            ids.append(srv.submit_raw(prob, method, due))
        bad = 0
        for rid in ids:
            st, _ = srv.wait(rid)
            bad += st != 0
        stats = srv.stats()
    finally:
        srv.close()
    torch.cuda.synchronize()
    # oracle check: a sample of the smaller requests (every entry) and the
    # largest request of each method in the large class (seeded rows)
    flops = np.array([float(d[0]) * d[1] * d[2] for d in wl.dims])
    small = [i for i in range(count) if flops[i] <= 1e8]
    sample = list(np.random.default_rng(3).choice(small, size=min(check, len(small)), replace=False)) if check else []
    large_checked = []
    if check:
        for is64 in (True, False):
            idx = [i for i in range(count) if bool(wl.is_f64[i]) == is64 and
                   int(wl.dims[i][0]) * int(wl.dims[i][1]) >= wl.LARGE_MN]
            if idx:
                large_checked.append(int(max(idx, key=lambda i: flops[i])))
    worst = 0.0
    checked = []
    for i in [*sample, *large_checked]:
        prob, method, (ra, ca, rb, cb), C = wl.reqs[i][:4]
        M, N, K = prob.M, prob.N, prob.K
        bank = wl.bank64 if method == mm.MM_F64 else wl.bank32
        rows = np.arange(M) if i in sample else np.unique(np.random.default_rng(int(i)).integers(0, M, 6))
        A = bank[0][ra:ra + M, ca:ca + K][rows]
        B = bank[1][rb:rb + K, cb:cb + N]
        got = C.cpu().numpy().astype(np.float64)[rows]
        if method == mm.MM_F64:
            R = oracle.gemm(A, B)
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F64)
        else:
            R = oracle.split_product(A, B, 6)
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(R)
        ratio = float((np.abs(got - R) / np.maximum(bound, 1e-300)).max())
        worst = max(worst, ratio)
        checked.append({"request": int(i), "method": "f64" if method == mm.MM_F64 else "split6", "M": M, "N": N,
                        "K": K, "rows": "all" if i in sample else [int(r) for r in rows],
                        "max_err_over_bound": ratio})
    # binary64 residual probe (Freivalds) of every served result, on the GPU
    freivalds = None
    if probe:
        res2 = torch.empty((count, 2), dtype=torch.float64, device="cuda")
        x_all = torch.from_numpy(I.probe_vector(4096)).cuda()
        rws = torch.empty(mm.lib().mm_residual_workspace_bytes(4096, 4096, 4096), dtype=torch.uint8, device="cuda")
        for i, (prob, method, _, C, A, B) in enumerate(wl.reqs):
            mm.residual_f64(A, B, C, x_all[:prob.N], out=res2[i], workspace=rws)
        r2z2 = res2.cpu().numpy()
        rel = np.sqrt(r2z2[:, 0] / np.maximum(r2z2[:, 1], 1e-300))
        f64_mask = np.array([m == mm.MM_F64 for _, m, *_ in wl.reqs])
        freivalds = {k: {"requests": int(msk.sum()), "median": float(np.median(rel[msk])), "max": float(rel[msk].max())}
                     for k, msk in (("f64", f64_mask), ("split6", ~f64_mask)) if msk.any()}
        del res2, rws
    flop = float(sum(2.0 * d[0] * d[1] * d[2] for d in wl.dims))
    span = float(t_arr[-1])
    mix_roof_s = sum(2.0 * d[0] * d[1] * d[2] / (PEAK["f64"] * 1e12) if f else
                     6 * 2.0 * d[0] * d[1] * d[2] / (PEAK["bf16"] * 1e12) for d, f in zip(wl.dims, wl.is_f64))
    res = {"requests": count, "rate_per_s": rate, "budget_bytes": budget, "slots": slots,
           "max_batch": max_batch, "large_mn": wl.LARGE_MN,
           "variants": {"f64": [small_v[0], large_v[0]], "split6": [small_v[3], large_v[3]]}, "failed": int(bad),
           "p50_ms": stats["p50_ms"], "p99_ms": stats["p99_ms"], "mean_ms": stats["mean_ms"],
           "max_ms": stats["max_ms"], "tflops": stats["tflops"], "useful_flop": flop,
           "offered_load_rho": mix_roof_s / span, "peak_bytes_in_flight": stats["peak_bytes"],
           "launches": stats["launches"], "mean_batch": stats["mean_batch"],
           "oracle_checked": len(checked), "oracle_max_err_over_bound": worst, "oracle_checks": checked,
           "freivalds_rel_residual_all": freivalds,
           "served_load_rho": stats["tflops"] * 1e12 * mix_roof_s / flop if flop else None}
    log(f"  serving {rate:.0f}/s budget {budget / 2**30:.2f} GiB slots={slots} batch={max_batch} v={variants}: "
        f"p50 {res['p50_ms']:.3f} ms p99 {res['p99_ms']:.3f} ms {res['tflops']:.1f} TFLOP/s, "
        f"rho {res['offered_load_rho']:.2f}, peak {res['peak_bytes_in_flight'] / 2**30:.2f} GiB, "
        f"{res['launches']} launches")
    return res


def serving_load_section(torch, mm, wl, variants):
    """The same 10,000 requests at higher arrival rates (offered load rho up to
    ~0.8 of the peak-rate mix roofline) and at the default rate under a budget
    small enough that admission binds: p50/p99, throughput and peak bytes."""
    points = []
    for rate, budget in ((40000.0, 64 << 30), (60000.0, 64 << 30), (20000.0, 1 << 30)):
        r = serving_section(torch, mm, wl=wl, variants=variants, budget=budget, check=0, rate=rate, probe=False)
        points.append({k: r[k] for k in ("rate_per_s", "budget_bytes", "offered_load_rho", "served_load_rho", "p50_ms", "p99_ms",
                                         "mean_ms", "max_ms", "tflops", "peak_bytes_in_flight", "launches",
                                         "mean_batch", "failed")})
    return points


def strassen_section(torch, mm, n=8192, reps=5):
    """binary64 at n by one Strassen-Winograd level: time, throughput counted
    as the definition's 2n^3, and the normwise error of sampled rows against
    the oracle's product."""
    import oracle
    A, B = I.pair("uniform_f64", n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(mm.lib().mm_strassen_workspace_bytes(n, n, n), dtype=torch.uint8, device="cuda")
    wall, ev, med, mn = timed_steps(torch, lambda: mm.gemm_strassen_f64(dA, dB, C=C, workspace=ws), reps, 2)
    Ch = C[:8].cpu().numpy()
    R = oracle.gemm(A[:8], B)
    out = {"ms": ev, "tflops_equiv": 2.0 * n ** 3 / (ev * 1e-3) / 1e12,
           "normwise_err_vs_oracle_rows0_7": float(np.linalg.norm(Ch - R) / np.linalg.norm(R))}
    log(f"  strassen: {ev:.3f} ms {out['tflops_equiv']:.2f} TFLOP/s-equivalent err {out['normwise_err_vs_oracle_rows0_7']:.2e}")
    del dA, dB, C, ws
    torch.cuda.empty_cache()
    return out


def peak_section(torch, achieved_f64=None):
    """MFMA-only throughput per dtype (libmm_peak.so, include/mm_peak.h): the
    ceiling the products' fractions of the datasheet peaks are read against.
    The best of 8, 16 or 32 independent accumulator chains per wave and 2, 4,
    8 or 16 four-wave workgroups per CU, each launch ~5-20 ms."""
    import ctypes
    from paper_2408_15384_amd import build as B
    lib = ctypes.CDLL(B.PEAK_LIB)
    fn = lib.mm_peak_mfma
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out_buf = torch.empty(16 * cus * 256, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = {}
    # total MFMAs per launch held fixed per dtype: per_cu * cus * 4 waves * iters * chains
    for name, code, flop, mfmas_per_wave in (("f64", 0, 2048, 48000 * 8 // 2), ("f32", 1, 2048, 96000 * 8 // 2),
                                             ("bf16", 2, 16384, 192000 * 8 // 2)):
        best = None
        for chains in (8, 16, 32):
            for per_cu in (2, 4, 8, 16):
                blocks = per_cu * cus
                iters = max(1, mfmas_per_wave // (per_cu * chains))
                if fn(code, chains, blocks, max(1, iters // 10), out_buf.data_ptr(), stream) != 0:
                    raise RuntimeError("mm_peak_mfma failed")
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                if fn(code, chains, blocks, iters, out_buf.data_ptr(), stream) != 0:
                    raise RuntimeError("mm_peak_mfma failed")
                e1.record()
                e1.synchronize()
                t = e0.elapsed_time(e1) * 1e-3
                tf = blocks * 4 * iters * chains * flop / t / 1e12
                if best is None or tf > best["tflops"]:
                    best = {"tflops": tf, "chains": chains, "workgroups_per_cu": per_cu}
        best["frac_of_datasheet"] = best["tflops"] / PEAK[name]
        res[name] = best
        log(f"  MFMA-only {name}: {best['tflops']:.1f} TFLOP/s ({best['frac_of_datasheet']:.1%} of {PEAK[name]}), "
            f"{best['chains']} chains, {best['workgroups_per_cu']} workgroups/CU")
    if achieved_f64:
        res["headline_frac_of_f64_ceiling"] = achieved_f64 / res["f64"]["tflops"]
    # Matrix waves and vector waves on the same SIMDs: does the SIMD overlap
    # them (both ~ the longer alone) or issue them in turn (both ~ the sum)?
    ov = lib.mm_peak_overlap
    ov.restype = ctypes.c_int32
    ov.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    blocks, iters = 2 * cus, 2000
    ovl = {}
    for role, key in ((1, "mfma_only_ms"), (2, "valu_only_ms"), (0, "both_ms")):
        if ov(role, blocks, 10, out_buf.data_ptr(), stream) != 0:
            raise RuntimeError("mm_peak_overlap failed")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            if ov(role, blocks, iters, out_buf.data_ptr(), stream) != 0:
                raise RuntimeError("mm_peak_overlap failed")
        e1.record()
        e1.synchronize()
        ovl[key] = e0.elapsed_time(e1) / 3
    ovl["both_over_sum"] = ovl["both_ms"] / (ovl["mfma_only_ms"] + ovl["valu_only_ms"])
    res["mfma_valu_overlap"] = ovl
    log(f"  matrix + vector waves on one SIMD: {ovl['both_ms']:.3f} ms against {ovl['mfma_only_ms']:.3f} + "
        f"{ovl['valu_only_ms']:.3f} ms alone")
    return res


def shard_section(torch, mm, n=8192, parts=8, reps=15):
    """One GPU's share of a row-sharded binary64 product at n: A's and C's rows
    [0, n/parts) times all of B.  Rows of C do not depend on how the rows are
    split, so the share must equal the same rows of the whole product bit for
    bit when both run the same tile variant."""
    m = n // parts
    A, B = I.pair("uniform_f64", n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    Cs = torch.empty((m, n), dtype=torch.float64, device="cuda")
    v = mm.select_variant("f64", m, n, n)
    wall, ev, med, mn = timed_steps(torch, lambda: mm.gemm_variant("f64", v, dA[:m], dB, Cs), reps, 3)
    Cf = torch.empty((n, n), dtype=torch.float64, device="cuda")
    mm.gemm_variant("f64", v, dA, dB, Cf)
    torch.cuda.synchronize()
    same = bool(torch.equal(Cs, Cf[:m]))
    out = {"M": m, "N": n, "K": n, "of_parts": parts, "tile_variant": v, "ms": ev, "ms_median": med,
           "tflops": 2.0 * m * n * n / (ev * 1e-3) / 1e12, "rows_equal_whole_product": same,
           "note": "compute of one GPU's share only; the all-gather of B is not part of this figure"}
    log(f"  shard {m}x{n}x{n}: {ev:.3f} ms {out['tflops']:.2f} TFLOP/s, rows equal: {same}")
    del dA, dB, Cs, Cf
    torch.cuda.empty_cache()
    return out


def layouts_section(torch, mm, n=8192, reps=5):
    """binary64 C = op(A).op(B) at n for every operand orientation: the cost of
    transposed storage (transpose into workspace + the row-major kernel)."""
    A, B = I.pair("uniform_f64", n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(mm.lib().mm_gemm_ex_workspace_bytes(0, 1, 1, n, n, n), dtype=torch.uint8, device="cuda")
    out = {}
    for ops in ("NN", "NT", "TN", "TT"):
        wall, ev, med, mn = timed_steps(torch, lambda: mm.gemm_ex("f64", dA, dB, ops[0], ops[1], C=C, workspace=ws),
                                        reps, 2)
        out[ops] = {"ms": ev, "tflops": 2.0 * n ** 3 / (ev * 1e-3) / 1e12}
        log(f"  layout {ops}: {ev:.3f} ms {out[ops]['tflops']:.2f} TFLOP/s")
    del dA, dB, C, ws
    torch.cuda.empty_cache()
    return out


# The paper's serial timings at -O3 (Tables I and II) and its 16-thread
# timings (section VI text), seconds, Cirrus Xeon E5-2695 2.1 GHz: context only.
PAPER_SERIAL_O3 = {"gcc": {32: 0.00003, 64: 0.00026, 128: 0.00228, 256: 0.02028, 512: 0.17037, 1024: 1.69891},
                   "intel": {32: 0.00003, 64: 0.00027, 128: 0.00215, 256: 0.02081, 512: 0.18232, 1024: 1.55254}}
PAPER_16_THREADS = {"gcc": {32: 2.8e-5, 1024: 0.88}, "intel": {32: 1.57e-5, 1024: 0.12}}


def paper_section(torch, mm, sizes=(32, 64, 128, 256, 512, 1024), reps=15):
    """The paper's experiment on this machine: Box-Muller N(0,1) inputs at its
    sizes, the product timed as the mean of 15 runs, on the GPU (binary64) and
    with the CPU oracle on one host core and on all of them; each GPU result
    checked against the oracle's per-entry bound."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    out = []
    n0 = oracle.get_threads()
    for n in sizes:
        A, B = I.pair("normal_f64", n, n, n, seed=0)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dC = torch.empty((n, n), dtype=torch.float64, device="cuda")
        wall, ev, med, mn = timed_steps(torch, lambda: mm.gemm_f64(dA, dB, dC), reps, 3)
        # the products alone: `reps` back-to-back launches captured in a graph
        # and replayed between two events (no per-call marshalling in between)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                mm.gemm_f64(dA, dB, dC)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        kern_s = e0.elapsed_time(e1) * 1e-3 / reps
        del g
        C = dC.cpu().numpy()
        row = {"n": n, "gpu_s": kern_s, "gpu_tflops": 2.0 * n ** 3 / kern_s / 1e12, "gpu_call_s": ev * 1e-3}
        for threads in (1, cores):
            oracle.set_threads(threads)
            r = reps if (threads > 1 or n <= 256) else max(1, 15 * 256 ** 3 // n ** 3)
            ts = []
            for _ in range(r):
                t0 = time.perf_counter()
                R = oracle.gemm(A, B)
                ts.append(time.perf_counter() - t0)
            row[f"oracle_{threads}t_s"] = float(np.mean(ts))
            row[f"oracle_{threads}t_reps"] = r
        if n == 1024:
            # the paper's thread scaling at 1024 (its section VII): the oracle
            # on 1, 2, 4, 8 and 16 host threads (one run each above 1 and 16)
            scale = {1: row["oracle_1t_s"], cores: row[f"oracle_{cores}t_s"]}
            for threads in (2, 4, 8, 16):
                if threads in scale or threads > cores:
                    continue
                oracle.set_threads(threads)
                t0 = time.perf_counter()
                oracle.gemm(A, B)
                scale[threads] = time.perf_counter() - t0
            row["oracle_thread_scaling_s"] = {str(k): v for k, v in sorted(scale.items())}
            row["paper_thread_scaling_s"] = {"gcc": {"1": 9.67, "16": 0.88}, "intel": {"1": 1.59, "16": 0.12}}
            log("  paper sizes n=1024 oracle threads " + ", ".join(f"{k}: {v:.3g} s" for k, v in sorted(scale.items())))
        bound = oracle.elementwise_bound(oracle.abs_product(A, B), n, oracle.U_F64)
        row["max_err_over_bound"] = float((np.abs(C - R) / np.maximum(bound, 1e-300)).max())
        row["paper_gcc_O3_serial_s"] = PAPER_SERIAL_O3["gcc"][n]
        row["paper_intel_O3_serial_s"] = PAPER_SERIAL_O3["intel"][n]
        if n in PAPER_16_THREADS["intel"]:
            row["paper_intel_16t_s"] = PAPER_16_THREADS["intel"][n]
            row["paper_gcc_16t_s"] = PAPER_16_THREADS["gcc"][n]
        log(f"  paper sizes n={n}: gpu {row['gpu_s']*1e6:.1f} us (per call from Python {row['gpu_call_s']*1e6:.1f} us), "
            f"oracle 1 core {row['oracle_1t_s']:.4g} s, "
            f"{cores} cores {row[f'oracle_{cores}t_s']:.4g} s, paper gcc -O3 {row['paper_gcc_O3_serial_s']} s")
        out.append(row)
    oracle.set_threads(n0)
    return {"inputs": "Box-Muller N(0,1), seed 0", "cores": cores, "reps": reps,
            "note": "gpu_s: mean of reps back-to-back products replayed from a graph; gpu_call_s: HIP events around "
                    "one call from Python (adds argument marshalling and launch); serial oracle runs above 256 use "
                    "fewer repetitions (oracle_1t_reps)", "rows": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--sections", default="peak,sizes,precision,grouped,serving,strassen,shard,layouts,paper,vendor",
                    help="comma list of sections to run after the headline (peak, sizes, precision, grouped, serving, strassen, "
                         "shard, layouts, paper, vendor; "
                         "or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the product runs on a single MI355X; sharding over several GPUs is "
              "not implemented (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2408_15384_amd import api as mm
    mm.load_library()
    mm.check(mm.lib().mm_init(0))
    n = args.n

    log(f"headline: binary64 GEMM M=N=K={n}")
    A, B = I.pair("uniform_f64", n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((n, n), dtype=torch.float64, device="cuda")
    # a plain copy of one operand: reference kernel for the HBM byte counters
    scratch = torch.empty_like(dA)
    scratch.copy_(dA)
    del scratch
    torch.cuda.synchronize()

    wall_ms, ev_ms, ev_med, ev_min = timed_steps(torch, lambda: mm.gemm_f64(dA, dB, dC), args.steps, args.warmup)
    flop = 2.0 * n ** 3
    value = flop / (wall_ms * 1e-3) / 1e12
    achieved = flop / (ev_ms * 1e-3) / 1e12
    variant = mm.select_variant("f64", n, n, n)
    traffic = read_traffic(variant) if n == 8192 else None
    C = dC.cpu().numpy()
    x = torch.from_numpy(I.probe_vector(n)).cuda()
    r2z2 = mm.residual_f64(dA, dB, dC, x).cpu().numpy()
    log(f"  {wall_ms:.3f} ms/step, kernel {ev_ms:.3f} ms -> {value:.2f} TFLOP/s ({achieved / PEAK['f64']:.1%} of peak)")

    line = {
        "metric": "GEMM TFLOP/s & % of dtype peak at N=8192; p50/p99 latency of request loop",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded uniform[-1,1) binary64, seed 0)",
        "config": {"workload": "fp64_gemm_8192", "M": n, "N": n, "K": n, "layout": "row-major NN",
                   "tile_variant": variant, "tile": list(mm.variant_info("f64", variant))},
        "pct_of_dtype_peak": value / PEAK["f64"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["f64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["f64"], "traffic": traffic,
                     "kernel_ms_mean": ev_ms, "kernel_ms_median": ev_med, "kernel_ms_min": ev_min,
                     "algorithmic_flop_per_launch": flop},
        "freivalds_rel_residual": float(np.sqrt(r2z2[0] / r2z2[1])),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a row sample)")
        line["cpu_baseline"] = cpu_baseline(A, B, C)
    del dA, dB, dC
    torch.cuda.empty_cache()
    sections = [x for x in args.sections.split(",") if x and x != "none"]
    if "peak" in sections:
        log("peak: MFMA-only throughput per dtype")
        line["mfma_peak"] = peak_section(torch, achieved)
    if "sizes" in sections:
        log("sizes: binary64 at N = 1024 and 4096")
        line["sizes"] = sizes_section(torch, mm)
    if "precision" in sections:
        log("precision: FP32 vs split-bf16 at N=8192")
        line["precision"] = precision_section(torch, mm, n, args.steps, args.warmup)
    if "grouped" in sections:
        log("grouped: 512 FP32 problems")
        line["grouped"] = grouped_section(torch, mm)
        torch.cuda.empty_cache()
    if "serving" in sections:
        log("serving: 10,000 requests")
        wl = ServingWorkload(torch, mm)
        variants = wl.tune(mm)
        line["serving"] = serving_section(torch, mm, wl=wl, variants=variants)
        line["serving"]["load_points"] = serving_load_section(torch, mm, wl, variants)
        del wl
        torch.cuda.empty_cache()
    if "strassen" in sections:
        log("strassen: one Strassen-Winograd level at N=8192")
        line["strassen"] = strassen_section(torch, mm)
    if "shard" in sections:
        log("shard: one GPU's share of a row-sharded product at N=8192")
        line["shard"] = shard_section(torch, mm)
    if "layouts" in sections:
        log("layouts: transposed operands at N=8192")
        line["layouts"] = layouts_section(torch, mm)
    if "paper" in sections:
        log("paper sizes: Box-Muller inputs, 32..1024")
        line["paper_sizes"] = paper_section(torch, mm)
    if "vendor" in sections:
        log("vendor: the same 8192 products in hipBLASLt / rocBLAS (torch.matmul), comparison only")
        from paper_2408_15384_amd.workloads import vendor_rates
        line["vendor_library"] = {"note": "torch.matmul on the same GPU, uniform inputs; context, not used by libmm",
                                  "n": n, **vendor_rates(torch, n)}
        vl = line["vendor_library"]
        prec = line.get("precision", {}).get("uniform_f32", {})
        if prec.get("fp32"):
            vl["libmm_f32_over_vendor"] = prec["fp32"]["tflops_useful"] / vl["f32"]["tflops"]
        # how hard each drives the bf16 matrix cores: the vendor's plain bf16
        # product against the split products' plane products (by time)
        vl["bf16"]["frac_of_datasheet"] = vl["bf16"]["tflops"] / PEAK["bf16"]
        for m in ("split3", "split6"):
            if prec.get(m):
                vl[f"libmm_{m}_mfma_frac_over_vendor_bf16"] = prec[m]["mfma_frac"] / vl["bf16"]["frac_of_datasheet"]
        line["vendor_library"]["libmm_f64_over_vendor"] = value / line["vendor_library"]["f64"]["tflops"]
    line["paper_context"] = {"note": "the paper's own CPU timings (Cirrus, Xeon E5-2695 2.1 GHz, 18 cores), "
                                     "context only", "serial_O3_gcc_1024_s": 1.69891,
                             "intel_16_threads_1024_s": 0.12}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
