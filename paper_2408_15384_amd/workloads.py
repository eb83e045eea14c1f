"""Named workloads of the library, run on their own so that a profiler's
output holds only their kernels.

    python -m paper_2408_15384_amd.workloads grouped --method split6 [--variant V --schedule S] [--reps 5]
    python -m paper_2408_15384_amd.workloads gemm --method f64 --n 8192 [--variant V] [--reps 5]
    python -m paper_2408_15384_amd.workloads vendor --n 8192 [--reps 10]
    (--sweep V:S,V:S,... or V,V,... times several configurations in one run)

grouped: the 512-problem batch (M, N, K each log-uniform on [32, 1024], seed 0,
FP32 entries uniform on [-1, 1)), one plan captured with the given tile variant
and schedule (default: the library's choice for the batch), replayed `reps`
times.  gemm: one square product of size n (binary64 or FP32 inputs by method,
uniform on [-1, 1), seed 0), launched `reps` times.  Each prints the mean
HIP-event time per launch.  vendor: the same square product in the vendor
libraries (torch.matmul, which calls hipBLASLt / rocBLAS) in binary64, FP32
and bfloat16, for comparison only: nothing in libmm calls them."""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _events(torch, fn, reps, warmup=1):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def grouped(method, variant, schedule, reps, sweep=None):
    import torch
    from paper_2408_15384_amd import api, inputs as I
    api.load_library()
    api.check(api.lib().mm_init(0))
    shapes = [tuple(int(v) for v in s) for s in I.grouped_shapes(512, 32, 1024, seed=0)]
    As, Bs, Cs = [], [], []
    for i, (M, N, K) in enumerate(shapes):
        A, B = I.pair("uniform_f32", M, N, K, seed=(0, i))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.empty((M, N), dtype=torch.float32, device="cuda"))
    configs = [(variant, schedule)] if not sweep else [tuple(int(x) for x in c.split(":")) for c in sweep.split(",")]
    for v, s in configs:
        plan = api.GroupedPlan(method, v, s)
        plan.run(As, Bs, Cs)
        ms = _events(torch, plan.replay, reps)
        info = plan.info()
        plan.close()
        print(f"grouped {method} variant {info['variant']} schedule {info['schedule']} tiles {info['tiles']}: "
              f"{ms:.4f} ms per replay", flush=True)


def gemm(method, n, variant, reps, sweep=None):
    import torch
    from paper_2408_15384_amd import api, inputs as I
    api.load_library()
    api.check(api.lib().mm_init(0))
    kind = "uniform_f64" if method == "f64" else "uniform_f32"
    A, B = I.pair(kind, n, n, n, seed=0)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B
    C = torch.empty((n, n), dtype=dA.dtype, device="cuda")
    ws = None
    if method in ("split3", "split6"):
        ws = torch.empty(api.split_workspace_bytes(n, n, n, 6), dtype=torch.uint8, device="cuda")
    variants = [int(x) for x in sweep.split(",")] if sweep else [
        variant if variant is not None else api.select_variant(method, n, n, n)]
    for v in variants:
        ms = _events(torch, lambda: api.gemm_variant(method, v, dA, dB, C, workspace=ws), reps)
        print(f"gemm {method} n={n} variant {v}: {ms:.4f} ms per launch, "
              f"{2.0 * n ** 3 / (ms * 1e-3) / 1e12:.1f} TFLOP/s", flush=True)


def vendor_rates(torch, n, reps=10):
    """TFLOP/s of torch.matmul on n x n operands (uniform on [-0.5, 0.5),
    seed 0) per dtype, HIP events over `reps` launches after 3 warm-ups."""
    g = torch.Generator(device="cuda").manual_seed(0)
    res = {}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.rand(n, n, dtype=dt, device="cuda", generator=g) - 0.5
        b = torch.rand(n, n, dtype=dt, device="cuda", generator=g) - 0.5
        c = torch.empty(n, n, dtype=dt, device="cuda")
        ms = _events(torch, lambda: torch.matmul(a, b, out=c), reps, warmup=3)
        res[name] = {"ms": ms, "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12}
        del a, b, c
    torch.cuda.empty_cache()
    return res


def vendor(n, reps):
    import torch
    for name, r in vendor_rates(torch, n, reps).items():
        print(f"vendor {name} n={n}: {r['ms']:.4f} ms per launch, {r['tflops']:.1f} TFLOP/s", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["grouped", "gemm", "vendor"])
    ap.add_argument("--method", default="f64", choices=["f64", "f32", "split3", "split6"])
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--schedule", type=int, default=None)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sweep", default=None,
                    help="grouped: comma list of variant:schedule pairs; gemm: comma list of variants")
    a = ap.parse_args(argv)
    if a.workload == "grouped":
        if a.method == "f64":
            ap.error("the grouped batch has FP32 inputs: --method f32, split3 or split6")
        grouped(a.method, a.variant, a.schedule, a.reps, a.sweep)
    elif a.workload == "vendor":
        vendor(a.n, a.reps)
    else:
        gemm(a.method, a.n, a.variant, a.reps, a.sweep)


if __name__ == "__main__":
    main()
