"""Command-line driver in the shape of the paper's test program (section VI):
three matrix sizes on the command line, one product C = A.B, the time taken.

    python -m paper_2408_15384_amd.cli M K N [--method f64] [--inputs uniform]
                                             [--reps 15] [--warmup 3] [--seed 0]
                                             [--trans-a] [--trans-b] [--json]

The three sizes are read as A being M x K and B being K x N (the paper's
m x n and n x p).  Inputs are seeded and synthetic; ``--inputs normal`` draws
them by the Box-Muller transform as in the paper's experiments (section IV).
Timing follows the paper's protocol (section V): warm-up runs, then a fixed
number of timed repetitions, each bracketed by HIP events on the stream; the
median, minimum and mean are printed with the rate 2MNK / t.  Every run ends
with the binary64 residual probe of the result (Freivalds), computed on the
GPU by the library.

Methods: f64, f32, split3, split6 (bfloat16 split products, FP32 output) and
strassen (one Winograd level on the binary64 product).  The product always
runs in libmm's kernels; without the built library or a GPU the command
exits with an error.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs as I

KINDS = {
    ("f64", "uniform"): "uniform_f64", ("f64", "int"): "int_f64", ("f64", "normal"): "normal_f64",
    ("f32", "uniform"): "uniform_f32", ("f32", "int"): "int_f32", ("f32", "m2e"): "m2e_f32",
}
METHOD_DTYPE = {"f64": "f64", "strassen": "f64", "f32": "f32", "split3": "f32", "split6": "f32"}


def parse(argv=None) -> argparse.Namespace:
    p = argparse.ArgumentParser(prog="python -m paper_2408_15384_amd.cli",
                                description="C = A.B on the GPU for A (M x K) and B (K x N), timed.")
    p.add_argument("M", type=int)
    p.add_argument("K", type=int)
    p.add_argument("N", type=int)
    p.add_argument("--method", choices=sorted(METHOD_DTYPE), default="f64")
    p.add_argument("--inputs", choices=["uniform", "normal", "int", "m2e"], default="uniform")
    p.add_argument("--reps", type=int, default=15)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--trans-a", action="store_true", help="pass A as the transpose of a stored K x M array")
    p.add_argument("--trans-b", action="store_true", help="pass B as the transpose of a stored N x K array")
    p.add_argument("--json", action="store_true", help="print one JSON object instead of text")
    a = p.parse_args(argv)
    if min(a.M, a.K, a.N) < 0:
        p.error("sizes must be non-negative")
    if a.reps < 1 or a.warmup < 0:
        p.error("--reps >= 1 and --warmup >= 0 required")
    dt = METHOD_DTYPE[a.method]
    if a.inputs == "normal" and dt == "f32":
        pass  # Box-Muller draws rounded to FP32
    elif (dt, a.inputs) not in KINDS:
        p.error(f"--inputs {a.inputs} is not defined for {a.method}")
    if a.method == "strassen" and (a.trans_a or a.trans_b):
        p.error("strassen takes untransposed operands")
    if a.method == "strassen" and (a.M % 2 or a.N % 2 or a.K % 2):
        p.error("strassen needs even M, K and N")
    return a


def host_operands(a: argparse.Namespace):
    """Seeded A (M x K) and B (K x N) as numpy arrays of the method's dtype."""
    dt = METHOD_DTYPE[a.method]
    if a.inputs == "normal" and dt == "f32":
        A, B = I.pair("normal_f64", a.M, a.N, a.K, seed=a.seed)
        return A.astype(np.float32), B.astype(np.float32)
    return I.pair(KINDS[(dt, a.inputs)], a.M, a.N, a.K, seed=a.seed)


def run(a: argparse.Namespace) -> dict:
    import torch
    from . import api

    api.load_library()
    api.check(api.lib().mm_init(0))
    A, B = host_operands(a)
    # a transposed operand is stored transposed and passed as a transposed view
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t() if a.trans_a else torch.from_numpy(A).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t() if a.trans_b else torch.from_numpy(B).cuda()
    dtype = torch.float64 if METHOD_DTYPE[a.method] == "f64" else torch.float32
    C = torch.empty((a.M, a.N), dtype=dtype, device="cuda")
    # workspace allocated once, outside the timed runs
    if a.method == "strassen":
        ws_bytes = api.lib().mm_strassen_workspace_bytes(a.M, a.N, a.K)
    else:
        ws_bytes = api.lib().mm_gemm_ex_workspace_bytes(api.METHODS[a.method], int(a.trans_a), int(a.trans_b),
                                                        a.M, a.N, a.K)
    ws = torch.empty(max(int(ws_bytes), 1), dtype=torch.uint8, device="cuda")

    def once():
        if a.method == "strassen":
            api.gemm_strassen_f64(dA, dB, C, workspace=ws)
        else:
            api.gemm_ex(a.method, dA.t() if a.trans_a else dA, dB.t() if a.trans_b else dB,
                        "T" if a.trans_a else "N", "T" if a.trans_b else "N", C, workspace=ws)

    for _ in range(a.warmup):
        once()
    torch.cuda.synchronize()
    times = []
    for _ in range(a.reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        once()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    rel = None
    if a.M and a.N and a.K:
        x = torch.from_numpy(I.probe_vector(a.N, a.seed)).cuda()
        r = api.residual_f64(dA.contiguous() if a.trans_a else dA, dB.contiguous() if a.trans_b else dB, C, x)
        r2, z2 = (float(v) for v in r.cpu().numpy())
        rel = float(np.sqrt(r2 / z2)) if z2 > 0 else float(np.sqrt(r2))
    times.sort()
    med = times[len(times) // 2]
    flop = 2.0 * a.M * a.N * a.K
    return {"M": a.M, "K": a.K, "N": a.N, "method": a.method, "inputs": a.inputs, "seed": a.seed,
            "layout": ("T" if a.trans_a else "N") + ("T" if a.trans_b else "N"),
            "reps": a.reps, "warmup": a.warmup, "median_s": med, "min_s": times[0],
            "mean_s": sum(times) / len(times), "tflops_median": flop / med / 1e12 if med > 0 else 0.0,
            "freivalds_rel_residual": rel}


def main(argv=None) -> int:
    a = parse(argv)
    res = run(a)
    if a.json:
        print(json.dumps(res))
    else:
        print(f"C = A.B  A {a.M}x{a.K}  B {a.K}x{a.N}  method {a.method}  layout {res['layout']}  "
              f"inputs {a.inputs} (seed {a.seed})")
        print(f"time over {a.reps} runs after {a.warmup} warm-up: median {res['median_s']:.6e} s, "
              f"min {res['min_s']:.6e} s, mean {res['mean_s']:.6e} s  ({res['tflops_median']:.2f} TFLOP/s)")
        if res["freivalds_rel_residual"] is not None:
            print(f"residual probe ||C.x - A.(B.x)|| / ||A.(B.x)|| = {res['freivalds_rel_residual']:.3e}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
