"""Benchmark: 3D free-space vector Poisson solves/s on one MI355X.

Workload (headline): 256^3 cell-centred grid on [0,1]^3, doubled to 512^3
(Hockney-Eastwood), Gaussian-regularised kernel G2 with sigma = 2H, 3-component
source of 32 seeded compact vortex rings (seed 4), outputs psi (3 components)
and its spectral curl (3 components).  Inputs and outputs stay resident in
HBM; a step is one hp_solve (every pass of the transform, multiply, curl and
inverse).  The FP32 solve is the headline value; the FP64 solve is timed the
same way and reported beside it, with the FP32 error against it.

Prints one JSON line (rank 0).  Usage: python bench.py [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3D Poisson solves/s + HBM GB/s at 256^3 unbounded, FP32 vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="grid of the oracle sample")
    return ap.parse_args()


def timed_solves(solver, steps, warmup):
    import torch
    from paper_2301_01145_amd import hp_pass_stats, hp_set_timing
    for _ in range(warmup):
        solver.run()
    torch.cuda.synchronize()
    hp_pass_stats(solver.plan)  # drop anything recorded so far
    hp_set_timing(solver.plan, True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(solver.stream)
    for _ in range(steps):
        solver.run()
    stop.record(solver.stream)
    torch.cuda.synchronize()
    hp_set_timing(solver.plan, False)
    ms = start.elapsed_time(stop) / steps
    return ms, hp_pass_stats(solver.plan)


def cpu_baseline(n_sample, n_full):
    """Time the FP64 oracle on the same workload recipe at a smaller grid."""
    import math

    import numpy as np

    import oracle
    from workloads import vortex_rings
    f = vortex_rings(n_sample, seed=4, count=32).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    oracle.solve("unbounded", "staggered", [n_sample] * 3, [0, 0, 0], [1, 1, 1], f, diff="curl")
    t = time.perf_counter() - t0
    # work of the dense FFT pipeline ~ M log M with M the doubled grid
    Ms, Mf = (2 * n_sample) ** 3, (2 * n_full) ** 3
    frac = (Ms * math.log2(Ms)) / (Mf * math.log2(Mf))
    return {
        "value": frac / t,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"full FP64 oracle solve (psi + curl, numpy pocketfft, single thread) of the "
                   f"same 32-ring workload at {n_sample}^3 (doubled {2 * n_sample}^3) took "
                   f"{t:.2f} s; scaled to a {n_full}^3 solve by the M log M ratio {frac:.4f}"),
        "sample_seconds": t,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2301_01145_amd import Solver
    from workloads import vortex_rings

    n = args.n
    f64 = vortex_rings(n, seed=4, count=32)
    f32 = f64.astype(np.float32)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    out = {}
    results = {}
    for prec, dtype in (("f32", torch.float32), ("f64", torch.float64)):
        if prec == "f64" and args.no_fp64:
            continue
        s = Solver("unbounded", "staggered", [n, n, n], diff="curl", dtype=dtype, ncomp=3, device=dev)
        src = [torch.as_tensor(f32[c], device=dev).to(dtype).contiguous() for c in range(3)]
        psi, u = s.bind(src)
        ms, passes = timed_solves(s, args.steps, args.warmup)
        fields = [p.double() for p in psi] + [x.double() for x in u]
        results[prec] = {"ms": ms, "passes": passes, "model_bytes": s.model_bytes(), "fields": fields}
        s.close()
        del src, psi, u
    r32 = results["f32"]
    value = 1000.0 / r32["ms"]
    # dominant kernel: the pass with the largest mean time
    name, pms, pbytes = max(r32["passes"], key=lambda x: x[1])
    achieved = pbytes / (pms * 1e-3) / 1e9
    out.update({
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"unbounded 3D vector Poisson, {n}^3 cell-centred on [0,1]^3 doubled "
                                f"to {2 * n}^3, G2 kernel sigma=2H, psi + spectral curl, 32 vortex "
                                "rings seed 4"),
                   "grid": n, "components": 3, "outputs": 6},
        "model_gbs": r32["model_bytes"] / (r32["ms"] * 1e-3) / 1e9,
        "model_bytes_per_solve": r32["model_bytes"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": name,
                     "kernel_ms": pms, "kernel_bytes": pbytes},
        "passes": [{"name": a, "ms": b, "model_gbs": c / (b * 1e-3) / 1e9 if b > 0 else None}
                   for a, b, c in r32["passes"]],
    })
    if "f64" in results:
        r64 = results["f64"]
        num = sum(float(torch.sum((a - b) ** 2)) for a, b in zip(r32["fields"], r64["fields"]))
        den = sum(float(torch.sum(b ** 2)) for b in r64["fields"])
        mx = max(float(torch.max(torch.abs(a - b))) for a, b in zip(r32["fields"], r64["fields"]))
        mref = max(float(torch.max(torch.abs(b))) for b in r64["fields"])
        out["fp64"] = {"value": 1000.0 / r64["ms"], "ms_per_step": r64["ms"],
                       "model_gbs": r64["model_bytes"] / (r64["ms"] * 1e-3) / 1e9}
        out["fp32_error_vs_fp64"] = {"rel_l2": (num / den) ** 0.5, "rel_max": mx / mref}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
