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
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3D Poisson solves/s + HBM GB/s at 256^3 unbounded, FP32 vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


# Sources of the free-space / periodic wavefront kernels (the headline's
# passes): their code, the wavefront FFT and the radix DFTs, plus the pass
# descriptor struct (PassArgs in hp_internal.hpp).  Changes elsewhere in the
# library do not change these kernels.
HEADLINE_SOURCES = ("hp_fast.hip", "hp_wavefft.hpp", "hp_device.hpp")


def _pass_args_text():
    with open(os.path.join(ROOT, "paper_2301_01145_amd", "csrc", "hp_internal.hpp"), "rb") as fh:
        t = fh.read()
    a = t.index(b"struct PassArgs {")
    return t[a:t.index(b"};", a) + 2]


def kernel_source_digest(files=HEADLINE_SOURCES):
    """sha256 over the named library sources (name + bytes, in the order
    given) and the PassArgs struct: counters recorded for one digest do not
    describe kernels built from another."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2301_01145_amd", "csrc")
    for f in files:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    h.update(_pass_args_text())
    return h.hexdigest()


# FP32 vector peak without packed math (the library is built with packed FP32
# disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def sandwich_flops(n):
    """Algorithmic flops of one launch of the x pass of the n^3 curl solve:
    (M/2 + 1) M pencils of length M = 2n, each with 3 forward and 5 backward
    complex FFTs at 5 M log2 M flops, the real Green's multiply of 3 spectra
    (2 flops per element) and the two x derivatives (2 flops per element)."""
    M = 2 * n
    fft = 5.0 * M * math.log2(M)
    per_pencil = 8 * fft + 3 * 2 * M + 2 * 2 * M
    return (M // 2 + 1) * M * per_pencil


def _profile_lines(path):
    """(source digest, {key: [values]}) of the machine-readable lines of a
    committed profile summary: `source_sha256: <hex>` and `<key>: <pass> <v>...`."""
    digest, rows = None, {}
    if not os.path.exists(path):
        return None, rows
    with open(path) as fh:
        for line in fh:
            t = line.strip().strip("`").split()
            if len(t) == 2 and t[0] == "source_sha256:":
                digest = t[1]
            elif len(t) >= 3 and t[0] in ("traffic_bytes:", "kernel_avg_us:"):
                rows.setdefault(t[0][:-1], {})[t[1]] = [float(v) for v in t[2:]]
    return digest, rows


def measured_traffic(pass_name, n):
    """HBM bytes per launch of `pass_name` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (already scaled by the copy-kernel
    factors), or None when there is none for these sources."""
    digest, rows = _profile_lines(os.path.join(PROFILES, f"unbounded{n}_curl_fp32_hbm_counters.md"))
    if digest != kernel_source_digest():
        return None
    v = rows.get("traffic_bytes", {}).get(pass_name)
    return None if v is None else v[0] + v[1]


def profiled_kernel_us(pass_name, n):
    """Average duration (us) of `pass_name`'s kernel in the committed
    rocprofv3 --kernel-trace --stats summary of this benchmark, or None when
    there is none for these sources."""
    digest, rows = _profile_lines(os.path.join(PROFILES, f"unbounded{n}_curl_fp32_kernel_trace.md"))
    if digest != kernel_source_digest():
        return None
    v = rows.get("kernel_avg_us", {}).get(pass_name)
    return None if v is None else v[0]


def six_field_model_bytes(n, es=4):
    """The pruned five-pass byte model with six stored spectral fields between
    the x pass and the backward y pass and the Green's octant in FP64: per
    component, A = (n+1) n n complex half-spectrum rows (P1 out), B = (n+1)
    2n n complex (P2 out); P1 3 (n^3 + A), P2 3 (A + B), P3 (3 + 6) B + octant,
    P4 6 (B + A), P5 6 (A + n^3)."""
    K = n + 1
    real = n ** 3 * es
    A = K * n * n * 2 * es
    B = K * 2 * n * n * 2 * es
    octant = K ** 3 * 8
    return 3 * (real + A) + 3 * (A + B) + 9 * B + octant + 6 * (B + A) + 6 * (A + real)


def _profile_view(name, n, pbytes):
    us = profiled_kernel_us(name, n)
    if us is None:
        return None
    gbs = pbytes / (us * 1e-6) / 1e9
    return {"kernel_avg_us": us, "achieved": gbs, "frac": gbs / HBM_PEAK_GBS,
            "source": f"profiles/unbounded{n}_curl_fp32_kernel_trace.md"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=256,
                    help="grid of the oracle sample (default: the benchmark's own 256^3)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-problem batched Neumann workload (prints its JSON object)")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the secondary workloads (2D periodic, 3D Dirichlet, batched Neumann, "
                         "differentiable 128^3)")
    return ap.parse_args()


def _time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def _time_graph(run, stream, steps, warmup):
    """Mean ms of `steps` replays of one solve captured into a hipGraph on
    `stream` (the plan's own stream, which must not be the default stream)."""
    import torch
    with torch.cuda.stream(stream):
        run()  # settles uploads of bound pointers before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        run()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        for _ in range(steps):
            g.replay()
        b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def neumann_batch64(steps, warmup):
    """64 batched Neumann problems (sizes from {32, 48, 64, 96, 128} per axis,
    seed 5), FP32: the default form and the autotuned one, replayed from a
    captured hipGraph (the plan lives on a side stream so that it can be
    captured)."""
    import numpy as np
    import torch

    from paper_2301_01145_amd.batched import BatchedSolver
    from workloads import neumann_batch
    probs = neumann_batch(64, seed=5)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bs = BatchedSolver("neumann", "staggered", [{"nc": list(p["shape"])} for p in probs], kernel="ps")
        psis32 = bs.bind([torch.as_tensor(p["f"].astype(np.float32), device="cuda") for p in probs])
    torch.cuda.synchronize()
    mode_default = bs.kernel_mode()
    ms_default = _time(bs.run, steps, warmup, bs.stream)
    ms_default_graph = _time_graph(bs.run, side, steps, warmup)
    # plan-time autotuning (kernel form, radix orders, tiles, work-item size),
    # outside the timed region
    with torch.cuda.stream(side):
        ntuned, tiles = bs.autotune(reps=5)
    ms_eager = _time(bs.run, steps, warmup, bs.stream)
    ms = _time_graph(bs.run, side, steps, warmup)
    forms = {0: "one persistent launch, general passes",
             1: "one persistent launch, wavefront tile bodies",
             2: "one launch per pass level, transform length and pass kind, wavefront tile bodies"}
    out = {"batches_per_s": 1000 / ms, "problems_per_s": 64000 / ms, "ms": ms,
           "timing": "hipGraph replays of the tuned batch",
           "kernel_form": forms[bs.kernel_mode()], "ms_eager": ms_eager,
           "default_form": forms[mode_default], "ms_default_graph": ms_default_graph,
           "ms_default_eager": ms_default,
           "tuned_pass_signatures": ntuned, "tiles_per_item": tiles,
           "model_bytes": bs.model_bytes(),
           "model_gbs": bs.model_bytes() / (ms * 1e-3) / 1e9,
           "error_flag": bs.error_flag()}
    with torch.cuda.stream(side):
        bs.run()
    torch.cuda.synchronize()
    got32 = [t.double() for t in psis32]
    bs.close()
    out["vs_fp64"] = _batch_vs_fp64(probs, got32, steps, warmup)
    return out


def _batch_vs_fp64(probs, got32, steps, warmup):
    """The same 64 problems as a batched FP64 plan and as 64 plain FP64 single
    plans on the same GPU: their times, and the error of the FP32 batch (and
    of the FP64 batch) against the plain FP64 solves."""
    import numpy as np
    import torch

    from paper_2301_01145_amd import Solver
    from paper_2301_01145_amd.batched import BatchedSolver
    side = torch.cuda.Stream()
    fs = [torch.as_tensor(p["f"].astype(np.float32).astype(np.float64), device="cuda") for p in probs]
    with torch.cuda.stream(side):
        b64 = BatchedSolver("neumann", "staggered", [{"nc": list(p["shape"])} for p in probs], kernel="ps",
                            dtype=torch.float64)
        psis64 = b64.bind(fs)
        b64.autotune(reps=3)  # FP64 batches run the general passes: tiles per item, radix orders
    torch.cuda.synchronize()
    ms_b64 = _time_graph(b64.run, side, steps, warmup)
    with torch.cuda.stream(side):
        b64.run()
    singles, outs = [], []
    with torch.cuda.stream(side):
        for i, p in enumerate(probs):
            s = Solver("neumann", "staggered", list(p["shape"]), kernel="ps", dtype=torch.float64)
            psi, _ = s.bind(fs[i])
            singles.append(s)
            outs.append(psi[0])

    def run_singles():
        for s in singles:
            s.run()
    torch.cuda.synchronize()
    ms_single = _time_graph(run_singles, side, steps, warmup)
    with torch.cuda.stream(side):
        run_singles()
    torch.cuda.synchronize()
    num32 = den = num64 = 0.0
    worst32 = 0.0
    for i in range(len(probs)):
        ref = outs[i]
        d32 = float(torch.sum((got32[i] - ref) ** 2))
        d64 = float(torch.sum((psis64[i] - ref) ** 2))
        r2 = float(torch.sum(ref ** 2))
        num32, num64, den = num32 + d32, num64 + d64, den + r2
        worst32 = max(worst32, (d32 / r2) ** 0.5 if r2 > 0 else 0.0)
    res = {"fp64_batched_ms": ms_b64, "fp64_single_plans_ms": ms_single,
           "timing": "hipGraph replays (FP64 batch: one tuned plan; single plans: 64 plans in one graph)",
           "fp32_batch_rel_l2_vs_fp64": (num32 / den) ** 0.5,
           "fp32_batch_worst_problem_rel_l2": worst32,
           "fp64_batch_rel_l2_vs_fp64_singles": (num64 / den) ** 0.5,
           "fp64_batch_error_flag": b64.error_flag()}
    for s in singles:
        s.close()
    b64.close()
    return res


def other_workloads(steps, warmup):
    """Secondary workloads: solves/s and model GB/s each (same timing method)."""
    import numpy as np
    import torch

    from paper_2301_01145_amd import Solver
    from paper_2301_01145_amd.autograd import poisson_solve
    from paper_2301_01145_amd.batched import BatchedSolver
    from workloads import dirichlet_3d, neumann_batch, periodic_modes_2d, vortex_rings
    res = {}
    # 2D periodic 64^2 FP64 PS
    # (one launch: its half spectrum fits one workgroup), eager and replayed from a captured graph
    f, _ = periodic_modes_2d(64, seed=1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver("periodic", "staggered", [64, 64], kernel="ps", dtype=torch.float64)
        s.bind(torch.as_tensor(f, device="cuda"))
    torch.cuda.synchronize()
    ms = _time(s.run, steps, warmup, s.stream)
    ms_graph = _time_graph(s.run, side, steps, warmup)
    # back-to-back launches on the stream are the faster form of this one-kernel
    # solve (a graph replay costs more host time than one kernel launch here)
    res["periodic2d_64_fp64"] = {"solves_per_s": 1000 / min(ms, ms_graph),
                                 "timing": "eager" if ms <= ms_graph else "graph",
                                 "ms_graph": ms_graph, "ms_eager": ms,
                                 "launches": int(s.passes()), "model_gbs": s.model_bytes() / (ms * 1e-3) / 1e9}
    s.close()
    # 3D Dirichlet 128^3 regular FD2 inhomogeneous FP32
    f, faces = dirichlet_3d(128)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver("dirichlet", "regular", [128] * 3, kernel="fd2", dtype=torch.float32, inhomogeneous=True)
        fd = {k: torch.as_tensor(v.astype(np.float32), device="cuda") for k, v in faces.items()}
        s.bind(torch.as_tensor(f.astype(np.float32), device="cuda"), fd)
    torch.cuda.synchronize()
    ms = _time(s.run, steps, warmup, s.stream)
    ms_graph = _time_graph(s.run, side, steps, warmup)
    res["dirichlet3d_128_fd2_fp32"] = {"solves_per_s": 1000 / ms, "ms": ms, "ms_graph": ms_graph,
                                       "launches": int(s.passes()),
                                       "model_gbs": s.model_bytes() / (ms * 1e-3) / 1e9}
    s.close()
    # the same source, homogeneous PS, psi and its gradient (sine -> cosine series)
    with torch.cuda.stream(side):
        s = Solver("dirichlet", "regular", [128] * 3, kernel="ps", diff="grad", dtype=torch.float32)
        s.bind(torch.as_tensor(f.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    ms = _time(s.run, steps, warmup, s.stream)
    ms_graph = _time_graph(s.run, side, steps, warmup)
    res["dirichlet3d_128_ps_grad_fp32"] = {"solves_per_s": 1000 / ms, "ms": ms, "ms_graph": ms_graph,
                                           "launches": int(s.passes()),
                                           "model_gbs": s.model_bytes() / (ms * 1e-3) / 1e9}
    s.close()
    # a condition per axis, and one free axis (FD2, FP32, seeded normal sources;
    # boundary values on the Dirichlet / Neumann faces), and a prime length
    rng = np.random.default_rng(12)
    for key, bcs, nc, inhom, diff in (("mixed3d_128_pdn_fd2_fp32", ["periodic", "dirichlet", "neumann"],
                                       [128, 128, 128], True, "none"),
                                      ("semi3d_128_free_pp_fd2_fp32", ["unbounded", "periodic", "periodic"],
                                       [128, 128, 128], False, "none"),
                                      # psi and its gradient: the free axis's derivative by the
                                      # odd kernel's rows, the periodic ones by the Hartley series
                                      ("semi3d_128_free_pp_fd2_grad_fp32", ["unbounded", "periodic", "periodic"],
                                       [128, 128, 128], False, "grad"),
                                      ("periodic3d_127_fp32", "periodic", [127, 127, 127], False, "none")):
        s = Solver(bcs, "staggered", nc, kernel="fd2", diff=diff, dtype=torch.float32, inhomogeneous=inhom)
        src = torch.as_tensor(rng.normal(size=s.in_shape).astype(np.float32), device="cuda")
        fd = None
        if inhom:
            fd = {}
            for a in range(3):
                if bcs[a] in ("dirichlet", "neumann"):
                    shp = tuple(s.out_shape[b] for b in range(3) if b != a)
                    for side in (0, 1):
                        fd[(a, side)] = torch.as_tensor(rng.normal(size=shp).astype(np.float32), device="cuda")
        s.bind(src, fd)
        ms = _time(s.run, steps, warmup, s.stream)
        res[key] = {"solves_per_s": 1000 / ms, "ms": ms, "launches": int(s.passes()),
                    "model_gbs": s.model_bytes() / (ms * 1e-3) / 1e9}
        s.close()
    res["neumann_batch64_fp32"] = neumann_batch64(steps, warmup)
    # free-space kernels (Section 2.5.2): plan time (Green's function on the doubled
    # grid, FP64 transform, octant) and solve time of the 256^3 curl plan, and the
    # FP64 error against the exact potential of a Gaussian blob at 64^3 and 128^3
    from scipy.special import erf
    kern = {}
    f_rings = [torch.as_tensor(vortex_rings(256, seed=4, count=32)[c].astype(np.float32), device="cuda")
               for c in range(3)]
    for kname in ("g2", "g4", "g6", "g8", "g10", "spectral"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Solver("unbounded", "staggered", [256] * 3, kernel=kname, diff="curl", dtype=torch.float32,
                   ncomp=3)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        s.bind(f_rings)
        solve_ms = _time(s.run, max(5, steps // 4), warmup, s.stream)
        s.close()
        errs = []
        for n in (64, 128):
            h = 1.0 / n
            x = (np.arange(n) + 0.5) * h
            c, A, sb = (0.5, 0.47, 0.52), 1.0, 0.06
            r = np.sqrt((x[:, None, None] - c[0]) ** 2 + (x[None, :, None] - c[1]) ** 2
                        + (x[None, None, :] - c[2]) ** 2)
            fb = A * np.exp(-r * r / (2 * sb * sb))
            exact = -A * (2 * np.pi * sb * sb) ** 1.5 * erf(r / (np.sqrt(2) * sb)) / (4 * np.pi * r)
            sb_ = Solver("unbounded", "staggered", [n] * 3, kernel=kname, dtype=torch.float64)
            psi, _ = sb_.solve(torch.as_tensor(fb, device="cuda"))
            torch.cuda.synchronize()
            errs.append(float(np.max(np.abs(psi[0].cpu().numpy() - exact)) / np.max(np.abs(exact))))
            sb_.close()
        kern[kname] = {"plan_ms": plan_ms, "solve_ms": solve_ms, "blob_rel_max_err_64": errs[0],
                       "blob_rel_max_err_128": errs[1], "observed_order": float(np.log2(errs[0] / errs[1]))}
    res["unbounded256_kernels"] = kern
    # 2D free space: FP64 error against the exact potential of a Gaussian blob at
    # 128^2 and 256^2 per kernel, and the FP32 solve time with the gradient at 2048^2
    from scipy.special import exp1
    k2d = {}
    for kname in ("g2", "g4", "g6", "g8", "g10", "spectral"):
        errs = []
        for n in (128, 256):
            h = 1.0 / n
            x = (np.arange(n) + 0.5) * h
            c, A, sb = (0.5, 0.47), 1.0, 0.06
            r = np.sqrt((x[:, None] - c[0]) ** 2 + (x[None, :] - c[1]) ** 2)
            fb = A * np.exp(-r * r / (2 * sb * sb))
            exact = A * sb * sb * (np.log(r) + 0.5 * exp1(0.5 * (r / sb) ** 2))
            s2 = Solver("unbounded", "staggered", [n, n], kernel=kname, dtype=torch.float64)
            psi, _ = s2.solve(torch.as_tensor(fb, device="cuda"))
            torch.cuda.synchronize()
            errs.append(float(np.max(np.abs(psi[0].cpu().numpy() - exact)) / np.max(np.abs(exact))))
            s2.close()
        k2d[kname] = {"blob_rel_max_err_128": errs[0], "blob_rel_max_err_256": errs[1],
                      "observed_order": float(np.log2(errs[0] / errs[1]))}
    s2 = Solver("unbounded", "staggered", [2048, 2048], kernel="g2", diff="grad", dtype=torch.float32)
    s2.bind(torch.randn(2048, 2048, device="cuda"))
    ms = _time(s2.run, max(5, steps // 4), warmup, s2.stream)
    res["unbounded2d"] = {"kernels": k2d, "grad_2048_fp32_ms": ms,
                          "grad_2048_fp32_model_gbs": s2.model_bytes() / (ms * 1e-3) / 1e9}
    s2.close()
    # Section 2.3.3's DIV (vector -> scalar) and NABLA on psi at 256^3, FP32 (general passes)
    for dname, nc_ in (("div", 3), ("nabla", 1)):
        s = Solver("unbounded", "staggered", [256] * 3, diff=dname, dtype=torch.float32, ncomp=nc_)
        s.bind(f_rings if nc_ == 3 else f_rings[0])
        ms = _time(s.run, max(5, steps // 4), warmup, s.stream)
        res[f"unbounded256_{dname}_fp32"] = {"solves_per_s": 1000 / ms, "ms": ms,
                                             "model_gbs": s.model_bytes() / (ms * 1e-3) / 1e9}
        s.close()
    # differentiable 128^3 curl solve: forward + backward of sum |u - u_t|^2, FP32
    n = 128
    fr = vortex_rings(n, seed=6, count=16, r_range=(0.08, 0.16), core_ratio=0.25).astype(np.float32)
    ft = vortex_rings(n, seed=7, count=16, r_range=(0.08, 0.16), core_ratio=0.25).astype(np.float32)
    s = Solver("unbounded", "staggered", [n] * 3, diff="curl", dtype=torch.float32, ncomp=3)
    _, ut = s.solve([torch.as_tensor(ft[c], device="cuda") for c in range(3)])
    ut = [u.clone() for u in ut]
    fin = [torch.as_tensor(fr[c], device="cuda").requires_grad_(True) for c in range(3)]

    def step():
        for x in fin:
            x.grad = None
        _, u = poisson_solve(s, fin)
        loss = sum(torch.sum((u[c] - ut[c]) ** 2) for c in range(3))
        loss.backward()

    ms = _time(step, steps, warmup, s.stream)
    res["autograd_unbounded128_curl_fp32"] = {"steps_per_s": 1000 / ms, "ms_fwd_bwd": ms}
    s.close()
    return res


def _device_copy(src, dst):
    from paper_2301_01145_amd import _lib
    import torch
    _lib.hp_device_copy(src.data_ptr(), dst.data_ptr(), src.numel() * src.element_size(),
                        torch.cuda.current_stream().cuda_stream)


def copy_reference():
    """A plain device copy of known size (the library's 16-byte streaming copy
    kernel, k_copy16), to calibrate FETCH_SIZE / WRITE_SIZE counters against
    bytes actually moved."""
    import torch
    n = 1 << 28  # 2^28 floats = 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        _device_copy(src, dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": 4 * n, "copies": 3}), flush=True)


def copy_ceiling(warmup=3, reps=20):
    """Measured HBM ceiling of a plain streaming copy (the library's k_copy16,
    1 GiB each way): bytes read + written per copy over its mean HIP-event time."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(warmup):
        _device_copy(src, dst)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        _device_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    return 2.0 * 4 * n / (ms * 1e-3) / 1e9, ok


def timed_solves(solver, steps, warmup):
    """Warmup; then `steps` solves with a HIP event pair around every pass (the
    per-pass breakdown); then the timed region: `steps` solves bracketed by
    synchronisation and HIP events on the plan's stream, with an event pair
    around the dominant pass only (its average duration there feeds the
    roofline; pairs around every pass add about 0.02 ms to a 256^3 solve).
    Returns (ms per solve, [(name, ms, bytes)] per pass, (name, ms, bytes) of
    the dominant pass in the timed region)."""
    import torch
    from paper_2301_01145_amd import hp_pass_stats, hp_set_timing
    for _ in range(warmup):
        solver.run()
    torch.cuda.synchronize()
    hp_pass_stats(solver.plan)  # drop anything recorded so far
    hp_set_timing(solver.plan, 1)
    for _ in range(steps):
        solver.run()
    hp_set_timing(solver.plan, 0)
    passes = hp_pass_stats(solver.plan)
    k = max(range(len(passes)), key=lambda i: passes[i][1])
    hp_set_timing(solver.plan, 2 + k)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(solver.stream)
    for _ in range(steps):
        solver.run()
    stop.record(solver.stream)
    torch.cuda.synchronize()
    hp_set_timing(solver.plan, 0)
    dominant = hp_pass_stats(solver.plan)[k]
    ms = start.elapsed_time(stop) / steps
    return ms, passes, dominant


_ORACLE_FIELDS = None  # (grid, [psi_x, psi_y, psi_z, u_x, u_y, u_z]) of the last oracle run


def cpu_baseline(n_sample, n_full):
    """Time the FP64 oracle on the same workload recipe at a smaller grid."""
    import math

    import numpy as np

    import oracle
    from workloads import vortex_rings
    f = vortex_rings(n_sample, seed=4, count=32).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    psi, curl = oracle.solve("unbounded", "staggered", [n_sample] * 3, [0, 0, 0], [1, 1, 1], f, diff="curl")
    t = time.perf_counter() - t0
    global _ORACLE_FIELDS
    _ORACLE_FIELDS = (n_sample, [psi[c] for c in range(3)] + list(curl))
    # work of the dense FFT pipeline ~ M log M with M the doubled grid
    Ms, Mf = (2 * n_sample) ** 3, (2 * n_full) ** 3
    frac = (Ms * math.log2(Ms)) / (Mf * math.log2(Mf))
    if n_sample == n_full:
        sample = (f"one full FP64 oracle solve (psi + curl, numpy pocketfft, single thread) of the "
                  f"same 32-ring {n_full}^3 workload (doubled {2 * n_full}^3) took {t:.2f} s")
    else:
        sample = (f"full FP64 oracle solve (psi + curl, numpy pocketfft, single thread) of the "
                  f"same 32-ring workload at {n_sample}^3 (doubled {2 * n_sample}^3) took "
                  f"{t:.2f} s; scaled to a {n_full}^3 solve by the M log M ratio {frac:.4f}")
    return {
        "value": frac / t,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": sample,
        "sample_seconds": t,
    }


def cpu_fft_context(n, threads):
    """Context beside the oracle baseline, in the role of the paper's CPU (FFTW)
    runs: the same pruned-free doubled-domain curl solve (R2C of the padded
    fields, Green's spectrum, curl, C2R) with scipy.fft on `threads` host
    threads, FP64 and FP32.  Not the oracle; labelled context only."""
    import numpy as np
    import scipy.fft as sfft
    from scipy.special import erf

    from workloads import vortex_rings
    h = 1.0 / n
    M = 2 * n
    sigma = 2 * h
    m = np.minimum(np.arange(M), M - np.arange(M)) * h
    out = {}
    f64 = vortex_rings(n, seed=4, count=32).astype(np.float64)
    for dt in (np.float64, np.float32):
        f = f64.astype(dt)
        t0 = time.perf_counter()
        r = np.sqrt(m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(r > 0, -erf(r / (np.sqrt(2) * sigma)) / (4 * np.pi * np.where(r > 0, r, 1)),
                         -1 / ((2 * np.pi) ** 1.5 * sigma))
        ghat = (sfft.rfftn(g.astype(dt), workers=threads) * h ** 3).real.astype(dt)
        del g, r
        t1 = time.perf_counter()
        k = 2 * np.pi * np.fft.fftfreq(M, d=h)
        k[M // 2] = 0
        kz = k[: M // 2 + 1].copy()
        kz[-1] = 0
        kx, ky, kzz = k[:, None, None].astype(dt), k[None, :, None].astype(dt), kz[None, None, :].astype(dt)
        ps = []
        for c in range(3):
            big = np.zeros((M, M, M), dtype=dt)
            big[:n, :n, :n] = f[c]
            ps.append(sfft.rfftn(big, workers=threads) * ghat)
        outs = [sfft.irfftn(p_, s=(M, M, M), workers=threads)[:n, :n, :n] for p_ in ps]
        curl = [1j * (ky * ps[2] - kzz * ps[1]), 1j * (kzz * ps[0] - kx * ps[2]), 1j * (kx * ps[1] - ky * ps[0])]
        outs += [sfft.irfftn(u, s=(M, M, M), workers=threads)[:n, :n, :n] for u in curl]
        t2 = time.perf_counter()
        out["fp64" if dt == np.float64 else "fp32"] = {"solve_s": t2 - t1, "green_setup_s": t1 - t0,
                                                        "solves_per_s": 1.0 / (t2 - t1)}
        del ps, outs, curl
    out.update({"kind": "context: scipy.fft (pocketfft) unpruned doubled-domain solve, not the oracle",
                "threads": threads, "grid": n})
    return out


def main():
    args = parse()
    if args.copy_ref:
        copy_reference()
        return
    if args.batch_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"neumann_batch64_fp32": neumann_batch64(args.steps, args.warmup)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); use --gpus 1",
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
        ms, passes, dominant = timed_solves(s, args.steps, args.warmup)
        fields = [p.double() for p in psi] + [x.double() for x in u]
        results[prec] = {"ms": ms, "passes": passes, "dominant": dominant, "model_bytes": s.model_bytes(),
                         "fields": fields}
        s.close()
        del src, psi, u
    r32 = results["f32"]
    value = 1000.0 / r32["ms"]
    # dominant kernel: the pass with the largest mean time, timed inside the
    # timed region
    name, pms, pbytes = r32["dominant"]
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
        # the same solve priced with six stored spectral fields between the x and
        # backward-y passes and an FP64 Green's octant (this library stores five,
        # and the octant in the solve precision)
        "model_bytes_six_field_fp64_green": six_field_model_bytes(n),
        "model_gbs_six_field_fp64_green": six_field_model_bytes(n) / (r32["ms"] * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, n),
                     "kernel": name, "kernel_ms": pms, "kernel_bytes": pbytes,
                     # the same bytes over the kernel's average in the committed
                     # rocprofv3 kernel trace of this benchmark (null: none for
                     # these sources)
                     "profile": _profile_view(name, n, pbytes),
                     # the same pass against the vector ALU (it issues VALU instructions
                     # about three quarters of its cycles; profiles/ SQ counters)
                     "alu_view": ({"bound": "alu", "achieved": sandwich_flops(n) / (pms * 1e-3) / 1e12,
                                   "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": sandwich_flops(n) / (pms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS,
                                   "flops": sandwich_flops(n)} if name == "sandwich_x" else None)},
        # per-pass means from the instrumented solves before the timed region
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
    # the same FP32 solve replayed from a captured hipGraph (extra field; `value`
    # stays the eager HIP-event time above)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver("unbounded", "staggered", [n, n, n], diff="curl", dtype=torch.float32, ncomp=3,
                   device=dev)
        s.bind([torch.as_tensor(f32[c], device=dev).contiguous() for c in range(3)])
    torch.cuda.synchronize()
    out["graph_ms_per_step"] = _time_graph(s.run, side, args.steps, args.warmup)
    s.close()
    # the same bytes against what a plain copy reaches on this device
    cgbs, cok = copy_ceiling()
    out["copy_ceiling"] = {"copy_gbs": cgbs, "kernel": "k_copy16 (16-byte nontemporal loads and stores, 1 GiB each way)",
                           "copy_correct": cok, "model_gbs_frac": out["model_gbs"] / cgbs,
                           "dominant_kernel_frac": out["roofline"]["achieved"] / cgbs}
    if not args.no_others:
        out["other_workloads"] = other_workloads(max(5, args.steps // 2), args.warmup)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, n)
        # the GPU results against that FP64 oracle solve (same input, every element)
        if _ORACLE_FIELDS is not None and _ORACLE_FIELDS[0] == n:
            err = {}
            ref = _ORACLE_FIELDS[1]
            for prec, r in results.items():
                num = den = 0.0
                mx = mref = 0.0
                per = []
                for a, b in zip(r["fields"], ref):
                    g = a.cpu().numpy()
                    d2 = float(np.sum((g - b) ** 2))
                    b2 = float(np.sum(b * b))
                    num, den = num + d2, den + b2
                    mx = max(mx, float(np.max(np.abs(g - b))))
                    mref = max(mref, float(np.max(np.abs(b))))
                    per.append((d2 / b2) ** 0.5)
                err[prec] = {"rel_l2": (num / den) ** 0.5, "rel_max": mx / mref,
                             "rel_l2_per_field": per}
            out["error_vs_oracle"] = err
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        out["cpu_fft_context"] = cpu_fft_context(n, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
