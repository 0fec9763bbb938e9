"""Batched persistent solve (one launch, many uneven problems) on the GPU.

* every problem of a batch equals the oracle (and the single-problem solve of
  the same problem bit for bit: the same tiles run the same device code);
* the 64-problem Neumann workload (DCT-II / DCT-III, PS, sizes drawn from
  {32, 48, 64, 96, 128} per axis, seed 5) matches the closed form of its
  cosine-mode sources and the oracle;
* replays of a captured hipGraph, with eager work in between, equal the eager
  result every time.
"""
import numpy as np
import pytest

from gpu_util import TOL, rel_l2, rel_max

pytestmark = pytest.mark.gpu


def _run_batch(bc, grid, kernel, shapes, prec, seed):
    import torch
    from paper_2301_01145_amd.batched import BatchedSolver
    from oracle import grid as og
    dtype = torch.float32 if prec == "f32" else torch.float64
    rnd = np.float32 if prec == "f32" else np.float64
    rng = np.random.default_rng(seed)
    probs = [{"nc": list(s), "lo": [0, 0, 0], "hi": [1.0, 1.5, 0.8]} for s in shapes]
    bs = BatchedSolver(bc, grid, probs, kernel=kernel, dtype=dtype)
    fs_np = [rng.normal(size=bs.in_shapes[i]).astype(rnd).astype(np.float64) for i in range(len(shapes))]
    fs = [torch.as_tensor(f, dtype=dtype, device="cuda") for f in fs_np]
    psis = bs.bind(fs)
    bs.run()
    torch.cuda.synchronize()
    assert bs.error_flag() == 0
    return bs, fs_np, fs, [p.double().cpu().numpy() for p in psis]


@pytest.mark.parametrize("bc,grid,kernel", [("neumann", "staggered", "ps"), ("neumann", "regular", "fd2"),
                                            ("dirichlet", "staggered", "fd2")])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_oracle_and_single(bc, grid, kernel, prec):
    import torch
    import oracle
    from paper_2301_01145_amd import Solver
    shapes = [(8, 12, 10), (16, 8, 24), (12, 12, 12), (30, 10, 8), (20, 40, 16)]
    bs, fs_np, fs, got = _run_batch(bc, grid, kernel, shapes, prec, seed=3)
    dtype = torch.float32 if prec == "f32" else torch.float64
    for i, s in enumerate(shapes):
        ref, _ = oracle.solve(bc, grid, list(s), [0, 0, 0], [1.0, 1.5, 0.8], fs_np[i], operator=kernel)
        l2, mx = TOL[prec]
        assert rel_l2(got[i], ref) <= l2 and rel_max(got[i], ref) <= mx, i
        single = Solver(bc, grid, list(s), [0, 0, 0], [1.0, 1.5, 0.8], kernel=kernel, dtype=dtype)
        psi, _ = single.solve(fs[i])
        torch.cuda.synchronize()
        assert np.array_equal(psi[0].double().cpu().numpy(), got[i]), i
        single.close()
    bs.close()


def test_neumann_batch_64():
    import torch
    import oracle
    from paper_2301_01145_amd.batched import BatchedSolver
    from workloads import neumann_batch, staggered_axis
    probs = neumann_batch(64, seed=5)
    bs = BatchedSolver("neumann", "staggered", [{"nc": list(p["shape"])} for p in probs], kernel="ps")
    assert bs.wavefront_kernel()  # every length is 64, 96, 128, 192 or 256
    fs = [torch.as_tensor(p["f"].astype(np.float32), device="cuda") for p in probs]
    psis = bs.bind(fs)
    bs.run()
    torch.cuda.synchronize()
    assert bs.error_flag() == 0
    worst = 0.0
    for i, p in enumerate(probs):
        got = psis[i].double().cpu().numpy()
        # closed form: each cosine product is an eigenfunction of the PS Laplacian
        xs = [staggered_axis(n) for n in p["shape"]]
        X, Y, Z = xs[0][:, None, None], xs[1][None, :, None], xs[2][None, None, :]
        ref = np.zeros(p["shape"])
        for (px, py, pz), A in p["modes"]:
            ref += A * np.cos(np.pi * px * X) * np.cos(np.pi * py * Y) * np.cos(np.pi * pz * Z) / (
                -np.pi ** 2 * (px * px + py * py + pz * pz))
        worst = max(worst, rel_l2(got, ref))
        if i < 8:
            f32 = fs[i].double().cpu().numpy()
            ora, _ = oracle.solve("neumann", "staggered", list(p["shape"]), [0, 0, 0], [1, 1, 1], f32)
            assert rel_l2(got, ora) <= 1e-5
    assert worst <= 1e-5, worst
    bs.close()


def test_batch_graph_replay():
    import torch
    side = torch.cuda.Stream()
    shapes = [(16, 24, 8), (32, 16, 16), (8, 8, 48)]
    with torch.cuda.stream(side):
        # the plan records the stream that is current when it is created
        bs, fs_np, fs, eager = _run_batch("neumann", "staggered", "ps", shapes, "f32", seed=9)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bs.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for p in bs._keep[1]:
            p.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, p in enumerate(bs._keep[1]):
            assert np.array_equal(p.double().cpu().numpy(), eager[i]), (rep, i)
        del junk
    assert bs.error_flag() == 0
    bs.close()


# Transform lengths 64, 96, 128, 192, 256 on every axis (FP32): the persistent
# launch runs the wavefront tile bodies (HP_Q_BATCH_KERNEL = 1).
WF_SHAPES = [(32, 48, 64), (96, 32, 48), (64, 64, 128), (128, 96, 32), (48, 48, 48), (32, 128, 96)]


@pytest.mark.parametrize("bc,grid,kernel", [("neumann", "staggered", "ps"), ("neumann", "regular", "fd2"),
                                            ("dirichlet", "staggered", "fd2"), ("dirichlet", "staggered", "ps")])
def test_batch_wavefront_matches_oracle_and_single(bc, grid, kernel):
    import torch
    import oracle
    from paper_2301_01145_amd import Solver
    print(f"wavefront batch {bc} {grid} {kernel}", flush=True)
    bs, fs_np, fs, got = _run_batch(bc, grid, kernel, WF_SHAPES, "f32", seed=21)
    assert bs.wavefront_kernel()
    for i, s in enumerate(WF_SHAPES):
        ref, _ = oracle.solve(bc, grid, list(s), [0, 0, 0], [1.0, 1.5, 0.8], fs_np[i], operator=kernel)
        l2, mx = TOL["f32"]
        assert rel_l2(got[i], ref) <= l2 and rel_max(got[i], ref) <= mx, i
        # single plans run the same wavefront FFTs on the same tiles: bit for bit
        single = Solver(bc, grid, list(s), [0, 0, 0], [1.0, 1.5, 0.8], kernel=kernel, dtype=torch.float32)
        psi, _ = single.solve(fs[i])
        torch.cuda.synchronize()
        assert np.array_equal(psi[0].double().cpu().numpy(), got[i]), i
        single.close()
    bs.close()


def test_batch_wavefront_matches_general(monkeypatch):
    """The same batch on the wavefront tile bodies and on the general passes."""
    import torch
    wf, fs_np, fs, got_wf = _run_batch("neumann", "staggered", "ps", WF_SHAPES, "f32", seed=23)
    assert wf.wavefront_kernel()
    wf.close()
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, _, _, got_gen = _run_batch("neumann", "staggered", "ps", WF_SHAPES, "f32", seed=23)
    assert not gen.wavefront_kernel()
    gen.close()
    for i in range(len(WF_SHAPES)):
        assert rel_l2(got_wf[i], got_gen[i]) <= 1e-5, i


def test_batch_wavefront_graph_replay():
    import torch
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bs, fs_np, fs, eager = _run_batch("neumann", "staggered", "ps", WF_SHAPES[:4], "f32", seed=25)
    assert bs.wavefront_kernel()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bs.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for p in bs._keep[1]:
            p.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, p in enumerate(bs._keep[1]):
            assert np.array_equal(p.double().cpu().numpy(), eager[i]), (rep, i)
        del junk
    assert bs.error_flag() == 0
    bs.close()


def test_batch_level_launches_match_persistent(monkeypatch):
    """The wavefront tile bodies as one launch per pass level give the same
    result as the single persistent launch, bit for bit."""
    one, _, _, got_one = _run_batch("neumann", "staggered", "ps", WF_SHAPES, "f32", seed=27)
    assert one.kernel_mode() == 1
    one.close()
    monkeypatch.setenv("HP_BATCH_LEVELS", "1")
    lev, _, _, got_lev = _run_batch("neumann", "staggered", "ps", WF_SHAPES, "f32", seed=27)
    assert lev.kernel_mode() == 2
    lev.close()
    for i in range(len(WF_SHAPES)):
        assert np.array_equal(got_one[i], got_lev[i]), i


def test_batch_level_launches_graph_replay(monkeypatch):
    """The level form captured into a graph (the groups of a level on forked
    streams, joined before the next level) replays the eager result bit for
    bit, with eager work between the replays."""
    import torch
    monkeypatch.setenv("HP_BATCH_LEVELS", "1")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bs, fs_np, fs, eager = _run_batch("neumann", "staggered", "ps", WF_SHAPES, "f32", seed=29)
    assert bs.kernel_mode() == 2
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bs.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for p in bs._keep[1]:
            p.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, p in enumerate(bs._keep[1]):
            assert np.array_equal(p.double().cpu().numpy(), eager[i]), (rep, i)
        del junk
    assert bs.error_flag() == 0
    bs.close()
