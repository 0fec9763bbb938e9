"""Solves captured into a hipGraph (torch.cuda.graph on a side stream) and
replayed: every replay, with eager work and synchronisations in between and
the outputs poisoned before it, equals the eager solve bit for bit.  Covers
the wavefront-FFT paths (free space with curl, periodic with gradient,
bounded with boundary values or with the gradient)."""
import numpy as np
import pytest

from gpu_util import case_input, rel_l2, to_dev

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]

CASES = [
    ("unbounded", "staggered", [32, 64, 32], "g2", "curl", 3, False),
    ("periodic", "staggered", [64, 64, 128], "ps", "grad", 1, False),
    ("dirichlet", "regular", [64, 32, 128], "fd2", "none", 1, True),
    ("neumann", "staggered", [32, 64, 64], "fd2", "none", 1, True),
    # general passes: operators, kernels, lower dimensions
    ("unbounded", "staggered", [24, 20, 30], "g4", "div", 3, False),
    ("unbounded", "staggered", [32, 64, 32], "g2", "div", 3, False),
    ("periodic", "staggered", [64, 64, 64], "fd2", "nabla", 3, False),
    ("periodic", "staggered", [30, 24, 20], "ps", "nabla", 3, False),
    ("unbounded", "staggered", [40, 36], "spectral", "curl", 1, False),
    ("unbounded", "staggered", [120], "g2", "grad", 1, False),
    # Dirichlet / Neumann gradient: wavefront and general passes
    ("dirichlet", "regular", [64, 32, 128], "ps", "grad", 1, False),
    ("neumann", "regular", [12, 10, 9], "fd2", "grad", 1, False),
]


@pytest.mark.parametrize("bc,grid,nc,kernel,diff,ncomp,inhom", CASES)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replay(bc, grid, nc, kernel, diff, ncomp, inhom, prec):
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    f, faces = case_input(bc, grid, nc, ncomp, inhom, prec, seed=41)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        # the plan records the stream that is current when it is created
        s = Solver(bc, grid, nc, LO[:len(nc)], HI[:len(nc)], kernel=kernel, diff=diff, dtype=dtype, ncomp=ncomp,
                   inhomogeneous=inhom)
        fin = [to_dev(f[c], dtype, torch) for c in range(3)] if ncomp == 3 else to_dev(f, dtype, torch)
        fd = {k: to_dev(v, dtype, torch) for k, v in faces.items()} if faces else None
        psi, der = s.solve(fin, fd)
    torch.cuda.synchronize()
    outs = list(psi) + list(der)
    eager = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert torch.equal(o, eager[i]), (rep, i)
        del junk
    s.close()


def test_bind_keeps_bound_tensors_alive():
    """bind() hands raw device pointers to the plan, so the solver must keep the
    bound tensors alive: temporaries passed to bind() and outputs the caller
    drops stay valid across torch.cuda.empty_cache() (which graph capture
    calls) and across graph replays."""
    import torch
    from gpu_util import oracle_solve
    from paper_2301_01145_amd import Solver
    nc = [32, 32, 64]
    f, _ = case_input("unbounded", "staggered", nc, 3, False, "f32", seed=51)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver("unbounded", "staggered", nc, LO, HI, kernel="g2", diff="curl", dtype=torch.float32,
                   ncomp=3)
        s.bind([to_dev(f[c], torch.float32, torch) for c in range(3)])  # temporaries, outputs dropped
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ref, rd = oracle_solve("unbounded", "staggered", nc, LO, HI, f, "g2", "curl", None)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        s.run()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        s.run()
    psi, der = s._keep[2], s._keep[3]
    for rep in range(2):
        for o in psi + der:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = np.stack([p.double().cpu().numpy() for p in psi])
        assert rel_l2(got, ref) <= 1e-5, rep
        for a in range(3):
            assert rel_l2(der[a].double().cpu().numpy(), rd[a]) <= 1e-5, (rep, a)
    del g
    s.close()
