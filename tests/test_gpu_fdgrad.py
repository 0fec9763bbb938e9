"""GRAD, CURL and DIV of Dirichlet / Neumann FD2 solves with boundary values
(FD2 differences of psi closed by the boundary rules) on the GPU against the
oracle, element by element: every BC x grid, 1D/2D/3D, FP32 and FP64, on the
general and on the wavefront passes; the eq. (tfih1D) paraboloid reproduces
eq. (tfih1Dgrad)."""
import numpy as np
import pytest

from gpu_util import TOL, case_input, gpu_solve, oracle_solve, rel_l2, rel_max

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]
BCG = [("dirichlet", "regular"), ("dirichlet", "staggered"), ("neumann", "regular"), ("neumann", "staggered")]


def check(got, ref, prec, what):
    l2, mx = TOL[prec]
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    assert e2 <= l2 and em <= mx, f"{what}: rel-L2 {e2:.3e} rel-max {em:.3e}"


@pytest.mark.parametrize("bc,grid", BCG)
@pytest.mark.parametrize("nc", [[12], [1], [12, 10], [9, 15], [12, 10, 9], [64, 32, 128]])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_inhomogeneous_gradient(bc, grid, nc, prec):
    nd = len(nc)
    if nc == [1] and (bc, grid) in (("dirichlet", "regular"), ("neumann", "regular")):
        pytest.skip("too few cells for this BC and grid")
    print(f"fd grad {bc} {grid} {nc} {prec}", flush=True)
    f, faces = case_input(bc, grid, nc, 1, True, prec, seed=151 + nd)
    got, gd = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, "fd2", "grad", prec, 1, faces)
    ref, rd = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, "fd2", "grad", faces)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd) == nd
    for a in range(nd):
        assert gd[a].shape == rd[a].shape
        check(gd[a], rd[a], prec, f"d/dx{a}")


@pytest.mark.parametrize("bc,grid", BCG)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_inhomogeneous_curl_2d(bc, grid, prec):
    nc = [12, 10]
    f, faces = case_input(bc, grid, nc, 1, True, prec, seed=157)
    _, gd = gpu_solve(bc, grid, nc, LO[:2], HI[:2], f, "fd2", "curl", prec, 1, faces)
    _, rd = oracle_solve(bc, grid, nc, LO[:2], HI[:2], f, "fd2", "curl", faces)
    for a in range(2):
        check(gd[a], rd[a], prec, f"curl {a}")


@pytest.mark.parametrize("bc,grid", BCG)
@pytest.mark.parametrize("diff", ["curl", "div"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_inhomogeneous_vector_operators(bc, grid, diff, prec):
    import oracle
    import torch
    from oracle import grid as og
    from paper_2301_01145_amd import Solver
    nc = [12, 10, 9]
    rng = np.random.default_rng(163)
    rnd = np.float32 if prec == "f32" else np.float64
    dtype = torch.float32 if prec == "f32" else torch.float64
    shape = tuple(og.unknowns(bc, grid, n) for n in nc)
    f = rng.normal(size=(3,) + shape).astype(rnd).astype(np.float64)
    faces = []
    for c in range(3):
        fc = {}
        for a in range(3):
            shp = tuple(og.output_points(bc, grid, nc[b]) for b in range(3) if b != a)
            for s in (0, 1):
                fc[(a, s)] = rng.normal(size=shp).astype(rnd).astype(np.float64)
        faces.append(fc)
    sv = Solver(bc, grid, nc, LO, HI, kernel="fd2", diff=diff, dtype=dtype, ncomp=3, inhomogeneous=True)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    fin = [dev(f[c]) for c in range(3)]
    psi = [sv.empty_output() for _ in range(3)]
    der = [sv.empty_output() for _ in range(sv.nderiv)]
    for c in range(3):
        from paper_2301_01145_amd import _lib
        _lib.hp_set_input(sv.plan, 0, c, fin[c].data_ptr(), 1)
        _lib.hp_bind_output(sv.plan, 0, c, psi[c].data_ptr())
        for (a, s), g in faces[c].items():
            gt = dev(g)
            fin.append(gt)  # keep alive
            _lib.hp_set_boundary(sv.plan, 0, a, s, c, gt.data_ptr(), 1)
    for k, t in enumerate(der):
        _lib.hp_bind_gradient(sv.plan, 0, k, t.data_ptr())
    sv.run()
    torch.cuda.synchronize()
    _, rd = oracle.solve(bc, grid, nc, LO, HI, f, operator="fd2", diff=diff, faces=faces)
    for k in range(len(rd)):
        check(der[k].double().cpu().numpy(), rd[k], prec, f"{diff} {k}")
    sv.close()


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("neumann", "regular"), ("neumann", "staggered")])
def test_paraboloid_gradient_on_gpu(bc, grid):
    import test_oracle_fdgrad as pf
    nc = [9, 8, 7]
    consts = [(0.7, -1.3), (2.1, 0.4), (-0.6, 1.1)]
    f, faces, _, grads = pf.paraboloid_case(bc, grid, nc, consts)
    _, gd = gpu_solve(bc, grid, nc, pf.LO, pf.HI, f, "fd2", "grad", "f64", 1, faces)
    scale = max(np.max(np.abs(g)) for g in grads)
    for a in range(3):
        assert np.max(np.abs(gd[a] - grads[a])) <= 1e-10 * scale, a


def test_inhomogeneous_gradient_graph_replay():
    """The solve with its derivative launches, replayed from a captured graph."""
    import torch
    from paper_2301_01145_amd import Solver
    nc = [12, 10, 9]
    f, faces = case_input("neumann", "staggered", nc, 1, True, "f64", seed=167)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver("neumann", "staggered", nc, LO, HI, kernel="fd2", diff="grad", dtype=torch.float64,
                   inhomogeneous=True)
        dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
        psi, der = s.bind(dev(f), {k: dev(v) for k, v in faces.items()})
        s.run()
    torch.cuda.synchronize()
    outs = list(psi) + list(der)
    eager = [t.cpu().numpy().copy() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, t in enumerate(outs):
            assert np.array_equal(t.cpu().numpy(), eager[i]), (rep, i)
        del junk
    s.close()
