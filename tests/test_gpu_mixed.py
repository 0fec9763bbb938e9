"""Mixed-boundary plans (a periodic, Dirichlet or Neumann condition per axis)
and semi-unbounded plans (one free axis beside them) on the GPU against the
oracle, element by element.

* every ordered pair of distinct conditions in 2D and four triples in 3D, both
  grids, PS and FD2, homogeneous and inhomogeneous (FD2), FP32 and FP64;
* lengths with prime factors (periodic axes run the Hartley transform on the
  general kernels at any length);
* Dirichlet / Neumann mixes at power-of-two transform lengths run the bounded
  wavefront kernels, also checked against the general ones;
* the zero mode of periodic / Neumann mixes; a 3-component field;
* GRAD, CURL, DIV and NABLA of mixed plans (series per axis; FD2 differences
  with boundary values), also on the wavefront passes;
* descriptor rules (NABLA of semi-unbounded plans refused, faces of
  periodic axes);
* semi-unbounded: three 2D and three 3D axis layouts, both grids, PS and FD2,
  boundary values, prime and power-of-two lengths, the kappa = 0 row, a
  3-component field, descriptor rules;
* GRAD, CURL and DIV of semi-unbounded plans (series along the bounded axes,
  the odd kernel's rows along the free one), the kappa = 0 row included;
* mixed and semi-unbounded plans at power-of-two lengths, where the passes
  along Dirichlet / Neumann axes run the wavefront kernels beside the general
  Hartley and free-axis passes, against the oracle and the all-general list;
* a seeded random sweep of mixed and semi-unbounded plans with derivative
  outputs at such lengths (HP_MIXED_SWEEP_CASES cases, 40 by default;
  HP_MIXED_SWEEP_SEED).
"""
import os

import numpy as np
import pytest

from gpu_util import TOL, rel_l2, rel_max

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]
PAIRS = [["periodic", "dirichlet"], ["dirichlet", "periodic"], ["periodic", "neumann"],
         ["neumann", "periodic"], ["dirichlet", "neumann"], ["neumann", "dirichlet"]]
TRIPLES = [["periodic", "dirichlet", "neumann"], ["neumann", "periodic", "dirichlet"],
           ["dirichlet", "neumann", "periodic"], ["periodic", "neumann", "neumann"]]


def mixed_input(bcs, gtype, nc, ncomp, inhom, prec, seed):
    from oracle import grid as og
    rng = np.random.default_rng(seed)
    nd = len(nc)
    shape = tuple(og.unknowns(bcs[a], gtype, nc[a]) for a in range(nd))
    f = rng.normal(size=((ncomp,) + shape) if ncomp == 3 else shape)
    faces = None
    if inhom:
        faces = {}
        for a in range(nd):
            if bcs[a] in ("periodic", "unbounded"):
                continue
            shp = tuple(og.output_points(bcs[b], gtype, nc[b]) for b in range(nd) if b != a)
            for s in (0, 1):
                faces[(a, s)] = rng.normal(size=shp)
    rnd = np.float32 if prec == "f32" else np.float64
    f = f.astype(rnd).astype(np.float64)
    if faces:
        faces = {k: v.astype(rnd).astype(np.float64) for k, v in faces.items()}
    return f, faces


def gpu_mixed(bcs, gtype, nc, f, kernel, prec, ncomp, faces):
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    nd = len(nc)
    s = Solver(list(bcs), gtype, nc, LO[:nd], HI[:nd], kernel=kernel, dtype=dtype, ncomp=ncomp,
               inhomogeneous=faces is not None)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    fin = [dev(f[c]) for c in range(3)] if ncomp == 3 else dev(f)
    fd = {k: dev(v) for k, v in faces.items()} if faces else None
    psi, _ = s.solve(fin, fd)
    torch.cuda.synchronize()
    out = np.stack([p.double().cpu().numpy() for p in psi]) if ncomp == 3 else psi[0].double().cpu().numpy()
    zm = s.zero_mode()
    npass = s.passes()
    s.close()
    return out, zm, npass


def check(got, ref, prec, what):
    l2, mx = TOL[prec]
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    assert e2 <= l2 and em <= mx, f"{what}: rel-L2 {e2:.3e} rel-max {em:.3e}"


def run_case(bcs, gtype, nc, kernel, inhom, prec, seed, ncomp=1):
    import oracle
    nd = len(nc)
    print(f"mixed {bcs} {gtype} {nc} {kernel} inhom={inhom} {prec} ncomp={ncomp}", flush=True)
    f, faces = mixed_input(bcs, gtype, nc, ncomp, inhom, prec, seed)
    got, zm, npass = gpu_mixed(bcs, gtype, nc, f, kernel, prec, ncomp, faces)
    ref, _ = oracle.solve(list(bcs), gtype, nc, LO[:nd], HI[:nd], f, operator=kernel,
                          faces=([faces] * 3 if (faces and ncomp == 3) else faces))
    assert got.shape == ref.shape
    check(got, ref, prec, "psi")
    if ncomp == 1:
        zr = oracle.zero_mode(list(bcs), gtype, nc, LO[:nd], HI[:nd], f, faces)
        assert abs(zm - zr) <= (1e-10 if prec == "f64" else 1e-4) * max(1.0, float(np.max(np.abs(f)))), (zm, zr)
    return got, npass


CASES = []
for bcs in PAIRS:
    for gtype in ("regular", "staggered"):
        for kernel, inhom in (("ps", False), ("fd2", False), ("fd2", True)):
            for prec in ("f64", "f32"):
                CASES.append((bcs, gtype, [12, 10], kernel, inhom, prec))
for bcs in TRIPLES:
    for gtype in ("regular", "staggered"):
        for kernel, inhom in (("ps", False), ("fd2", True)):
            for prec in ("f64", "f32"):
                CASES.append((bcs, gtype, [12, 10, 9], kernel, inhom, prec))


@pytest.mark.parametrize("bcs,gtype,nc,kernel,inhom,prec", CASES)
def test_mixed_matches_oracle(bcs, gtype, nc, kernel, inhom, prec):
    run_case(bcs, gtype, nc, kernel, inhom, prec, seed=101 + len(nc))


@pytest.mark.parametrize("bcs,nc", [(["periodic", "dirichlet"], [7, 13]), (["neumann", "periodic"], [11, 127]),
                                    (["periodic", "neumann", "dirichlet"], [13, 7, 11])])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_prime_lengths(bcs, nc, prec):
    run_case(bcs, "staggered", nc, "fd2", True, prec, seed=103)


@pytest.mark.parametrize("bcs", [["dirichlet", "neumann", "dirichlet"], ["neumann", "dirichlet", "neumann"]])
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_wavefront_matches_general(bcs, gtype, prec, monkeypatch):
    # transform lengths 64 / 128 on every axis: the bounded wavefront kernels
    if gtype == "staggered":
        nc = [32, 64, 32]
    else:  # DST-I 2 N_c, DCT-I 2 N_c
        nc = [32, 64, 32]
    fast, npass = run_case(bcs, gtype, nc, "fd2", True, prec, seed=107)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, _ = run_case(bcs, gtype, nc, "fd2", True, prec, seed=107)
    check(fast, gen, prec, "wavefront vs general")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_vector(prec):
    run_case(["periodic", "dirichlet", "neumann"], "staggered", [16, 12, 10], "ps", False, prec, seed=109,
             ncomp=3)


def test_mixed_constant_source_zero_mode():
    import torch
    from paper_2301_01145_amd import Solver
    s = Solver(["periodic", "neumann"], "regular", [12, 10], LO[:2], HI[:2], kernel="fd2", dtype=torch.float64)
    f = torch.full(s.in_shape, 2.5, dtype=torch.float64, device="cuda")
    psi, _ = s.solve(f)
    torch.cuda.synchronize()
    assert abs(s.zero_mode() - 2.5) <= 1e-12
    assert float(psi[0].abs().max()) <= 1e-12
    s.close()


def test_mixed_descriptor_rules():
    import ctypes
    import torch
    from paper_2301_01145_amd import HipoissonError, Solver, _lib, make_desc
    d = make_desc(["periodic", "unbounded"], "staggered", [8, 8], diff="nabla")
    out = ctypes.c_void_p()
    assert _lib.lib().hp_plan_create(ctypes.byref(d), None, ctypes.byref(out)) == _lib.HP_E_UNSUPPORTED
    s = Solver(["periodic", "dirichlet"], "staggered", [8, 8], kernel="fd2", dtype=torch.float64,
               inhomogeneous=True)
    g = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(HipoissonError):
        _lib.hp_set_boundary(s.plan, 0, 0, 0, 0, g.data_ptr(), 1)  # axis 0 is periodic
    _lib.hp_set_boundary(s.plan, 0, 1, 0, 0, g.data_ptr(), 1)     # axis 1 is Dirichlet
    s.close()


# ----------------------------------------------------------- semi-unbounded
SEMI2 = [["unbounded", "periodic"], ["dirichlet", "unbounded"], ["unbounded", "neumann"]]
SEMI3 = [["periodic", "unbounded", "dirichlet"], ["unbounded", "neumann", "periodic"],
         ["neumann", "dirichlet", "unbounded"]]
SEMI_CASES = []
for bcs in SEMI2:
    for gtype in ("regular", "staggered"):
        for kernel, inhom in (("ps", False), ("fd2", False), ("fd2", True)):
            if inhom and bcs == ["unbounded", "periodic"]:
                continue  # no face takes boundary values
            for prec in ("f64", "f32"):
                SEMI_CASES.append((bcs, gtype, [12, 10], kernel, inhom, prec))
for bcs in SEMI3:
    for gtype in ("regular", "staggered"):
        for kernel, inhom in (("ps", False), ("fd2", True)):
            for prec in ("f64", "f32"):
                SEMI_CASES.append((bcs, gtype, [12, 10, 9], kernel, inhom, prec))


@pytest.mark.parametrize("bcs,gtype,nc,kernel,inhom,prec", SEMI_CASES)
def test_semi_matches_oracle(bcs, gtype, nc, kernel, inhom, prec):
    run_case(bcs, gtype, nc, kernel, inhom, prec, seed=113 + len(nc))


@pytest.mark.parametrize("bcs,nc", [(["unbounded", "dirichlet"], [7, 13]), (["periodic", "unbounded"], [11, 127]),
                                    (["unbounded", "neumann", "dirichlet"], [13, 7, 11]),
                                    (["neumann", "periodic", "unbounded"], [32, 16, 64])])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_lengths(bcs, nc, prec):
    run_case(bcs, "staggered", nc, "fd2", "dirichlet" in bcs or "neumann" in bcs, prec, seed=127)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_zero_eigenvalue_row(prec):
    # a source constant along the periodic / Neumann axes: only the kappa = 0
    # row (G = |x| / 2) acts
    import oracle
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    nc = [16, 6, 5]
    bcs = ["unbounded", "periodic", "neumann"]
    x = np.random.default_rng(131).normal(size=16)
    f = np.broadcast_to(x[:, None, None], (16, 6, 5)).copy()
    f = f.astype(np.float32 if prec == "f32" else np.float64).astype(np.float64)
    s = Solver(bcs, "staggered", nc, LO, HI, kernel="fd2", dtype=dtype)
    psi, _ = s.solve(torch.as_tensor(f, dtype=dtype, device="cuda"))
    torch.cuda.synchronize()
    got = psi[0].double().cpu().numpy()
    ref, _ = oracle.solve(bcs, "staggered", nc, LO, HI, f, operator="fd2")
    check(got, ref, prec, "psi")
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_vector(prec):
    run_case(["dirichlet", "periodic", "unbounded"], "staggered", [10, 12, 16], "ps", False, prec, seed=137,
             ncomp=3)


def test_semi_descriptor_rules():
    import ctypes
    import torch
    from paper_2301_01145_amd import HipoissonError, Solver, _lib, make_desc
    out = ctypes.c_void_p()
    for kw, st in ((dict(bc=["unbounded", "unbounded"], grid="staggered", nc=[8, 8]), _lib.HP_E_ARG),
                   (dict(bc=["unbounded", "unbounded", "periodic"], grid="staggered", nc=[8, 8, 8]),
                    _lib.HP_E_UNSUPPORTED)):
        d = make_desc(**kw)
        assert _lib.lib().hp_plan_create(ctypes.byref(d), None, ctypes.byref(out)) == st
    s = Solver(["unbounded", "dirichlet"], "staggered", [8, 8], kernel="fd2", dtype=torch.float64,
               inhomogeneous=True)
    g = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(HipoissonError):
        _lib.hp_set_boundary(s.plan, 0, 0, 0, 0, g.data_ptr(), 1)  # the free axis
    s.close()


@pytest.mark.parametrize("bcs,kernel,inhom", [(["periodic", "dirichlet", "neumann"], "fd2", True),
                                              (["neumann", "unbounded", "periodic"], "ps", False)])
def test_mixed_and_semi_graph_replay(bcs, kernel, inhom):
    """Replays of a captured solve (eager work in between) equal the eager solve."""
    import torch
    from paper_2301_01145_amd import Solver
    nc = [12, 10, 16]
    f, faces = mixed_input(bcs, "staggered", nc, 1, inhom, "f64", seed=139)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = Solver(bcs, "staggered", nc, LO, HI, kernel=kernel, dtype=torch.float64, inhomogeneous=inhom)
        dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
        fd = {k: dev(v) for k, v in faces.items()} if faces else None
        psi, _ = s.bind(dev(f), fd)
        s.run()
    torch.cuda.synchronize()
    eager = psi[0].cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.run()
    torch.cuda.synchronize()
    for rep in range(3):
        psi[0].fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(psi[0].cpu().numpy(), eager), rep
        del junk
    s.close()


def _sweep_cases(count, seed):
    """Seeded random mixed / semi-unbounded cases: conditions per axis, grid,
    operator, boundary values, precision and sizes of any factorization."""
    from oracle import grid as og
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        nd = int(rng.integers(2, 4))
        bcs = [str(rng.choice(["periodic", "dirichlet", "neumann"])) for _ in range(nd)]
        if rng.random() < 0.35:
            bcs[int(rng.integers(0, nd))] = "unbounded"
        if len(set(bcs)) == 1:
            continue  # a uniform plan: covered by the main sweep
        gtype = str(rng.choice(["regular", "staggered"]))
        kernel = str(rng.choice(["ps", "fd2"]))
        faces_ok = any(b in ("dirichlet", "neumann") for b in bcs)
        inhom = kernel == "fd2" and faces_ok and bool(rng.random() < 0.5)
        prec = str(rng.choice(["f32", "f64"]))
        hi_n = 64 if nd == 2 else 20
        nc = []
        for b in bcs:
            while True:
                n = int(rng.integers(2, hi_n + 1))
                if og.unknowns(b, gtype, n) >= (2 if (b == "neumann" and gtype == "regular") else 1):
                    break
            nc.append(n)
        ncomp = 3 if (nd == 3 and rng.random() < 0.2) else 1
        out.append((bcs, gtype, nc, kernel, inhom and ncomp == 1, prec, ncomp, int(rng.integers(0, 1 << 20))))
    return out


@pytest.mark.parametrize("bcs,gtype,nc,kernel,inhom,prec,ncomp,seed", _sweep_cases(60, seed=2301))
def test_mixed_sweep(bcs, gtype, nc, kernel, inhom, prec, ncomp, seed):
    run_case(bcs, gtype, nc, kernel, inhom, prec, seed=seed, ncomp=ncomp)


# ------------------------------------------------ derivatives of mixed plans
DERIV_CASES = []
for bcs in PAIRS:
    for gtype in ("regular", "staggered"):
        for kernel, inhom, diff in (("ps", False, "grad"), ("fd2", False, "nabla"), ("fd2", True, "grad"),
                                    ("ps", False, "curl")):
            for prec in ("f64", "f32"):
                DERIV_CASES.append((bcs, gtype, [12, 10], kernel, inhom, diff, prec, 1))
for bcs in TRIPLES:
    for gtype in ("regular", "staggered"):
        for kernel, inhom, diff, ncomp in (("ps", False, "grad", 1), ("fd2", False, "curl", 3),
                                           ("ps", False, "div", 3), ("ps", False, "nabla", 3),
                                           ("fd2", True, "grad", 1)):
            for prec in ("f64", "f32"):
                DERIV_CASES.append((bcs, gtype, [12, 10, 9], kernel, inhom, diff, prec, ncomp))


@pytest.mark.parametrize("bcs,gtype,nc,kernel,inhom,diff,prec,ncomp", DERIV_CASES)
def test_mixed_derivatives(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp):
    run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=173 + len(nc))


def run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed, f=None):
    import oracle
    import torch
    from paper_2301_01145_amd import Solver
    nd = len(nc)
    print(f"mixed deriv {bcs} {gtype} {nc} {kernel} inhom={inhom} {diff} {prec} ncomp={ncomp}", flush=True)
    faces = None
    if f is None:
        f, faces = mixed_input(bcs, gtype, nc, ncomp, inhom, prec, seed=seed)
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver(list(bcs), gtype, nc, LO[:nd], HI[:nd], kernel=kernel, diff=diff, dtype=dtype, ncomp=ncomp,
               inhomogeneous=inhom)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    fin = [dev(f[c]) for c in range(3)] if ncomp == 3 else dev(f)
    psi, der = s.solve(fin, {k: dev(v) for k, v in faces.items()} if faces else None)
    torch.cuda.synchronize()
    got = np.stack([p.double().cpu().numpy() for p in psi]) if ncomp == 3 else psi[0].double().cpu().numpy()
    ref, rd = oracle.solve(list(bcs), gtype, nc, LO[:nd], HI[:nd], f, operator=kernel, diff=diff,
                           faces=([faces] * 3 if (faces and ncomp == 3) else faces))
    check(got, ref, prec, "psi")
    assert len(der) == len(rd)
    dout = [d.double().cpu().numpy() for d in der]
    for a in range(len(rd)):
        check(dout[a], rd[a], prec, f"{diff} {a}")
    s.close()
    return got, dout


@pytest.mark.parametrize("bcs", [["dirichlet", "neumann", "dirichlet"], ["neumann", "dirichlet", "neumann"]])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_derivatives_wavefront_matches_general(bcs, prec, monkeypatch):
    # Dirichlet / Neumann mixes at power-of-two transform lengths: the series
    # derivative passes on the wavefront kernels against the general ones
    import torch
    from paper_2301_01145_amd import Solver
    nc = [32, 64, 32]
    f, _ = mixed_input(bcs, "staggered", nc, 1, False, prec, seed=179)
    dtype = torch.float32 if prec == "f32" else torch.float64

    def run():
        s = Solver(bcs, "staggered", nc, LO, HI, kernel="ps", diff="grad", dtype=dtype)
        psi, der = s.solve(torch.as_tensor(f, dtype=dtype, device="cuda"))
        torch.cuda.synchronize()
        out = [d.double().cpu().numpy() for d in der]
        s.close()
        return out

    fast = run()
    monkeypatch.setenv("HP_GENERIC", "1")
    gen = run()
    for a in range(3):
        check(fast[a], gen[a], prec, f"d/dx{a}")


# ----------------------------------------- derivatives of semi-unbounded plans
SEMI_DERIV_CASES = []
for bcs in SEMI2:
    for gtype in ("regular", "staggered"):
        for kernel, diff in (("ps", "grad"), ("fd2", "curl")):
            for prec in ("f64", "f32"):
                SEMI_DERIV_CASES.append((bcs, gtype, [12, 10], kernel, diff, prec, 1))
for bcs in SEMI3:
    for gtype in ("regular", "staggered"):
        for kernel, diff, ncomp in (("ps", "grad", 1), ("fd2", "curl", 3), ("ps", "div", 3)):
            for prec in ("f64", "f32"):
                SEMI_DERIV_CASES.append((bcs, gtype, [12, 10, 9], kernel, diff, prec, ncomp))


@pytest.mark.parametrize("bcs,gtype,nc,kernel,diff,prec,ncomp", SEMI_DERIV_CASES)
def test_semi_derivatives(bcs, gtype, nc, kernel, diff, prec, ncomp):
    run_deriv_case(bcs, gtype, nc, kernel, False, diff, prec, ncomp, seed=181 + len(nc))


@pytest.mark.parametrize("bcs,nc", [(["unbounded", "dirichlet"], [7, 13]), (["periodic", "unbounded"], [11, 127]),
                                    (["neumann", "periodic", "unbounded"], [32, 16, 64])])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_derivative_lengths(bcs, nc, prec):
    run_deriv_case(bcs, "staggered", nc, "fd2", False, "grad", prec, 1, seed=191)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_derivative_zero_eigenvalue_row(prec):
    # a source constant along the periodic / Neumann axes: the free-axis
    # derivative takes only the kappa = 0 row (G' = sign(x) / 2); the others
    # vanish (to rounding, measured against the free-axis derivative's size)
    import oracle
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    nc = [16, 6, 5]
    bcs = ["unbounded", "periodic", "neumann"]
    x = np.random.default_rng(193).normal(size=16)
    f = np.broadcast_to(x[:, None, None], (16, 6, 5)).copy()
    f = f.astype(np.float32 if prec == "f32" else np.float64).astype(np.float64)
    s = Solver(bcs, "staggered", nc, LO, HI, kernel="fd2", diff="grad", dtype=dtype)
    psi, der = s.solve(torch.as_tensor(f, dtype=dtype, device="cuda"))
    torch.cuda.synchronize()
    ref, rd = oracle.solve(bcs, "staggered", nc, LO, HI, f, operator="fd2", diff="grad")
    check(psi[0].double().cpu().numpy(), ref, prec, "psi")
    d0 = der[0].double().cpu().numpy()
    check(d0, rd[0], prec, "d/dx0")
    scale = float(np.max(np.abs(rd[0])))
    for a in (1, 2):
        assert np.max(np.abs(rd[a])) <= 1e-13 * scale
        assert np.max(np.abs(der[a].double().cpu().numpy())) <= TOL[prec][1] * scale, a
    s.close()


# a periodic (Hartley) axis beside Dirichlet / Neumann axes at power-of-two
# transform lengths: the Dirichlet / Neumann passes run the wavefront kernels,
# the Hartley passes the general ones
MIX_WF = [["periodic", "dirichlet", "neumann"], ["neumann", "periodic", "dirichlet"],
          ["dirichlet", "neumann", "periodic"]]


@pytest.mark.parametrize("bcs", MIX_WF)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("kernel,inhom,diff", [("fd2", True, "none"), ("ps", False, "grad"), ("fd2", False, "curl")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_periodic_axis_wavefront(bcs, gtype, kernel, inhom, diff, prec, monkeypatch):
    nc = [32, 64, 32]
    ncomp = 3 if diff == "curl" else 1
    got, dout = run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=197)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, dgen = run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=197)
    check(got, gen, prec, "psi wavefront vs general")
    for a in range(len(dgen)):
        check(dout[a], dgen[a], prec, f"{diff} {a} wavefront vs general")


# semi-unbounded plans with Dirichlet / Neumann axes at power-of-two transform
# lengths: their passes run the wavefront kernels, the free axis's sandwich
# the general ones
SEMI_WF = [["neumann", "dirichlet", "unbounded"], ["unbounded", "dirichlet", "neumann"],
           ["dirichlet", "unbounded", "neumann"]]


@pytest.mark.parametrize("bcs", SEMI_WF)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("kernel,inhom,diff", [("fd2", True, "none"), ("ps", False, "grad"), ("fd2", False, "curl")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_semi_bounded_axes_wavefront(bcs, gtype, kernel, inhom, diff, prec, monkeypatch):
    nc = [32, 64, 32]
    ncomp = 3 if diff == "curl" else 1
    got, dout = run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=199)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, dgen = run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=199)
    check(got, gen, prec, "psi wavefront vs general")
    for a in range(len(dgen)):
        check(dout[a], dgen[a], prec, f"{diff} {a} wavefront vs general")


@pytest.mark.parametrize("bcs", [["periodic", "dirichlet", "neumann"], ["neumann", "dirichlet", "unbounded"]])
def test_wavefront_passes_beside_general_ones(bcs):
    """At power-of-two lengths a mixed plan's Dirichlet / Neumann passes run
    the wavefront kernels while its Hartley or free-axis passes stay general."""
    import torch
    from paper_2301_01145_amd import Solver, hp_pass_stats, hp_set_timing
    nc = [32, 64, 32]
    f, _ = mixed_input(bcs, "staggered", nc, 1, False, "f32", seed=201)
    s = Solver(bcs, "staggered", nc, LO, HI, kernel="fd2", dtype=torch.float32)
    s.bind(torch.as_tensor(f.astype(np.float32), device="cuda"))
    hp_pass_stats(s.plan)
    hp_set_timing(s.plan, 1)
    s.run()
    hp_set_timing(s.plan, 0)
    names = [p[0] for p in hp_pass_stats(s.plan)]
    s.close()
    assert any(n.startswith("r2r_") for n in names), names
    assert any(not n.startswith("r2r_") for n in names), names



def _deriv_sweep_cases(count, seed):
    """Seeded random mixed / semi-unbounded plans with derivative outputs:
    Dirichlet / Neumann axes of 32 or 64 cells (power-of-two transform
    lengths: their passes run the wavefront kernels), periodic and free axes of
    any small size; every operator the plan allows."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        nd = int(rng.integers(2, 4))
        bcs = [str(rng.choice(["periodic", "dirichlet", "neumann"])) for _ in range(nd)]
        free = rng.random() < 0.35
        if free:
            bcs[int(rng.integers(0, nd))] = "unbounded"
        if len(set(bcs)) == 1 or not any(b in ("dirichlet", "neumann") for b in bcs):
            continue
        gtype = str(rng.choice(["regular", "staggered"]))
        kernel = str(rng.choice(["ps", "fd2"]))
        prec = str(rng.choice(["f32", "f64"]))
        ncomp = 3 if (nd == 3 and rng.random() < 0.4) else 1
        inhom = kernel == "fd2" and not free and bool(rng.random() < 0.4)
        if ncomp == 3:
            choices = ["curl", "div"] + ([] if (free or inhom) else ["nabla"])
        else:
            choices = ["grad"] + (["curl"] if nd == 2 else []) + ([] if (free or inhom) else ["nabla"])
        diff = str(rng.choice(choices))
        nc = [int(rng.choice([32, 64] if nd == 2 else [32])) if b in ("dirichlet", "neumann")
              else int(rng.integers(3, 21)) for b in bcs]
        out.append((bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, int(rng.integers(0, 1 << 20))))
    return out


@pytest.mark.parametrize("bcs,gtype,nc,kernel,inhom,diff,prec,ncomp,seed",
                         _deriv_sweep_cases(int(os.environ.get("HP_MIXED_SWEEP_CASES", "40")),
                                            seed=int(os.environ.get("HP_MIXED_SWEEP_SEED", "2302"))))
def test_mixed_derivative_sweep(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed):
    run_deriv_case(bcs, gtype, nc, kernel, inhom, diff, prec, ncomp, seed=seed)



@pytest.mark.parametrize("bcs", [["dirichlet", "dirichlet", "dirichlet"], ["periodic", "dirichlet", "neumann"],
                                 ["neumann", "neumann", "dirichlet"]])
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("diff", ["none", "curl", "div"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_vector_boundary_values(bcs, gtype, diff, prec):
    """A 3-component field with boundary values: the same face arrays bound for
    every component (FD2; psi, and CURL / DIV by differences)."""
    run_deriv_case(bcs, gtype, [12, 10, 9], "fd2", True, diff, prec, 3, seed=211)


def test_vector_boundary_values_per_component():
    """One face dict per component: each component solved with its own values,
    equal to three scalar solves."""
    import torch
    from paper_2301_01145_amd import Solver
    bcs, nc = ["dirichlet", "neumann", "periodic"], [12, 10, 9]
    fs, fcs = [], []
    for c in range(3):
        f, faces = mixed_input(bcs, "staggered", nc, 1, True, "f64", seed=221 + c)
        fs.append(f)
        fcs.append(faces)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    s = Solver(bcs, "staggered", nc, LO, HI, kernel="fd2", dtype=torch.float64, ncomp=3, inhomogeneous=True)
    psi, _ = s.solve([dev(f) for f in fs], [{k: dev(v) for k, v in fc.items()} for fc in fcs])
    torch.cuda.synchronize()
    got = [p.double().cpu().numpy() for p in psi]
    s.close()
    for c in range(3):
        ref, _, _ = gpu_mixed(bcs, "staggered", nc, fs[c], "fd2", "f64", 1, fcs[c])
        check(got[c], ref, "f64", f"component {c}")
    with pytest.raises(ValueError):
        s2 = Solver(bcs, "staggered", nc, LO, HI, kernel="fd2", dtype=torch.float64, ncomp=3,
                    inhomogeneous=True)
        try:
            s2.bind([dev(f) for f in fs], [{k: dev(v) for k, v in fcs[0].items()}] * 2)
        finally:
            s2.close()
