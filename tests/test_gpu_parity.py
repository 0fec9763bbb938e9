"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, small grids.

Each case draws a seeded source (and boundary values), rounds it to the solve
precision, runs libhipoisson.so and the oracle on the same values and
compares every output element: rel-L2 <= 1e-12 / rel-max <= 1e-11 in FP64,
rel-L2 <= 1e-5 / rel-max <= 1e-4 in FP32.  Sizes span several tiles, odd and
mixed-radix lengths and ragged last tiles.
"""
import itertools

import numpy as np
import pytest

from gpu_util import (TOL, case_input, gpu_solve, laplacian_rounding_tol, oracle_solve, rel_l2, rel_max,
                      to_dev)

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]


def check(got, ref, prec, what=""):
    l2, mx = TOL[prec]
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    assert e2 <= l2 and em <= mx, f"{what}: rel-L2 {e2:.3e} rel-max {em:.3e}"


BOUNDED = []
for bc, grid, kernel, nd, prec in itertools.product(
        ["dirichlet", "neumann"], ["regular", "staggered"], ["ps", "fd2"], [1, 2, 3], ["f64", "f32"]):
    BOUNDED.append((bc, grid, kernel, nd, prec, False))
    if kernel == "fd2":
        BOUNDED.append((bc, grid, kernel, nd, prec, True))


@pytest.mark.parametrize("bc,grid,kernel,nd,prec,inhom", BOUNDED)
def test_bounded_small(bc, grid, kernel, nd, prec, inhom):
    nc = [12, 10, 9][:nd]
    f, faces = case_input(bc, grid, nc, 1, inhom, prec, seed=nd * 7 + inhom)
    got, _ = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", prec, 1, faces)
    ref, _ = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", faces)
    check(got, ref, prec, "psi")


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                     ("neumann", "regular"), ("neumann", "staggered")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bounded_tiles(bc, grid, prec):
    nc = [40, 36, 48]
    f, faces = case_input(bc, grid, nc, 1, True, prec, seed=3)
    got, _ = gpu_solve(bc, grid, nc, LO, HI, f, "fd2", "none", prec, 1, faces)
    ref, _ = oracle_solve(bc, grid, nc, LO, HI, f, "fd2", "none", faces)
    check(got, ref, prec, "psi")


# Power-of-two transform lengths in [64, 512] on every axis: the wavefront-FFT
# bounded kernels (ragged 32-pencil tiles where an axis has N_c - 1 or
# N_c + 1 unknowns).
FASTB = [([64, 32, 128], "fd2", True), ([32, 64, 32], "ps", False), ([64, 128], "fd2", True),
         ([128, 32], "ps", False), ([256, 32, 32], "fd2", True), ([32, 32, 256], "ps", False),
         # lengths 96 and 192 (radix-12 first stage; FP32 on the wavefront kernels)
         ([48, 96, 64], "fd2", True), ([96, 48], "ps", False), ([32, 48, 96], "ps", False)]


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                     ("neumann", "regular"), ("neumann", "staggered")])
@pytest.mark.parametrize("nc,kernel,inhom", FASTB)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bounded_fast(bc, grid, nc, kernel, inhom, prec):
    nd = len(nc)
    f, faces = case_input(bc, grid, nc, 1, inhom, prec, seed=17 + nd)
    got, _ = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", prec, 1, faces)
    ref, _ = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", faces)
    check(got, ref, prec, "psi")


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("neumann", "staggered"),
                                     ("dirichlet", "staggered"), ("neumann", "regular")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nc", [[64, 32, 128], [96, 48, 64]])
def test_bounded_fast_matches_general(bc, grid, prec, nc, monkeypatch):
    """The same 3D problem (transform lengths 2^k, 96, 192) on the wavefront
    and the general kernels."""
    f, faces = case_input(bc, grid, nc, 1, True, prec, seed=29)
    fast, _ = gpu_solve(bc, grid, nc, LO, HI, f, "fd2", "none", prec, 1, faces)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, _ = gpu_solve(bc, grid, nc, LO, HI, f, "fd2", "none", prec, 1, faces)
    ref, _ = oracle_solve(bc, grid, nc, LO, HI, f, "fd2", "none", faces)
    check(fast, ref, prec, "wavefront vs oracle")
    check(gen, ref, prec, "general vs oracle")
    check(fast, gen, prec, "wavefront vs general")


# Dirichlet / Neumann gradient: small ragged sizes on the general passes, and
# power-of-two transform lengths on the wavefront passes (also checked against
# the general ones).  psi is the same with and without the gradient.
BGRAD = [[12], [9], [12, 10], [9, 15], [12, 10, 9], [64, 32, 128], [128, 64]]


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                     ("neumann", "regular"), ("neumann", "staggered")])
@pytest.mark.parametrize("nc", BGRAD)
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bounded_grad(bc, grid, nc, kernel, prec, monkeypatch):
    nd = len(nc)
    f, _ = case_input(bc, grid, nc, 1, False, prec, seed=5 + nd)
    got, gd = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "grad", prec, 1, None)
    ref, rd = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "grad", None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd) == nd
    for a in range(nd):
        assert gd[a].shape == rd[a].shape
        check(gd[a], rd[a], prec, f"d/dx{a}")
    plain, _ = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", prec, 1, None)
    assert np.array_equal(plain, got)
    if max(nc) >= 64:
        monkeypatch.setenv("HP_GENERIC", "1")
        _, gen = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "grad", prec, 1, None)
        for a in range(nd):
            check(gd[a], gen[a], prec, f"wavefront vs general d/dx{a}")


@pytest.mark.parametrize("nd,nc", [(1, [12]), (1, [9]), (2, [12, 10]), (2, [9, 15]), (3, [12, 10, 9]),
                                   (3, [20, 24, 30])])
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("diff", ["none", "grad"])
def test_periodic(nd, nc, kernel, prec, diff):
    f, _ = case_input("periodic", "staggered", nc, 1, False, prec, seed=nd)
    got, gd = gpu_solve("periodic", "staggered", nc, LO[:nd], HI[:nd], f, kernel, diff, prec, 1, None)
    ref, rd = oracle_solve("periodic", "staggered", nc, LO[:nd], HI[:nd], f, kernel, diff, None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd)
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"grad {a}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nc", [[12, 10, 9], [16, 20, 24]])
def test_periodic_curl(prec, nc):
    f, _ = case_input("periodic", "staggered", nc, 3, False, prec, seed=5)
    got, gd = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", "curl", prec, 3, None)
    ref, rd = oracle_solve("periodic", "staggered", nc, LO, HI, f, "ps", "curl", None)
    check(got, ref, prec, "psi")
    for a in range(3):
        check(gd[a], rd[a], prec, f"curl {a}")


# 3D periodic plans with power-of-two sizes in [64, 1024]: the wavefront
# passes of the free-space path on undoubled pencils.
PERF = [([64, 64, 128], 1, "none"), ([128, 64, 64], 1, "grad"), ([64, 128, 64], 3, "curl"),
        ([64, 64, 64], 3, "none"),
        # length 1024 (16 elements per lane) on each axis in turn
        ([1024, 64, 64], 1, "grad"), ([64, 1024, 64], 3, "curl"), ([64, 64, 1024], 1, "none")]


@pytest.mark.parametrize("nc,ncomp,diff", PERF)
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_periodic_fast(nc, ncomp, diff, kernel, prec):
    if max(nc) == 1024 and kernel == "fd2":
        pytest.skip("length-1024 cases: one operator")
    f, _ = case_input("periodic", "staggered", nc, ncomp, False, prec, seed=13)
    got, gd = gpu_solve("periodic", "staggered", nc, LO, HI, f, kernel, diff, prec, ncomp, None)
    ref, rd = oracle_solve("periodic", "staggered", nc, LO, HI, f, kernel, diff, None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd)
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"deriv {a}")


def test_periodic_fast_matches_general(monkeypatch):
    nc = [64, 128, 64]
    f, _ = case_input("periodic", "staggered", nc, 3, False, "f64", seed=31)
    fast, fd = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", "curl", "f64", 3, None)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, gdr = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", "curl", "f64", 3, None)
    check(fast, gen, "f64", "psi fast vs general")
    for a in range(3):
        check(fd[a], gdr[a], "f64", f"curl {a} fast vs general")


UNB = [([8, 10, 12], 1, "none"), ([8, 10, 12], 1, "grad"), ([8, 10, 12], 3, "curl"),
       ([20, 18, 24], 3, "curl"), ([20, 18, 24], 3, "none"), ([30, 16, 15], 1, "grad"),
       # power-of-two doubled lengths: wavefront-FFT kernels
       ([32, 32, 32], 3, "curl"), ([64, 32, 128], 3, "curl"), ([32, 128, 64], 1, "grad"),
       ([64, 64, 32], 1, "none"), ([512, 32, 32], 1, "none"),
       # doubled length 1024 (16 elements per lane) along y and along z
       ([32, 512, 32], 3, "curl"), ([32, 32, 512], 1, "grad")]


@pytest.mark.parametrize("nc,ncomp,diff", UNB)
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("grid", ["staggered", "regular"])
def test_unbounded(nc, ncomp, diff, prec, grid):
    if grid == "regular" and nc[0] != 8:
        pytest.skip("regular grid: one size")
    if grid == "regular":
        nc = [9, 14, 11]  # N_c + 1 nodes -> doubled 20, 30, 24
    f, _ = case_input("unbounded", grid, nc, ncomp, False, prec, seed=11)
    got, gd = gpu_solve("unbounded", grid, nc, LO, HI, f, "g2", diff, prec, ncomp, None)
    ref, rd = oracle_solve("unbounded", grid, nc, LO, HI, f, "g2", diff, None)
    check(got, ref, prec, "psi")
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"deriv {a}")


@pytest.mark.parametrize("diff,ncomp", [("curl", 3), ("grad", 1), ("nabla", 1)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_regular_wavefront(diff, ncomp, prec):
    # node-centred free space with N_c + 1 = 32, 64, 32 nodes: doubled lengths
    # 64, 128, 64, so the wavefront passes run
    from paper_2301_01145_amd import hp_pass_stats, hp_set_timing
    import torch
    from paper_2301_01145_amd import Solver
    nc = [31, 63, 31]
    f, _ = case_input("unbounded", "regular", nc, ncomp, False, prec, seed=59)
    got, gd = gpu_solve("unbounded", "regular", nc, LO, HI, f, "g2", diff, prec, ncomp, None)
    ref, rd = oracle_solve("unbounded", "regular", nc, LO, HI, f, "g2", diff, None)
    check(got, ref, prec, "psi")
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"{diff} {a}")
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "regular", nc, LO, HI, diff=diff, dtype=dtype, ncomp=ncomp)
    s.bind([to_dev(f[c], dtype, torch) for c in range(3)] if ncomp == 3 else to_dev(f, dtype, torch))
    hp_set_timing(s.plan, True)
    s.run()
    torch.cuda.synchronize()
    hp_set_timing(s.plan, False)
    names = [p[0] for p in hp_pass_stats(s.plan)]
    s.close()
    assert names == ["r2c_z", "fwd_y", "sandwich_x", "inv_y", "c2r_z"], names


def test_single_pass_timing():
    """hp_set_timing(plan, 2 + k) records events around pass k only: every
    pass keeps its name and bytes, only pass k has a time; a negative mode is
    refused."""
    import torch
    from paper_2301_01145_amd import HipoissonError, Solver, hp_pass_stats, hp_set_timing
    nc = [32, 32, 32]
    f, _ = case_input("unbounded", "staggered", nc, 3, False, "f32", seed=61)
    s = Solver("unbounded", "staggered", nc, LO, HI, diff="curl", dtype=torch.float32, ncomp=3)
    s.bind([to_dev(f[c], torch.float32, torch) for c in range(3)])
    hp_pass_stats(s.plan)
    hp_set_timing(s.plan, 2 + 2)
    for _ in range(3):
        s.run()
    hp_set_timing(s.plan, 0)
    st = hp_pass_stats(s.plan)
    assert [p[0] for p in st] == ["r2c_z", "fwd_y", "sandwich_x", "inv_y", "c2r_z"], st
    assert st[2][1] > 0.0 and all(st[i][1] == 0.0 for i in (0, 1, 3, 4)), st
    assert all(p[2] > 0.0 for p in st), st
    with pytest.raises(HipoissonError):
        hp_set_timing(s.plan, -1)
    s.close()


NEW_KERNELS = ["g4", "g6", "g8", "g10", "spectral"]


@pytest.mark.parametrize("kernel", NEW_KERNELS)
@pytest.mark.parametrize("nc,ncomp,diff", [([10, 12, 8], 1, "none"), ([24, 20, 16], 1, "grad"),
                                           ([32, 32, 64], 3, "curl"), ([9, 15, 10], 1, "none")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_kernels(kernel, nc, ncomp, diff, prec):
    # higher-order Gaussian and spectral kernels (anisotropic cells: the
    # spectral cutoff uses the largest spacing); general and wavefront passes
    f, _ = case_input("unbounded", "staggered", nc, ncomp, False, prec, seed=23)
    got, gd = gpu_solve("unbounded", "staggered", nc, LO, HI, f, kernel, diff, prec, ncomp, None)
    ref, rd = oracle_solve("unbounded", "staggered", nc, LO, HI, f, kernel, diff, None)
    check(got, ref, prec, "psi")
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"deriv {a}")


@pytest.mark.parametrize("kernel", ["g6", "spectral"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_kernels_adjoint(kernel, prec):
    import torch
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    nc = [16, 12, 20]
    rng = np.random.default_rng(29)
    rnd = np.float32 if prec == "f32" else np.float64
    gpsi = rng.normal(size=(3,) + tuple(nc)).astype(rnd).astype(np.float64)
    gder = [rng.normal(size=tuple(nc)).astype(rnd).astype(np.float64) for _ in range(3)]
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "staggered", nc, LO, HI, kernel=kernel, diff="curl", dtype=dtype, ncomp=3)
    dev = lambda x: torch.as_tensor(x, dtype=dtype, device="cuda")
    out = s.adjoint([dev(gpsi[c]) for c in range(3)], [dev(g) for g in gder])
    torch.cuda.synchronize()
    got = np.stack([o.double().cpu().numpy() for o in out])
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(3)]
    ref = ub.adjoint_unbounded(gpsi, gder, hs, 2.0 * max(hs), "curl", kernel=kernel)
    s.close()
    check(got, ref, prec, "adjoint")


@pytest.mark.parametrize("bc,nc", [("periodic", [12, 10, 8]), ("periodic", [64, 32, 64]),
                                   ("periodic", [64, 64, 128]), ("unbounded", [10, 12, 8]),
                                   ("unbounded", [32, 32, 64])])
@pytest.mark.parametrize("diff,ncomp", [("div", 3), ("nabla", 1), ("nabla", 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_div_nabla(bc, nc, diff, ncomp, prec):
    # Section 2.3.3's DIV and NABLA on psi: general passes at ragged sizes,
    # wavefront passes where every transform length is a power of two >= 64
    kernel = "ps" if bc == "periodic" else "g2"
    f, _ = case_input(bc, "staggered", nc, ncomp, False, prec, seed=37)
    got, gd = gpu_solve(bc, "staggered", nc, LO, HI, f, kernel, diff, prec, ncomp, None)
    ref, rd = oracle_solve(bc, "staggered", nc, LO, HI, f, kernel, diff, None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd) == (1 if diff == "div" else ncomp)
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"{diff} {a}")


@pytest.mark.parametrize("nd,nc", [(1, [24]), (2, [12, 20]), (2, [64, 64])])
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_periodic_nabla_low_dim(nd, nc, kernel, prec):
    f, _ = case_input("periodic", "staggered", nc, 1, False, prec, seed=38)
    got, gd = gpu_solve("periodic", "staggered", nc, LO[:nd], HI[:nd], f, kernel, "nabla", prec, 1, None)
    ref, rd = oracle_solve("periodic", "staggered", nc, LO[:nd], HI[:nd], f, kernel, "nabla", None)
    check(got, ref, prec, "psi")
    check(gd[0], rd[0], prec, "nabla")


@pytest.mark.parametrize("diff,ncomp", [("div", 3), ("nabla", 1), ("nabla", 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("with_psi", [True, False])
@pytest.mark.parametrize("nc", [[16, 12, 20], [32, 64, 32]])
def test_div_nabla_adjoint(diff, ncomp, prec, with_psi, nc):
    import torch
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    rng = np.random.default_rng(41)
    rnd = np.float32 if prec == "f32" else np.float64
    shape = tuple(nc)
    gpsi = rng.normal(size=((ncomp,) + shape) if ncomp == 3 else shape).astype(rnd).astype(np.float64)
    nder = 1 if diff == "div" else ncomp
    gder = [rng.normal(size=shape).astype(rnd).astype(np.float64) for _ in range(nder)]
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "staggered", nc, LO, HI, diff=diff, dtype=dtype, ncomp=ncomp)
    dev = lambda x: torch.as_tensor(x, dtype=dtype, device="cuda")
    gp = ([dev(gpsi[c]) for c in range(3)] if ncomp == 3 else [dev(gpsi)]) if with_psi else None
    out = s.adjoint(gp, [dev(g) for g in gder])
    torch.cuda.synchronize()
    got = np.stack([o.double().cpu().numpy() for o in out]) if ncomp == 3 else out[0].double().cpu().numpy()
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(3)]
    ref = ub.adjoint_unbounded(gpsi if with_psi else None, gder, hs, 2.0 * max(hs), diff)
    s.close()
    check(got, ref, prec, "adjoint")


@pytest.mark.parametrize("bc,nc", [("unbounded", [32, 64, 32]), ("periodic", [64, 128, 64])])
@pytest.mark.parametrize("diff,ncomp", [("div", 3), ("nabla", 1), ("nabla", 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_div_nabla_fast_matches_general(bc, nc, diff, ncomp, prec, monkeypatch):
    """DIV / NABLA on the wavefront passes against the general passes (same input)."""
    kernel = "ps" if bc == "periodic" else "g2"
    f, _ = case_input(bc, "staggered", nc, ncomp, False, prec, seed=53)
    fast, fd = gpu_solve(bc, "staggered", nc, LO, HI, f, kernel, diff, prec, ncomp, None)
    monkeypatch.setenv("HP_GENERIC", "1")
    gen, gd = gpu_solve(bc, "staggered", nc, LO, HI, f, kernel, diff, prec, ncomp, None)
    check(fast, gen, prec, "psi")
    for a in range(len(gd)):
        check(fd[a], gd[a], prec, f"{diff} {a}")


LOW_DIM = [(d, k) for d in (2, 1) for k in ["g2", "g4", "g6", "g8", "g10", "spectral"]]


@pytest.mark.parametrize("nd,kernel", LOW_DIM)
@pytest.mark.parametrize("diff", ["none", "grad", "nabla"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_low_dim(nd, kernel, diff, prec):
    # 2D / 1D free space (run as 3D plans with unit, undoubled trailing axes)
    for nc in ([[24, 20], [64, 48]] if nd == 2 else [[40], [256]]):
        f, _ = case_input("unbounded", "staggered", nc, 1, False, prec, seed=43)
        got, gd = gpu_solve("unbounded", "staggered", nc, LO[:nd], HI[:nd], f, kernel, diff, prec, 1, None)
        ref, rd = oracle_solve("unbounded", "staggered", nc, LO[:nd], HI[:nd], f, kernel, diff, None)
        check(got, ref, prec, f"psi {nc}")
        assert len(gd) == len(rd)
        for a in range(len(rd)):
            if diff == "nabla" and prec == "f64":
                # the Laplacian multiplies the spectrum by k^2 <= (pi / H)^2: the FP64
                # rounding of the transform of the slowly decaying 1D / 2D kernel (set by
                # its largest values) grows by up to (n / 128)^2 against the O(1) output,
                # and in general by the amplification of laplacian_rounding_tol
                hs = [(HI[b] - LO[b]) / nc[b] for b in range(nd)]
                tol = max(1e-12 * max(1.0, (max(nc) / 128.0) ** 2),
                          laplacian_rounding_tol(ref, rd[a], hs, [2 * n for n in nc]))
                e2 = rel_l2(gd[a], rd[a])
                assert e2 <= tol and rel_max(gd[a], rd[a]) <= 10 * tol, (nc, e2)
            else:
                check(gd[a], rd[a], prec, f"{diff} {a} {nc}")


@pytest.mark.parametrize("nd,kernel", [(2, "g2"), (2, "spectral"), (1, "g2"), (1, "spectral")])
@pytest.mark.parametrize("diff", ["none", "grad"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_low_dim_regular(nd, kernel, diff, prec):
    # node-centred 2D / 1D free space: N_c + 1 nodes doubled to 2 (N_c + 1)
    for nc in ([[23, 19], [63, 47]] if nd == 2 else [[39], [255]]):
        f, _ = case_input("unbounded", "regular", nc, 1, False, prec, seed=47)
        got, gd = gpu_solve("unbounded", "regular", nc, LO[:nd], HI[:nd], f, kernel, diff, prec, 1, None)
        ref, rd = oracle_solve("unbounded", "regular", nc, LO[:nd], HI[:nd], f, kernel, diff, None)
        assert got.shape == tuple(n + 1 for n in nc)
        check(got, ref, prec, f"psi {nc}")
        assert len(gd) == len(rd)
        for a in range(len(rd)):
            check(gd[a], rd[a], prec, f"{diff} {a} {nc}")


@pytest.mark.parametrize("bc,kernel", [("periodic", "ps"), ("periodic", "fd2"), ("unbounded", "g2"),
                                       ("unbounded", "g6"), ("unbounded", "spectral")])
@pytest.mark.parametrize("nc", [[24, 20], [64, 48]])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_curl_2d(bc, kernel, nc, prec):
    # 2D curl of a scalar: (d_y psi, -d_x psi)
    f, _ = case_input(bc, "staggered", nc, 1, False, prec, seed=47)
    got, gd = gpu_solve(bc, "staggered", nc, LO[:2], HI[:2], f, kernel, "curl", prec, 1, None)
    ref, rd = oracle_solve(bc, "staggered", nc, LO[:2], HI[:2], f, kernel, "curl", None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd) == 2
    for a in range(2):
        check(gd[a], rd[a], prec, f"curl {a}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_curl_2d_adjoint(prec):
    import torch
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    nc = [30, 24]
    rng = np.random.default_rng(48)
    rnd = np.float32 if prec == "f32" else np.float64
    gpsi = rng.normal(size=tuple(nc)).astype(rnd).astype(np.float64)
    gder = [rng.normal(size=tuple(nc)).astype(rnd).astype(np.float64) for _ in range(2)]
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "staggered", nc, LO[:2], HI[:2], kernel="g4", diff="curl", dtype=dtype)
    dev = lambda x: torch.as_tensor(x, dtype=dtype, device="cuda")
    out = s.adjoint([dev(gpsi)], [dev(g) for g in gder])
    torch.cuda.synchronize()
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(2)]
    ref = ub.adjoint_unbounded(gpsi, gder, hs, 2.0 * max(hs), "curl", kernel="g4")
    s.close()
    check(out[0].double().cpu().numpy(), ref, prec, "adjoint")


@pytest.mark.parametrize("nd", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unbounded_low_dim_adjoint(nd, prec):
    import torch
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    nc = [36, 20][:nd] if nd == 2 else [50]
    rng = np.random.default_rng(44)
    rnd = np.float32 if prec == "f32" else np.float64
    gpsi = rng.normal(size=tuple(nc)).astype(rnd).astype(np.float64)
    gder = [rng.normal(size=tuple(nc)).astype(rnd).astype(np.float64) for _ in range(nd)]
    dtype = torch.float32 if prec == "f32" else torch.float64
    kernel = "g4" if nd == 2 else "spectral"
    s = Solver("unbounded", "staggered", nc, LO[:nd], HI[:nd], kernel=kernel, diff="grad", dtype=dtype)
    dev = lambda x: torch.as_tensor(x, dtype=dtype, device="cuda")
    out = s.adjoint([dev(gpsi)], [dev(g) for g in gder])
    torch.cuda.synchronize()
    got = out[0].double().cpu().numpy()
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(nd)]
    ref = ub.adjoint_unbounded(gpsi, gder, hs, 2.0 * max(hs), "grad", kernel=kernel)
    s.close()
    check(got, ref, prec, "adjoint")


@pytest.mark.parametrize("bc,grid,nc,inhom,ncomp", [
    ("periodic", "staggered", [40], False, 1), ("periodic", "regular", [12, 20], False, 1),
    ("periodic", "staggered", [16, 12, 10], False, 3), ("neumann", "regular", [30], True, 1),
    ("neumann", "staggered", [24, 18], True, 1), ("neumann", "regular", [12, 10, 15], True, 1),
    ("neumann", "staggered", [64, 32, 64], False, 1), ("dirichlet", "staggered", [8, 8], False, 1)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zero_mode_query(bc, grid, nc, inhom, ncomp, prec):
    import torch
    import oracle
    from paper_2301_01145_amd import Solver
    nd = len(nc)
    f, faces = case_input(bc, grid, nc, ncomp, inhom, prec, seed=53)
    f = f + 0.37  # incompatible source
    rnd = np.float32 if prec == "f32" else np.float64
    f = f.astype(rnd).astype(np.float64)
    dtype = torch.float32 if prec == "f32" else torch.float64
    kernel = "fd2" if inhom else "ps"
    s = Solver(bc, grid, nc, LO[:nd], HI[:nd], kernel=kernel, dtype=dtype, ncomp=ncomp, inhomogeneous=inhom,
               diff="curl" if ncomp == 3 else "none")
    fin = [to_dev(f[c], dtype, torch) for c in range(3)] if ncomp == 3 else to_dev(f, dtype, torch)
    fd = {k: to_dev(v, dtype, torch) for k, v in faces.items()} if faces else None
    s.bind(fin, fd)
    got = s.zero_mode()
    comps = [f[c] for c in range(3)] if ncomp == 3 else [f]
    refs = [oracle.zero_mode(bc, grid, nc, LO[:nd], HI[:nd], c, faces) for c in comps]
    ref = max(refs, key=abs)
    assert abs(got - ref) <= 1e-12 * max(1.0, float(np.max(np.abs(f)))), (got, ref)
    s.close()


@pytest.mark.parametrize("generic", [False, True])
def test_unbounded_generic_matches_fast(generic, monkeypatch):
    """The same power-of-two problem through the general passes and the wavefront kernels."""
    if generic:
        monkeypatch.setenv("HP_GENERIC", "1")
    nc = [32, 64, 32]
    f, _ = case_input("unbounded", "staggered", nc, 3, False, "f32", seed=2)
    got, gd = gpu_solve("unbounded", "staggered", nc, LO, HI, f, "g2", "curl", "f32", 3, None)
    ref, rd = oracle_solve("unbounded", "staggered", nc, LO, HI, f, "g2", "curl", None)
    check(got, ref, "f32", "psi")
    for a in range(3):
        check(gd[a], rd[a], "f32", f"curl {a}")


@pytest.mark.parametrize("diff,ncomp", [("none", 1), ("grad", 1), ("curl", 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("with_psi", [True, False])
@pytest.mark.parametrize("nc", [[10, 12, 8], [32, 64, 32]])
def test_unbounded_adjoint(diff, ncomp, prec, with_psi, nc):
    import torch
    from oracle import grid as og
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    if diff == "none" and not with_psi:
        pytest.skip("no upstream gradient")
    rng = np.random.default_rng(21)
    shape = tuple(nc)
    rnd = np.float32 if prec == "f32" else np.float64
    gpsi = rng.normal(size=((ncomp,) + shape) if ncomp == 3 else shape).astype(rnd).astype(np.float64)
    nder = 3 if diff != "none" else 0
    gder = [rng.normal(size=shape).astype(rnd).astype(np.float64) for _ in range(nder)]
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "staggered", nc, LO, HI, diff=diff, dtype=dtype, ncomp=ncomp)
    dev = lambda x: torch.as_tensor(x, dtype=dtype, device="cuda")
    gp = ([dev(gpsi[c]) for c in range(3)] if ncomp == 3 else [dev(gpsi)]) if with_psi else None
    gd = [dev(g) for g in gder] if nder else None
    out = s.adjoint(gp, gd)
    torch.cuda.synchronize()
    got = np.stack([o.double().cpu().numpy() for o in out]) if ncomp == 3 else out[0].double().cpu().numpy()
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(3)]
    ref = ub.adjoint_unbounded(gpsi if with_psi else None, gder, hs, 2.0 * max(hs), diff)
    s.close()
    check(got, ref, prec, "adjoint")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nc", [[10, 12, 8], [32, 64, 32]])
def test_unbounded_adjoint_partial_gradients(prec, nc):
    """Plain vector adjoint with only one upstream gradient bound: the other
    components of grad_f are the transpose applied to zero, i.e. zero."""
    import torch
    from oracle import unbounded as ub
    from paper_2301_01145_amd import Solver
    rng = np.random.default_rng(23)
    shape = tuple(nc)
    rnd = np.float32 if prec == "f32" else np.float64
    g1 = rng.normal(size=shape).astype(rnd).astype(np.float64)
    gpsi = np.zeros((3,) + shape)
    gpsi[1] = g1
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("unbounded", "staggered", nc, LO, HI, diff="none", dtype=dtype, ncomp=3)
    gp = [None, torch.as_tensor(g1, dtype=dtype, device="cuda"), None]
    # poison the outputs: every component must be written
    gf = [torch.full(shape, float("nan"), dtype=dtype, device="cuda") for _ in range(3)]
    out = s.adjoint(gp, None, gf)
    torch.cuda.synchronize()
    got = np.stack([o.double().cpu().numpy() for o in out])
    hs = [(HI[a] - LO[a]) / nc[a] for a in range(3)]
    ref = ub.adjoint_unbounded(gpsi, None, hs, 2.0 * max(hs), "none")
    s.close()
    assert np.all(got[0] == 0) and np.all(got[2] == 0)
    check(got[1], ref[1], prec, "adjoint component 1")


@pytest.mark.parametrize("bc,grid,nc", [("periodic", "staggered", [1, 8]), ("neumann", "regular", [1]),
                                        ("dirichlet", "staggered", [1]), ("dirichlet", "regular", [2, 3]),
                                        ("periodic", "regular", [4096]), ("dirichlet", "regular", [2048]),
                                        ("neumann", "staggered", [2, 1, 3])])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_degenerate_and_long(bc, grid, nc, prec):
    """Axes of one or two cells, and the longest single-axis transforms."""
    nd = len(nc)
    kernel = "fd2"
    f, _ = case_input(bc, grid, nc, 1, False, prec, seed=13)
    got, _ = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", prec, 1, None)
    ref, _ = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, "none", None)
    check(got, ref, prec, "psi")


@pytest.mark.parametrize("bc", ["periodic", "neumann", "dirichlet", "unbounded"])
def test_zero_source(bc):
    nc = [8, 8, 8]
    f = np.zeros(tuple(nc) if bc != "neumann" else (8, 8, 8))
    kernel = "g2" if bc == "unbounded" else "ps"
    got, _ = gpu_solve(bc, "staggered", nc, LO, HI, f, kernel, "none", "f32", 1, None)
    assert np.all(got == 0.0)


@pytest.mark.parametrize("slab", ["8", "16"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_unbounded_kz_slabs(slab, prec, monkeypatch):
    """The y / x passes run slab by slab along kz (uneven last slab)."""
    monkeypatch.setenv("HP_SLAB", slab)
    nc = [64, 32, 128]
    f, _ = case_input("unbounded", "staggered", nc, 3, False, prec, seed=4)
    got, gd = gpu_solve("unbounded", "staggered", nc, LO, HI, f, "g2", "curl", prec, 3, None)
    ref, rd = oracle_solve("unbounded", "staggered", nc, LO, HI, f, "g2", "curl", None)
    check(got, ref, prec, "psi")
    for a in range(3):
        check(gd[a], rd[a], prec, f"curl {a}")


# NABLA, DIV and CURL on Dirichlet / Neumann plans (homogeneous): small ragged
# sizes on the general passes and power-of-two / 96 transform lengths on the
# wavefront passes, against the oracle's derivatives of the eigenfunction series.
BOPS = [([12, 10, 9], "nabla", 1), ([10, 12, 8], "nabla", 3), ([9, 12, 10], "div", 3),
        ([10, 9, 12], "curl", 3), ([12, 10], "curl", 1), ([16], "nabla", 1), ([12, 15], "nabla", 1),
        ([64, 32, 32], "div", 3), ([32, 64, 32], "curl", 3), ([64, 32], "curl", 1),
        ([32, 32, 64], "nabla", 3), ([48, 32, 64], "curl", 3)]


@pytest.mark.parametrize("bc,grid", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                     ("neumann", "regular"), ("neumann", "staggered")])
@pytest.mark.parametrize("nc,diff,ncomp", BOPS)
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bounded_operators(bc, grid, nc, diff, ncomp, kernel, prec):
    nd = len(nc)
    f, _ = case_input(bc, grid, nc, ncomp, False, prec, seed=71 + nd)
    got, gd = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, prec, ncomp, None)
    ref, rd = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd)
    for a in range(len(rd)):
        if diff == "nabla":
            # the Laplacian amplifies the transform rounding by up to k_max^2
            hs = [(HI[b] - LO[b]) / nc[b] for b in range(nd)]
            psi_c = ref[a] if ncomp == 3 else ref
            l2 = TOL[prec][0] if prec == "f32" else max(
                TOL[prec][0], laplacian_rounding_tol(psi_c, rd[a], hs, [2 * n for n in nc]))
            assert rel_l2(gd[a], rd[a]) <= l2, (a, rel_l2(gd[a], rd[a]), l2)
        else:
            check(gd[a], rd[a], prec, f"{diff} {a}")
