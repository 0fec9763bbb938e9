"""Cell counts whose transform lengths have prime factors above 5 (the direct
prime-radix stages of the general kernels), for every boundary condition and
grid, against the oracle element by element: N_c = 7, 11, 13 and 127 (and the
regular-grid free-space N_c = 64, doubled to 2 (N_c + 1) = 130 = 2 5 13)."""
import pytest

from gpu_util import TOL, case_input, gpu_solve, oracle_solve, rel_l2, rel_max

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]

BCS = [("periodic", "staggered", "ps"), ("periodic", "regular", "fd2"),
       ("dirichlet", "regular", "fd2"), ("dirichlet", "staggered", "ps"),
       ("neumann", "regular", "ps"), ("neumann", "staggered", "fd2"),
       ("unbounded", "staggered", "g2"), ("unbounded", "regular", "g4")]
SIZES = [[7], [127], [11, 13], [127, 7], [7, 11, 13], [13, 127, 11]]


def check(got, ref, prec, what):
    l2, mx = TOL[prec]
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    assert e2 <= l2 and em <= mx, f"{what}: rel-L2 {e2:.3e} rel-max {em:.3e}"


@pytest.mark.parametrize("bc,grid,kernel", BCS)
@pytest.mark.parametrize("nc", SIZES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_prime_lengths(bc, grid, kernel, nc, prec):
    nd = len(nc)
    print(f"any length {bc} {grid} {kernel} {nc} {prec}", flush=True)
    diff = "grad" if bc in ("periodic", "unbounded") or kernel == "ps" else "none"
    inhom = kernel == "fd2" and bc in ("dirichlet", "neumann")
    f, faces = case_input(bc, grid, nc, 1, inhom, prec, seed=83 + nd)
    got, gd = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, prec, 1, faces)
    ref, rd = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, faces)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd)
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"d/dx{a}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("diff,ncomp", [("none", 1), ("curl", 3)])
def test_unbounded_regular_64(prec, diff, ncomp):
    nc = [64, 64, 64] if prec == "f32" else [64, 20, 12]
    f, _ = case_input("unbounded", "regular", nc, ncomp, False, prec, seed=89)
    got, gd = gpu_solve("unbounded", "regular", nc, LO, HI, f, "g2", diff, prec, ncomp, None)
    ref, rd = oracle_solve("unbounded", "regular", nc, LO, HI, f, "g2", diff, None)
    check(got, ref, prec, "psi")
    for a in range(len(rd)):
        check(gd[a], rd[a], prec, f"curl {a}")
