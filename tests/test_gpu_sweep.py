"""Seeded random sweep of GPU-vs-oracle parity cases: boundary condition, grid,
dimension, kernel, operator, precision, boundary values and sizes are drawn
together (any size: transform lengths with prime factors above 5 included),
and every output element is compared at the library's tolerances."""
import os

import numpy as np
import pytest

from gpu_util import TOL, case_input, gpu_solve, laplacian_rounding_tol, oracle_solve, rel_l2, rel_max
from oracle import grid as og

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]


def _cells(rng, bc, grid, lo, hi):
    """Any cell count whose transform length is at least 2 (lengths with prime
    factors above 5 run the direct prime-radix stages)."""
    while True:
        nc = int(rng.integers(lo, hi + 1))
        L = nc if bc == "periodic" else (2 * (nc + 1) if bc == "unbounded" and grid == "regular" else 2 * nc)
        if L >= 2:
            return nc


def _cases(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        bc = str(rng.choice(["periodic", "dirichlet", "neumann", "unbounded"]))
        nd = int(rng.integers(1, 4))
        grid = str(rng.choice(["regular", "staggered"]))
        if bc == "unbounded" and (nd < 3 or rng.random() < 0.7):
            grid = "staggered"
        prec = str(rng.choice(["f32", "f64"]))
        ncomp, diff, inhom = 1, "none", False
        if bc in ("dirichlet", "neumann"):
            kernel = str(rng.choice(["ps", "fd2"]))
            inhom = kernel == "fd2" and bool(rng.random() < 0.5)
        elif bc == "periodic":
            kernel = str(rng.choice(["ps", "fd2"]))
        else:
            kernel = str(rng.choice(["g2", "g4", "g6", "g8", "g10", "spectral"]))
        if bc in ("periodic", "unbounded"):
            choices = ["none", "grad", "nabla"]
            if nd == 2:
                choices.append("curl")
            if nd == 3:
                choices += ["curl", "div"]
            diff = str(rng.choice(choices))
            if nd == 3 and diff in ("curl", "div"):
                ncomp = 3
            elif nd == 3 and diff == "nabla" and rng.random() < 0.5:
                ncomp = 3
        hi_n = {1: 300, 2: 64, 3: 28}[nd]
        nc = [_cells(rng, bc, grid, 2, hi_n) for _ in range(nd)]
        seed = int(rng.integers(0, 1 << 30))
        if bc in ("dirichlet", "neumann") and not inhom and seed % 2 == 0:
            diff = "grad"  # homogeneous Dirichlet / Neumann gradient (no extra draw)
        out.append((bc, grid, nc, kernel, diff, ncomp, inhom, prec, seed))
    return out


CASES = _cases(int(os.environ.get("HP_SWEEP_CASES", "120")), seed=int(os.environ.get("HP_SWEEP_SEED", "2023")))


@pytest.mark.parametrize("bc,grid,nc,kernel,diff,ncomp,inhom,prec,seed", CASES)
def test_sweep(bc, grid, nc, kernel, diff, ncomp, inhom, prec, seed):
    nd = len(nc)
    print(f"sweep {bc} {grid} {nc} {kernel} {diff} ncomp={ncomp} inhom={inhom} {prec}", flush=True)
    f, faces = case_input(bc, grid, nc, ncomp, inhom, prec, seed=seed % 100000)
    got, gd = gpu_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, prec, ncomp, faces)
    ref, rd = oracle_solve(bc, grid, nc, LO[:nd], HI[:nd], f, kernel, diff, faces)
    l2, mx = TOL[prec]
    assert rel_l2(got, ref) <= l2 and rel_max(got, ref) <= mx, (rel_l2(got, ref), rel_max(got, ref))
    assert len(gd) == len(rd)
    for a in range(len(rd)):
        scale = 1.0
        if diff == "nabla" and prec == "f64" and bc == "unbounded" and nd < 3:
            # derived bounds for 1D / 2D Laplacians (growing kernels; amplification
            # of the FP64 rounding by k^2, laplacian_rounding_tol)
            hs = [(HI[b] - LO[b]) / nc[b] for b in range(nd)]
            doubled = [2 * og.unknowns(bc, grid, n) for n in nc]
            scale = max(1.0, (max(nc) / 128.0) ** 2,
                        laplacian_rounding_tol(ref, rd[a], hs, doubled) / l2)  # scalar source in 1D / 2D
        assert rel_l2(gd[a], rd[a]) <= l2 * scale and rel_max(gd[a], rd[a]) <= mx * scale, (
            a, rel_l2(gd[a], rd[a]), rel_max(gd[a], rd[a]))
