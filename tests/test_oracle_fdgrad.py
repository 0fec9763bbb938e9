"""Pins of the oracle's derivatives with inhomogeneous boundary values
(oracle.bounded.fd_derivative: centred FD2 differences closed by the ghost
rules of the boundary weighting).

What pins what:
  * The paraboloid of eq. (tfih1D), which the FD2 solve reproduces exactly on
    REGULAR Dirichlet and both Neumann grids: GRAD of the solve equals
    eq. (tfih1Dgrad) at every output point, boundary nodes included; CURL and
    DIV of a vector of such paraboloids equal their closed forms.
  * A quadratic on the STAGGERED Dirichlet grid with its face values: the
    derivative is exact (the one-sided closure is the quadratic's derivative).
  * Second-order convergence for a smooth non-polynomial field, every BC x
    grid, with face values taken from the field; and of GRAD through the whole
    FD2 solve of a manufactured solution (first order on STAGGERED Dirichlet,
    whose solve uses the linear ghost of the boundary weighting).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import bounded, grid

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]


def parab(x, L, a, b):
    t = x / L
    return a * (1 - t) ** 2 + b * t ** 2


def parab_grad(x, L, a, b):
    t = x / L
    return (2 * a * (t - 1) + 2 * b * t) / L  # eq. (tfih1Dgrad) divided by L (reading R8)


def paraboloid_case(bc, gtype, nc, consts):
    nd = len(nc)
    lengths = [HI[a] - LO[a] for a in range(nd)]
    xo = [grid.positions(bc, gtype, LO[a], HI[a], nc[a]) - LO[a] for a in range(nd)]
    xi = [x[1:-1] if (bc == "dirichlet" and gtype == "regular") else x for x in xo]
    shape_in = tuple(len(x) for x in xi)
    f = np.full(shape_in, sum(2.0 * (consts[a][0] + consts[a][1]) / lengths[a] ** 2 for a in range(nd)))
    mesh = np.meshgrid(*xo, indexing="ij")
    psi = sum(parab(mesh[a], lengths[a], *consts[a]) for a in range(nd))
    grads = [parab_grad(mesh[a], lengths[a], *consts[a]) for a in range(nd)]
    faces = {}
    for a in range(nd):
        for side in (0, 1):
            idx = [slice(None)] * nd
            idx[a] = 0 if side == 0 else -1
            src = psi if bc == "dirichlet" else grads[a]
            if gtype == "regular":  # the boundary nodes lie on the face
                faces[(a, side)] = src[tuple(idx)]
            else:  # STAGGERED: psi (Dirichlet) or d psi / d x_a (Neumann) on the face itself
                xs = [x for x in xo]
                xs[a] = np.array([0.0 if side == 0 else lengths[a]])
                m = np.meshgrid(*xs, indexing="ij")
                if bc == "dirichlet":
                    val = sum(parab(m[b], lengths[b], *consts[b]) for b in range(nd))
                else:
                    val = parab_grad(m[a], lengths[a], *consts[a]) + 0.0 * m[0]
                faces[(a, side)] = val.squeeze(axis=a)
    return f, faces, psi, grads


@pytest.mark.parametrize("bc,gtype", [("dirichlet", "regular"), ("neumann", "regular"), ("neumann", "staggered")])
@pytest.mark.parametrize("nd", [1, 2, 3])
def test_paraboloid_gradient_is_tfih1dgrad(bc, gtype, nd):
    nc = [9, 8, 7][:nd]
    consts = [(0.7, -1.3), (2.1, 0.4), (-0.6, 1.1)][:nd]
    f, faces, psi_ex, grads = paraboloid_case(bc, gtype, nc, consts)
    psi, der = oracle.solve(bc, gtype, nc, LO[:nd], HI[:nd], f, operator="fd2", diff="grad", faces=faces)
    scale = max(np.max(np.abs(g)) for g in grads)
    for a in range(nd):
        assert np.max(np.abs(der[a] - grads[a])) <= 1e-10 * scale, a


@pytest.mark.parametrize("bc,gtype", [("dirichlet", "regular"), ("neumann", "regular"), ("neumann", "staggered")])
def test_paraboloid_curl_and_div(bc, gtype):
    nc = [7, 6, 5]
    comps = [[(0.7, -1.3), (2.1, 0.4), (-0.6, 1.1)], [(0.2, 0.9), (-1.0, 0.3), (0.5, 0.5)],
             [(1.4, -0.2), (0.8, 1.9), (-0.3, -0.7)]]
    fs, faces, grads = [], [], []
    for c in range(3):
        f, fc, _, g = paraboloid_case(bc, gtype, nc, comps[c])
        fs.append(f)
        faces.append(fc)
        grads.append(g)
    f = np.stack(fs)
    _, curl = oracle.solve(bc, gtype, nc, LO, HI, f, operator="fd2", diff="curl", faces=faces)
    _, div = oracle.solve(bc, gtype, nc, LO, HI, f, operator="fd2", diff="div", faces=faces)
    g = grads
    ref_curl = [g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]]
    scale = max(np.max(np.abs(x)) for x in ref_curl)
    for c in range(3):
        assert np.max(np.abs(curl[c] - ref_curl[c])) <= 1e-10 * scale, c
    ref_div = g[0][0] + g[1][1] + g[2][2]
    assert np.max(np.abs(div[0] - ref_div)) <= 1e-10 * np.max(np.abs(ref_div))


def test_dirichlet_staggered_quadratic_is_exact():
    L, n = 1.3, 11
    h = L / n
    x = (np.arange(n) + 0.5) * h
    psi = 0.4 + 2.5 * x - 1.7 * x * x
    d = bounded.fd_derivative(psi, "dirichlet", "staggered", h, 0, 0.4, 0.4 + 2.5 * L - 1.7 * L * L)
    assert np.max(np.abs(d - (2.5 - 3.4 * x))) <= 1e-12


@pytest.mark.parametrize("bc,gtype", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                      ("neumann", "regular"), ("neumann", "staggered")])
def test_fd_derivative_second_order(bc, gtype):
    errs = []
    for nc in (16, 32, 64):
        L = 1.0
        x = grid.positions(bc, gtype, 0.0, L, nc)
        u = np.sin(2.3 * x) + 0.3 * np.cos(5.1 * x)
        du = 2.3 * np.cos(2.3 * x) - 0.3 * 5.1 * np.sin(5.1 * x)
        f = lambda t: math.sin(2.3 * t) + 0.3 * math.cos(5.1 * t)
        df = lambda t: 2.3 * math.cos(2.3 * t) - 0.3 * 5.1 * math.sin(5.1 * t)
        lo, hi = (f(0.0), f(L)) if bc == "dirichlet" else (df(0.0), df(L))
        h = grid.spacing(0.0, L, nc)
        d = bounded.fd_derivative(u, bc, gtype, h, 0, lo, hi)
        errs.append(np.max(np.abs(d - du)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


@pytest.mark.parametrize("bc,gtype", [("dirichlet", "regular"), ("dirichlet", "staggered"),
                                      ("neumann", "regular"), ("neumann", "staggered")])
def test_solve_gradient_second_order(bc, gtype):
    # psi = sin(1.7 x + 0.3) cos(1.1 y) + the eq. (tfih1D) paraboloid in x; f = lap psi,
    # face values from psi: GRAD of the FD2 solve converges at O(H^2) (O(H) on
    # STAGGERED Dirichlet)
    def psi_f(x, y):
        return np.sin(1.7 * x + 0.3) * np.cos(1.1 * y) + parab(x, 1.0, 0.6, -0.9)

    def grad_f(x, y):
        return (1.7 * np.cos(1.7 * x + 0.3) * np.cos(1.1 * y) + parab_grad(x, 1.0, 0.6, -0.9),
                -1.1 * np.sin(1.7 * x + 0.3) * np.sin(1.1 * y))

    def lap_f(x, y):
        return -(1.7 ** 2 + 1.1 ** 2) * np.sin(1.7 * x + 0.3) * np.cos(1.1 * y) + 2.0 * (0.6 - 0.9)

    errs = []
    for n in (16, 32, 64):
        nc = [n, n]
        lo, hi = [0.0, 0.0], [1.0, 1.0]
        xo = [grid.positions(bc, gtype, lo[a], hi[a], nc[a]) for a in range(2)]
        xi = [x[1:-1] if (bc == "dirichlet" and gtype == "regular") else x for x in xo]
        X, Y = np.meshgrid(*xi, indexing="ij")
        f = lap_f(X, Y)
        faces = {}
        for a in range(2):
            for side in (0, 1):
                pos = [xo[0], xo[1]]
                pos[a] = np.array([lo[a] if side == 0 else hi[a]])
                PX, PY = np.meshgrid(*pos, indexing="ij")
                val = psi_f(PX, PY) if bc == "dirichlet" else grad_f(PX, PY)[a]
                faces[(a, side)] = val.squeeze(axis=a)
        _, der = oracle.solve(bc, gtype, nc, lo, hi, f, operator="fd2", diff="grad", faces=faces)
        XO, YO = np.meshgrid(*xo, indexing="ij")
        ref = grad_f(XO, YO)
        errs.append(max(np.max(np.abs(der[a] - ref[a])) for a in range(2)))
    # STAGGERED Dirichlet: the solve's linear ghost (2 g - psi_0, R4) leaves an
    # O(H) slope error in the first cells, which the gradient shows in the max
    # norm; the other grids are second order to the faces
    rate = 1.8 if (bc == "dirichlet" and gtype == "staggered") else 3.3
    assert errs[0] / errs[1] > rate and errs[1] / errs[2] > rate, errs


def test_periodic_axis_difference_closed_form():
    # the wrapped centred difference of sin(k x) is k cos(k x) sin(k H) / (k H)
    L, n = 1.7, 24
    h = L / n
    x = np.arange(n) * h
    k = 2 * np.pi * 3 / L
    d = bounded.fd_derivative(np.sin(k * x), "periodic", "regular", h, 0)
    assert np.max(np.abs(d - k * np.cos(k * x) * np.sin(k * h) / (k * h))) <= 1e-12


def test_mixed_boundary_values_gradient_second_order():
    # a periodic x axis beside a Neumann y axis with boundary values: GRAD of the
    # FD2 solve of psi = cos(2 pi x + 0.2) * (y^2 - y / 3) + sin(4 pi x) converges at O(H^2)
    def psi_f(x, y):
        return np.cos(2 * np.pi * x + 0.2) * (y * y - y / 3) + np.sin(4 * np.pi * x)

    def grad_f(x, y):
        return (-2 * np.pi * np.sin(2 * np.pi * x + 0.2) * (y * y - y / 3) + 4 * np.pi * np.cos(4 * np.pi * x),
                np.cos(2 * np.pi * x + 0.2) * (2 * y - 1 / 3))

    def lap_f(x, y):
        return (-(2 * np.pi) ** 2 * np.cos(2 * np.pi * x + 0.2) * (y * y - y / 3) + 2 * np.cos(2 * np.pi * x + 0.2)
                - (4 * np.pi) ** 2 * np.sin(4 * np.pi * x))

    errs = []
    bcs = ["periodic", "neumann"]
    for n in (16, 32, 64):
        nc, lo, hi = [n, n], [0.0, 0.0], [1.0, 1.0]
        xo = [grid.positions(bcs[a], "staggered", lo[a], hi[a], nc[a]) for a in range(2)]
        X, Y = np.meshgrid(*xo, indexing="ij")
        faces = {}
        for side in (0, 1):
            yv = np.array([lo[1] if side == 0 else hi[1]])
            PX, PY = np.meshgrid(xo[0], yv, indexing="ij")
            faces[(1, side)] = grad_f(PX, PY)[1].squeeze(axis=1)
        _, der = oracle.solve(bcs, "staggered", nc, lo, hi, lap_f(X, Y), operator="fd2", diff="grad", faces=faces)
        ref = grad_f(X, Y)
        errs.append(max(np.max(np.abs(der[a] - ref[a])) for a in range(2)))
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs
