"""Pins of the oracle's semi-unbounded solve (oracle.bounded.solve_semi): one
free axis, the others periodic, Dirichlet or Neumann.

What pins what:
  * FD2: a dense matrix-function solve that uses neither the sine / cosine /
    Fourier transforms nor the doubling: with A the dense FD2 matrix of the
    bounded axes (ghost points eliminated by the boundary rules), every pair of
    free-axis points is coupled by H_u G(|x_u - x_u'|) evaluated as a function of
    A through its eigendecomposition, G = -exp(-sqrt(-A) |x|) / (2 sqrt(-A))
    (|x| / 2 on the null space).
  * PS: products of a bounded-axis eigenfunction and any profile along the free
    axis equal the eigenfunction times the direct 1D sum of that profile
    against the Green's function of kappa^2 = -(eigenvalue sum).
  * The Green's function itself: it solves psi'' - kappa^2 psi = delta
    (a Gaussian source of width s has a closed-form solution with erfc, which
    the solve reaches at O(H^2) on the free axis).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import bounded, grid

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]


def fd2_matrix_1d(bc, gtype, n, h):
    """1D FD2 Laplacian on the unknowns with the homogeneous boundary rule
    eliminated (the ghost equations of the dense model, written per BC)."""
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = -2.0
        if i > 0:
            A[i, i - 1] = 1.0
        if i < n - 1:
            A[i, i + 1] = 1.0
    if bc == "periodic":
        A[0, n - 1] += 1.0
        A[n - 1, 0] += 1.0
    elif bc == "dirichlet" and gtype == "staggered":
        A[0, 0] -= 1.0  # ghost = -psi_0
        A[n - 1, n - 1] -= 1.0
    elif bc == "neumann" and gtype == "regular":
        A[0, 1] += 1.0  # ghost = psi_1
        A[n - 1, n - 2] += 1.0
    elif bc == "neumann":
        A[0, 0] += 1.0  # ghost = psi_0
        A[n - 1, n - 1] += 1.0
    return A / (h * h)


def dense_semi_fd2(f, bcs, gtype, hs):
    nd = f.ndim
    u = bcs.index("unbounded")
    bounded_axes = [a for a in range(nd) if a != u]
    # Kronecker sum of the bounded axes' matrices, in the array order of those axes
    mats = [fd2_matrix_1d(bcs[a], gtype, f.shape[a], hs[a]) for a in bounded_axes]
    A = mats[0]
    for m in mats[1:]:
        A = np.kron(A, np.eye(m.shape[0])) + np.kron(np.eye(A.shape[0]), m)
    w, V = np.linalg.eig(A)
    w = w.real
    Vi = np.linalg.inv(V)
    kappa = np.sqrt(np.maximum(-w, 0.0))
    zero = np.abs(w) < 1e-9 * np.max(np.abs(w))
    n = f.shape[u]
    xu = (np.arange(n)) * hs[u]
    # rows: bounded modes flattened; f moved to [bounded..., u]
    fb = np.moveaxis(f, u, -1).reshape(-1, n)
    c = Vi @ fb  # coefficients per eigenvector
    out = np.zeros_like(c, dtype=np.complex128)
    for i in range(n):
        d = np.abs(xu[i] - xu)
        G = np.where(zero[:, None], 0.5 * d[None, :],
                     -np.exp(-np.where(zero, 1.0, kappa)[:, None] * d[None, :]) /
                     (2.0 * np.where(zero, 1.0, kappa)[:, None]))
        out[:, i] = hs[u] * np.sum(G * c, axis=1)
    psi = (V @ out).real
    shape_b = [f.shape[a] for a in bounded_axes]
    return np.moveaxis(psi.reshape(shape_b + [n]), -1, u)


SEMI = [["unbounded", "periodic"], ["dirichlet", "unbounded"], ["unbounded", "neumann"],
        ["periodic", "unbounded", "dirichlet"], ["unbounded", "neumann", "periodic"],
        ["neumann", "dirichlet", "unbounded"]]


@pytest.mark.parametrize("bcs", SEMI)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
def test_semi_fd2_matches_dense_matrix_function(bcs, gtype):
    nd = len(bcs)
    nc = [7, 6, 5][:nd]
    lo, hi = LO[:nd], HI[:nd]
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    shape = tuple(grid.unknowns(bcs[a], gtype, nc[a]) for a in range(nd))
    f = np.random.default_rng(5 + nd).normal(size=shape)
    psi, _ = oracle.solve(bcs, gtype, nc, lo, hi, f, operator="fd2")
    ref = dense_semi_fd2(f, bcs, gtype, hs)
    if "dirichlet" in bcs and gtype == "regular":
        d = bcs.index("dirichlet")
        psi = np.take(psi, np.arange(1, psi.shape[d] - 1), axis=d)
    assert psi.shape == ref.shape
    assert np.max(np.abs(psi - ref)) <= 1e-11 * np.max(np.abs(ref))


def _eigenfunction(bc, m, x, lo, length):
    t = (x - lo) / length
    if bc == "dirichlet":
        return np.sin(np.pi * m * t), -(np.pi * m / length) ** 2
    if bc == "neumann":
        return np.cos(np.pi * m * t), -(np.pi * m / length) ** 2
    return np.cos(2 * np.pi * m * t + 0.7), -(2 * np.pi * m / length) ** 2


@pytest.mark.parametrize("bcs", SEMI)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("zero_mode", [False, True])
def test_semi_ps_eigenfunction_times_direct_sum(bcs, gtype, zero_mode):
    if zero_mode and "dirichlet" in bcs:
        pytest.skip("no zero eigenvalue with a Dirichlet axis")
    nd = len(bcs)
    u = bcs.index("unbounded")
    nc = [12, 10, 9][:nd]
    lo, hi = LO[:nd], HI[:nd]
    xs_out = [grid.positions(bcs[a], gtype, lo[a], hi[a], nc[a]) for a in range(nd)]
    xs_in = [x[1:-1] if (bcs[a] == "dirichlet" and gtype == "regular") else x for a, x in enumerate(xs_out)]
    rng = np.random.default_rng(17)
    prof = rng.normal(size=len(xs_in[u]))  # any profile along the free axis
    f_in = np.ones([len(x) for x in xs_in])
    f_out = np.ones([len(x) if a != u else 1 for a, x in enumerate(xs_out)])
    lam = 0.0
    for a in range(nd):
        view = [1] * nd
        view[a] = -1
        if a == u:
            f_in = f_in * prof.reshape(view)
            continue
        m = 0 if zero_mode else 1 + a % 2
        vi, la = _eigenfunction(bcs[a], m, xs_in[a], lo[a], hi[a] - lo[a])
        vo, _ = _eigenfunction(bcs[a], m, xs_out[a], lo[a], hi[a] - lo[a])
        f_in = f_in * vi.reshape(view)
        f_out = f_out * vo.reshape(view)
        lam += la
    kappa = math.sqrt(-lam)
    xu = xs_in[u]
    hu = grid.spacing(lo[u], hi[u], nc[u])
    conv = np.array([hu * np.sum(bounded.helmholtz_kernel_1d(kappa, xu[i] - xu) * prof)
                     for i in range(len(xu))])
    view = [1] * nd
    view[u] = -1
    ref = f_out * conv.reshape(view)
    psi, _ = oracle.solve(bcs, gtype, nc, lo, hi, f_in, operator="ps")
    assert psi.shape == ref.shape
    assert np.max(np.abs(psi - ref)) <= 1e-12 * np.max(np.abs(ref))


def gaussian_helmholtz(x, kappa, s):
    """Solution of u'' - kappa^2 u = exp(-x^2 / (2 s^2)) on the line."""
    c = s * math.sqrt(math.pi / 2.0) * math.exp(kappa * kappa * s * s / 2.0)
    t1 = np.exp(-kappa * x) * special.erfc((kappa * s * s - x) / (s * math.sqrt(2.0)))
    t2 = np.exp(kappa * x) * special.erfc((kappa * s * s + x) / (s * math.sqrt(2.0)))
    return -c * (t1 + t2) / (2.0 * kappa)


def test_gaussian_closed_form_is_the_green_convolution():
    kappa, s = math.pi, 0.1
    for x in (-0.3, 0.0, 0.17):
        quad, _ = integrate.quad(lambda t: -math.exp(-kappa * abs(x - t)) / (2 * kappa) *
                                 math.exp(-t * t / (2 * s * s)), -2, 2, points=[x], limit=200)
        assert abs(quad - gaussian_helmholtz(np.array(x), kappa, s)) <= 1e-10


@pytest.mark.parametrize("other", ["dirichlet", "periodic"])
def test_semi_second_order_along_the_free_axis(other):
    # f = sin(pi y) exp(-x^2 / 2 s^2) (periodic: cos(2 pi y)) on x in [-1, 1] free
    s = 0.12
    errs = []
    for n in (32, 64, 128):
        nc = [n, 8]
        lo, hi = [-1.0, 0.0], [1.0, 1.0]
        x = grid.positions("unbounded", "staggered", lo[0], hi[0], n)
        y = grid.positions(other, "staggered", lo[1], hi[1], 8)
        fy, lam = _eigenfunction(other, 1, y, 0.0, 1.0)
        f = np.exp(-x[:, None] ** 2 / (2 * s * s)) * fy[None, :]
        psi, _ = oracle.solve(["unbounded", other], "staggered", nc, lo, hi, f, operator="ps")
        ref = gaussian_helmholtz(x, math.sqrt(-lam), s)[:, None] * fy[None, :]
        errs.append(np.max(np.abs(psi - ref)) / np.max(np.abs(ref)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[2] < 5e-3


@pytest.mark.parametrize("bcs", SEMI)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
def test_semi_gradient_eigenfunction_times_direct_sums(bcs, gtype):
    # psi = phi_B(x_B) conv(x_u): d/dx_b psi = phi_B' conv, d/dx_u psi = phi_B conv'
    # with conv' the direct sum of the profile against G' (0 at distance 0);
    # every eigenvalue here is nonzero, so kappa > 0
    nd = len(bcs)
    u = bcs.index("unbounded")
    nc = [12, 10, 9][:nd]
    lo, hi = LO[:nd], HI[:nd]
    xs_out = [grid.positions(bcs[a], gtype, lo[a], hi[a], nc[a]) for a in range(nd)]
    xs_in = [x[1:-1] if (bcs[a] == "dirichlet" and gtype == "regular") else x for a, x in enumerate(xs_out)]
    prof = np.random.default_rng(19).normal(size=len(xs_in[u]))
    f_in = np.ones([len(x) for x in xs_in])
    facs, dfacs = [], []
    lam = 0.0
    for a in range(nd):
        view = [1] * nd
        view[a] = -1
        if a == u:
            f_in = f_in * prof.reshape(view)
            facs.append(None)
            dfacs.append(None)
            continue
        m = 1 + a % 2
        vi, la = _eigenfunction(bcs[a], m, xs_in[a], lo[a], hi[a] - lo[a])
        f_in = f_in * vi.reshape(view)
        t = (xs_out[a] - lo[a]) / (hi[a] - lo[a])
        L = hi[a] - lo[a]
        if bcs[a] == "dirichlet":
            v, dv = np.sin(np.pi * m * t), np.pi * m / L * np.cos(np.pi * m * t)
        elif bcs[a] == "neumann":
            v, dv = np.cos(np.pi * m * t), -np.pi * m / L * np.sin(np.pi * m * t)
        else:
            v, dv = np.cos(2 * np.pi * m * t + 0.7), -2 * np.pi * m / L * np.sin(2 * np.pi * m * t + 0.7)
        facs.append(v.reshape(view))
        dfacs.append(dv.reshape(view))
        lam += la
    kappa = math.sqrt(-lam)
    xu = xs_in[u]
    hu = grid.spacing(lo[u], hi[u], nc[u])
    conv = np.array([hu * np.sum(bounded.helmholtz_kernel_1d(kappa, xu[i] - xu) * prof) for i in range(len(xu))])
    # G'(x) = -kappa sign(x) G(x) for kappa > 0, from the pinned kernel itself
    dconv = np.array([hu * np.sum(-kappa * np.sign(xu[i] - xu) * bounded.helmholtz_kernel_1d(kappa, xu[i] - xu) * prof)
                      for i in range(len(xu))])
    view = [1] * nd
    view[u] = -1
    _, der = oracle.solve(bcs, gtype, nc, lo, hi, f_in, operator="ps", diff="grad")
    for g in range(nd):
        ref = (dconv if g == u else conv).reshape(view) * 1.0
        for a in range(nd):
            if a != u:
                ref = ref * (dfacs[a] if a == g else facs[a])
        assert der[g].shape == ref.shape
        assert np.max(np.abs(der[g] - ref)) <= 1e-11 * np.max(np.abs(ref)), g


@pytest.mark.parametrize("other", ["dirichlet", "periodic"])
def test_semi_free_derivative_second_order(other):
    # d/dx of the Gaussian-profile solution, against quadrature of G' * g
    s = 0.12
    errs = []
    for n in (32, 64, 128):
        nc = [n, 8]
        lo, hi = [-1.0, 0.0], [1.0, 1.0]
        x = grid.positions("unbounded", "staggered", lo[0], hi[0], n)
        y = grid.positions(other, "staggered", lo[1], hi[1], 8)
        fy, lam = _eigenfunction(other, 1, y, 0.0, 1.0)
        kappa = math.sqrt(-lam)
        f = np.exp(-x[:, None] ** 2 / (2 * s * s)) * fy[None, :]
        _, der = oracle.solve(["unbounded", other], "staggered", nc, lo, hi, f, operator="ps", diff="grad")
        ref = np.array([integrate.quad(lambda t: 0.5 * math.copysign(1.0, xi - t) * math.exp(-kappa * abs(xi - t))
                                       * math.exp(-t * t / (2 * s * s)), -1.5, 1.5, points=[xi], limit=200)[0]
                        for xi in x])[:, None] * fy[None, :]
        errs.append(np.max(np.abs(der[0] - ref)) / np.max(np.abs(ref)))
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs
