"""Pins of the oracle's bounded solves (oracle.bounded).

What pins what:
  * FD2 solves (homogeneous and inhomogeneous, every BC x grid, 1D/2D/3D) are
    compared with a dense linear solve of the finite-difference equations
    written on a grid extended by one ghost / boundary layer per face, with the
    boundary condition stated as its own equation (no elimination by hand).
    The null space of periodic / Neumann problems is fixed by the same
    constraint the zero-mode rule implies (weighted mean of psi = 0), and the
    incompatible part of the source is an extra unknown constant.
  * Table 1 FD2 eigenvalues are the eigenvalues of the dense 1D FD matrix.
  * PS solves of the products of eq. (tfb) are the closed forms (exact).
  * The quadratic of eq. (tfih1D) is reproduced exactly by FD2 for REGULAR
    Dirichlet and both Neumann grids (Section 4.2).
  * FD2 converges at O(H^2) (Fig. BS / Fig. IH claims).
  * The Dirichlet / Neumann gradient of a product of eigenfunctions (PS and
    FD2, one mode per axis, the top modes included) is the analytic
    derivative of the closed-form psi, boundary nodes included.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import bounded, grid

CASES = [("dirichlet", "regular"), ("dirichlet", "staggered"),
         ("neumann", "regular"), ("neumann", "staggered"), ("periodic", "staggered"),
         ("periodic", "regular")]


# --------------------------------------------------------------- dense FD model
def dense_fd_solve(f, bc, gtype, hs, faces, return_constant=False):
    """Solve the FD2 equations directly on an extended grid (test-side model).
    Periodic and Neumann systems carry one more unknown, the constant removed
    from the source (returned as well with return_constant=True)."""
    shape = f.shape
    nd = len(shape)
    periodic = bc == "periodic"
    ext = shape if periodic else tuple(n + 2 for n in shape)
    off = 0 if periodic else 1
    idx = {p: i for i, p in enumerate(itertools.product(*[range(e) for e in ext]))}
    nvar = len(idx)
    singular = bc in ("periodic", "neumann")
    size = nvar + (1 if singular else 0)
    A = np.zeros((size, size))
    b = np.zeros(size)

    def is_inner(p):
        return all(off <= p[a] < off + shape[a] for a in range(nd))

    for p, i in idx.items():
        if is_inner(p):
            for a in range(nd):
                for s in (-1, 1):
                    q = list(p)
                    q[a] = (q[a] + s) % ext[a] if periodic else q[a] + s
                    A[i, idx[tuple(q)]] += 1.0 / hs[a] ** 2
                A[i, i] -= 2.0 / hs[a] ** 2
            b[i] = f[tuple(p[a] - off for a in range(nd))]
            if singular:
                A[i, nvar] = 1.0  # unknown constant removed from the source
            continue
        ghost_axes = [a for a in range(nd) if not (off <= p[a] < off + shape[a])]
        if len(ghost_axes) > 1:
            # edge / corner of the extended grid: not in any stencil
            if bc == "dirichlet" and gtype == "regular":
                a = max(ghost_axes)
                side = 0 if p[a] == 0 else 1
                g = faces.get((a, side)) if faces else None
                others = [d for d in range(nd) if d != a]
                A[i, i] = 1.0
                b[i] = 0.0 if g is None else g[tuple(p[d] for d in others)]
            else:
                A[i, i] = 1.0
            continue
        a = ghost_axes[0]
        side = 0 if p[a] == 0 else 1
        others = [d for d in range(nd) if d != a]
        g = faces.get((a, side)) if faces else None
        if g is None:
            gv = 0.0
        elif bc == "dirichlet" and gtype == "regular":
            gv = g[tuple(p[d] for d in others)]
        else:
            gv = g[tuple(p[d] - 1 for d in others)]
        h = hs[a]
        inward = list(p)
        inward[a] = 1 if side == 0 else shape[a]
        inward2 = list(p)
        inward2[a] = 2 if side == 0 else shape[a] - 1
        i1, i2 = idx[tuple(inward)], idx[tuple(inward2)]
        if bc == "dirichlet" and gtype == "regular":
            A[i, i] = 1.0
        elif bc == "dirichlet":
            A[i, i] = 0.5
            A[i, i1] = 0.5
        elif bc == "neumann" and gtype == "regular":
            # (psi_{+1} - psi_{-1}) / (2H) = g along +x_a
            if side == 0:
                A[i, i2] = 1.0 / (2 * h)
                A[i, i] = -1.0 / (2 * h)
            else:
                A[i, i] = 1.0 / (2 * h)
                A[i, i2] = -1.0 / (2 * h)
        else:
            # (psi_inside - psi_ghost) / H on the lower face, reversed above
            if side == 0:
                A[i, i1] = 1.0 / h
                A[i, i] = -1.0 / h
            else:
                A[i, i] = 1.0 / h
                A[i, i1] = -1.0 / h
        b[i] = gv
    if singular:
        # weighted mean of psi over the unknowns is zero: trapezoid weights for
        # REGULAR Neumann (DCT-I zero mode), plain sum otherwise
        for p, i in idx.items():
            if is_inner(p):
                w = 1.0
                if bc == "neumann" and gtype == "regular":
                    for a in range(nd):
                        if p[a] in (off, off + shape[a] - 1):
                            w *= 0.5
                A[nvar, i] = w
    sol_all = np.linalg.solve(A, b)
    sol = sol_all[:nvar]
    const = float(sol_all[nvar]) if singular else 0.0
    full = np.zeros(ext)
    for p, i in idx.items():
        full[p] = sol[i]
    if bc == "dirichlet" and gtype == "regular":
        out = full
    elif periodic:
        out = full
    else:
        out = full[tuple(slice(1, 1 + n) for n in shape)]
    return (out, const) if return_constant else out


def random_faces(bc, gtype, nc, nd, rng):
    faces = {}
    for a in range(nd):
        for s in (0, 1):
            shp = tuple(grid.output_points(bc, gtype, nc[d]) for d in range(nd) if d != a)
            faces[(a, s)] = rng.normal(size=shp)
    return faces


@pytest.mark.parametrize("bc,gtype", CASES)
@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("inhom", [False, True])
def test_fd2_matches_dense_solve(bc, gtype, nd, inhom):
    if inhom and bc == "periodic":
        pytest.skip("periodic has no boundary values")
    rng = np.random.default_rng(nd * 10 + inhom)
    nc = [7, 6, 5][:nd]
    lo = [0.0, -0.5, 1.0][:nd]
    hi = [1.0, 1.3, 2.5][:nd]
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    shape = tuple(grid.unknowns(bc, gtype, nc[a]) for a in range(nd))
    f = rng.normal(size=shape)
    faces = random_faces(bc, gtype, nc, nd, rng) if inhom else None
    psi, _ = oracle.solve(bc, gtype, nc, lo, hi, f, operator="fd2", faces=faces)
    ref = dense_fd_solve(f, bc, gtype, hs, faces or {})
    assert psi.shape == ref.shape
    assert np.max(np.abs(psi - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc,gtype", CASES)
def test_fd2_eigenvalues_match_dense_matrix(bc, gtype):
    nc, L = 9, 2.0
    h = L / nc
    n = grid.unknowns(bc, gtype, nc)
    # columns of the dense FD operator from unit sources on the homogeneous model
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        # apply the operator by finite differences with the ghost rules
        ext = np.zeros(n + 2)
        ext[1:-1] = e
        if bc == "periodic":
            ext[0], ext[-1] = e[-1], e[0]
        elif bc == "dirichlet" and gtype == "regular":
            ext[0] = ext[-1] = 0.0
        elif bc == "dirichlet":
            ext[0], ext[-1] = -e[0], -e[-1]
        elif gtype == "regular":
            ext[0], ext[-1] = e[1], e[-2]
        else:
            ext[0], ext[-1] = e[0], e[-1]
        M[:, j] = (ext[:-2] - 2 * ext[1:-1] + ext[2:]) / h**2
    ev = np.sort(np.linalg.eigvals(M).real)
    lam = np.sort(bounded.eigenvalues(bc, gtype, "fd2", n, L, h))
    assert np.allclose(ev, lam, atol=1e-10 * np.max(np.abs(lam)))


def s_fn(x, L):
    return np.sin(4 * np.pi * x / L)


def c_fn(x, L):
    return np.cos(4 * np.pi * x / L)


@pytest.mark.parametrize("bc,gtype", CASES)
@pytest.mark.parametrize("nd", [1, 2, 3])
def test_ps_closed_form(bc, gtype, nd):
    """eq. (tfb)/(tfb3D): psi = -f / ((4 pi)^2 sum_a L_a^-2) (read as in the
    dimensionally consistent form; the printed prefactor is garbled)."""
    nc = [12, 10, 8][:nd]
    lo = [0.0, 1.0, -2.0][:nd]
    hi = [1.0, 3.0, 1.0][:nd]
    fn = s_fn if bc == "dirichlet" else c_fn
    f = 1.0
    psi_a = None
    lam = -(4 * np.pi) ** 2 * sum(1.0 / (hi[a] - lo[a]) ** 2 for a in range(nd))
    xs_unk = []
    xs_out = []
    for a in range(nd):
        x = grid.positions(bc, gtype, lo[a], hi[a], nc[a]) - lo[a]
        xs_out.append(x)
        if bc == "dirichlet" and gtype == "regular":
            x = x[1:-1]
        xs_unk.append(x)
    f = np.ones([len(x) for x in xs_unk])
    fo = np.ones([len(x) for x in xs_out])
    for a in range(nd):
        view = [1] * nd
        view[a] = -1
        f = f * fn(xs_unk[a], hi[a] - lo[a]).reshape(view)
        fo = fo * fn(xs_out[a], hi[a] - lo[a]).reshape(view)
    if bc == "periodic":
        # add a cross term so both sine and cosine modes are present
        view = [1] * nd
        view[0] = -1
        extra = s_fn(xs_unk[0], hi[0] - lo[0]).reshape(view) * np.ones_like(f)
        f = f + extra
        lam_extra = -(4 * np.pi / (hi[0] - lo[0])) ** 2
        psi_a = fo / lam + extra / lam_extra
    else:
        psi_a = fo / lam
    psi, _ = oracle.solve(bc, gtype, nc, lo, hi, f, operator="ps")
    assert np.max(np.abs(psi - psi_a)) <= 1e-13 * np.max(np.abs(psi_a))


def test_periodic_2d_modes_closed_form():
    """64 x 64 periodic PS source of random Fourier modes: exact per mode."""
    from workloads import periodic_modes_2d
    f, modes = periodic_modes_2d(64, seed=1)
    x = (np.arange(64) + 0.5) / 64
    X, Y = x[:, None], x[None, :]
    psi_a = np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) / (-8 * np.pi**2)
    for p, q, a, b in modes:
        ph = 2 * np.pi * (p * X + q * Y)
        psi_a = psi_a + (a * np.cos(ph) + b * np.sin(ph)) / (-4 * np.pi**2 * (p * p + q * q))
    psi, _ = oracle.solve("periodic", "staggered", [64, 64], [0, 0], [1, 1], f, operator="ps")
    err = np.linalg.norm(psi - psi_a) / np.linalg.norm(psi_a)
    assert err < 1e-14


@pytest.mark.parametrize("bc,gtype", [("dirichlet", "regular"), ("neumann", "regular"),
                                      ("neumann", "staggered")])
def test_inhomogeneous_quadratic_exact(bc, gtype):
    """eq. (tfih1D): the paraboloid sum is reproduced exactly by FD2."""
    nd = 3
    nc = [10, 8, 6]
    lo = [0.0, 0.0, 0.0]
    hi = [1.0, 2.0, 1.5]
    rng = np.random.default_rng(7)
    ab = rng.normal(size=(nd, 2))
    Ls = [hi[a] - lo[a] for a in range(nd)]

    def psi_fn(coords):
        out = 0.0
        for a in range(nd):
            t = coords[a] / Ls[a]
            out = out + ab[a, 0] * (1 - t) ** 2 + ab[a, 1] * t ** 2
        return out

    fval = sum(2.0 * (ab[a, 0] + ab[a, 1]) / Ls[a] ** 2 for a in range(nd))
    xs = [grid.positions(bc, gtype, lo[a], hi[a], nc[a]) for a in range(nd)]
    unk = [x[1:-1] if (bc == "dirichlet" and gtype == "regular") else x for x in xs]
    f = np.full([len(u) for u in unk], fval)
    faces = {}
    for a in range(nd):
        others = [d for d in range(nd) if d != a]
        mesh = np.meshgrid(*[xs[d] for d in others], indexing="ij")
        for s in (0, 1):
            xa = 0.0 if s == 0 else Ls[a]
            if bc == "dirichlet":
                coords = [None] * nd
                coords[a] = np.full_like(mesh[0], xa)
                for d, m in zip(others, mesh):
                    coords[d] = m
                faces[(a, s)] = psi_fn(coords)
            else:
                # d(psi)/dx_a on the face (eq. tfih1Dgrad with the 1/L factor)
                g = (2 * ab[a, 0] * (xa / Ls[a] - 1) + 2 * ab[a, 1] * xa / Ls[a]) / Ls[a]
                faces[(a, s)] = np.full(mesh[0].shape, g)
    psi, _ = oracle.solve(bc, gtype, nc, lo, hi, f, operator="fd2", faces=faces)
    Xs = np.meshgrid(*xs, indexing="ij")
    psi_a = psi_fn(Xs)
    if bc == "neumann":
        psi = psi - psi.mean()
        psi_a = psi_a - psi_a.mean()
    assert np.max(np.abs(psi - psi_a)) <= 1e-11 * np.max(np.abs(psi_a))


@pytest.mark.parametrize("bc,gtype", CASES[:5])
def test_fd2_second_order(bc, gtype):
    """FD2 error against the exact solution falls by ~4 per grid doubling."""
    errs = []
    for nc in (16, 32, 64):
        x = grid.positions(bc, gtype, 0.0, 1.0, nc)
        fn = s_fn if bc in ("dirichlet", "periodic") else c_fn
        psi_a = np.outer(fn(x, 1.0), fn(x, 1.0)) / (-(4 * np.pi) ** 2 * 2)
        xu = x[1:-1] if (bc == "dirichlet" and gtype == "regular") else x
        f = np.outer(fn(xu, 1.0), fn(xu, 1.0))
        psi, _ = oracle.solve(bc, gtype, [nc, nc], [0, 0], [1, 1], f, operator="fd2")
        errs.append(np.max(np.abs(psi - psi_a)) / np.max(np.abs(psi_a)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2


def test_dirichlet_staggered_inhomogeneous_second_order():
    """The linear ghost is second order (not exact) for the paraboloid + S."""
    errs = []
    for nc in (16, 32, 64):
        x = grid.positions("dirichlet", "staggered", 0.0, 1.0, nc)
        a, b = 0.7, -1.3

        def psi_fn(t):
            return a * (1 - t) ** 2 + b * t**2 + np.sin(4 * np.pi * t) / (-(4 * np.pi) ** 2)

        f = np.full(nc, 2.0 * (a + b)) + np.sin(4 * np.pi * x)
        faces = {(0, 0): np.array(psi_fn(0.0)), (0, 1): np.array(psi_fn(1.0))}
        psi, _ = oracle.solve("dirichlet", "staggered", [nc], [0], [1], f, operator="fd2", faces=faces)
        errs.append(np.max(np.abs(psi - psi_fn(x))))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_periodic_gradient_bandlimited():
    n, L = 16, 2.0
    x = grid.positions("periodic", "staggered", 0.0, L, n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    psi = np.sin(2 * np.pi * 3 * X / L) * np.cos(2 * np.pi * 2 * Y / L)
    gx, gy = bounded.periodic_gradient(psi, [L, L])
    ex = (2 * np.pi * 3 / L) * np.cos(2 * np.pi * 3 * X / L) * np.cos(2 * np.pi * 2 * Y / L)
    ey = -(2 * np.pi * 2 / L) * np.sin(2 * np.pi * 3 * X / L) * np.sin(2 * np.pi * 2 * Y / L)
    assert np.max(np.abs(gx - ex)) < 1e-12 and np.max(np.abs(gy - ey)) < 1e-12


def test_ps_inhomogeneous_rejected():
    with pytest.raises(ValueError):
        oracle.solve("dirichlet", "regular", [4], [0], [1], np.zeros(3), operator="ps",
                     faces={(0, 0): np.array(1.0)})


@pytest.mark.parametrize("bc,gtype", [("neumann", "regular"), ("neumann", "staggered"),
                                      ("periodic", "staggered"), ("periodic", "regular")])
@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("inhom", [False, True])
def test_zero_mode_is_the_removed_constant(bc, gtype, nd, inhom):
    """oracle.zero_mode equals the constant c of the dense FD2 model
    L_h psi + c = f (with the boundary values), the part of the source that no
    solution can match."""
    if inhom and bc == "periodic":
        pytest.skip("periodic has no boundary values")
    rng = np.random.default_rng(nd * 10 + inhom + 5)
    nc = [7, 6, 5][:nd]
    lo = [0.0, -0.5, 1.0][:nd]
    hi = [1.0, 1.3, 2.5][:nd]
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    shape = tuple(grid.unknowns(bc, gtype, nc[a]) for a in range(nd))
    f = rng.normal(size=shape) + 0.7  # incompatible on purpose
    faces = random_faces(bc, gtype, nc, nd, rng) if inhom else None
    _, c = dense_fd_solve(f, bc, gtype, hs, faces or {}, return_constant=True)
    got = oracle.zero_mode(bc, gtype, nc, lo, hi, f, faces)
    assert abs(got - c) <= 1e-11 * max(1.0, abs(c)), (got, c)
    # a compatible source (the constant removed) has no zero mode
    assert abs(oracle.zero_mode(bc, gtype, nc, lo, hi, f - c, faces)) <= 1e-11 * max(1.0, abs(c))


def test_zero_mode_zero_without_a_zero_eigenvalue():
    f = np.ones((4, 5))
    assert oracle.zero_mode("dirichlet", "staggered", [4, 5], [0, 0], [1, 1], f) == 0.0
    assert oracle.zero_mode("unbounded", "staggered", [4, 5], [0, 0], [1, 1], f) == 0.0


# ------------------------------------------------------- bounded gradient
def _mode(bc, m, length):
    """Eigenfunction of mode m (sin(pi m x / L) or cos(pi m x / L)) and its
    analytic derivative, as functions of x measured from X_l."""
    w = np.pi * m / length
    if bc == "dirichlet":
        return (lambda x: np.sin(w * x)), (lambda x: w * np.cos(w * x)), w
    return (lambda x: np.cos(w * x)), (lambda x: -w * np.sin(w * x)), w


def _mode_product_case(bc, gtype, nc, lo, hi, modes, operator):
    """Source = product of one eigenfunction per axis at the unknown points.
    psi is the same product over the eigenvalue sum (PS: -w^2; FD2: the
    three-point stencil applied to a sampled sinusoid, -(4/H^2) sin^2(w H/2)),
    and d psi / d x_a replaces the factor of axis a by its derivative."""
    nd = len(nc)
    xs_out, xs_unk, fns = [], [], []
    lam = 0.0
    for a in range(nd):
        length = hi[a] - lo[a]
        h = length / nc[a]
        x = grid.positions(bc, gtype, lo[a], hi[a], nc[a]) - lo[a]
        xs_out.append(x)
        xs_unk.append(x[1:-1] if (bc == "dirichlet" and gtype == "regular") else x)
        g, dg, w = _mode(bc, modes[a], length)
        fns.append((g, dg))
        lam += -w * w if operator == "ps" else -(4.0 / h**2) * np.sin(w * h / 2) ** 2

    def product(xs, deriv_axis=None):
        out = np.ones([len(x) for x in xs])
        for a in range(nd):
            view = [1] * nd
            view[a] = -1
            fn = fns[a][1] if a == deriv_axis else fns[a][0]
            out = out * fn(xs[a]).reshape(view)
        return out

    f = product(xs_unk)
    psi_a = product(xs_out) / lam
    grad_a = [product(xs_out, a) / lam for a in range(nd)]
    return f, psi_a, grad_a


@pytest.mark.parametrize("bc,gtype", CASES[:4])
@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("operator", ["ps", "fd2"])
def test_bounded_gradient_of_eigenmodes(bc, gtype, nd, operator):
    nc = [12, 10, 8][:nd]
    lo = [0.0, 1.0, -2.0][:nd]
    hi = [1.0, 3.0, 1.0][:nd]
    f, psi_a, grad_a = _mode_product_case(bc, gtype, nc, lo, hi, [3, 2, 5][:nd], operator)
    psi, grad = oracle.solve(bc, gtype, nc, lo, hi, f, operator=operator, diff="grad")
    scale = max(np.max(np.abs(g)) for g in grad_a)
    assert np.max(np.abs(psi - psi_a)) <= 1e-13 * np.max(np.abs(psi_a))
    assert len(grad) == nd
    for a in range(nd):
        assert np.max(np.abs(grad[a] - grad_a[a])) <= 1e-12 * scale, a


@pytest.mark.parametrize("bc,gtype,top", [("dirichlet", "regular", 9), ("dirichlet", "staggered", 10),
                                          ("neumann", "regular", 10), ("neumann", "staggered", 9)])
def test_bounded_gradient_top_mode(bc, gtype, top):
    """The highest eigenfunction of each basis (10 cells): staggered sine and
    regular cosine tops alternate in sign on the points, where their derivative
    is exactly zero; the other two are ordinary modes."""
    f, psi_a, grad_a = _mode_product_case(bc, gtype, [10], [0.0], [2.0], [top], "ps")
    _, grad = oracle.solve(bc, gtype, [10], [0.0], [2.0], f, operator="ps", diff="grad")
    scale = max(1.0, np.max(np.abs(grad_a[0])))
    assert np.max(np.abs(grad[0] - grad_a[0])) <= 1e-12 * scale
    if (bc, gtype) in (("dirichlet", "staggered"), ("neumann", "regular")):
        assert np.max(np.abs(grad_a[0])) < 1e-12 * np.pi * top / 2.0


@pytest.mark.parametrize("bc,gtype", CASES[:4])
@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("operator", ["ps", "fd2"])
def test_bounded_laplacian_of_eigenmodes(bc, gtype, nd, operator):
    """NABLA of a product of eigenfunctions: every second derivative brings
    -w_a^2, so NABLA psi = sum_a (-w_a^2) x the product / the eigenvalue sum
    at the output points (boundary nodes included).  With PS that sum is the
    eigenvalue itself and NABLA psi is the source."""
    nc = [12, 10, 8][:nd]
    lo = [0.0, 1.0, -2.0][:nd]
    hi = [1.0, 3.0, 1.0][:nd]
    modes = [3, 2, 5][:nd]
    f, psi_a, _ = _mode_product_case(bc, gtype, nc, lo, hi, modes, operator)
    w2 = sum((np.pi * modes[a] / (hi[a] - lo[a])) ** 2 for a in range(nd))
    lap_a = -w2 * psi_a  # psi_a = product / eigenvalue sum at the output points
    psi, lap = oracle.solve(bc, gtype, nc, lo, hi, f, operator=operator, diff="nabla")
    assert len(lap) == 1
    assert np.max(np.abs(lap[0] - lap_a)) <= 1e-11 * np.max(np.abs(lap_a))
    if operator == "ps":
        # the eigenfunction product itself: the source, now at the output points
        _, prod, _ = _mode_product_case(bc, gtype, nc, lo, hi, modes, "ps")
        prod = -w2 * prod
        assert np.max(np.abs(lap[0] - prod)) <= 1e-11 * np.max(np.abs(prod))


def _vector_mode_case(bc, gtype, nc, lo, hi, operator):
    """A 3D vector whose component c is a product of eigenfunctions with its
    own modes: sources, potentials and every first derivative in closed form."""
    modes = [[3, 2, 1], [1, 3, 2], [2, 1, 4]]
    f, psi, grads = [], [], []
    for c in range(3):
        fc, pc, gc = _mode_product_case(bc, gtype, nc, lo, hi, modes[c], operator)
        f.append(fc)
        psi.append(pc)
        grads.append(gc)
    return np.stack(f), psi, grads


@pytest.mark.parametrize("bc,gtype", CASES[:4])
@pytest.mark.parametrize("operator", ["ps", "fd2"])
def test_bounded_curl_and_div_of_eigenmodes(bc, gtype, operator):
    """CURL and DIV of a 3D vector of eigenfunction products, from the closed
    forms of every d psi_c / d x_a (the curl's components and signs, the
    divergence's diagonal terms)."""
    nc, lo, hi = [10, 8, 12], [0.0, 1.0, -2.0], [1.0, 3.0, 1.0]
    f, psi_a, g = _vector_mode_case(bc, gtype, nc, lo, hi, operator)
    psi, curl = oracle.solve(bc, gtype, nc, lo, hi, f, operator=operator, diff="curl")
    curl_a = [g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]]
    scale = max(np.max(np.abs(c)) for c in curl_a)
    for c in range(3):
        assert np.max(np.abs(psi[c] - psi_a[c])) <= 1e-12 * np.max(np.abs(psi_a[c]))
        assert np.max(np.abs(curl[c] - curl_a[c])) <= 1e-11 * scale, c
    _, div = oracle.solve(bc, gtype, nc, lo, hi, f, operator=operator, diff="div")
    div_a = g[0][0] + g[1][1] + g[2][2]
    assert len(div) == 1
    assert np.max(np.abs(div[0] - div_a)) <= 1e-11 * max(np.max(np.abs(x[i])) for i, x in enumerate(g))


@pytest.mark.parametrize("bc,gtype", CASES[:4])
def test_bounded_curl_2d_of_eigenmodes(bc, gtype):
    nc, lo, hi = [12, 10], [0.0, 1.0], [1.0, 3.0]
    f, psi_a, g = _mode_product_case(bc, gtype, nc, lo, hi, [3, 2], "ps")
    _, curl = oracle.solve(bc, gtype, nc, lo, hi, f, operator="ps", diff="curl")
    scale = max(np.max(np.abs(x)) for x in g)
    assert np.max(np.abs(curl[0] - g[1])) <= 1e-12 * scale
    assert np.max(np.abs(curl[1] + g[0])) <= 1e-12 * scale


def test_bounded_laplacian_inhomogeneous_rejected():
    # with boundary values only first derivatives are defined (FD2 differences)
    f = np.zeros((6,))
    with pytest.raises(NotImplementedError):
        oracle.solve("dirichlet", "staggered", [6], [0.0], [1.0], f, operator="fd2", diff="nabla",
                     faces={(0, 0): np.array(1.0)})
