"""Pins of the oracle's mixed-boundary solve (oracle.bounded.solve_mixed): a
periodic, Dirichlet or Neumann condition per axis.

What pins what:
  * FD2 solves (homogeneous and inhomogeneous, both grids, 2D and 3D axis
    combinations) equal a dense linear solve of the finite-difference
    equations on a grid extended by one ghost / boundary layer on the faces of
    every Dirichlet / Neumann axis and wrapped along periodic axes, with each
    face condition stated as its own equation (the same equations as the
    uniform-BC dense model of test_oracle_bounded.py, chosen per axis).
  * PS solves of products of per-axis eigenfunctions (sin for Dirichlet, cos
    for Neumann, cos / sin of 2 pi m x / L for periodic axes) are the closed
    forms f / sum_a lambda_a.
  * A mixed solve whose axes all carry the same condition is the uniform solve.
  * The zero mode: a constant source on an all periodic / Neumann mix is
    removed entirely; with a Dirichlet axis nothing is removed.
  * Derivatives (bounded.mixed_derivative): GRAD and NABLA of a product of
    per-axis eigenfunctions (PS and FD2) are the analytic derivatives of the
    product over the eigenvalue sum at the output points; CURL and DIV of a
    3D vector with a different mode triple per component are their closed
    forms.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import bounded, grid

LO = [0.0, -0.5, 1.0]
HI = [1.0, 1.3, 2.5]
NC = [7, 6, 5]
BC3 = ("periodic", "dirichlet", "neumann")


def dense_fd_solve_mixed(f, bcs, gtype, hs, faces):
    """FD2 equations per axis condition, solved directly (test-side model)."""
    shape = f.shape
    nd = len(shape)
    per = [b == "periodic" for b in bcs]
    dreg = [b == "dirichlet" and gtype == "regular" for b in bcs]
    ext = tuple(n if per[a] else n + 2 for a, n in enumerate(shape))
    off = [0 if per[a] else 1 for a in range(nd)]
    idx = {p: i for i, p in enumerate(itertools.product(*[range(e) for e in ext]))}
    nvar = len(idx)
    singular = all(b in ("periodic", "neumann") for b in bcs)
    size = nvar + (1 if singular else 0)
    A = np.zeros((size, size))
    b = np.zeros(size)

    def inside(p, a):
        return off[a] <= p[a] < off[a] + shape[a]

    def face_value(a, side, p):
        g = faces.get((a, side)) if faces else None
        if g is None:
            return 0.0
        # face arrays span the output points of the other axes
        return g[tuple(p[d] if (dreg[d] or per[d]) else p[d] - 1 for d in range(nd) if d != a)]

    for p, i in idx.items():
        ghost_axes = [a for a in range(nd) if not inside(p, a)]
        if not ghost_axes:
            for a in range(nd):
                for s in (-1, 1):
                    q = list(p)
                    q[a] = (q[a] + s) % ext[a] if per[a] else q[a] + s
                    A[i, idx[tuple(q)]] += 1.0 / hs[a] ** 2
                A[i, i] -= 2.0 / hs[a] ** 2
            b[i] = f[tuple(p[a] - off[a] for a in range(nd))]
            if singular:
                A[i, nvar] = 1.0  # unknown constant removed from the source
            continue
        if len(ghost_axes) > 1:
            # edge / corner of the extended grid: in no stencil; an output
            # node only where every such axis is a REGULAR Dirichlet axis
            A[i, i] = 1.0
            if all(dreg[a] for a in ghost_axes):
                a = max(ghost_axes)
                b[i] = face_value(a, 0 if p[a] == 0 else 1, p)
            continue
        a = ghost_axes[0]
        side = 0 if p[a] == 0 else 1
        gv = face_value(a, side, p)
        h = hs[a]
        inward = list(p)
        inward[a] = 1 if side == 0 else shape[a]
        inward2 = list(p)
        inward2[a] = 2 if side == 0 else shape[a] - 1
        i1, i2 = idx[tuple(inward)], idx[tuple(inward2)]
        if bcs[a] == "dirichlet" and gtype == "regular":
            A[i, i] = 1.0
        elif bcs[a] == "dirichlet":
            A[i, i] = 0.5
            A[i, i1] = 0.5
        elif gtype == "regular":
            if side == 0:
                A[i, i2] = 1.0 / (2 * h)
                A[i, i] = -1.0 / (2 * h)
            else:
                A[i, i] = 1.0 / (2 * h)
                A[i, i2] = -1.0 / (2 * h)
        else:
            if side == 0:
                A[i, i1] = 1.0 / h
                A[i, i] = -1.0 / h
            else:
                A[i, i] = 1.0 / h
                A[i, i1] = -1.0 / h
        b[i] = gv
    if singular:
        for p, i in idx.items():
            if all(inside(p, a) for a in range(nd)):
                w = 1.0
                for a in range(nd):
                    if bcs[a] == "neumann" and gtype == "regular" and p[a] in (off[a], off[a] + shape[a] - 1):
                        w *= 0.5
                A[nvar, i] = w
    sol = np.linalg.solve(A, b)[:nvar]
    full = np.zeros(ext)
    for p, i in idx.items():
        full[p] = sol[i]
    return full[tuple(slice(None) if (dreg[a] or per[a]) else slice(1, 1 + shape[a]) for a in range(nd))]


def mixed_faces(bcs, gtype, nc, rng):
    nd = len(bcs)
    faces = {}
    for a in range(nd):
        if bcs[a] == "periodic":
            continue
        for s in (0, 1):
            shp = tuple(grid.output_points(bcs[d], gtype, nc[d]) for d in range(nd) if d != a)
            faces[(a, s)] = rng.normal(size=shp)
    return faces


COMBOS = [list(c) for c in itertools.permutations(BC3, 2)] + \
    [["periodic", "dirichlet", "neumann"], ["neumann", "periodic", "dirichlet"],
     ["dirichlet", "neumann", "periodic"], ["periodic", "neumann", "neumann"]]


@pytest.mark.parametrize("bcs", COMBOS)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("inhom", [False, True])
def test_mixed_fd2_matches_dense_solve(bcs, gtype, inhom):
    nd = len(bcs)
    rng = np.random.default_rng(7 * nd + inhom + (gtype == "regular"))
    nc, lo, hi = NC[:nd], LO[:nd], HI[:nd]
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    shape = tuple(grid.unknowns(bcs[a], gtype, nc[a]) for a in range(nd))
    f = rng.normal(size=shape)
    faces = mixed_faces(bcs, gtype, nc, rng) if inhom else None
    psi, _ = oracle.solve(bcs, gtype, nc, lo, hi, f, operator="fd2", faces=faces)
    ref = dense_fd_solve_mixed(f, bcs, gtype, hs, faces or {})
    assert psi.shape == ref.shape
    assert np.max(np.abs(psi - ref)) <= 1e-11 * np.max(np.abs(ref))


def _eigenmode(bc, m, x, lo, length):
    t = (x - lo) / length
    if bc == "dirichlet":
        return np.sin(np.pi * m * t), -(np.pi * m / length) ** 2
    if bc == "neumann":
        return np.cos(np.pi * m * t), -(np.pi * m / length) ** 2
    # periodic: a phase-shifted cosine (both parities of the mode)
    return np.cos(2 * np.pi * m * t + 0.3), -(2 * np.pi * m / length) ** 2


@pytest.mark.parametrize("bcs", COMBOS)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
def test_mixed_ps_closed_form(bcs, gtype):
    nd = len(bcs)
    nc, lo, hi = [12, 10, 8][:nd], LO[:nd], HI[:nd]
    lengths = [hi[a] - lo[a] for a in range(nd)]
    xs_in = []
    xs_out = []
    for a in range(nd):
        h = grid.spacing(lo[a], hi[a], nc[a])
        xo = grid.positions(bcs[a], gtype, lo[a], hi[a], nc[a])
        xs_out.append(xo)
        xs_in.append(xo[1:-1] if (bcs[a] == "dirichlet" and gtype == "regular") else xo)
        assert len(xs_in[-1]) == grid.unknowns(bcs[a], gtype, nc[a]), h
    rng = np.random.default_rng(3)
    shape_in = tuple(len(x) for x in xs_in)
    shape_out = tuple(len(x) for x in xs_out)
    f = np.zeros(shape_in)
    psi_ref = np.zeros(shape_out)
    # one mode of every axis per term; mode numbers well inside each axis's band
    for _ in range(3):
        ms = []
        for a in range(nd):
            top = max(1, grid.unknowns(bcs[a], gtype, nc[a]) // 3)
            ms.append(int(rng.integers(1, top + 1)))
        amp = rng.normal()
        fin, fout, lam = amp, amp, 0.0
        for a in range(nd):
            view = [1] * nd
            view[a] = -1
            vi, la = _eigenmode(bcs[a], ms[a], xs_in[a], lo[a], lengths[a])
            vo, _ = _eigenmode(bcs[a], ms[a], xs_out[a], lo[a], lengths[a])
            fin = fin * vi.reshape(view)
            fout = fout * vo.reshape(view)
            lam += la
        f = f + fin
        psi_ref = psi_ref + fout / lam
    psi, _ = oracle.solve(bcs, gtype, nc, lo, hi, f, operator="ps")
    assert psi.shape == shape_out
    assert np.max(np.abs(psi - psi_ref)) <= 1e-12 * np.max(np.abs(psi_ref))


@pytest.mark.parametrize("bc", BC3)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("operator", ["ps", "fd2"])
def test_mixed_uniform_is_the_uniform_solve(bc, gtype, operator):
    nd = 3
    rng = np.random.default_rng(11)
    nc, lo, hi = NC, LO, HI
    shape = tuple(grid.unknowns(bc, gtype, nc[a]) for a in range(nd))
    f = rng.normal(size=shape)
    faces = mixed_faces([bc] * nd, gtype, nc, rng) if (operator == "fd2" and bc != "periodic") else None
    mixed, _ = oracle.solve([bc] * nd, gtype, nc, lo, hi, f, operator=operator, faces=faces)
    uniform, _ = oracle.solve(bc, gtype, nc, lo, hi, f, operator=operator, faces=faces)
    assert np.max(np.abs(mixed - uniform)) <= 1e-12 * np.max(np.abs(uniform))
    zm = oracle.zero_mode([bc] * nd, gtype, nc, lo, hi, f, faces)
    zu = oracle.zero_mode(bc, gtype, nc, lo, hi, f, faces)
    assert abs(zm - zu) <= 1e-12 * max(1.0, abs(zu))


@pytest.mark.parametrize("bcs", COMBOS)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
def test_mixed_zero_mode_of_a_constant(bcs, gtype):
    nd = len(bcs)
    nc, lo, hi = NC[:nd], LO[:nd], HI[:nd]
    shape = tuple(grid.unknowns(bcs[a], gtype, nc[a]) for a in range(nd))
    z = oracle.zero_mode(bcs, gtype, nc, lo, hi, np.full(shape, 2.5))
    if "dirichlet" in bcs:
        assert z == 0.0
    else:
        assert abs(z - 2.5) <= 1e-13
        # the solve of a constant source is then zero
        psi, _ = oracle.solve(bcs, gtype, nc, lo, hi, np.full(shape, 2.5), operator="fd2")
        assert np.max(np.abs(psi)) <= 1e-12


def test_periodic_axis_has_no_faces():
    f = np.zeros((6, 5))
    with pytest.raises(ValueError):
        bounded.solve_mixed(f, ["periodic", "dirichlet"], "staggered", "fd2", [1.0, 1.0], [1 / 6, 1 / 5],
                            {(0, 0): np.zeros(5)})


# ------------------------------------------------ derivatives of mixed plans
def _mode_and_derivs(bc, m, x, lo, length):
    """Eigenfunction of one axis, its first and second derivative, eigenvalue."""
    t = (x - lo) / length
    if bc == "dirichlet":
        w = np.pi * m / length
        return np.sin(w * (x - lo)), w * np.cos(w * (x - lo)), -w * w * np.sin(w * (x - lo)), -w * w
    if bc == "neumann":
        w = np.pi * m / length
        return np.cos(w * (x - lo)), -w * np.sin(w * (x - lo)), -w * w * np.cos(w * (x - lo)), -w * w
    w = 2 * np.pi * m / length
    return (np.cos(w * (x - lo) + 0.4), -w * np.sin(w * (x - lo) + 0.4), -w * w * np.cos(w * (x - lo) + 0.4),
            -w * w)


@pytest.mark.parametrize("bcs", COMBOS)
@pytest.mark.parametrize("gtype", ["regular", "staggered"])
@pytest.mark.parametrize("operator", ["ps", "fd2"])
def test_mixed_gradient_and_laplacian_of_eigenmodes(bcs, gtype, operator):
    # psi of one product of per-axis eigenfunctions is that product over the
    # eigenvalue sum; its gradient and Laplacian are the analytic ones (the
    # FD2 eigenvalues enter only through the sum)
    nd = len(bcs)
    nc, lo, hi = [12, 10, 9][:nd], LO[:nd], HI[:nd]
    xs_out = [grid.positions(bcs[a], gtype, lo[a], hi[a], nc[a]) for a in range(nd)]
    xs_in = [x[1:-1] if (bcs[a] == "dirichlet" and gtype == "regular") else x for a, x in enumerate(xs_out)]
    ms = [1 + (a % 2) for a in range(nd)]
    lam = 0.0
    fin = np.ones([len(x) for x in xs_in])
    parts = []
    for a in range(nd):
        view = [1] * nd
        view[a] = -1
        v, _, _, la = _mode_and_derivs(bcs[a], ms[a], xs_in[a], lo[a], hi[a] - lo[a])
        fin = fin * v.reshape(view)
        parts.append([p.reshape(view) for p in _mode_and_derivs(bcs[a], ms[a], xs_out[a], lo[a], hi[a] - lo[a])[:3]])
        if operator == "ps":
            lam += la
    if operator == "fd2":
        lam = sum(bounded.eigenvalues(bcs[a], gtype, "fd2", len(xs_in[a]), hi[a] - lo[a],
                                      grid.spacing(lo[a], hi[a], nc[a]))[ms[a] - (1 if bcs[a] == "dirichlet" else 0)
                                                                       if bcs[a] != "periodic" else ms[a]]
                  for a in range(nd))
    psi, grads = oracle.solve(bcs, gtype, nc, lo, hi, fin, operator=operator, diff="grad")
    _, lap = oracle.solve(bcs, gtype, nc, lo, hi, fin, operator=operator, diff="nabla")

    def prod(sel):
        out = 1.0
        for a in range(nd):
            out = out * parts[a][sel[a]]
        return out

    ref_psi = prod([0] * nd) / lam
    assert np.max(np.abs(psi - ref_psi)) <= 1e-11 * np.max(np.abs(ref_psi))
    for g in range(nd):
        ref = prod([1 if a == g else 0 for a in range(nd)]) / lam
        assert np.max(np.abs(grads[g] - ref)) <= 1e-10 * np.max(np.abs(ref)), g
    ref_lap = sum(prod([2 if a == g else 0 for a in range(nd)]) for g in range(nd)) / lam
    assert np.max(np.abs(lap[0] - ref_lap)) <= 1e-10 * np.max(np.abs(ref_lap))


def test_mixed_curl_and_div_closed_form():
    bcs = ["periodic", "dirichlet", "neumann"]
    gtype = "staggered"
    nc, lo, hi = [12, 10, 9], LO, HI
    xs = [grid.positions(bcs[a], gtype, lo[a], hi[a], nc[a]) for a in range(3)]
    comps, psis, dps = [], [], []
    for c, ms in enumerate([(1, 2, 1), (2, 1, 3), (1, 3, 2)]):
        fin, lam, parts = 1.0, 0.0, []
        for a in range(3):
            view = [1, 1, 1]
            view[a] = -1
            v, dv, _, la = _mode_and_derivs(bcs[a], ms[a], xs[a], lo[a], hi[a] - lo[a])
            fin = fin * v.reshape(view)
            parts.append((v.reshape(view), dv.reshape(view)))
            lam += la
        comps.append(fin)
        psis.append(fin / lam)
        dps.append([parts[0][g == 0] * parts[1][g == 1] * parts[2][g == 2] / lam for g in range(3)])
    f = np.stack(comps)
    _, curl = oracle.solve(bcs, gtype, nc, lo, hi, f, operator="ps", diff="curl")
    _, div = oracle.solve(bcs, gtype, nc, lo, hi, f, operator="ps", diff="div")
    d = dps
    ref_curl = [d[2][1] - d[1][2], d[0][2] - d[2][0], d[1][0] - d[0][1]]
    for c in range(3):
        assert np.max(np.abs(curl[c] - ref_curl[c])) <= 1e-10 * np.max(np.abs(ref_curl[c])), c
    ref_div = d[0][0] + d[1][1] + d[2][2]
    assert np.max(np.abs(div[0] - ref_div)) <= 1e-10 * np.max(np.abs(ref_div))
