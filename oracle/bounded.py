"""Bounded solves (periodic, Dirichlet, Neumann) of the oracle.

The solve follows the four steps of Section 2.2: forward transform, pointwise
multiply by the spectral multiplier, (optional spectral operation), backward
transform.  Table 1 (tab:Bounded) names the transform pair and the 1D
eigenvalue for every BC / grid / operator combination; eq. (pois_spec) sums
the per-axis eigenvalues in 2D and 3D.  The zero wavenumber, where the
eigenvalue vanishes (periodic and Neumann), is set to zero (the remark after
eq. (spect_sol)).

Inhomogeneous Dirichlet / Neumann values (Section 2.4.2 and Section 4.2) are
only available with the FD2 eigenvalues.  The paper names the technique
("simple weighting of the boundary source terms") without writing it out; the
reading used here moves each boundary value into the right-hand side of the
layer of unknowns next to the face, through the ghost-point rule of each
grid (g is the boundary value for Dirichlet and d(psi)/dx_a, not the outward
normal derivative, for Neumann, as in eq. (tfih1Dgrad)):

  Dirichlet REGULAR    psi at the boundary node is g:   f_first -= g / H^2
  Dirichlet STAGGERED  ghost = 2 g - psi_0:             f_first -= 2 g / H^2
  Neumann  REGULAR     ghost = psi_1 -+ 2 H g:          f_first += 2 g / H,
                                                        f_last  -= 2 g / H
  Neumann  STAGGERED   face difference (psi_0 - ghost) / H = g:
                                                        f_first += g / H,
                                                        f_last  -= g / H

In several dimensions every face adds to its own adjacent layer, so edges and
corners collect the terms of every face that touches them.
"""
import numpy as np

from . import grid as _grid
from . import transforms as _tr

# Table 1: forward transform, backward transform, and the factor c(n) with
# backward(forward(x)) = c(n) x for the unnormalised definitions.
TRANSFORM_PAIRS = {
    ("dirichlet", "regular"): ("dst1", "dst1", lambda n: 2.0 * (n + 1)),
    ("dirichlet", "staggered"): ("dst2", "dst3", lambda n: 2.0 * n),
    ("neumann", "regular"): ("dct1", "dct1", lambda n: 2.0 * (n - 1)),
    # Table 1 prints "DST-III" as the backward transform here; the inverse of
    # DCT-II is DCT-III, which is what is used.
    ("neumann", "staggered"): ("dct2", "dct3", lambda n: 2.0 * n),
}


def eigenvalues(bc, grid, operator, n, length, h):
    """1D eigenvalues of Table 1 for k = 0 .. n-1 (N of the table is n).

    operator is "ps" (pseudo-spectral) or "fd2" (second-order finite
    difference).  length is L = X_u - X_l, h the cell size H.
    """
    k = np.arange(n, dtype=np.float64)
    L = float(length)
    if operator == "ps":
        if bc == "dirichlet":
            return -((np.pi * (k + 1.0) / L) ** 2)
        if bc == "neumann":
            return -((np.pi * k / L) ** 2)
        if bc == "periodic":
            kk = np.where(k < n / 2.0, k, n - k)
            return -((2.0 * np.pi * kk / L) ** 2)
    elif operator == "fd2":
        s = -4.0 / (h * h)
        if bc == "dirichlet" and grid == "regular":
            return s * np.sin(np.pi * (k + 1.0) / (2.0 * (n + 1))) ** 2
        if bc == "dirichlet" and grid == "staggered":
            return s * np.sin(np.pi * (k + 1.0) / (2.0 * n)) ** 2
        if bc == "neumann" and grid == "regular":
            return s * np.sin(np.pi * k / (2.0 * (n - 1))) ** 2
        if bc == "neumann" and grid == "staggered":
            return s * np.sin(np.pi * k / (2.0 * n)) ** 2
        if bc == "periodic":
            return s * np.sin(np.pi * k / n) ** 2
    raise ValueError((bc, grid, operator))


def multiplier(bc, grid, operator, shape, lengths, hs):
    """Sum of the per-axis eigenvalues on the spectral grid (eq. pois_spec)."""
    lam = np.zeros(shape)
    for a, n in enumerate(shape):
        la = eigenvalues(bc, grid, operator, n, lengths[a], hs[a])
        view = [1] * len(shape)
        view[a] = n
        lam = lam + la.reshape(view)
    return lam


def _divide(fhat, lam):
    """psi_hat = f_hat / lambda, with the zero eigenvalue mapped to zero."""
    out = np.zeros_like(fhat)
    nz = lam != 0.0
    out[nz] = fhat[nz] / lam[nz]
    return out


def apply_boundary_values(f, bc, grid, hs, faces):
    """Move boundary values into the right-hand side (FD2 only).

    f has the unknown shape.  faces maps (axis, side) with side 0 = lower,
    1 = upper to an array with the output shape of the other axes.  For
    REGULAR Dirichlet only the entries at interior nodes of the other axes
    enter the right-hand side.
    """
    f = np.array(f, dtype=np.float64, copy=True)
    nd = f.ndim
    for (axis, side), g in faces.items():
        g = np.asarray(g, dtype=np.float64)
        if bc == "dirichlet" and grid == "regular":
            g = g[tuple(slice(1, -1) for _ in range(nd - 1))]
        h = hs[axis]
        if bc == "dirichlet" and grid == "regular":
            term = -g / h**2
        elif bc == "dirichlet" and grid == "staggered":
            term = -2.0 * g / h**2
        elif bc == "neumann" and grid == "regular":
            term = (2.0 * g / h) if side == 0 else (-2.0 * g / h)
        elif bc == "neumann" and grid == "staggered":
            term = (g / h) if side == 0 else (-g / h)
        else:
            raise ValueError("boundary values need a Dirichlet or Neumann BC")
        idx = [slice(None)] * nd
        idx[axis] = 0 if side == 0 else f.shape[axis] - 1
        f[tuple(idx)] += term
    return f


def dirichlet_regular_output(psi_inner, faces):
    """Embed interior nodes into the node grid and write the boundary nodes.

    Boundary nodes take the value of their face; a node on several faces takes
    the value of the face with the highest axis index.  Missing faces are 0.
    """
    nd = psi_inner.ndim
    out = np.zeros(tuple(n + 2 for n in psi_inner.shape))
    out[tuple(slice(1, -1) for _ in range(nd))] = psi_inner
    for axis in range(nd):
        for side in (0, 1):
            g = faces.get((axis, side)) if faces else None
            idx = [slice(None)] * nd
            idx[axis] = 0 if side == 0 else out.shape[axis] - 1
            out[tuple(idx)] = 0.0 if g is None else np.asarray(g, dtype=np.float64)
    return out


def solve_bounded(f, bc, grid, operator, lengths, hs, faces=None):
    """Solve lap(psi) = f on a bounded grid.

    f has the unknown shape (grid.unknowns per axis).  Returns psi on the
    output points (grid.output_points per axis).
    """
    f = np.asarray(f, dtype=np.float64)
    if faces:
        if operator != "fd2":
            raise ValueError("inhomogeneous boundary values need the FD2 operator")
        f = apply_boundary_values(f, bc, grid, hs, faces)
    lam = multiplier(bc, grid, operator, f.shape, lengths, hs)
    if bc == "periodic":
        psi = np.fft.ifftn(_divide(np.fft.fftn(f), lam)).real
        return psi
    fwd, bwd, norm = TRANSFORM_PAIRS[(bc, grid)]
    fhat = f
    for a in range(f.ndim):
        fhat = _tr.apply(fwd, fhat, a)
    psihat = _divide(fhat, lam)
    psi = psihat
    for a in reversed(range(f.ndim)):
        psi = _tr.apply(bwd, psi, a) / norm(f.shape[a])
    if bc == "dirichlet" and grid == "regular":
        psi = dirichlet_regular_output(psi, faces or {})
    return psi


def periodic_gradient(psi, lengths):
    """Spectral gradient of a periodic field (Section 2.3.3, eq. ft_sd).

    Multiplies the DFT by i k_a, k_a = 2 pi m / L_a with m taken in
    (-n/2, n/2); the Nyquist mode m = n/2 has no real derivative and is set to
    zero (the paper does not say what it does with it).
    """
    psi = np.asarray(psi, dtype=np.float64)
    ph = np.fft.fftn(psi)
    out = []
    for a, n in enumerate(psi.shape):
        m = np.fft.fftfreq(n, d=1.0 / n)
        if n % 2 == 0:
            m[n // 2] = 0.0
        k = 2.0 * np.pi * m / float(lengths[a])
        view = [1] * psi.ndim
        view[a] = n
        out.append(np.fft.ifftn(1j * k.reshape(view) * ph).real)
    return out


def periodic_curl(psi, lengths):
    """Spectral curl u = i k x psi^ of a periodic 3D vector field (Section
    2.3.3, eq. ft_sd; the curl output of Section 4.3, eq. poisscurl):
    u_x = d_y psi_z - d_z psi_y, u_y = d_z psi_x - d_x psi_z,
    u_z = d_x psi_y - d_y psi_x, each derivative from periodic_gradient."""
    g = [periodic_gradient(p, lengths) for p in psi]
    return [g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]]


def eigenfunctions(bc, n, length, x):
    """The n eigenfunctions of Table 1 along one axis at positions x measured
    from X_l, and their derivatives: sin(pi (k+1) x / L) for Dirichlet,
    cos(pi k x / L) for Neumann, k = 0 .. n-1.  Returns (phi, dphi), each of
    shape (len(x), n)."""
    x = np.asarray(x, dtype=np.float64)[:, None]
    k = np.arange(n, dtype=np.float64)[None, :]
    if bc == "dirichlet":
        w = np.pi * (k + 1.0) / float(length)
        return np.sin(w * x), w * np.cos(w * x)
    if bc == "neumann":
        w = np.pi * k / float(length)
        return np.cos(w * x), -w * np.sin(w * x)
    raise ValueError(bc)


def bounded_derivative(psi, bc, grid, nc, lengths, axis, order=1):
    """Derivative of order 1 or 2 along `axis` of a Dirichlet / Neumann
    solution with homogeneous boundary values.  Section 2.3.3 defines the
    spectral derivative for the Fourier basis; for the sine / cosine bases of
    Table 1 it is read here as the derivative of the eigenfunction series that
    passes through psi at the unknown points, evaluated at the output points:
    along `axis` the matrix d^m phi(x_out) phi(x_unk)^-1 applied to every line
    of psi, the other axes untouched.  The first derivative turns a sine series
    into a cosine series and back; the second keeps the basis, each
    eigenfunction times -w^2.  REGULAR Dirichlet output includes the boundary
    nodes (the normal derivative there; 0 along the faces)."""
    psi = np.asarray(psi, dtype=np.float64)
    a = axis
    n = _grid.unknowns(bc, grid, nc[a])
    x_out = _grid.positions(bc, grid, 0.0, lengths[a], nc[a])
    dreg = bc == "dirichlet" and grid == "regular"
    x_unk = x_out[1:-1] if dreg else x_out
    phi, _ = eigenfunctions(bc, n, lengths[a], x_unk)
    phi_out, dphi = eigenfunctions(bc, n, lengths[a], x_out)
    if order == 1:
        deriv = dphi
    elif order == 2:
        w = np.pi * (np.arange(n) + (1.0 if bc == "dirichlet" else 0.0)) / float(lengths[a])
        deriv = phi_out * (-w * w)[None, :]
    else:
        raise ValueError(order)
    dmat = deriv @ np.linalg.inv(phi)
    vals = np.moveaxis(psi, a, 0)
    if dreg:
        vals = vals[1:-1]
    return np.moveaxis(np.tensordot(dmat, vals, axes=1), 0, a)


def bounded_gradient(psi, bc, grid, nc, lengths):
    """Spectral gradient of a Dirichlet / Neumann solution with homogeneous
    boundary values: the first derivative of the eigenfunction series along
    every axis (bounded_derivative)."""
    psi = np.asarray(psi, dtype=np.float64)
    return [bounded_derivative(psi, bc, grid, nc, lengths, a, 1) for a in range(psi.ndim)]


def bounded_laplacian(psi, bc, grid, nc, lengths):
    """NABLA of Section 2.3.3 on a Dirichlet / Neumann solution: the sum over
    the axes of the second derivative of the eigenfunction series."""
    psi = np.asarray(psi, dtype=np.float64)
    return sum(bounded_derivative(psi, bc, grid, nc, lengths, a, 2) for a in range(psi.ndim))


def bounded_curl(psi, bc, grid, nc, lengths):
    """Curl of a 3D vector Dirichlet / Neumann solution (component c of psi on
    its own sine / cosine series): u_x = d_y psi_z - d_z psi_y,
    u_y = d_z psi_x - d_x psi_z, u_z = d_x psi_y - d_y psi_x, each derivative
    from bounded_derivative."""
    d = lambda c, a: bounded_derivative(psi[c], bc, grid, nc, lengths, a, 1)
    return [d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)]


# ------------------------------------------------------------------ mixed BCs
# Section 2.6 describes building a solve from 1D transforms per axis, a DFT,
# DST or DCT chosen per direction, so that each axis can carry its own
# boundary condition.  The paper plans this without implementing it; the
# oracle writes it out directly: every axis takes the forward transform of its
# own condition (the complex DFT for a periodic axis, the Table 1 pair
# otherwise), the spectrum is divided by the sum of the per-axis Table 1
# eigenvalues (eq. pois_spec), and every axis takes its backward transform.

def _apply_real_pair(kind, x, axis):
    """A real-to-real transform applied to the real and imaginary parts."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return _tr.apply(kind, x.real, axis) + 1j * _tr.apply(kind, x.imag, axis)
    return _tr.apply(kind, x, axis)


def apply_boundary_values_mixed(f, bcs, grid, hs, faces):
    """apply_boundary_values with a condition per axis: each face takes the
    weight of its own axis's condition; the face arrays span the output points
    of the other axes, so their boundary nodes are dropped along REGULAR
    Dirichlet axes only."""
    f = np.array(f, dtype=np.float64, copy=True)
    nd = f.ndim
    for (axis, side), g in faces.items():
        bc = bcs[axis]
        if bc == "periodic":
            raise ValueError("a periodic axis has no faces")
        g = np.asarray(g, dtype=np.float64)
        rest = [b for b in range(nd) if b != axis]
        g = g[tuple(slice(1, -1) if (bcs[b] == "dirichlet" and grid == "regular") else slice(None)
                    for b in rest)]
        h = hs[axis]
        if bc == "dirichlet" and grid == "regular":
            term = -g / h**2
        elif bc == "dirichlet":
            term = -2.0 * g / h**2
        elif grid == "regular":
            term = (2.0 * g / h) if side == 0 else (-2.0 * g / h)
        else:
            term = (g / h) if side == 0 else (-g / h)
        idx = [slice(None)] * nd
        idx[axis] = 0 if side == 0 else f.shape[axis] - 1
        f[tuple(idx)] += term
    return f


def mixed_output(psi_inner, bcs, grid, faces):
    """Embed the unknowns into the output points: REGULAR Dirichlet axes gain
    their two boundary nodes, which take their face's value (a node on several
    faces: the face of the highest axis index; missing faces are 0)."""
    nd = psi_inner.ndim
    dreg = [bcs[a] == "dirichlet" and grid == "regular" for a in range(nd)]
    out = np.zeros(tuple(n + 2 if dreg[a] else n for a, n in enumerate(psi_inner.shape)))
    out[tuple(slice(1, -1) if dreg[a] else slice(None) for a in range(nd))] = psi_inner
    for axis in range(nd):
        if not dreg[axis]:
            continue
        for side in (0, 1):
            g = faces.get((axis, side)) if faces else None
            idx = [slice(None)] * nd
            idx[axis] = 0 if side == 0 else out.shape[axis] - 1
            out[tuple(idx)] = 0.0 if g is None else np.asarray(g, dtype=np.float64)
    return out


def solve_mixed(f, bcs, grid, operator, lengths, hs, faces=None):
    """Solve lap(psi) = f with condition bcs[a] ("periodic", "dirichlet" or
    "neumann") on axis a.  f has the unknown shape; returns psi on the output
    points."""
    f = np.asarray(f, dtype=np.float64)
    nd = f.ndim
    if faces:
        if operator != "fd2":
            raise ValueError("inhomogeneous boundary values need the FD2 operator")
        f = apply_boundary_values_mixed(f, bcs, grid, hs, faces)
    lam = np.zeros(f.shape)
    for a in range(nd):
        view = [1] * nd
        view[a] = f.shape[a]
        lam = lam + eigenvalues(bcs[a], grid, operator, f.shape[a], lengths[a], hs[a]).reshape(view)
    fhat = f.astype(np.complex128)
    for a in range(nd):
        if bcs[a] == "periodic":
            fhat = np.fft.fft(fhat, axis=a)
        else:
            fhat = _apply_real_pair(TRANSFORM_PAIRS[(bcs[a], grid)][0], fhat, a)
    psi = _divide(fhat, lam)
    for a in reversed(range(nd)):
        if bcs[a] == "periodic":
            psi = np.fft.ifft(psi, axis=a)
        else:
            _, bwd, norm = TRANSFORM_PAIRS[(bcs[a], grid)]
            psi = _apply_real_pair(bwd, psi, a) / norm(f.shape[a])
    return mixed_output(psi.real, bcs, grid, faces or {})


# ------------------------------------------------------- semi-unbounded axes
# Section 2.6: transforming the bounded directions splits the Laplacian, and
# what remains along the free directions is a Helmholtz equation per mode.
# With one free axis u and bounded-mode eigenvalue sum Lambda <= 0, the mode
# solves psi'' - kappa^2 psi = f along u, kappa^2 = -Lambda, whose free-space
# Green's function is G(x) = -exp(-kappa |x|) / (2 kappa) (|x| / 2 for
# kappa = 0).  The oracle convolves with it by the Hockney-Eastwood doubling of
# Section 2.5 along u: M = 2 n points, G sampled at min(m, M - m) H_u, times
# the cell length H_u.

def helmholtz_kernel_1d(kappa, x):
    """Free-space Green's function of d^2/dx^2 - kappa^2 in 1D."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    kappa = np.asarray(kappa, dtype=np.float64)
    safe = np.where(kappa > 0.0, kappa, 1.0)
    return np.where(kappa > 0.0, -np.exp(-safe * x) / (2.0 * safe), 0.5 * x)


def helmholtz_kernel_1d_derivative(kappa, x):
    """d/dx of helmholtz_kernel_1d: sign(x) exp(-kappa |x|) / 2 (sign(x) / 2
    for kappa = 0), 0 at x = 0 (the mean of its one-sided limits, so that the
    sampled convolution stays second order across the jump)."""
    x = np.asarray(x, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    return 0.5 * np.sign(x) * np.exp(-kappa * np.abs(x))


def solve_semi(f, bcs, grid, operator, lengths, hs, faces=None, free_derivative=False):
    """solve_mixed with one axis "unbounded": that axis is convolved with the
    1D Helmholtz Green's function of each bounded mode (doubled to M = 2 n).
    free_derivative: d psi / d x_u instead, the convolution with the kernel's
    derivative (odd: sampled as sign(m) G'(|m| H) on the doubled axis, with
    the entry m = n, which no output in the window reads, set to 0)."""
    f = np.asarray(f, dtype=np.float64)
    nd = f.ndim
    u = bcs.index("unbounded")
    if faces:
        if operator != "fd2":
            raise ValueError("inhomogeneous boundary values need the FD2 operator")
        if any(a == u for (a, _) in faces):
            raise ValueError("a free axis has no faces")
        f = apply_boundary_values_mixed(f, bcs, grid, hs, faces)
    lam = np.zeros([1 if a == u else f.shape[a] for a in range(nd)])
    for a in range(nd):
        if a == u:
            continue
        view = [1] * nd
        view[a] = f.shape[a]
        lam = lam + eigenvalues(bcs[a], grid, operator, f.shape[a], lengths[a], hs[a]).reshape(view)
    fhat = f.astype(np.complex128)
    for a in range(nd):
        if a == u:
            continue
        if bcs[a] == "periodic":
            fhat = np.fft.fft(fhat, axis=a)
        else:
            fhat = _apply_real_pair(TRANSFORM_PAIRS[(bcs[a], grid)][0], fhat, a)
    n = f.shape[u]
    M = 2 * n
    m = np.arange(M)
    dist = np.minimum(m, M - m) * hs[u]
    kappa = np.sqrt(np.maximum(-lam, 0.0))
    gshape = [1] * nd
    gshape[u] = M
    if free_derivative:
        signed = np.where(m < n, m, m - M) * hs[u]
        signed[n] = 0.0
        g_ext = helmholtz_kernel_1d_derivative(kappa, signed.reshape(gshape))
    else:
        g_ext = helmholtz_kernel_1d(kappa, dist.reshape(gshape))  # broadcast over the bounded modes
    pad = [(0, 0)] * nd
    pad[u] = (0, M - n)
    conv = np.fft.ifft(np.fft.fft(np.pad(fhat, pad), axis=u) * np.fft.fft(g_ext, axis=u), axis=u)
    psi = np.take(conv, np.arange(n), axis=u) * hs[u]
    for a in reversed(range(nd)):
        if a == u:
            continue
        if bcs[a] == "periodic":
            psi = np.fft.ifft(psi, axis=a)
        else:
            _, bwd, norm = TRANSFORM_PAIRS[(bcs[a], grid)]
            psi = _apply_real_pair(bwd, psi, a) / norm(f.shape[a])
    return mixed_output(psi.real, bcs, grid, faces or {})


# ------------------------------------------- derivatives with boundary values
# With inhomogeneous FD2 boundary values the unknowns' sine / cosine series does
# not carry g (bounded_derivative needs homogeneous values).  The derivative is
# then taken the way the FD2 eigenvalues discretise the operator: the centred
# second-order difference (psi_{i+1} - psi_{i-1}) / (2 H) at every output point,
# closed at the faces by the Neumann ghost rules that also weight the boundary
# terms:
#   Neumann  REGULAR     ghost = psi_1 -+ 2 H g        (centred derivative = g)
#   Neumann  STAGGERED   ghost = psi_0 -+ H g          (face difference = g)
# and by one-sided second-order differences next to Dirichlet faces: on
# REGULAR boundary nodes (where no FD2 equation holds) -+(3 psi_0 - 4 psi_1 +
# psi_2) / (2 H); at the first STAGGERED centre the derivative of the
# quadratic through the face value g and the two nearest centres,
# -+(4 g / 3 - psi_0 - psi_1 / 3) / H (the linear ghost 2 g - psi_0 of the
# solve would make that point first order only).

def fd_derivative(psi, bc, grid, h, axis, g_lo=None, g_hi=None):
    """d psi / d x_axis at the output points of a bounded FD2 solve (psi on the
    output points; g_lo, g_hi the face values of this axis, None = 0)."""
    psi = np.asarray(psi, dtype=np.float64)
    if bc == "periodic":  # a periodic axis of a mixed plan: the grid wraps
        return (np.roll(psi, -1, axis=axis) - np.roll(psi, 1, axis=axis)) / (2.0 * h)
    x = np.moveaxis(psi, axis, 0)
    n = x.shape[0]
    lo = 0.0 if g_lo is None else np.asarray(g_lo, dtype=np.float64)
    hi = 0.0 if g_hi is None else np.asarray(g_hi, dtype=np.float64)
    out = np.empty_like(x)
    if bc == "dirichlet" and grid == "regular":
        out[1:-1] = (x[2:] - x[:-2]) / (2.0 * h)
        out[0] = (-3.0 * x[0] + 4.0 * x[1] - x[2]) / (2.0 * h)
        out[-1] = (3.0 * x[-1] - 4.0 * x[-2] + x[-3]) / (2.0 * h)
        return np.moveaxis(out, 0, axis)
    if bc == "dirichlet":
        if n == 1:
            out[0] = (hi - lo) / h
            return np.moveaxis(out, 0, axis)
        out[1:-1] = (x[2:] - x[:-2]) / (2.0 * h)
        out[0] = (x[1] / 3.0 + x[0] - 4.0 * lo / 3.0) / h
        out[-1] = (4.0 * hi / 3.0 - x[-1] - x[-2] / 3.0) / h
        return np.moveaxis(out, 0, axis)
    if grid == "regular":
        below, above = x[1] - 2.0 * h * lo, x[n - 2] + 2.0 * h * hi
    else:
        below, above = x[0] - h * lo, x[-1] + h * hi
    ext = np.concatenate([below[None] if np.ndim(below) else np.full((1,) + x.shape[1:], below), x,
                          above[None] if np.ndim(above) else np.full((1,) + x.shape[1:], above)], axis=0)
    out[:] = (ext[2:] - ext[:-2]) / (2.0 * h)
    return np.moveaxis(out, 0, axis)


def fd_gradient(psi, bc, grid, hs, faces):
    """fd_derivative along every axis; faces {(axis, side): g} (output points
    of the other axes)."""
    faces = faces or {}
    return [fd_derivative(psi, bc, grid, hs[a], a, faces.get((a, 0)), faces.get((a, 1)))
            for a in range(np.ndim(psi))]


def periodic_derivative(psi, length, axis, order=1):
    """Spectral derivative of order 1 or 2 along one periodic axis (Section
    2.3.3, eq. ft_sd; the Nyquist wavenumber zeroed, as in periodic_gradient)."""
    psi = np.asarray(psi, dtype=np.float64)
    n = psi.shape[axis]
    m = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        m[n // 2] = 0.0
    k = 2.0 * np.pi * m / float(length)
    view = [1] * psi.ndim
    view[axis] = n
    factor = (1j * k) ** order
    return np.fft.ifft(factor.reshape(view) * np.fft.fft(psi, axis=axis), axis=axis).real


def mixed_derivative(psi, bcs, grid, nc, lengths, axis, order=1):
    """Derivative along `axis` of a mixed-boundary solution with homogeneous
    values: the eigenfunction series of that axis's own condition
    (bounded_derivative for Dirichlet / Neumann, periodic_derivative for a
    periodic axis), the other axes untouched."""
    if bcs[axis] == "periodic":
        return periodic_derivative(psi, lengths[axis], axis, order)
    return bounded_derivative(psi, bcs[axis], grid, nc, lengths, axis, order)


def fd_gradient_mixed(psi, bcs, grid, hs, faces):
    """fd_derivative along every axis of a mixed-boundary solve, each axis
    closed by its own condition."""
    faces = faces or {}
    return [fd_derivative(psi, bcs[a], grid, hs[a], a, faces.get((a, 0)), faces.get((a, 1)))
            for a in range(np.ndim(psi))]
