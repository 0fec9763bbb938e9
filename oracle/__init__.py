"""FP64 CPU oracle for the spectral Poisson solve -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the GPU library is checked
against.  It follows the paper (SailFFish, Section 2): forward transform,
pointwise spectral multiply, optional spectral derivative, backward
transform, for periodic, Dirichlet and Neumann boundaries (Table 1) and for
free space by domain doubling (Section 2.5).  Every transform is either its
textbook definition written out (the sine / cosine transforms) or a library
DFT (numpy.fft), in float64.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library.

Parity status of each function is recorded next to its pins in tests/.
"""
import numpy as np

from . import bounded, grid, transforms, unbounded

__all__ = ["bounded", "grid", "transforms", "unbounded", "solve", "zero_mode"]


def zero_mode(bc, grid_type, nc, lo, hi, f, faces=None):
    """The part of the source that the k = 0 projection removes (Section 2.2,
    the zero eigenvalue of periodic and Neumann problems): the k = 0
    coefficient of the forward transform of the right-hand side (boundary
    terms included, FD2) divided by the k = 0 coefficient of a field of ones.
    Zero for Dirichlet and free-space problems, and for compatible sources."""
    nd = len(nc)
    if isinstance(bc, (list, tuple)):
        # a condition per axis: a zero eigenvalue sum only without Dirichlet
        # (or free) axes
        if any(b not in ("periodic", "neumann") for b in bc):
            return 0.0
        hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
        f = np.asarray(f, dtype=np.float64)
        if faces:
            f = bounded.apply_boundary_values_mixed(f, list(bc), grid_type, hs, faces)
        a_hat, o_hat = f, np.ones_like(f)
        for a in range(nd):
            if bc[a] == "periodic":
                a_hat, o_hat = np.fft.fft(a_hat, axis=a).real, np.fft.fft(o_hat, axis=a).real
            else:
                fwd = bounded.TRANSFORM_PAIRS[(bc[a], grid_type)][0]
                a_hat, o_hat = transforms.apply(fwd, a_hat, a), transforms.apply(fwd, o_hat, a)
        return float(a_hat.flat[0] / o_hat.flat[0])
    if bc not in ("periodic", "neumann"):
        return 0.0
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    f = np.asarray(f, dtype=np.float64)
    if faces:
        f = bounded.apply_boundary_values(f, bc, grid_type, hs, faces)
    one = np.ones_like(f)
    if bc == "periodic":
        return float(np.fft.fftn(f).flat[0].real / np.fft.fftn(one).flat[0].real)
    fwd = bounded.TRANSFORM_PAIRS[(bc, grid_type)][0]
    a_hat, o_hat = f, one
    for a in range(nd):
        a_hat = transforms.apply(fwd, a_hat, a)
        o_hat = transforms.apply(fwd, o_hat, a)
    return float(a_hat.flat[0] / o_hat.flat[0])


def solve(bc, grid_type, nc, lo, hi, f, operator="ps", diff="none",
          faces=None, sigma_cells=2.0):
    """One solve described like the library's plan descriptor.

    bc: "periodic" | "dirichlet" | "neumann" | "unbounded", or one condition
        per axis (a list) for a mixed-boundary solve, at most one of them
        "unbounded" (a semi-unbounded solve, bounded.solve_semi)
    grid_type: "regular" | "staggered"
    nc, lo, hi: per-axis cell count and domain bounds (length = ndim)
    f: source on the unknown points (scalar), or (3, ...) for a 3D vector
    operator: "ps" | "fd2" for bounded BCs; for unbounded, the Green's kernel
              ("g2", "g4", "g6", "g8", "g10", "spectral"; anything else: "g2")
    diff: "none" | "grad" | "curl" | "div" | "nabla" (Section 2.3.3's operators,
          applied to psi: gradient of a scalar, curl or divergence of a 3D
          vector, Laplacian of every component; in 2D the curl of a scalar
          is (d_y psi, -d_x psi)).  Dirichlet / Neumann plans take every
          operator with homogeneous boundary values, as derivatives of the
          eigenfunction series (bounded.bounded_derivative)
    faces: {(axis, side): g} boundary values (FD2 Dirichlet / Neumann)
    Returns (psi, derivs) on the output points.
    """
    nd = len(nc)
    hs = [grid.spacing(lo[a], hi[a], nc[a]) for a in range(nd)]
    lengths = [float(hi[a]) - float(lo[a]) for a in range(nd)]
    f = np.asarray(f, dtype=np.float64)
    if isinstance(bc, (list, tuple)):
        # a condition per axis (bounded.solve_mixed, bounded.solve_semi);
        # derivatives of homogeneous solves per bounded axis by its own series
        # (bounded.mixed_derivative), along a free axis by the kernel's
        # derivative; with boundary values by FD2 differences
        bcs = list(bc)
        free = "unbounded" in bcs
        if diff != "none" and ((free and (faces or diff == "nabla")) or (faces and diff == "nabla")):
            raise NotImplementedError("mixed-boundary derivatives: no NABLA with boundary values or a free "
                                      "axis; free-axis plans homogeneous")
        vector = f.ndim == nd + 1
        comps = [f[c] for c in range(f.shape[0])] if vector else [f]
        solver = bounded.solve_semi if "unbounded" in bcs else bounded.solve_mixed
        psi = [solver(c, bcs, grid_type, operator, lengths, hs,
                      (faces[i] if (faces and vector) else faces))
               for i, c in enumerate(comps)]
        if free and diff != "none":
            # semi-unbounded: bounded axes by their series, the free axis by the
            # convolution with the kernel's derivative (bounded.solve_semi)
            u = bcs.index("unbounded")
            dfree = [bounded.solve_semi(c, bcs, grid_type, operator, lengths, hs, None, free_derivative=True)
                     for c in comps]
            d1 = lambda c, a: (dfree[c] if a == u else
                               bounded.mixed_derivative(psi[c], bcs, grid_type, nc, lengths, a, 1))
        elif faces and diff != "none":
            # boundary values: FD2 differences per axis (bounded.fd_gradient_mixed)
            face_c = (lambda c: faces[c]) if vector else (lambda c: faces)
            grads = [bounded.fd_gradient_mixed(psi[c], bcs, grid_type, hs, face_c(c)) for c in range(len(psi))]
            d1 = lambda c, a: grads[c][a]
        else:
            d1 = lambda c, a: bounded.mixed_derivative(psi[c], bcs, grid_type, nc, lengths, a, 1)
        if diff == "none":
            derivs = []
        elif diff == "grad" and not vector:
            derivs = [d1(0, a) for a in range(nd)]
        elif diff == "curl" and nd == 2 and not vector:
            derivs = [d1(0, 1), -d1(0, 0)]
        elif diff == "curl" and vector and nd == 3:
            derivs = [d1(2, 1) - d1(1, 2), d1(0, 2) - d1(2, 0), d1(1, 0) - d1(0, 1)]
        elif diff == "div" and vector and nd == 3:
            derivs = [d1(0, 0) + d1(1, 1) + d1(2, 2)]
        elif diff == "nabla":
            derivs = [sum(bounded.mixed_derivative(p, bcs, grid_type, nc, lengths, a, 2) for a in range(nd))
                      for p in psi]
        else:
            raise ValueError(diff)
        return (np.stack(psi) if vector else psi[0]), derivs
    if bc == "unbounded":
        sigma = float(sigma_cells) * max(hs)
        kernel = operator if operator in unbounded.KERNELS else "g2"
        return unbounded.solve_unbounded(f, hs, sigma, diff, kernel)
    vector = f.ndim == nd + 1
    comps = [f[c] for c in range(f.shape[0])] if vector else [f]
    psi = [bounded.solve_bounded(c, bc, grid_type, operator, lengths, hs, faces if not vector else (faces[i] if faces else None))
           for i, c in enumerate(comps)]
    derivs = []
    if diff != "none" and bc != "periodic" and faces:
        # boundary values: centred FD2 differences closed by the ghost rules
        # (bounded.fd_derivative); first-derivative operators only
        face_c = (lambda c: faces[c]) if vector else (lambda c: faces)
        grads = [bounded.fd_gradient(psi[c], bc, grid_type, hs, face_c(c)) for c in range(len(psi))]
        if diff == "grad" and not vector:
            derivs = grads[0]
        elif diff == "curl" and nd == 2 and not vector:
            derivs = [grads[0][1], -grads[0][0]]
        elif diff == "curl" and vector and nd == 3:
            g = grads
            derivs = [g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]]
        elif diff == "div" and vector and nd == 3:
            derivs = [grads[0][0] + grads[1][1] + grads[2][2]]
        else:
            raise NotImplementedError("boundary values: GRAD, CURL and DIV")
    elif diff != "none" and bc != "periodic":
        if diff == "grad":
            if vector:
                raise NotImplementedError("gradient: scalar only")
            derivs = bounded.bounded_gradient(psi[0], bc, grid_type, nc, lengths)
        elif diff == "nabla":
            derivs = [bounded.bounded_laplacian(p, bc, grid_type, nc, lengths) for p in psi]
        elif diff == "div":
            if not vector or nd != 3:
                raise NotImplementedError("divergence: 3D vector only")
            derivs = [sum(bounded.bounded_derivative(psi[c], bc, grid_type, nc, lengths, c, 1)
                          for c in range(3))]
        elif diff == "curl" and nd == 2 and not vector:
            g = bounded.bounded_gradient(psi[0], bc, grid_type, nc, lengths)
            derivs = [g[1], -g[0]]
        elif diff == "curl":
            if not vector or nd != 3:
                raise NotImplementedError("curl: 3D vector or 2D scalar")
            derivs = bounded.bounded_curl(psi, bc, grid_type, nc, lengths)
        else:
            raise ValueError(diff)
    elif diff == "grad":
        if vector:
            raise NotImplementedError("periodic gradient: scalar only")
        derivs = bounded.periodic_gradient(psi[0], lengths)
    elif diff == "curl" and nd == 2 and not vector:
        # 2D curl of a scalar (stream function): (d_y psi, -d_x psi)
        g = bounded.periodic_gradient(psi[0], lengths)
        derivs = [g[1], -g[0]]
    elif diff == "curl":
        if not vector or nd != 3:
            raise NotImplementedError("curl: 3D vector or 2D scalar")
        derivs = bounded.periodic_curl(psi, lengths)
    elif diff == "div":
        if not vector or nd != 3:
            raise NotImplementedError("divergence: 3D vector only")
        derivs = [sum(bounded.periodic_gradient(psi[c], lengths)[c] for c in range(3))]
    elif diff == "nabla":
        # the spectral first derivative (Nyquist zeroed) applied twice per axis
        derivs = [sum(bounded.periodic_gradient(bounded.periodic_gradient(p, lengths)[a], lengths)[a]
                      for a in range(nd)) for p in psi]
    elif diff != "none":
        raise ValueError(diff)
    return (np.stack(psi) if vector else psi[0]), derivs
