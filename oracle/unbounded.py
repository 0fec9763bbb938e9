"""Unbounded (free-space) solves of the oracle: the Hockney-Eastwood method.

Section 2.5 (sec:unbounded): the Green's function is laid out on a domain
doubled in every dimension and mirrored about the point N, the source is
doubled too with the added region set to zero, the periodic convolution is
done with DFTs, and the solution in the physical window is kept.  For real
data the R2C / C2R forms are used (Section 2.5.1); numpy's rfftn / irfftn
serve as those library primitives.

Readings of points the paper leaves open:
  * mirroring: per axis G_ext(m) = G(min(m, 2n - m) H) for m = 0 .. 2n-1;
  * quadrature: the discrete convolution carries the cell volume prod_a H_a;
  * kernel G2 (Section 2.5.2; formula not printed): the Gaussian-regularised
    3D kernel G(r) = -erf(r / (sqrt(2) sigma)) / (4 pi r), with
    G(0) = -1 / ((2 pi)^(3/2) sigma), which solves lap(G) = zeta_sigma, a unit
    Gaussian of standard deviation sigma; the sign follows lap(psi) = f of
    eq. (pois); sigma defaults to 2 H;
  * spectral derivatives (Section 2.3.3, eq. ft_sd) on the doubled grid use
    k_a = 2 pi m / (2 n_a H_a), m in (-n_a, n_a); the Nyquist mode m = n_a is
    given a zero derivative.
The curl output solves the curl Poisson problem of Section 4.3
(eq. poisscurl): psi = G * f first, then u = curl(psi) spectrally.
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def green_g2(r, sigma):
    """Gaussian-regularised 3D free-space Green's function (reading above)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    zero = r == 0.0
    rr = r[~zero]
    out[~zero] = -erf(rr / (SQRT2 * sigma)) / (4.0 * np.pi * rr)
    out[zero] = -1.0 / ((2.0 * np.pi) ** 1.5 * sigma)
    return out


def mirrored_distance(n, h):
    """Per-axis distances min(m, 2n - m) * H on the doubled grid."""
    m = np.arange(2 * n)
    return np.minimum(m, 2 * n - m).astype(np.float64) * float(h)


def green_extended(shape, hs, sigma):
    """G_ext on the doubled grid of the given physical shape (3D)."""
    if len(shape) != 3:
        raise NotImplementedError("the G2 kernel is the 3D kernel")
    dx = mirrored_distance(shape[0], hs[0])[:, None, None]
    dy = mirrored_distance(shape[1], hs[1])[None, :, None]
    dz = mirrored_distance(shape[2], hs[2])[None, None, :]
    return green_g2(np.sqrt(dx * dx + dy * dy + dz * dz), sigma)


def green_spectrum(shape, hs, sigma):
    """Ghat = DFT(G_ext) * prod(H) on the doubled grid (R2C layout)."""
    g = green_extended(shape, hs, sigma)
    return np.fft.rfftn(g) * float(np.prod(hs))


def wavenumbers(shape, hs):
    """Angular wavenumbers of the doubled grid in the R2C layout.

    Returns one broadcastable array per axis; the Nyquist entry is zero.
    """
    nd = len(shape)
    ks = []
    for a, n in enumerate(shape):
        mfull = 2 * n
        if a == nd - 1:
            m = np.arange(n + 1, dtype=np.float64)
        else:
            m = np.arange(mfull, dtype=np.float64)
            m = np.where(m < n, m, m - mfull)
        m[np.abs(m) == n] = 0.0
        k = 2.0 * np.pi * m / (mfull * float(hs[a]))
        view = [1] * nd
        view[a] = k.size
        ks.append(k.reshape(view))
    return ks


def _pad(f):
    big = np.zeros(tuple(2 * n for n in f.shape))
    big[tuple(slice(0, n) for n in f.shape)] = f
    return big


def _back(spec, shape):
    full = np.fft.irfftn(spec, s=tuple(2 * n for n in shape), axes=tuple(range(len(shape))))
    return full[tuple(slice(0, n) for n in shape)]


def solve_unbounded(f, hs, sigma, diff="none"):
    """Free-space solve of lap(psi) = f for a scalar or a 3-component field.

    f has shape (n_x, n_y, n_z) or (3, n_x, n_y, n_z).  Returns
    (psi, derivs): psi like f; derivs is [] for diff="none", the gradient
    components of a scalar psi for "grad", the curl of a 3-component psi for
    "curl".
    """
    f = np.asarray(f, dtype=np.float64)
    vector = f.ndim == 4
    comps = [f[c] for c in range(3)] if vector else [f]
    shape = comps[0].shape
    ghat = green_spectrum(shape, hs, sigma)
    psihat = [ghat * np.fft.rfftn(_pad(c)) for c in comps]
    psi = [_back(p, shape) for p in psihat]
    ks = wavenumbers(shape, hs)
    derivs = []
    if diff == "grad":
        if vector:
            raise ValueError("grad is defined here for a scalar field")
        derivs = [_back(1j * ks[a] * psihat[0], shape) for a in range(3)]
    elif diff == "curl":
        if not vector:
            raise ValueError("curl needs a 3-component field")
        kx, ky, kz = ks
        px, py, pz = psihat
        derivs = [
            _back(1j * (ky * pz - kz * py), shape),
            _back(1j * (kz * px - kx * pz), shape),
            _back(1j * (kx * py - ky * px), shape),
        ]
    elif diff != "none":
        raise ValueError(diff)
    psi_out = np.stack(psi) if vector else psi[0]
    return psi_out, derivs


def adjoint_unbounded(g_psi, g_derivs, hs, sigma, diff="none"):
    """Transpose of the map f -> (psi, derivs) of solve_unbounded.

    The forward map is K = R D G P: P pads to the doubled grid, G is the
    convolution with the real, even G_ext (symmetric), D the spectral
    derivative, R keeps the physical window.  Its transpose is P^T = R,
    G^T = G, R^T = P, and D^T: the curl (with the Nyquist mode zeroed) is
    symmetric, the gradient's transpose is minus the divergence.  So
    grad_f = R G P g_psi + R G C P g_u (curl) or R G P g_psi - R G div P g_grad.
    g_psi may be None (no upstream gradient on psi).
    """
    derivs = [np.asarray(d, dtype=np.float64) for d in (g_derivs or [])]
    if g_psi is not None:
        g_psi = np.asarray(g_psi, dtype=np.float64)
        vector = g_psi.ndim == 4
        shape = g_psi.shape[1:] if vector else g_psi.shape
    else:
        vector = diff == "curl"
        shape = derivs[0].shape
    ghat = green_spectrum(shape, hs, sigma)
    ks = wavenumbers(shape, hs)
    ncomp = 3 if vector else 1
    acc = []
    for c in range(ncomp):
        if g_psi is None:
            acc.append(np.zeros(ghat.shape, dtype=np.complex128))
        else:
            acc.append(np.fft.rfftn(_pad(g_psi[c] if vector else g_psi)))
    if diff == "curl":
        gu = [np.fft.rfftn(_pad(d)) for d in derivs]
        kx, ky, kz = ks
        acc[0] = acc[0] + 1j * (ky * gu[2] - kz * gu[1])
        acc[1] = acc[1] + 1j * (kz * gu[0] - kx * gu[2])
        acc[2] = acc[2] + 1j * (kx * gu[1] - ky * gu[0])
    elif diff == "grad":
        for a in range(3):
            acc[0] = acc[0] - 1j * ks[a] * np.fft.rfftn(_pad(derivs[a]))
    elif diff != "none":
        raise ValueError(diff)
    out = [_back(ghat * s, shape) for s in acc]
    return np.stack(out) if vector else out[0]


def psi_at(points, f, hs, sigma):
    """psi at selected output points by the direct sum of the discrete convolution.

    psi_i = prod(H) * sum_j G_ext(i - j) f_j, which is what the doubled-domain
    convolution computes inside the physical window (i - j never reaches the
    mirror point n).  points is a list of integer index triples.
    """
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape
    vol = float(np.prod(hs))
    out = []
    for p in points:
        dx = np.abs(np.arange(shape[0]) - p[0]) * hs[0]
        dy = np.abs(np.arange(shape[1]) - p[1]) * hs[1]
        dz = np.abs(np.arange(shape[2]) - p[2]) * hs[2]
        r = np.sqrt(dx[:, None, None] ** 2 + dy[None, :, None] ** 2 + dz[None, None, :] ** 2)
        out.append(vol * float(np.sum(green_g2(r, sigma) * f)))
    return np.array(out)
