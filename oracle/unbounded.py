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

Higher-order and spectral kernels (Section 2.5.2 names kernels of orders 2 to
10 and a spectral kernel without printing them).  Reading used here: each is
defined by its spectrum, G^(k) = -zeta^(k) / k^2, with
  * Gaussian order 2m: zeta^(k) = exp(-s) sum_{j<m} s^j / j!, s = k^2 sigma^2 / 2
    (the Gaussian times its own Taylor series truncated after m terms, so
    1 - zeta^ = O(k^(2m)) and the regularisation error is O(sigma^(2m)));
  * spectral: zeta^(k) = 1 for |k| <= k_c = pi / H, else 0 (H = max_a H_a).
Their radial inverse transforms G(r) = -(1 / (2 pi^2 r)) int_0^inf zeta^(k)
sin(k r) / k dk are, with rho = r / sigma and He_n the probabilists' Hermite
polynomials,
  G_2m(r) = -(1 / (4 pi r)) [erf(rho / sqrt2)
            + sqrt(2 / pi) exp(-rho^2 / 2) sum_{j=1}^{m-1} (-1)^(j-1) He_{2j-1}(rho) / (2^j j!)]
  (each j term from int_0^inf exp(-u^2/2) u^(2j-1) sin(u rho) du
   = (-1)^(j-1) sqrt(pi/2) He_{2j-1}(rho) exp(-rho^2/2)), and
  G_spectral(r) = -Si(k_c r) / (2 pi^2 r).
At r = 0 the limits are G_2m(0) = -(1 / ((2 pi)^(3/2) sigma)) sum_{j<m} C(2j, j) / 4^j
and G_spectral(0) = -k_c / (2 pi^2).  The closed forms are checked against the
spectral integrals by quadrature in the tests.

Lower dimensions (Section 2.5.2: spectral kernels in 1D, 2D and 3D, Gaussian
kernels of orders 2-10; in 1D the paper has only the spectral one, and the
Gaussian orders are added here), read through the same spectra; the
additive constant of each is fixed so that G approaches the unregularised
fundamental solution ((1 / 2 pi) ln r in 2D, |x| / 2 in 1D) at large r:
  2D, order 2m: G = (1 / 2 pi) [ln r + E1(rho^2 / 2) / 2
                 - sum_{j=1}^{m-1} exp(-rho^2 / 2) L_{j-1}(rho^2 / 2) / (2 j)]
     (L_n Laguerre polynomials; each j term from int_0^inf exp(-u^2/2)
      u^(2j-1) J0(u rho) du = 2^(j-1) (j-1)! exp(-rho^2/2) L_{j-1}(rho^2/2));
  2D, spectral:  G = (1 / 2 pi) [F(k_c r) - ln(k_c / 2) - gamma],
     F(x) = int_0^x (1 - J0(t)) / t dt;
  1D, order 2:   G = (x / 2) erf(x / (sqrt2 sigma)) + sigma exp(-x^2 / (2 sigma^2)) / sqrt(2 pi);
  1D, order 2m:  G2 + (sigma / sqrt(2 pi)) e^{-rho^2/2} sum_{j=1}^{m-1} (-1)^j He_{2j-2}(rho) / (2^j j!);
  1D, spectral:  G = (|x| Si(k_c |x|) + cos(k_c x) / k_c) / pi.
"""
import functools
import math

import numpy as np
from numpy.polynomial import hermite_e
from scipy import integrate
from scipy.special import erf, eval_hermitenorm, eval_laguerre, exp1, j0, sici

SQRT2 = math.sqrt(2.0)
EULER_GAMMA = 0.57721566490153286060651209008240243

# Green's kernels of the free-space solve: name -> Gaussian order (0: spectral)
KERNELS = {"g2": 2, "g4": 4, "g6": 6, "g8": 8, "g10": 10, "spectral": 0}


def green_g2(r, sigma):
    """Gaussian-regularised 3D free-space Green's function (reading above)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    zero = r == 0.0
    rr = r[~zero]
    out[~zero] = -erf(rr / (SQRT2 * sigma)) / (4.0 * np.pi * rr)
    out[zero] = -1.0 / ((2.0 * np.pi) ** 1.5 * sigma)
    return out


def green_gauss(r, sigma, order):
    """Gaussian-regularised 3D kernel of even order 2m (reading above)."""
    m = order // 2
    if order != 2 * m or m < 1:
        raise ValueError("order must be 2, 4, ..., 10")
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    zero = r == 0.0
    rr = r[~zero]
    rho = rr / sigma
    acc = erf(rho / SQRT2)
    for j in range(1, m):
        c = np.zeros(2 * j)
        c[2 * j - 1] = 1.0  # He_{2j-1}
        acc = acc + math.sqrt(2.0 / math.pi) * np.exp(-0.5 * rho * rho) * (
            (-1) ** (j - 1) * hermite_e.hermeval(rho, c) / (2.0 ** j * math.factorial(j)))
    out[~zero] = -acc / (4.0 * np.pi * rr)
    out[zero] = -sum(math.comb(2 * j, j) / 4.0 ** j for j in range(m)) / ((2.0 * np.pi) ** 1.5 * sigma)
    return out


def green_spectral(r, h):
    """Spectrally truncated 3D kernel, cutoff k_c = pi / h (reading above)."""
    kc = math.pi / h
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    zero = r == 0.0
    rr = r[~zero]
    out[~zero] = -sici(kc * rr)[0] / (2.0 * np.pi ** 2 * rr)
    out[zero] = -kc / (2.0 * np.pi ** 2)
    return out


def green_gauss_2d(r, sigma, order):
    """2D Gaussian-regularised kernel of order 2m (reading above)."""
    m = order // 2
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    zero = r == 0.0
    t = 0.5 * (r[~zero] / sigma) ** 2
    acc = np.log(r[~zero]) + 0.5 * exp1(t)
    for j in range(1, m):
        acc = acc - np.exp(-t) * eval_laguerre(j - 1, t) / (2.0 * j)
    out[~zero] = acc / (2.0 * np.pi)
    # r -> 0: ln r + E1(t)/2 -> (ln(2 sigma^2) - gamma) / 2, L_{j-1}(0) = 1
    out[zero] = (0.5 * (math.log(2.0 * sigma * sigma) - EULER_GAMMA)
                 - sum(1.0 / (2.0 * j) for j in range(1, m))) / (2.0 * np.pi)
    return out


@functools.lru_cache(maxsize=None)
def _one_minus_j0_integral(x):
    """F(x) = int_0^x (1 - J0(t)) / t dt by adaptive quadrature."""
    if x == 0.0:
        return 0.0
    pts = [j * math.pi for j in range(1, int(x / math.pi) + 1)][:500] or None
    val, _ = integrate.quad(lambda t: (1.0 - j0(t)) / t if t > 0 else 0.0, 0.0, x, limit=2000,
                            points=pts, epsabs=1e-15, epsrel=1e-14)
    return val


def green_spectral_2d(r, h):
    """2D spectrally truncated kernel, cutoff k_c = pi / h (reading above)."""
    kc = math.pi / h
    r = np.asarray(r, dtype=np.float64)
    F = np.vectorize(lambda x: _one_minus_j0_integral(float(x)))(kc * r)
    return (F - math.log(0.5 * kc) - EULER_GAMMA) / (2.0 * np.pi)


def green_g2_1d(x, sigma):
    """1D Gaussian-regularised kernel (reading above)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    return 0.5 * x * erf(x / (SQRT2 * sigma)) + sigma * np.exp(-0.5 * (x / sigma) ** 2) / math.sqrt(2.0 * np.pi)


def green_gauss_1d(x, sigma, order):
    """1D Gaussian-regularised kernel of order 2m (reading above): the order-2m
    source is the Gaussian times sum_{j<m} (-1)^j He_{2j}(rho) / (2^j j!), and
    since d^2/d rho^2 [e^{-rho^2/2} He_n] = e^{-rho^2/2} He_{n+2}, integrating
    twice adds (sigma / sqrt(2 pi)) e^{-rho^2/2} sum_{j=1}^{m-1} (-1)^j
    He_{2j-2}(rho) / (2^j j!) to the G2 kernel (no linear term: G stays even
    and keeps the far field |x| / 2)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    rho = x / sigma
    corr = np.zeros_like(x)
    for j in range(1, order // 2):
        corr = corr + (-1.0) ** j * eval_hermitenorm(2 * j - 2, rho) / (2.0 ** j * math.factorial(j))
    return green_g2_1d(x, sigma) + sigma * np.exp(-0.5 * rho * rho) / math.sqrt(2.0 * np.pi) * corr


def green_spectral_1d(x, h):
    """1D spectrally truncated kernel, cutoff k_c = pi / h (reading above)."""
    kc = math.pi / h
    x = np.abs(np.asarray(x, dtype=np.float64))
    return (x * sici(kc * x)[0] + np.cos(kc * x) / kc) / np.pi


def green(kernel, r, sigma, h, dim=3):
    """Kernel `kernel` of KERNELS in `dim` dimensions at distances r (sigma:
    Gaussian width, h: cutoff spacing)."""
    order = KERNELS[kernel]
    if dim == 2:
        return green_spectral_2d(r, h) if order == 0 else green_gauss_2d(r, sigma, order)
    if dim == 1:
        if order == 0:
            return green_spectral_1d(r, h)
        if order == 2:
            return green_g2_1d(r, sigma)
        return green_gauss_1d(r, sigma, order)
    if order == 0:
        return green_spectral(r, h)
    if order == 2:
        return green_g2(r, sigma)
    return green_gauss(r, sigma, order)


def mirrored_distance(n, h):
    """Per-axis distances min(m, 2n - m) * H on the doubled grid."""
    m = np.arange(2 * n)
    return np.minimum(m, 2 * n - m).astype(np.float64) * float(h)


def green_extended(shape, hs, sigma, kernel="g2"):
    """G_ext on the doubled grid of the given physical shape (1D, 2D or 3D)."""
    nd = len(shape)
    r2 = 0.0
    for a in range(nd):
        view = [1] * nd
        view[a] = 2 * shape[a]
        d = mirrored_distance(shape[a], hs[a]).reshape(view)
        r2 = r2 + d * d
    return green(kernel, np.sqrt(r2), sigma, max(hs), nd)


def green_spectrum(shape, hs, sigma, kernel="g2"):
    """Ghat = DFT(G_ext) * prod(H) on the doubled grid (R2C layout)."""
    g = green_extended(shape, hs, sigma, kernel)
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


def solve_unbounded(f, hs, sigma, diff="none", kernel="g2"):
    """Free-space solve of lap(psi) = f for a scalar or a 3-component field.

    f has shape (n_x,), (n_x, n_y), (n_x, n_y, n_z) or (3, n_x, n_y, n_z).  Returns
    (psi, derivs): psi like f; derivs is [] for diff="none", the gradient
    components of a scalar psi for "grad", the curl of a 3-component psi for
    "curl", its divergence for "div" and the Laplacian of every component for
    "nabla" (the spectral first derivative, Nyquist zeroed, applied twice per
    axis).  `kernel` names the Green's kernel (KERNELS).
    """
    f = np.asarray(f, dtype=np.float64)
    vector = f.ndim == 4
    comps = [f[c] for c in range(3)] if vector else [f]
    shape = comps[0].shape
    ghat = green_spectrum(shape, hs, sigma, kernel)
    psihat = [ghat * np.fft.rfftn(_pad(c)) for c in comps]
    psi = [_back(p, shape) for p in psihat]
    ks = wavenumbers(shape, hs)
    derivs = []
    if diff == "grad":
        if vector:
            raise ValueError("grad is defined here for a scalar field")
        derivs = [_back(1j * ks[a] * psihat[0], shape) for a in range(len(shape))]
    elif diff == "curl" and len(shape) == 2 and not vector:
        # 2D curl of a scalar (stream function): (d_y psi, -d_x psi)
        derivs = [_back(1j * ks[1] * psihat[0], shape), _back(-1j * ks[0] * psihat[0], shape)]
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
    elif diff == "div":
        if not vector:
            raise ValueError("div needs a 3-component field")
        derivs = [_back(sum(1j * ks[a] * psihat[a] for a in range(3)), shape)]
    elif diff == "nabla":
        # sum over axes of the spectral first derivative applied twice
        derivs = [_back(sum((1j * ks[a]) ** 2 for a in range(len(shape))) * p, shape) for p in psihat]
    elif diff != "none":
        raise ValueError(diff)
    psi_out = np.stack(psi) if vector else psi[0]
    return psi_out, derivs


def adjoint_unbounded(g_psi, g_derivs, hs, sigma, diff="none", kernel="g2"):
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
        shape = derivs[0].shape
        vector = (diff == "curl" and len(shape) == 3) or diff == "div" or (diff == "nabla" and len(derivs) == 3)
    ghat = green_spectrum(shape, hs, sigma, kernel)
    ks = wavenumbers(shape, hs)
    ncomp = 3 if vector else 1
    acc = []
    for c in range(ncomp):
        if g_psi is None:
            acc.append(np.zeros(ghat.shape, dtype=np.complex128))
        else:
            acc.append(np.fft.rfftn(_pad(g_psi[c] if vector else g_psi)))
    if diff == "curl" and len(shape) == 2:
        # transpose of (d_y, -d_x): -d_y g_0 + d_x g_1
        acc[0] = acc[0] - 1j * ks[1] * np.fft.rfftn(_pad(derivs[0])) + 1j * ks[0] * np.fft.rfftn(_pad(derivs[1]))
    elif diff == "curl":
        gu = [np.fft.rfftn(_pad(d)) for d in derivs]
        kx, ky, kz = ks
        acc[0] = acc[0] + 1j * (ky * gu[2] - kz * gu[1])
        acc[1] = acc[1] + 1j * (kz * gu[0] - kx * gu[2])
        acc[2] = acc[2] + 1j * (kx * gu[1] - ky * gu[0])
    elif diff == "grad":
        for a in range(len(shape)):
            acc[0] = acc[0] - 1j * ks[a] * np.fft.rfftn(_pad(derivs[a]))
    elif diff == "div":
        # the divergence's transpose is minus the gradient
        gd = np.fft.rfftn(_pad(derivs[0]))
        for c in range(3):
            acc[c] = acc[c] - 1j * ks[c] * gd
    elif diff == "nabla":
        # the Laplacian (a real even multiplier) is its own transpose
        lap = sum((1j * ks[a]) ** 2 for a in range(len(shape)))
        for c in range(ncomp):
            acc[c] = acc[c] + lap * np.fft.rfftn(_pad(derivs[c]))
    elif diff != "none":
        raise ValueError(diff)
    out = [_back(ghat * s, shape) for s in acc]
    return np.stack(out) if vector else out[0]


def psi_at(points, f, hs, sigma, kernel="g2"):
    """psi at selected output points by the direct sum of the discrete convolution.

    psi_i = prod(H) * sum_j G_ext(i - j) f_j, which is what the doubled-domain
    convolution computes inside the physical window (i - j never reaches the
    mirror point n).  points is a list of integer index triples.
    """
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape
    vol = float(np.prod(hs))
    nd = f.ndim
    out = []
    for p in points:
        r2 = 0.0
        for a in range(nd):
            view = [1] * nd
            view[a] = shape[a]
            r2 = r2 + ((np.arange(shape[a]) - p[a]) * hs[a]).reshape(view) ** 2
        out.append(vol * float(np.sum(green(kernel, np.sqrt(r2), sigma, max(hs), nd) * f)))
    return np.array(out)
