"""Pins of the oracle's higher-order Gaussian and spectral free-space kernels
(3D, and the 2D / 1D kernels).

Each kernel is defined by its spectrum G^(k) = -zeta^(k) / k^2 (the reading of
Section 2.5.2 stated in oracle/unbounded.py).  The checks here do not reuse
the closed forms they test:
  * the closed form equals the radial inverse transform of the spectrum,
    -(1 / (2 pi^2 r)) int zeta^(k) sin(k r) / k dk, done by adaptive
    quadrature of the definition;
  * r -> 0 limits and the far field -1 / (4 pi r);
  * the order: with a unit Gaussian source the regularisation error of the
    order-2m kernel falls by 4^m when sigma halves;
  * whole free-space solves (domain doubling) of a resolved Gaussian blob
    match its potential: the order-2m kernel's closed form (the same
    derivation with the source width folded in), and for the spectral kernel
    the exact unregularised potential (the band limit removes nothing a
    resolved blob holds).
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf

from oracle import unbounded as ub

ORDERS = [2, 4, 6, 8, 10]


def zeta_hat(k, sigma, order):
    s = 0.5 * (k * sigma) ** 2
    return math.exp(-s) * sum(s ** j / math.factorial(j) for j in range(order // 2))


def radial_inverse(zh, r, kmax, points=None):
    """-(1 / (2 pi^2 r)) int_0^kmax zh(k) sin(k r) / k dk by adaptive quadrature."""
    def f(k):
        return zh(k) * (math.sin(k * r) / k if k > 0 else r)
    val, err = integrate.quad(f, 0.0, kmax, limit=2000, epsabs=1e-16, epsrel=1e-14, points=points)
    return -val / (2.0 * math.pi ** 2 * r)


@pytest.mark.parametrize("order", ORDERS)
def test_gauss_kernel_is_its_spectral_integral(order):
    sigma = 0.1
    rs = np.array([1e-3, 0.05, 0.3, 1.0, 2.5, 5.0, 9.0]) * sigma
    got = ub.green_gauss(rs, sigma, order) if order > 2 else ub.green_g2(rs, sigma)
    for r, g in zip(rs, got):
        # split the range at the zeros of sin(k r) that fall inside it
        kmax = 40.0 / sigma
        pts = [j * math.pi / r for j in range(1, int(kmax * r / math.pi) + 1)][:200]
        ref = radial_inverse(lambda k: zeta_hat(k, sigma, order), r, kmax, pts or None)
        assert abs(g - ref) <= 1e-10 * abs(ref), (order, r, g, ref)


@pytest.mark.parametrize("order", ORDERS[1:])
def test_gauss_kernel_limits(order):
    sigma = 0.07
    g0 = ub.green_gauss(np.array([0.0]), sigma, order)[0]
    g_small = ub.green_gauss(np.array([1e-7 * sigma]), sigma, order)[0]
    assert abs(g_small - g0) <= 1e-12 * abs(g0)
    far = np.array([40.0, 60.0]) * sigma
    assert np.allclose(ub.green_gauss(far, sigma, order), -1.0 / (4 * np.pi * far), rtol=1e-14, atol=0)
    # at order 2 the general form reduces to the G2 kernel
    r = np.linspace(0.0, 5 * sigma, 11)
    assert np.allclose(ub.green_gauss(r, sigma, 2), ub.green_g2(r, sigma), rtol=1e-14, atol=0)


def test_spectral_kernel_is_its_spectral_integral():
    h = 0.02
    kc = math.pi / h
    rs = np.array([1e-3, 0.3, 1.0, 5.0, 20.0, 70.0]) * h
    got = ub.green_spectral(rs, h)
    for r, g in zip(rs, got):
        pts = [j * math.pi / r for j in range(1, int(kc * r / math.pi) + 1)] or None
        ref = radial_inverse(lambda k: 1.0, r, kc, pts)
        assert abs(g - ref) <= 1e-11 * abs(ref), (r, g, ref)
    g0 = ub.green_spectral(np.array([0.0]), h)[0]
    assert abs(ub.green_spectral(np.array([1e-8 * h]), h)[0] - g0) <= 1e-12 * abs(g0)
    assert abs(g0 + kc / (2 * math.pi ** 2)) <= 1e-15 * abs(g0)


def blob_potential_gauss(r, Q, s, sigma, order):
    """Potential of A exp(-r^2 / (2 s^2)) (charge Q) through the order-2m kernel."""
    S = math.sqrt(s * s + sigma * sigma)
    rho = r / S
    acc = erf(rho / math.sqrt(2))
    for j in range(1, order // 2):
        he = np.polynomial.hermite_e.hermeval(rho, [0] * (2 * j - 1) + [1])
        acc = acc + math.sqrt(2 / math.pi) * np.exp(-0.5 * rho * rho) * (sigma / S) ** (2 * j) * (
            (-1) ** (j - 1) * he / (2 ** j * math.factorial(j)))
    return -Q * acc / (4 * np.pi * r)


@pytest.mark.parametrize("order", ORDERS)
def test_gauss_regularisation_order(order):
    # unit-width source; the error against the exact potential scales as sigma^order
    r = np.linspace(0.05, 6.0, 400)
    exact = -erf(r / math.sqrt(2)) / (4 * np.pi * r)
    # (order 10 at sigma = 0.05 reaches the FP64 floor: one step coarser there)
    sigmas = (0.2, 0.1) if order == 10 else (0.1, 0.05)
    e = [np.max(np.abs(blob_potential_gauss(r, 1.0, 1.0, sg, order) - exact)) for sg in sigmas]
    rate = math.log2(e[0] / e[1])
    assert abs(rate - order) < 0.2, (order, rate)


def _blob_grid(n, c, A, s):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    return h, r, A * np.exp(-r * r / (2 * s * s))


@pytest.mark.parametrize("order", [4, 6, 8, 10])
def test_gauss_kernel_blob_solve(order):
    n, c, A, s = 48, (0.5, 0.47, 0.52), 1.3, 0.06
    h, r, f = _blob_grid(n, c, A, s)
    sigma = 2 * h
    psi, _ = ub.solve_unbounded(f, [h] * 3, sigma, kernel=f"g{order}")
    Q = A * (2 * np.pi * s * s) ** 1.5
    ref = blob_potential_gauss(r, Q, s, sigma, order)
    assert np.max(np.abs(psi - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_spectral_kernel_blob_solve():
    n, c, A, s = 48, (0.5, 0.47, 0.52), 0.9, 0.06
    h, r, f = _blob_grid(n, c, A, s)
    psi, _ = ub.solve_unbounded(f, [h] * 3, 2 * h, kernel="spectral")
    Q = A * (2 * np.pi * s * s) ** 1.5
    ref = -Q * erf(r / (math.sqrt(2) * s)) / (4 * np.pi * r)
    assert np.max(np.abs(psi - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kernel", ["g6", "spectral"])
def test_new_kernels_direct_sum(kernel):
    # the doubled-domain convolution equals the direct sum of the discrete convolution
    rng = np.random.default_rng(21)
    f = rng.normal(size=(6, 5, 7))
    hs = [0.1, 0.13, 0.09]
    psi, _ = ub.solve_unbounded(f, hs, 0.2, kernel=kernel)
    pts = [(0, 0, 0), (5, 4, 6), (2, 3, 1), (4, 0, 5)]
    assert np.allclose(ub.psi_at(pts, f, hs, 0.2, kernel=kernel), [psi[p] for p in pts], rtol=1e-13, atol=0)


# ------------------------------------------------------------------ 1D and 2D
from scipy.special import exp1, j0 as bessel_j0


def radial_inverse_2d_diff(zh, r, r0, kmax):
    """G(r) - G(r0) = -(1 / 2 pi) int_0^kmax zh(k) (J0(k r) - J0(k r0)) / k dk."""
    pts = sorted(set([j * math.pi / r for j in range(1, int(kmax * r / math.pi) + 1)][:300]
                     + [j * math.pi / r0 for j in range(1, int(kmax * r0 / math.pi) + 1)][:300])) or None
    val, _ = integrate.quad(lambda k: zh(k) * (bessel_j0(k * r) - bessel_j0(k * r0)) / k if k > 0 else 0.0,
                            0.0, kmax, limit=4000, points=pts, epsabs=1e-15, epsrel=1e-13)
    return -val / (2 * math.pi)


@pytest.mark.parametrize("order", ORDERS)
def test_gauss_2d_kernel_is_its_spectral_integral(order):
    sigma = 0.1
    r0 = 0.5 * sigma
    g0 = ub.green(f"g{order}", np.array([r0]), sigma, 1.0, dim=2)[0]
    for r in np.array([0.0, 0.05, 1.0, 2.5, 6.0]) * sigma:
        g = ub.green(f"g{order}", np.array([r]), sigma, 1.0, dim=2)[0]
        ref = radial_inverse_2d_diff(lambda k: zeta_hat(k, sigma, order), r, r0, 40.0 / sigma)
        assert abs((g - g0) - ref) <= 1e-10 * max(abs(ref), 1e-3), (order, r, g - g0, ref)
    far = np.array([40.0, 80.0]) * sigma
    assert np.allclose(ub.green(f"g{order}", far, sigma, 1.0, dim=2), np.log(far) / (2 * np.pi),
                       rtol=1e-13, atol=0)


def test_spectral_2d_kernel_is_its_spectral_integral():
    h = 0.05
    kc = math.pi / h
    r0 = 0.7 * h
    g0 = ub.green("spectral", np.array([r0]), 0.1, h, dim=2)[0]
    for r in np.array([0.0, 0.3, 1.0, 4.0, 11.0]) * h:
        g = ub.green("spectral", np.array([r]), 0.1, h, dim=2)[0]
        ref = radial_inverse_2d_diff(lambda k: 1.0, r, r0, kc)
        assert abs((g - g0) - ref) <= 1e-10 * max(abs(ref), 1e-3), (r, g - g0, ref)
    # large r: the unregularised (1 / 2 pi) ln r, up to an O(1 / (k_c r)^(3/2)) oscillation
    far = np.array([3000.0, 7000.0]) * h
    assert np.allclose(ub.green("spectral", far, 0.1, h, dim=2), np.log(far) / (2 * np.pi), rtol=0,
                       atol=2e-4)


@pytest.mark.parametrize("kernel", ["g2", "g4", "g6", "g8", "g10", "spectral"])
def test_1d_kernels_are_their_spectral_integrals(kernel):
    sigma, h = 0.1, 0.05
    kc = math.pi / h
    zh = (lambda k: zeta_hat(k, sigma, int(kernel[1:]))) if kernel != "spectral" else (lambda k: 1.0)
    kmax = kc if kernel == "spectral" else 40.0 / sigma
    g0 = ub.green(kernel, np.array([0.0]), sigma, h, dim=1)[0]
    for x in [0.02, 0.1, 0.37, 1.3]:
        g = ub.green(kernel, np.array([x]), sigma, h, dim=1)[0]
        # G(x) - G(0) = -(1 / pi) int zh(k) (cos(k x) - 1) / k^2 dk (break points at the
        # zeros of cos(k x) - 1 for the cutoff spectrum; the Gaussian spectra are smooth)
        pts = ([j * math.pi / x for j in range(1, int(kmax * x / math.pi) + 1)][:300] or None
               if kernel == "spectral" else None)
        val, _ = integrate.quad(lambda k: zh(k) * (math.cos(k * x) - 1) / (k * k) if k > 0 else -0.5 * x * x,
                                0.0, kmax, limit=4000, points=pts, epsabs=1e-16, epsrel=1e-14)
        ref = -val / math.pi  # (the spectral kernel's spectrum stops at k_c)
        assert abs((g - g0) - ref) <= 1e-10 * abs(ref), (kernel, x, g - g0, ref)
    assert np.allclose(ub.green(kernel, np.array([50.0, 80.0]), sigma, h, dim=1), [25.0, 40.0], rtol=0,
                       atol=1e-3)


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10])
def test_1d_gauss_kernel_second_derivative_is_its_source(order):
    """G'' = zeta_2m, the Gaussian times sum_{j<m} (-1)^j He_2j(rho) / (2^j j!) (the
    inverse transform of zeta^ = exp(-s) sum_{j<m} s^j / j!), by central differences."""
    from scipy.special import eval_hermitenorm
    sigma = 0.1
    d = 1e-3 * sigma
    for x in (0.0, 0.07, 0.19, 0.33):
        G = lambda y: ub.green(f"g{order}", np.array([y]), sigma, 1.0, dim=1)[0]
        gpp = (G(x + d) - 2 * G(x) + G(x - d)) / d ** 2
        rho = x / sigma
        zeta = math.exp(-0.5 * rho * rho) / (math.sqrt(2 * math.pi) * sigma) * sum(
            (-1) ** j * eval_hermitenorm(2 * j, rho) / (2 ** j * math.factorial(j)) for j in range(order // 2))
        assert abs(gpp - zeta) <= 1e-5 * max(abs(zeta), 1.0 / sigma), (order, x, gpp, zeta)


@pytest.mark.parametrize("kernel", ["g2", "g4", "g6", "spectral"])
def test_2d_blob_solve(kernel):
    n = 64
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    c, A, s = (0.5, 0.47), 1.2, 0.06
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2)
    f = A * np.exp(-r * r / (2 * s * s))
    sigma = 2 * h
    psi, _ = ub.solve_unbounded(f, [h, h], sigma, kernel=kernel)
    Q = A * 2 * np.pi * s * s
    S = s if kernel == "spectral" else math.sqrt(s * s + sigma * sigma)
    t = 0.5 * (r / S) ** 2
    ref = np.log(r) + 0.5 * exp1(t)
    if kernel != "spectral":
        from scipy.special import eval_laguerre
        for j in range(1, int(kernel[1:]) // 2):
            ref = ref - (sigma / S) ** (2 * j) * np.exp(-t) * eval_laguerre(j - 1, t) / (2 * j)
    ref = Q * ref / (2 * np.pi)
    assert np.max(np.abs(psi - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kernel,dim", [("g4", 2), ("spectral", 2), ("g2", 1), ("g8", 1), ("spectral", 1)])
def test_low_dim_direct_sum(kernel, dim):
    rng = np.random.default_rng(22)
    shape = (7, 5)[:dim] if dim == 2 else (9,)
    f = rng.normal(size=shape)
    hs = [0.1, 0.13][:dim]
    psi, _ = ub.solve_unbounded(f, hs, 0.2, kernel=kernel)
    pts = [(0, 0), (6, 4), (3, 2)] if dim == 2 else [(0,), (8,), (4,)]
    assert np.allclose(ub.psi_at(pts, f, hs, 0.2, kernel=kernel), [psi[p] for p in pts], rtol=1e-13, atol=0)
