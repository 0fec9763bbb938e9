"""Pins of the oracle's free-space solves (oracle.unbounded).

  * Domain doubling (Section 2.5) equals the direct sum of the discrete
    convolution psi_i = prod(H) sum_j G(|x_i - x_j|) f_j (brute force written
    here, independent of the oracle's FFT path).
  * The G2 kernel satisfies lap(G) = unit Gaussian of width sigma (checked on
    its radial form by finite differences), tends to -1/(4 pi r), and is
    continuous at r = 0.
  * For a Gaussian source the G2 potential has the closed form
    -Q erf(r / (sqrt(2) s_eff)) / (4 pi r), Q = A (2 pi s^2)^(3/2),
    s_eff^2 = s^2 + sigma^2; the HE solve reproduces it to rounding.
  * Spectral gradient / curl (eq. ft_sd): transpose identities with the
    oracle's adjoint, the closed-form derivative of the Gaussian potential,
    and a divergence-free curl output.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import unbounded as ub


def brute_force(f, hs, sigma):
    nx, ny, nz = f.shape
    out = np.zeros_like(f)
    X, Y, Z = np.meshgrid(np.arange(nx) * hs[0], np.arange(ny) * hs[1], np.arange(nz) * hs[2], indexing="ij")
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                r = np.sqrt((X - i * hs[0]) ** 2 + (Y - j * hs[1]) ** 2 + (Z - k * hs[2]) ** 2)
                g = np.where(r > 0, -erf(r / (math.sqrt(2) * sigma)) / (4 * np.pi * np.where(r > 0, r, 1)),
                             -1.0 / ((2 * np.pi) ** 1.5 * sigma))
                out[i, j, k] = np.sum(g * f) * hs[0] * hs[1] * hs[2]
    return out


def test_doubling_equals_direct_sum():
    rng = np.random.default_rng(0)
    f = rng.normal(size=(6, 5, 7))
    hs = [0.1, 0.13, 0.09]
    psi, _ = ub.solve_unbounded(f, hs, 0.2)
    ref = brute_force(f, hs, 0.2)
    assert np.max(np.abs(psi - ref)) <= 1e-13 * np.max(np.abs(ref))
    pts = [(0, 0, 0), (5, 4, 6), (2, 3, 1)]
    assert np.allclose(ub.psi_at(pts, f, hs, 0.2), [ref[p] for p in pts], rtol=1e-13, atol=0)


def test_g2_kernel_properties():
    sigma = 0.3
    r = np.array([0.05, 0.2, 0.5, 1.0])
    d = 1e-4
    rg = lambda x: x * ub.green_g2(x, sigma)
    lap = (rg(r + d) - 2 * rg(r) + rg(r - d)) / d**2 / r
    gauss = np.exp(-r**2 / (2 * sigma**2)) / ((2 * np.pi) ** 1.5 * sigma**3)
    assert np.allclose(lap, gauss, rtol=1e-6)
    far = np.array([20 * sigma, 50 * sigma])
    assert np.allclose(ub.green_g2(far, sigma), -1 / (4 * np.pi * far), rtol=1e-15)
    assert abs(ub.green_g2(np.array([1e-7]), sigma)[0] - ub.green_g2(np.array([0.0]), sigma)[0]) < 1e-12


def blob_potential(X, Y, Z, c, A, s, sigma):
    Q = A * (2 * np.pi * s * s) ** 1.5
    se = math.sqrt(s * s + sigma * sigma)
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    rs = np.where(r > 0, r, 1.0)
    psi = np.where(r > 0, -Q * erf(rs / (math.sqrt(2) * se)) / (4 * np.pi * rs),
                   -Q * math.sqrt(2 / np.pi) / (4 * np.pi * se))
    # radial derivative dpsi/dr
    dpsi = np.where(r > 0, Q * erf(rs / (math.sqrt(2) * se)) / (4 * np.pi * rs**2)
                    - Q * math.sqrt(2 / np.pi) / se * np.exp(-rs**2 / (2 * se * se)) / (4 * np.pi * rs), 0.0)
    return psi, dpsi, r, (X - c[0], Y - c[1], Z - c[2])


@pytest.mark.parametrize("n", [32, 48])
def test_gaussian_closed_form(n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    c, A, s = (0.5, 0.47, 0.52), 1.3, 0.06
    f = A * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    sigma = 2 * h
    psi, _ = ub.solve_unbounded(f, [h, h, h], sigma)
    ref, _, _, _ = blob_potential(X, Y, Z, c, A, s, sigma)
    assert np.max(np.abs(psi - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_gradient_and_curl_closed_form():
    n = 48
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    c, A, s = (0.5, 0.5, 0.5), 1.0, 0.05
    sigma = 2 * h
    f = A * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * s * s))
    _, dpsi, r, d = blob_potential(X, Y, Z, c, A, s, sigma)
    rs = np.where(r > 0, r, 1.0)
    grad_a = [dpsi * d[a] / rs for a in range(3)]
    _, grad = ub.solve_unbounded(f, [h] * 3, sigma, "grad")
    scale = max(np.max(np.abs(g)) for g in grad_a)
    err = max(np.max(np.abs(grad[a] - grad_a[a])) for a in range(3)) / scale
    assert err < 1e-12
    # curl of psi e_z: (d_y psi, -d_x psi, 0)
    fv = np.stack([0 * f, 0 * f, f])
    _, curl = ub.solve_unbounded(fv, [h] * 3, sigma, "curl")
    ref = [grad_a[1], -grad_a[0], 0 * f]
    err = max(np.max(np.abs(curl[a] - ref[a])) for a in range(3)) / scale
    assert err < 1e-12


def test_curl_is_divergence_free():
    rng = np.random.default_rng(3)
    n = 16
    f = rng.normal(size=(3, n, n, n))
    h = 1.0 / n
    _, u = ub.solve_unbounded(f, [h] * 3, 2 * h, "curl")
    # divergence by the same spectral derivative on the doubled grid, computed here
    M = 2 * n
    m = np.fft.fftfreq(M, d=1.0 / M)
    m[M // 2] = 0
    k = 2 * np.pi * m / (M * h)
    full = [np.fft.irfftn(ub.green_spectrum((n, n, n), [h] * 3, 2 * h) * np.fft.rfftn(np.pad(fc, ((0, n),) * 3)), s=(M,) * 3, axes=(0, 1, 2)) for fc in f]
    spec = [np.fft.fftn(p) for p in full]
    K = np.meshgrid(k, k, k, indexing="ij")
    uhat = [1j * (K[1] * spec[2] - K[2] * spec[1]), 1j * (K[2] * spec[0] - K[0] * spec[2]),
            1j * (K[0] * spec[1] - K[1] * spec[0])]
    div = np.fft.ifftn(sum(1j * K[a] * uhat[a] for a in range(3))).real
    assert np.max(np.abs(div)) < 1e-10 * max(np.max(np.abs(x)) for x in u)
    # the window of that spectral curl is the oracle's curl
    for a in range(3):
        ua = np.fft.ifftn(uhat[a]).real[:n, :n, :n]
        assert np.max(np.abs(ua - u[a])) < 1e-12 * np.max(np.abs(u[a]))


@pytest.mark.parametrize("diff", ["none", "grad", "curl"])
def test_adjoint_identity(diff):
    rng = np.random.default_rng(11)
    shape = (6, 7, 5)
    hs = [0.1, 0.12, 0.08]
    sigma = 0.2
    vec = diff == "curl"
    a = rng.normal(size=((3,) + shape) if vec else shape)
    Ka_psi, Ka_d = ub.solve_unbounded(a, hs, sigma, diff)
    b_psi = rng.normal(size=Ka_psi.shape)
    b_d = [rng.normal(size=shape) for _ in Ka_d]
    lhs = np.sum(Ka_psi * b_psi) + sum(np.sum(x * y) for x, y in zip(Ka_d, b_d))
    rhs = np.sum(a * ub.adjoint_unbounded(b_psi, b_d, hs, sigma, diff))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300) * 10 + 1e-14
    if diff != "none":
        # derivative part alone (no upstream gradient on psi)
        lhs2 = sum(np.sum(x * y) for x, y in zip(Ka_d, b_d))
        rhs2 = np.sum(a * ub.adjoint_unbounded(None, b_d, hs, sigma, diff))
        assert abs(lhs2 - rhs2) <= 1e-11 * abs(lhs2)


def test_curl_operator_symmetric():
    """K = R curl G P maps 3 fields to 3 fields and is symmetric."""
    rng = np.random.default_rng(5)
    shape = (8, 8, 8)
    hs = [1 / 8] * 3
    a = rng.normal(size=(3,) + shape)
    b = rng.normal(size=(3,) + shape)
    _, Ka = ub.solve_unbounded(a, hs, 0.25, "curl")
    _, Kb = ub.solve_unbounded(b, hs, 0.25, "curl")
    lhs = sum(np.sum(Ka[c] * b[c]) for c in range(3))
    rhs = sum(np.sum(a[c] * Kb[c]) for c in range(3))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_regular_grid_is_the_node_convolution():
    """REGULAR free space (reading of the node count): N_c + 1 nodes per axis at
    spacing L / N_c, doubled to 2 (N_c + 1); the solve equals the direct sum of
    the discrete convolution over those nodes (3D brute force, 2D / 1D direct sums)."""
    import oracle
    rng = np.random.default_rng(3)
    nc = [5, 4, 6]
    hs = [0.1, 0.13, 0.09]
    lo = [0.0, -0.2, 0.5]
    hi = [lo[a] + hs[a] * nc[a] for a in range(3)]
    f = rng.normal(size=tuple(n + 1 for n in nc))
    psi, _ = oracle.solve("unbounded", "regular", nc, lo, hi, f, operator="g2", sigma_cells=2.0)
    assert psi.shape == f.shape
    ref = brute_force(f, hs, 2.0 * max(hs))
    assert np.max(np.abs(psi - ref)) <= 1e-13 * np.max(np.abs(ref))
    for nd, kernel in ((2, "g4"), (1, "spectral")):
        f = rng.normal(size=tuple(n + 1 for n in nc[:nd]))
        psi, _ = oracle.solve("unbounded", "regular", nc[:nd], lo[:nd], hi[:nd], f, operator=kernel,
                              sigma_cells=2.0)
        pts = [(0, 0), (5, 4), (2, 3)] if nd == 2 else [(0,), (5,), (3,)]
        got = [psi[p] for p in pts]
        want = ub.psi_at(pts, f, hs[:nd], 2.0 * max(hs[:nd]), kernel=kernel)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14), (nd, got, want)
