"""Pins of the oracle's DIV and NABLA operators (Section 2.3.3 lists DIV, GRAD,
CURL and NABLA; they act on psi after the convolution, as in Section 4.3).

NABLA is read as the spectral first derivative (Nyquist mode zeroed) applied
twice per axis and summed; DIV as the sum of the components' own derivatives.
  * periodic PS: for a source of Fourier modes below the Nyquist index the
    Laplacian of psi is the source itself, and the divergence of psi is a
    closed form per mode;
  * free space, spectral kernel: the Laplacian of psi of a resolved Gaussian
    blob is the blob itself;
  * free space, G2 kernel: the divergence of psi of the field (blob, 0, 0) is
    the closed-form x-derivative of the blob's potential;
  * the transposes used by the adjoint: <K a, b> = <a, K^T b>.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle import unbounded as ub


def _modes(rng, n, lengths, count):
    out = []
    for _ in range(count):
        m = [int(rng.integers(-(na // 2) + 1, na // 2)) for na in n]
        if all(v == 0 for v in m):
            m[0] = 1
        out.append((m, rng.normal(), rng.uniform(0, 2 * np.pi)))
    return out


def _grid(n, lo, hi):
    xs = [lo[a] + (np.arange(n[a]) + 0.5) * (hi[a] - lo[a]) / n[a] for a in range(len(n))]
    return np.meshgrid(*xs, indexing="ij")


def test_periodic_nabla_returns_source():
    rng = np.random.default_rng(31)
    n, lo, hi = (12, 10, 8), [0.0, -0.5, 1.0], [1.0, 1.3, 2.5]
    L = [hi[a] - lo[a] for a in range(3)]
    X = _grid(n, lo, hi)
    f = np.zeros(n)
    for m, A, ph in _modes(rng, n, L, 6):
        f += A * np.cos(sum(2 * np.pi * m[a] * (X[a] - lo[a]) / L[a] for a in range(3)) + ph)
    psi, (lap,) = oracle.solve("periodic", "staggered", list(n), lo, hi, f, operator="ps", diff="nabla")
    assert np.max(np.abs(lap - f)) <= 1e-12 * np.max(np.abs(f))


def test_periodic_div_closed_form():
    rng = np.random.default_rng(32)
    n, lo, hi = (10, 12, 14), [0.0, 0.0, 0.0], [1.0, 1.5, 0.8]
    L = [hi[a] - lo[a] for a in range(3)]
    X = _grid(n, lo, hi)
    f = np.zeros((3,) + n)
    ref = np.zeros(n)
    for c in range(3):
        for m, A, ph in _modes(rng, n, L, 3):
            k = [2 * np.pi * m[a] / L[a] for a in range(3)]
            th = sum(k[a] * (X[a] - lo[a]) for a in range(3)) + ph
            f[c] += A * np.cos(th)
            k2 = sum(v * v for v in k)
            # psi_c = -A cos(th) / |k|^2, d_c psi_c = A k_c sin(th) / |k|^2
            ref += A * k[c] * np.sin(th) / k2
    _, (div,) = oracle.solve("periodic", "staggered", list(n), lo, hi, f, operator="ps", diff="div")
    assert np.max(np.abs(div - ref)) <= 1e-12 * np.max(np.abs(ref))


def _blob(n, c, A, s):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    d = (X - c[0], Y - c[1], Z - c[2])
    r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
    return h, r, d, A * np.exp(-r * r / (2 * s * s))


def test_unbounded_spectral_nabla_returns_source():
    h, r, _, f = _blob(48, (0.5, 0.47, 0.52), 1.1, 0.06)
    _, (lap,) = ub.solve_unbounded(f, [h] * 3, 2 * h, "nabla", kernel="spectral")
    assert np.max(np.abs(lap - f)) <= 1e-11 * np.max(np.abs(f))


def test_unbounded_g2_div_closed_form():
    h, r, d, b = _blob(48, (0.5, 0.5, 0.47), 0.8, 0.05)
    sigma = 2 * h
    fv = np.stack([b, 0 * b, 0 * b])
    _, (div,) = ub.solve_unbounded(fv, [h] * 3, sigma, "div")
    Q = 0.8 * (2 * np.pi * 0.05 ** 2) ** 1.5
    se = math.sqrt(0.05 ** 2 + sigma ** 2)
    dpsi = (Q * erf(r / (math.sqrt(2) * se)) / (4 * np.pi * r ** 2)
            - Q * math.sqrt(2 / np.pi) / se * np.exp(-r ** 2 / (2 * se * se)) / (4 * np.pi * r))
    ref = dpsi * d[0] / r
    assert np.max(np.abs(div - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("diff,vec", [("div", True), ("nabla", False), ("nabla", True)])
def test_div_nabla_transposes(diff, vec):
    rng = np.random.default_rng(12)
    shape = (6, 7, 5)
    hs = [0.1, 0.12, 0.08]
    a = rng.normal(size=((3,) + shape) if vec else shape)
    Ka_psi, Ka_d = ub.solve_unbounded(a, hs, 0.2, diff)
    b_psi = rng.normal(size=Ka_psi.shape)
    b_d = [rng.normal(size=shape) for _ in Ka_d]
    lhs = np.sum(Ka_psi * b_psi) + sum(np.sum(x * y) for x, y in zip(Ka_d, b_d))
    rhs = np.sum(a * ub.adjoint_unbounded(b_psi, b_d, hs, 0.2, diff))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    lhs2 = sum(np.sum(x * y) for x, y in zip(Ka_d, b_d))
    rhs2 = np.sum(a * ub.adjoint_unbounded(None, b_d, hs, 0.2, diff))
    assert abs(lhs2 - rhs2) <= 1e-11 * abs(lhs2)


def test_unbounded_2d_curl_closed_form():
    # spectral kernel: psi is the exact potential of the resolved blob
    n = 64
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    c, A, s = (0.5, 0.47), 1.0, 0.06
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2)
    f = A * np.exp(-r * r / (2 * s * s))
    _, (u0, u1) = ub.solve_unbounded(f, [h, h], 2 * h, "curl", kernel="spectral")
    Q = A * 2 * np.pi * s * s
    dpsi = Q * (1 - np.exp(-r * r / (2 * s * s))) / (2 * np.pi * r)  # d psi / d r
    ref0, ref1 = dpsi * (Y - c[1]) / r, -dpsi * (X - c[0]) / r
    scale = np.max(np.abs(ref0))
    assert np.max(np.abs(u0 - ref0)) <= 1e-11 * scale and np.max(np.abs(u1 - ref1)) <= 1e-11 * scale


def test_periodic_2d_curl_closed_form():
    n, lo, hi = (12, 10), [0.0, 0.0], [1.0, 1.5]
    L = [1.0, 1.5]
    x = [(np.arange(n[a]) + 0.5) * L[a] / n[a] for a in range(2)]
    X, Y = np.meshgrid(*x, indexing="ij")
    kx, ky = 2 * np.pi * 2 / L[0], 2 * np.pi * 3 / L[1]
    f = np.cos(kx * X + ky * Y + 0.3)
    _, (u0, u1) = oracle.solve("periodic", "staggered", list(n), lo, hi, f, operator="ps", diff="curl")
    k2 = kx * kx + ky * ky
    # psi = -cos(th) / k2: d_y psi = ky sin(th) / k2, -d_x psi = -kx sin(th) / k2
    th = kx * X + ky * Y + 0.3
    assert np.max(np.abs(u0 - ky * np.sin(th) / k2)) <= 1e-13 and np.max(np.abs(u1 + kx * np.sin(th) / k2)) <= 1e-13


def test_unbounded_2d_curl_transpose():
    rng = np.random.default_rng(14)
    shape, hs = (7, 9), [0.1, 0.12]
    a = rng.normal(size=shape)
    Ka_psi, Ka_d = ub.solve_unbounded(a, hs, 0.2, "curl")
    b_psi = rng.normal(size=shape)
    b_d = [rng.normal(size=shape) for _ in Ka_d]
    lhs = np.sum(Ka_psi * b_psi) + sum(np.sum(x * y) for x, y in zip(Ka_d, b_d))
    rhs = np.sum(a * ub.adjoint_unbounded(b_psi, b_d, hs, 0.2, "curl"))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _vector_modes_3d(seed, n, lo, hi, per_comp):
    """A 3-component source of Fourier modes below the Nyquist index on an
    anisotropic periodic box, with the closed forms of the PS solution per
    mode: f_c = A cos(th), th = k.(x - lo) + phase; psi_c = -A cos(th) / |k|^2
    and d_a psi_c = A k_a sin(th) / |k|^2 (Section 2.2, eq. spect_sol with the
    PS multiplier -|k|^2; eq. ft_sd for the derivative)."""
    rng = np.random.default_rng(seed)
    L = [hi[a] - lo[a] for a in range(3)]
    X = _grid(n, lo, hi)
    f = np.zeros((3,) + tuple(n))
    psi = np.zeros_like(f)
    dpsi = np.zeros((3, 3) + tuple(n))  # [component][axis]
    for c in range(3):
        for m, A, ph in _modes(rng, n, L, per_comp):
            k = [2 * np.pi * m[a] / L[a] for a in range(3)]
            th = sum(k[a] * (X[a] - lo[a]) for a in range(3)) + ph
            k2 = sum(v * v for v in k)
            f[c] += A * np.cos(th)
            psi[c] -= A * np.cos(th) / k2
            for a in range(3):
                dpsi[c, a] += A * k[a] * np.sin(th) / k2
    return f, psi, dpsi


def test_periodic_3d_curl_closed_form():
    # u = curl psi per mode: u_x = d_y psi_z - d_z psi_y, u_y = d_z psi_x -
    # d_x psi_z, u_z = d_x psi_y - d_y psi_x (Section 4.3, eq. poisscurl)
    n, lo, hi = (12, 10, 14), [0.0, -0.4, 0.3], [1.0, 1.1, 1.1]
    f, psi_ref, d = _vector_modes_3d(41, n, lo, hi, 4)
    psi, u = oracle.solve("periodic", "staggered", list(n), lo, hi, f, operator="ps", diff="curl")
    ref = [d[2, 1] - d[1, 2], d[0, 2] - d[2, 0], d[1, 0] - d[0, 1]]
    assert np.max(np.abs(psi - psi_ref)) <= 1e-12 * np.max(np.abs(psi_ref))
    for c in range(3):
        scale = max(np.max(np.abs(r)) for r in ref)
        assert np.max(np.abs(u[c] - ref[c])) <= 1e-12 * scale, c


def test_periodic_3d_gradient_closed_form():
    n, lo, hi = (10, 12, 8), [0.2, 0.0, -1.0], [1.0, 1.7, 0.5]
    f, psi_ref, d = _vector_modes_3d(42, n, lo, hi, 5)
    psi, g = oracle.solve("periodic", "staggered", list(n), lo, hi, f[0], operator="ps", diff="grad")
    assert np.max(np.abs(psi - psi_ref[0])) <= 1e-12 * np.max(np.abs(psi_ref[0]))
    scale = np.max(np.abs(d[0]))
    for a in range(3):
        assert np.max(np.abs(g[a] - d[0, a])) <= 1e-12 * scale, a
