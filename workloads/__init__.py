"""Seeded synthetic inputs for the Poisson solves (shared by tests and bench).

This module only draws random numbers and evaluates source / boundary
functions on grid points.  It holds none of the solver's arithmetic and
imports neither the library nor the oracle.  Every generator returns float64
arrays; callers cast to the solve precision and feed the same (rounded)
values to both sides.

The workloads follow the paper's test inputs: products of sines and cosines
(eq. tfb), smooth compactly supported sources (eq. bump1D), vortex rings
(Section 4.3), Gaussian sources with closed-form potentials.
"""
import numpy as np


def staggered_axis(n, lo=0.0, hi=1.0):
    h = (hi - lo) / n
    return lo + h * (np.arange(n) + 0.5)


def regular_axis(npts, nc, lo=0.0, hi=1.0):
    h = (hi - lo) / nc
    return lo + h * np.arange(npts)


# ---------------------------------------------------------------- 2D periodic
def periodic_modes_2d(n=64, seed=1, count=8, kmax2=64):
    """sin(2 pi x) sin(2 pi y) plus `count` random Fourier modes, mean removed.

    Modes (p, q) are drawn without replacement from the half plane
    {p > 0, or p == 0 and q > 0} with p^2 + q^2 <= kmax2; each carries
    a cos(2 pi (p x + q y)) + b sin(2 pi (p x + q y)), a, b ~ N(0, 1).
    Grid: n x n cell centres on [0, 1)^2.
    Returns (f, modes) with modes = [(p, q, a, b), ...].
    """
    rng = np.random.default_rng(seed)
    cand = [(p, q) for p in range(0, 9) for q in range(-8, 9)
            if (p > 0 or (p == 0 and q > 0)) and p * p + q * q <= kmax2]
    pick = rng.choice(len(cand), size=count, replace=False)
    ab = rng.normal(size=(count, 2))
    modes = [(cand[i][0], cand[i][1], ab[j, 0], ab[j, 1]) for j, i in enumerate(pick)]
    x = staggered_axis(n)[:, None]
    y = staggered_axis(n)[None, :]
    f = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    for p, q, a, b in modes:
        ph = 2 * np.pi * (p * x + q * y)
        f = f + a * np.cos(ph) + b * np.sin(ph)
    f = f - f.mean()
    return f, modes


# ------------------------------------------------------------- 3D Dirichlet
def boundary_sinusoids(seed=2, count=4, kmax=3):
    """Parameters of g(x) = sum_j c_j sin(2 pi k_j . x + phi_j)."""
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k.astype(np.float64))
    c = rng.normal(size=count)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=count)
    return np.array(ks), c, phi


def eval_sinusoids(params, x, y, z):
    ks, c, phi = params
    out = 0.0
    for j in range(len(c)):
        out = out + c[j] * np.sin(2 * np.pi * (ks[j, 0] * x + ks[j, 1] * y + ks[j, 2] * z) + phi[j])
    return out


def gaussian_blobs_params(seed=3, count=16, lo=0.15, hi=0.85):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(count, 3))
    amps = rng.normal(size=count)
    return centres, amps


def eval_blobs(params, sigma, x, y, z):
    centres, amps = params
    out = 0.0
    for b in range(len(amps)):
        r2 = (x - centres[b, 0]) ** 2 + (y - centres[b, 1]) ** 2 + (z - centres[b, 2]) ** 2
        out = out + amps[b] * np.exp(-r2 / (2.0 * sigma * sigma))
    return out


def dirichlet_3d(nc=128, seed_bc=2, seed_src=3, sigma=0.05):
    """3D Dirichlet, REGULAR grid on [0,1]^3 with nc cells.

    Returns (f, faces): f on the (nc-1)^3 interior nodes (16 Gaussian blobs),
    faces {(axis, side): g} on the (nc+1)^2 nodes of each face.
    """
    nodes = regular_axis(nc + 1, nc)
    inner = nodes[1:-1]
    bp = boundary_sinusoids(seed_bc)
    sp = gaussian_blobs_params(seed_src)
    f = eval_blobs(sp, sigma, inner[:, None, None], inner[None, :, None], inner[None, None, :])
    faces = {}
    for axis in range(3):
        for side in (0, 1):
            v = nodes[0] if side == 0 else nodes[-1]
            a, b = np.meshgrid(nodes, nodes, indexing="ij")
            coords = [None, None, None]
            others = [d for d in range(3) if d != axis]
            coords[axis] = np.full_like(a, v)
            coords[others[0]] = a
            coords[others[1]] = b
            faces[(axis, side)] = eval_sinusoids(bp, *coords)
    return f, faces


# ------------------------------------------------------------ vortex rings
def vortex_ring_params(seed, count, r_range, core_ratio, centre_range=(0.2, 0.8)):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(centre_range[0], centre_range[1], size=(count, 3))
    radii = rng.uniform(r_range[0], r_range[1], size=count)
    normals = rng.normal(size=(count, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    gammas = rng.normal(size=count)
    cores = radii * core_ratio
    return centres, radii, cores, normals, gammas


def vortex_rings(n, seed, count, r_range=(0.05, 0.10), core_ratio=0.2, dtype=np.float64):
    """3-component vorticity of `count` compact Gaussian vortex rings.

    Cell-centred n^3 grid on [0, 1]^3.  A ring with centre c, radius R, unit
    normal e and circulation Gamma contributes
    Gamma / (2 pi s^2) exp(-rho^2 / (2 s^2)) t, with s = core_ratio * R, rho
    the distance to the ring's centre line and t the unit tangent, for
    rho <= 4 s (zero beyond).  Returns an array of shape (3, n, n, n).
    """
    centres, radii, cores, normals, gammas = vortex_ring_params(seed, count, r_range, core_ratio)
    w = np.zeros((3, n, n, n), dtype=np.float64)
    h = 1.0 / n
    for c, R, s, e, G in zip(centres, radii, cores, normals, gammas):
        reach = R + 4.0 * s
        lo = np.clip(np.floor((c - reach) / h - 0.5).astype(int), 0, n)
        hi = np.clip(np.ceil((c + reach) / h - 0.5).astype(int) + 1, 0, n)
        xs = [(np.arange(lo[a], hi[a]) + 0.5) * h - c[a] for a in range(3)]
        dx, dy, dz = np.meshgrid(*xs, indexing="ij")
        along = dx * e[0] + dy * e[1] + dz * e[2]
        px, py, pz = dx - along * e[0], dy - along * e[1], dz - along * e[2]
        rp = np.sqrt(px * px + py * py + pz * pz)
        rho2 = (rp - R) ** 2 + along ** 2
        mask = (rho2 <= (4.0 * s) ** 2) & (rp > 0.0)
        amp = np.where(mask, G / (2.0 * np.pi * s * s) * np.exp(-rho2 / (2.0 * s * s)), 0.0)
        inv = np.where(rp > 0.0, 1.0 / np.where(rp > 0.0, rp, 1.0), 0.0)
        tx = (e[1] * pz - e[2] * py) * inv
        ty = (e[2] * px - e[0] * pz) * inv
        tz = (e[0] * py - e[1] * px) * inv
        sl = (slice(lo[0], hi[0]), slice(lo[1], hi[1]), slice(lo[2], hi[2]))
        w[(0,) + sl] += amp * tx
        w[(1,) + sl] += amp * ty
        w[(2,) + sl] += amp * tz
    return w.astype(dtype, copy=False)


def gaussian_blobs_vector(n, seed=8, per_comp=3, s=0.03, centre_range=(0.3, 0.7)):
    """Accuracy twin: `per_comp` Gaussian blobs A exp(-r^2 / (2 s^2)) per component.

    Returns (f, params) with f of shape (3, n, n, n) on cell centres of
    [0, 1]^3 and params[c] = (centres, amps) for the closed-form potential.
    """
    rng = np.random.default_rng(seed)
    x = staggered_axis(n)
    X, Y, Z = x[:, None, None], x[None, :, None], x[None, None, :]
    f = np.zeros((3, n, n, n))
    params = []
    for c in range(3):
        centres = rng.uniform(centre_range[0], centre_range[1], size=(per_comp, 3))
        amps = rng.normal(size=per_comp)
        f[c] = eval_blobs((centres, amps), s, X, Y, Z)
        params.append((centres, amps))
    return f, params


# ------------------------------------------------------- batched Neumann
BATCH_SIZES = (32, 48, 64, 96, 128)


def neumann_batch(count=64, seed=5, nmodes=6):
    """`count` independent 3D Neumann problems on STAGGERED grids of [0,1]^3.

    Per-axis sizes are drawn independently from BATCH_SIZES.  Each source is a
    sum of `nmodes` products prod_a cos(pi p_a x_a) with p != 0 and
    p_a <= min(n_a / 4, 8), amplitudes N(0, 1), so it has zero mean.
    Returns a list of dicts {"shape", "f", "modes": [(p, A), ...]}.
    """
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(count):
        shape = tuple(int(v) for v in rng.choice(BATCH_SIZES, size=3))
        pmax = [min(nn // 4, 8) for nn in shape]
        modes = []
        while len(modes) < nmodes:
            p = tuple(int(rng.integers(0, pmax[a] + 1)) for a in range(3))
            if any(p):
                modes.append((p, float(rng.normal())))
        xs = [staggered_axis(nn) for nn in shape]
        X, Y, Z = xs[0][:, None, None], xs[1][None, :, None], xs[2][None, None, :]
        f = np.zeros(shape)
        for p, A in modes:
            f = f + A * np.cos(np.pi * p[0] * X) * np.cos(np.pi * p[1] * Y) * np.cos(np.pi * p[2] * Z)
        probs.append({"shape": shape, "f": f, "modes": modes})
    return probs


def random_directions(shape, seeds=range(1000, 1064)):
    """Unit-variance Gaussian direction fields, one per seed."""
    return [np.random.default_rng(s).normal(size=shape) for s in seeds]
