"""Helpers of the GPU parity tests: run the library and the oracle on the same input."""
import numpy as np

import oracle

RNG_SEED = 1234


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)


TOL = {"f64": (1e-12, 1e-11), "f32": (1e-5, 1e-4)}


def to_dev(x, dtype, torch):
    x = np.asarray(x)
    return torch.as_tensor(x if x.ndim == 0 else np.ascontiguousarray(x), dtype=dtype, device="cuda")


def case_input(bc, grid, nc, ncomp, inhomogeneous, prec, seed):
    """Seeded random source and faces, rounded to the solve precision."""
    from oracle import grid as og
    rng = np.random.default_rng(seed)
    nd = len(nc)
    shape = tuple(og.unknowns(bc, grid, n) for n in nc)
    f = rng.normal(size=((ncomp,) + shape) if ncomp == 3 else shape)
    faces = None
    if inhomogeneous:
        faces = {}
        for a in range(nd):
            shp = tuple(og.output_points(bc, grid, nc[b]) for b in range(nd) if b != a)
            for s in (0, 1):
                faces[(a, s)] = rng.normal(size=shp)
    rnd = np.float32 if prec == "f32" else np.float64
    f = f.astype(rnd).astype(np.float64)
    if faces:
        faces = {k: v.astype(rnd).astype(np.float64) for k, v in faces.items()}
    return f, faces


def gpu_solve(bc, grid, nc, lo, hi, f, kernel, diff, prec, ncomp, faces, sigma_cells=0.0):
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver(bc, grid, nc, lo, hi, kernel=kernel, diff=diff, dtype=dtype, ncomp=ncomp,
               inhomogeneous=faces is not None, sigma_cells=sigma_cells)
    fin = [to_dev(f[c], dtype, torch) for c in range(3)] if ncomp == 3 else to_dev(f, dtype, torch)
    fd = {k: to_dev(v, dtype, torch) for k, v in faces.items()} if faces else None
    psi, der = s.solve(fin, fd)
    torch.cuda.synchronize()
    psi = np.stack([p.double().cpu().numpy() for p in psi]) if ncomp == 3 else psi[0].double().cpu().numpy()
    der = [d.double().cpu().numpy() for d in der]
    s.close()
    return psi, der


def oracle_solve(bc, grid, nc, lo, hi, f, kernel, diff, faces, sigma_cells=0.0):
    op = kernel  # bounded: "ps" | "fd2"; free space: the Green's kernel name
    return oracle.solve(bc, grid, nc, lo, hi, f, operator=op, diff=diff, faces=faces,
                        sigma_cells=sigma_cells if sigma_cells > 0 else 2.0)


def laplacian_rounding_tol(psi, lap, hs, doubled):
    """Rounding bound for a Laplacian taken in spectral space from FP64 data:
    an FFT of N points rounds psi-hat by at most about eps log2(N) relative
    (once on each side compared: the GPU and the oracle), and multiplying by
    |k|^2 <= sum_a (pi / H_a)^2 amplifies that against the output by
    A = k_max^2 ||psi|| / ||lap psi||.  Returns the rel-L2 bound 2 eps log2(N) A."""
    eps = np.finfo(np.float64).eps
    k2 = sum((np.pi / h) ** 2 for h in hs)
    amp = k2 * np.linalg.norm(psi) / np.linalg.norm(lap)
    return 2.0 * eps * np.log2(float(np.prod(doubled))) * amp
