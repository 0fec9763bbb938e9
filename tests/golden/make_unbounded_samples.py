"""Write tests/golden/unbounded256_curl_samples.npz from the FP64 oracle.

Workload: the 32 vortex rings of seed 4 on the 256^3 cell-centred grid of
[0, 1]^3 (rounded to float32, as the GPU receives them), free-space solve with
the G2 kernel (sigma = 2 H) and its curl, computed by oracle.solve on the
doubled 512^3 grid.  Stored: 512 seeded sample indices and psi / curl at those
points, plus the L2 norms of every full output field.  Calls only oracle/ and
workloads/.  Run: python tests/golden/make_unbounded_samples.py  (~10 GB RAM)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import vortex_rings  # noqa: E402

N = 256
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "unbounded256_curl_samples.npz")


def main():
    t0 = time.time()
    f = vortex_rings(N, seed=4, count=32).astype(np.float32).astype(np.float64)
    psi, u = oracle.solve("unbounded", "staggered", [N] * 3, [0, 0, 0], [1, 1, 1], f, diff="curl")
    rng = np.random.default_rng(2024)
    idx = rng.integers(0, N, size=(512, 3))
    sl = (idx[:, 0], idx[:, 1], idx[:, 2])
    np.savez(OUT, idx=idx, psi=np.stack([psi[c][sl] for c in range(3)]),
             curl=np.stack([u[c][sl] for c in range(3)]),
             psi_norm=np.array([np.linalg.norm(psi[c]) for c in range(3)]),
             curl_norm=np.array([np.linalg.norm(u[c]) for c in range(3)]),
             psi_absmax=np.array([np.abs(psi[c]).max() for c in range(3)]),
             curl_absmax=np.array([np.abs(u[c]).max() for c in range(3)]))
    print(f"wrote {OUT} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
