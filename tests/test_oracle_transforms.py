"""Pins of the oracle's sine / cosine transforms (module oracle.transforms).

The definitions follow the FFTW real-to-real transforms that Section 2.4.1
points to.  Each dense matrix is pinned against scipy.fft's unnormalised
transform of the same type (an independent library implementation), and the
inverse pairs of Table 1 are pinned by their exact scaling identities.
"""
import numpy as np
import pytest
import scipy.fft as sf

from oracle import transforms as tr

pytestmark = pytest.mark.filterwarnings("ignore")

LIB = {
    "dst1": lambda x: sf.dst(x, type=1),
    "dst2": lambda x: sf.dst(x, type=2),
    "dst3": lambda x: sf.dst(x, type=3),
    "dct1": lambda x: sf.dct(x, type=1),
    "dct2": lambda x: sf.dct(x, type=2),
    "dct3": lambda x: sf.dct(x, type=3),
}


@pytest.mark.parametrize("kind", sorted(LIB))
@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 64, 127])
def test_matrix_matches_library(kind, n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n)
    y = tr.apply(kind, x, 0)
    ref = LIB[kind](x)
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("fwd,bwd,scale", [
    ("dst1", "dst1", lambda n: 2 * (n + 1)),
    ("dst2", "dst3", lambda n: 2 * n),
    ("dct1", "dct1", lambda n: 2 * (n - 1)),
    ("dct2", "dct3", lambda n: 2 * n),
])
@pytest.mark.parametrize("n", [2, 7, 16, 33])
def test_inverse_pairs(fwd, bwd, scale, n):
    m = tr.MATRICES[bwd](n) @ tr.MATRICES[fwd](n)
    assert np.allclose(m, scale(n) * np.eye(n), atol=1e-11 * n)


def test_apply_along_axis():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(4, 5, 6))
    for axis in range(3):
        ref = sf.dct(x, type=2, axis=axis)
        assert np.allclose(tr.apply("dct2", x, axis), ref, atol=1e-12)
