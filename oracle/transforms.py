"""Discrete transforms of the oracle, written as their definitions.

Section 2.1, eq. (dft) gives the forward DFT (no scaling) and the inverse DFT
(scaled by 1/N); the oracle takes both from numpy.fft as library primitives.

Section 2.4.1 and Table 1 (tab:Bounded) pair Dirichlet and Neumann BCs with the
real-to-real sine and cosine transforms DST-I/II/III and DCT-I/II/III; the
paper points to FFTW for their definitions.  They are written out below as
dense matrices from the unnormalised definitions (row k, column j):

  DST-I   Y_k = 2 sum_j x_j sin(pi (j+1)(k+1) / (n+1))
  DST-II  Y_k = 2 sum_j x_j sin(pi (j+1/2)(k+1) / n)
  DST-III Y_k = (-1)^k x_{n-1} + 2 sum_{j<n-1} x_j sin(pi (j+1)(k+1/2) / n)
  DCT-I   Y_k = x_0 + (-1)^k x_{n-1} + 2 sum_{0<j<n-1} x_j cos(pi j k / (n-1))
  DCT-II  Y_k = 2 sum_j x_j cos(pi (j+1/2) k / n)
  DCT-III Y_k = x_0 + 2 sum_{j>=1} x_j cos(pi j (k+1/2) / n)

Angles are formed as pi * p / q with the integer p reduced modulo 2q before the
floating-point multiply, so large index products lose no accuracy.
"""
import numpy as np


def _trig(fn, p, q):
    """fn(pi * p / q) for integer arrays p and an integer q > 0."""
    r = np.mod(np.asarray(p, dtype=np.int64), 2 * q)
    return fn(np.pi * r.astype(np.float64) / q)


def dst1_matrix(n):
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return 2.0 * _trig(np.sin, (j + 1) * (k + 1), n + 1)


def dst2_matrix(n):
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return 2.0 * _trig(np.sin, (2 * j + 1) * (k + 1), 2 * n)


def dst3_matrix(n):
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    m = 2.0 * _trig(np.sin, (j + 1) * (2 * k + 1), 2 * n)
    m[:, n - 1] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return m


def dct1_matrix(n):
    if n < 2:
        raise ValueError("DCT-I needs n >= 2")
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    m = 2.0 * _trig(np.cos, j * k, n - 1)
    m[:, 0] = 1.0
    m[:, n - 1] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return m


def dct2_matrix(n):
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return 2.0 * _trig(np.cos, (2 * j + 1) * k, 2 * n)


def dct3_matrix(n):
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    m = 2.0 * _trig(np.cos, j * (2 * k + 1), 2 * n)
    m[:, 0] = 1.0
    return m


MATRICES = {
    "dst1": dst1_matrix,
    "dst2": dst2_matrix,
    "dst3": dst3_matrix,
    "dct1": dct1_matrix,
    "dct2": dct2_matrix,
    "dct3": dct3_matrix,
}


def apply(kind, x, axis):
    """Apply the named real-to-real transform along one axis of x."""
    x = np.asarray(x, dtype=np.float64)
    m = MATRICES[kind](x.shape[axis])
    y = np.tensordot(m, x, axes=([1], [axis]))
    return np.moveaxis(y, 0, axis)
