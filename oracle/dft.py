"""Naive unitary DFT as an explicit matrix (test infrastructure only).

Section III.C, eq. (RDA): F and F^H are the DFT matrix and its inverse.  The
oracle never uses an FFT: the N x N matrix is built from an N-entry table of
exp(-2 pi i k / N) indexed by (j * k) mod N, and applied by a matrix product.
Scaling is unitary (1/sqrt(N) each way), which keeps the pairs F, F^H
consistent as rule i) of Section III.C asks.
"""

import functools

import numpy as np


@functools.lru_cache(maxsize=6)
def dft_matrix(n):
    """Unitary DFT matrix F_n[k, j] = exp(-2 pi i (k j mod n) / n) / sqrt(n)."""
    n = int(n)
    if n <= 0:
        raise ValueError("DFT length must be positive")
    table = np.exp(-2j * np.pi * np.arange(n, dtype=np.float64) / n)
    k = np.arange(n, dtype=np.int64)
    idx = np.multiply.outer(k, k) % n
    mat = table[idx] / np.sqrt(n)
    mat.setflags(write=False)
    return mat


def dft(x, axis):
    """Unitary DFT of ``x`` along ``axis`` (0 or 1 of a 2-D array, or a 1-D
    vector with axis 0)."""
    x = np.asarray(x, dtype=np.complex128)
    f = dft_matrix(x.shape[axis])
    if x.ndim == 1:
        return f @ x
    if axis == 0:
        return f @ x
    return x @ f.T


def idft(x, axis):
    """Inverse (= conjugate transpose) of :func:`dft` along ``axis``."""
    x = np.asarray(x, dtype=np.complex128)
    f = dft_matrix(x.shape[axis])
    fh = f.conj().T
    if x.ndim == 1:
        return fh @ x
    if axis == 0:
        return fh @ x
    return x @ fh.T


def idft_rows_at(x, cols):
    """Inverse DFT along axis 1, evaluated only at output columns ``cols``
    (rows of F^H restricted to those outputs)."""
    x = np.asarray(x, dtype=np.complex128)
    f = dft_matrix(x.shape[1])
    fh = f.conj().T
    return x @ fh[np.asarray(cols)].T


def freq_index(n):
    """Signed frequency index nu(k) = k for k < n/2 and k - n otherwise
    (the Nyquist bin of an even length is negative)."""
    k = np.arange(n, dtype=np.int64)
    return np.where(k < (n + 1) // 2, k, k - n)
