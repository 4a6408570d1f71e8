"""Pins for the oracle's naive DFT (Section III.C eq. (RDA): F and F^H)."""

import numpy as np
import pytest

import inputs
from oracle import dft


@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 16, 48, 64])
def test_impulse_gives_exponential(n):
    # Closed form: DFT of delta[j - j0] is exp(-2 pi i k j0 / n) / sqrt(n).
    for j0 in {0, n // 3, n - 1}:
        x = np.zeros(n, complex)
        x[j0] = 1.0
        want = np.exp(-2j * np.pi * np.arange(n) * j0 / n) / np.sqrt(n)
        np.testing.assert_allclose(dft.dft(x, 0), want, atol=1e-14)


@pytest.mark.parametrize("n", [4, 6, 16, 96])
def test_exponential_gives_impulse(n):
    # Closed form: DFT of exp(+2 pi i k0 j / n) is sqrt(n) delta[k - k0].
    for k0 in range(0, n, max(1, n // 5)):
        x = np.exp(2j * np.pi * k0 * np.arange(n) / n)
        want = np.zeros(n, complex)
        want[k0] = np.sqrt(n)
        np.testing.assert_allclose(dft.dft(x, 0), want, atol=1e-12)


def test_constant_and_alternating():
    n = 32
    np.testing.assert_allclose(dft.dft(np.ones(n), 0)[0], np.sqrt(n), atol=1e-13)
    alt = (-1.0) ** np.arange(n)
    y = dft.dft(alt, 0)
    assert abs(y[n // 2] - np.sqrt(n)) < 1e-12
    assert np.max(np.abs(np.delete(y, n // 2))) < 1e-12


@pytest.mark.parametrize("n", [8, 12, 64, 256])
def test_unitary_and_inverse(n):
    f = dft.dft_matrix(n)
    np.testing.assert_allclose(f.conj().T @ f, np.eye(n), atol=1e-12)
    x = inputs.random_complex((n, 5), seed=n)
    np.testing.assert_allclose(dft.idft(dft.dft(x, 0), 0), x, atol=1e-12)


def test_axes_of_2d_arrays():
    x = inputs.random_complex((12, 20), seed=3)
    cols = np.stack([dft.dft(x[:, j], 0) for j in range(20)], axis=1)
    rows = np.stack([dft.dft(x[i, :], 0) for i in range(12)], axis=0)
    np.testing.assert_allclose(dft.dft(x, 0), cols, atol=1e-13)
    np.testing.assert_allclose(dft.dft(x, 1), rows, atol=1e-13)


def test_restricted_inverse_rows():
    x = inputs.random_complex((6, 24), seed=4)
    full = dft.idft(x, 1)
    cols = [0, 5, 23, 11]
    np.testing.assert_allclose(dft.idft_rows_at(x, cols), full[:, cols], atol=1e-13)


@pytest.mark.parametrize("n", [16, 96, 512])
def test_cross_check_against_library_fft(n):
    # Independent cross-check against numpy's FFT (a different algorithm).
    x = inputs.random_complex(n, seed=7 + n)
    np.testing.assert_allclose(dft.dft(x, 0), np.fft.fft(x, norm="ortho"), atol=1e-11)


def test_freq_index_matches_fftfreq_order():
    for n in (1, 2, 7, 8, 1536):
        np.testing.assert_array_equal(dft.freq_index(n),
                                      np.round(np.fft.fftfreq(n) * n).astype(int))
