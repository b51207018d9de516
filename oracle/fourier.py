"""Oracle: unitary 2D discrete Fourier transform (Methods 3.3, Eq. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: the far-field operator is the unitary DFT with forward kernel
exp(-2 pi i k n / N) and a 1/N factor per 2D transform (1/sqrt(N) per
axis), so Parseval holds exactly and the adjoint equals the inverse.  The
detector-centred intensity of the paper has its zero frequency at
(N/2, N/2); ``to_fft_order`` moves it to (0, 0).
"""
from __future__ import annotations

import numpy as np


def fft2u(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2D DFT over the last two axes."""
    return np.fft.fft2(x, norm="ortho")


def ifft2u(X: np.ndarray) -> np.ndarray:
    """Unitary inverse 2D DFT over the last two axes."""
    return np.fft.ifft2(X, norm="ortho")


def to_fft_order(I_centred: np.ndarray) -> np.ndarray:
    """Detector-centred pattern -> FFT order (zero frequency at index 0)."""
    return np.fft.ifftshift(I_centred, axes=(-2, -1))


def to_detector_order(I_fft: np.ndarray) -> np.ndarray:
    """FFT order -> detector-centred pattern (zero frequency at N/2)."""
    return np.fft.fftshift(I_fft, axes=(-2, -1))


def dft_matrix(n: int) -> np.ndarray:
    """Unitary 1D DFT matrix built element by element from its definition."""
    F = np.empty((n, n), np.complex128)
    for k in range(n):
        for m in range(n):
            F[k, m] = np.exp(-2j * np.pi * k * m / n) / np.sqrt(n)
    return F


def brute_dft2(x: np.ndarray) -> np.ndarray:
    """Unitary 2D DFT by direct O(N^4) summation (tiny sizes only)."""
    ny, nx = x.shape
    out = np.zeros((ny, nx), np.complex128)
    for ky in range(ny):
        for kx in range(nx):
            s = 0.0 + 0.0j
            for y in range(ny):
                for xx in range(nx):
                    s += x[y, xx] * np.exp(-2j * np.pi * (ky * y / ny + kx * xx / nx))
            out[ky, kx] = s / np.sqrt(ny * nx)
    return out
