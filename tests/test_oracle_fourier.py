"""Pins of the unitary DFT oracle (Eq. 3) against brute-force summation and
the transform's textbook identities.  CPU only."""
import numpy as np
import pytest

from oracle import fourier


@pytest.mark.parametrize("shape", [(2, 2), (3, 3), (4, 4), (6, 6), (8, 8), (12, 12), (3, 4), (6, 8)])
def test_fft_equals_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np.testing.assert_allclose(fourier.fft2u(x), fourier.brute_dft2(x), rtol=0, atol=1e-13)


def test_dft_matrix_unitary_and_matches_fft():
    for n in (5, 16, 24):
        F = fourier.dft_matrix(n)
        np.testing.assert_allclose(F.conj().T @ F, np.eye(n), atol=1e-13)
        x = np.random.default_rng(n).standard_normal((n, n)) + 0j
        np.testing.assert_allclose(F @ x @ F.T, fourier.fft2u(x), atol=1e-12)


def test_parseval_and_inverse():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((64, 48)) + 1j * rng.standard_normal((64, 48))
    X = fourier.fft2u(x)
    assert np.isclose(np.sum(np.abs(X) ** 2), np.sum(np.abs(x) ** 2), rtol=1e-13)
    np.testing.assert_allclose(fourier.ifft2u(X), x, atol=1e-13)


def test_delta_gives_constant_and_shift_theorem():
    n = 16
    d = np.zeros((n, n), complex)
    d[0, 0] = 1.0
    np.testing.assert_allclose(fourier.fft2u(d), 1.0 / n, atol=1e-15)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n)) + 0j
    a, b = 3, 5
    ky, kx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    phase = np.exp(-2j * np.pi * (ky * a + kx * b) / n)
    np.testing.assert_allclose(fourier.fft2u(np.roll(x, (a, b), axis=(0, 1))),
                               fourier.fft2u(x) * phase, atol=1e-12)


def test_detector_order_puts_dc_at_centre():
    n = 8
    X = fourier.fft2u(np.ones((n, n), complex))
    D = fourier.to_detector_order(X)
    assert np.isclose(D[n // 2, n // 2], n)
    np.testing.assert_allclose(fourier.to_fft_order(D), X)
