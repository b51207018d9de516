"""Pins of the linear fusion baselines and image metrics (oracle/baselines.py)
against hand computations and the Poisson maximum-likelihood closed form."""
import numpy as np

from oracle import baselines


def test_linear_integration_of_scaled_frames_is_exact():
    rate = np.array([[0.5, 3.0], [12.0, 7.25]])
    t = [1.0, 4.0, 16.0]
    raw = np.stack([rate * tk for tk in t])[None]
    out = baselines.linear_integration(raw, t, sat=1e9)
    assert np.allclose(out[0], rate, rtol=0, atol=1e-12)


def test_linear_integration_is_the_poisson_rate_estimate_by_hand():
    # counts 3, 35, 290 in t = 1, 10, 100: MLE of the rate = 328 / 111 per unit time
    raw = np.array([3.0, 35.0, 290.0]).reshape(1, 3, 1, 1)
    t = [1.0, 10.0, 100.0]
    assert abs(baselines.linear_integration(raw, t, sat=4095)[0, 0, 0] - 328.0 / 111.0) < 1e-12
    # the third frame saturated (sat = 290): only 3 + 35 counts in 11 time units
    assert abs(baselines.linear_integration(raw, t, sat=290)[0, 0, 0] - 38.0 / 11.0) < 1e-12
    # every frame saturated: the shortest frame's value
    assert baselines.linear_integration(raw, t, sat=3)[0, 0, 0] == 3.0
    # the dark level comes off every frame before the sum
    assert abs(baselines.linear_integration(raw + 2.0, t, sat=4095, dark=2.0)[0, 0, 0] - 328.0 / 111.0) < 1e-12


def test_single_exposure_is_the_shortest_frame():
    raw = np.arange(2 * 3 * 4 * 4, dtype=float).reshape(2, 3, 4, 4)
    assert np.array_equal(baselines.single_exposure(raw, dark=1.0), raw[:, 0] - 1.0)


def test_metrics_closed_forms():
    C = np.array([[4.0, 0.0], [2.0, 0.0]])
    F = C * 1.01
    assert abs(baselines.radiometric_deviation(F, C) - 0.01) < 1e-12
    assert abs(baselines.snr_db(F, C) - 40.0) < 1e-9
    F2 = C + np.array([[0.0, 1.0], [0.0, -1.0]])
    assert baselines.background_variance(F2, C) == 1.0


# ------------------------------------------------------------------- MTF

def test_inscribed_square_of_a_disk_and_a_full_mask():
    yy, xx = np.mgrid[0:101, 0:101]
    disk = (yy - 50) ** 2 + (xx - 50) ** 2 <= 40 ** 2
    y0, x0, n = baselines.inscribed_square(disk)
    assert disk[y0:y0 + n, x0:x0 + n].all()
    assert abs(n - 40 * np.sqrt(2)) <= 3          # the disk's inscribed square
    assert baselines.inscribed_square(np.ones((32, 32), bool)) == (0, 0, 32)


def test_mtf_of_the_truth_and_of_a_scaled_copy_is_one():
    rng = np.random.default_rng(1)
    T = np.exp(1j * rng.standard_normal((48, 48)))
    mask = np.ones(T.shape, bool)
    for R in (T, (0.3 - 0.7j) * T):
        f, H = baselines.mtf(R, T, mask, nbins=8)
        np.testing.assert_allclose(H, 1.0, rtol=1e-12)
        np.testing.assert_allclose(f, (np.arange(8) + 0.5) / 16)


def test_mtf_of_a_gaussian_blur_on_a_white_object():
    # T with a flat spectrum (unit modulus, random phases; mean 1) blurred by a
    # periodic Gaussian of transfer g(k) = exp(-2 pi^2 s^2 |k|^2), g(0) = 1: H
    # in each annulus is the plain mean of g over the annulus's frequencies
    n, s = 64, 1.3
    rng = np.random.default_rng(2)
    Th = np.exp(2j * np.pi * rng.random((n, n)))
    Th[0, 0] = n * n
    T = np.fft.ifft2(Th)
    f = np.fft.fftfreq(n)
    k2 = f[:, None] ** 2 + f[None, :] ** 2
    g = np.exp(-2 * np.pi ** 2 * s ** 2 * k2)
    R = np.fft.ifft2(Th * g)
    fc, H = baselines.mtf(R, T, np.ones((n, n), bool), nbins=8)
    edges = np.linspace(0, 0.5, 9)
    for b in range(8):
        vals = [g[i, j] for i in range(n) for j in range(n)
                if (i or j) and edges[b] <= np.sqrt(k2[i, j]) and (np.sqrt(k2[i, j]) < edges[b + 1]
                                                                   or (b == 7 and np.sqrt(k2[i, j]) <= 0.5))]
        assert abs(H[b] - np.mean(vals)) < 1e-12
    assert np.all(np.diff(H) < 0)                 # a blur transfers less at higher frequency


def test_mtf_ignores_noise_uncorrelated_with_the_object():
    rng = np.random.default_rng(3)
    T = np.exp(1j * rng.standard_normal((128, 128)))
    noise = 0.3 * (rng.standard_normal(T.shape) + 1j * rng.standard_normal(T.shape))
    _, H = baselines.mtf(T + noise, T, np.ones(T.shape, bool), nbins=4)
    np.testing.assert_allclose(H, 1.0, atol=0.05)


def test_benchmark_mtf_helper_matches_the_oracle():
    import bench
    rng = np.random.default_rng(4)
    yy, xx = np.mgrid[0:90, 0:90]
    mask = (yy - 44) ** 2 + (xx - 47) ** 2 <= 38 ** 2
    T = np.exp(1j * rng.standard_normal((90, 90)))
    R = (0.5 + 0.2j) * T + 0.2 * (rng.standard_normal(T.shape) + 1j * rng.standard_normal(T.shape))
    _, H = baselines.mtf(R, T, mask, nbins=16)
    np.testing.assert_allclose(bench._mtf(R, T, mask, nbins=16), H, rtol=1e-10)
