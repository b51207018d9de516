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
