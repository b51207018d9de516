"""Pins of the fusion oracle (Methods 3.4, Eqs. 5-10) against closed forms,
brute force and the invariants the equations imply.  CPU only."""
import math

import numpy as np
import pytest

from oracle import mnf


def _reflect101(i, n):
    # x[-1] = x[1], x[-2] = x[2], x[n] = x[n-2], x[n+1] = x[n-3]
    if i < 0:
        return -i
    if i >= n:
        return 2 * (n - 1) - i
    return i


def _brute_reduce(g):
    w = [1 / 16, 4 / 16, 6 / 16, 4 / 16, 1 / 16]
    h, wd = g.shape
    out = np.zeros((h // 2, wd // 2))
    for i in range(h // 2):
        for j in range(wd // 2):
            s = 0.0
            for a in range(-2, 3):
                for b in range(-2, 3):
                    s += w[a + 2] * w[b + 2] * g[_reflect101(2 * i + a, h), _reflect101(2 * j + b, wd)]
            out[i, j] = s
    return out


def _closed_expand_1d(g):
    n = len(g)
    gm = lambda i: g[1] if i < 0 else (g[n - 1] if i >= n else g[i])
    out = np.zeros(2 * n)
    for i in range(n):
        out[2 * i] = (gm(i - 1) + 6 * gm(i) + gm(i + 1)) / 8
        out[2 * i + 1] = (gm(i) + gm(i + 1)) / 2
    return out


def _closed_expand(g):
    a = np.stack([_closed_expand_1d(g[:, j]) for j in range(g.shape[1])], axis=1)
    return np.stack([_closed_expand_1d(a[i]) for i in range(a.shape[0])], axis=0)


def test_reduce_matches_brute_force_nonsquare():
    rng = np.random.default_rng(0)
    g = rng.standard_normal((8, 12))
    np.testing.assert_allclose(mnf.reduce(g), _brute_reduce(g), rtol=0, atol=1e-13)


def test_expand_matches_closed_form_nonsquare():
    rng = np.random.default_rng(1)
    g = rng.standard_normal((5, 7))
    np.testing.assert_allclose(mnf.expand(g), _closed_expand(g), rtol=0, atol=1e-13)


def test_constant_pyramid_is_constant():
    g = np.full((32, 16), 3.25)
    for G in mnf.gaussian_pyramid(g, 3):
        np.testing.assert_allclose(G, 3.25, atol=1e-14)
    np.testing.assert_allclose(mnf.expand(np.full((4, 4), -2.0)), -2.0, atol=1e-14)


def test_laplacian_collapse_is_exact():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((64, 32)) * 100
    G = mnf.gaussian_pyramid(g, 4)
    Lp = mnf.laplacian_pyramid(G)
    np.testing.assert_allclose(mnf.collapse(G[-1], Lp), g, rtol=0, atol=1e-11)


def test_weight_closed_form_values():
    mu, s = 0.5, 0.2
    assert mnf.raw_weight(np.array(mu), mu, s) == 1.0
    assert math.isclose(mnf.raw_weight(np.array(mu + s), mu, s), math.exp(-0.5), rel_tol=1e-15)
    assert math.isclose(mnf.raw_weight(np.array(mu - 2 * s), mu, s), math.exp(-2.0), rel_tol=1e-15)
    # a saturated pixel is penalised, not removed: exp(-0.25 / 0.08)
    assert math.isclose(mnf.raw_weight(np.array(1.0), mu, s), math.exp(-3.125), rel_tol=1e-14)


def test_normalised_intensity_clamps():
    I = np.array([-5.0, 0.0, 50.0, 4095.0, 5000.0])
    np.testing.assert_allclose(mnf.normalised_intensity(I, 4095.0, 0.0),
                               [0.0, 0.0, 50 / 4095, 1.0, 1.0])
    np.testing.assert_allclose(mnf.normalised_intensity(np.array([10.0]), 110.0, 10.0), [0.0])


def test_weights_sum_to_one():
    rng = np.random.default_rng(3)
    raw = rng.integers(0, 4096, size=(3, 4, 16, 24)).astype(np.float64)
    W = mnf.weights(raw, mnf.FuseParams(sat=4095.0))
    np.testing.assert_allclose(W.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(W > 0)


@pytest.mark.parametrize("K,L", [(1, 0), (2, 1), (3, 4), (5, 3)])
def test_identical_exposures_return_input(K, L):
    rng = np.random.default_rng(10 + K)
    img = rng.uniform(0, 4000, size=(32, 48))
    raw = np.repeat(img[None], K, axis=0)
    p = mnf.FuseParams(levels=L, sat=4095.0)
    out = mnf.fuse_position(raw, [1.0] * K, p)
    np.testing.assert_allclose(out, img, rtol=1e-13, atol=1e-10)


def test_scaled_exposures_return_shortest_exposure():
    # linearly scaled, unsaturated exposures: every I_tilde_k equals I_1, the
    # weights differ per exposure but sum to one, so I_MNF = I_1 exactly.
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 600, size=(32, 32))
    t = [1.0, 10.0, 100.0]
    raw = np.stack([img * tk for tk in t])
    assert raw.max() < 65535
    p = mnf.FuseParams(levels=3, sat=65535.0)
    out, W, _ = mnf.fuse_position(raw, t, p, return_parts=True)
    assert np.ptp(W[0]) > 0.1  # weights genuinely vary
    np.testing.assert_allclose(out, img, rtol=1e-12, atol=1e-10)


def test_zero_levels_is_weighted_average():
    rng = np.random.default_rng(6)
    raw = rng.integers(0, 4096, size=(3, 8, 8)).astype(np.float64)
    t = [1.0, 2.0, 4.0]
    p = mnf.FuseParams(levels=0, sat=4095.0)
    W = mnf.normalised_weights(raw / 4095.0, 0.5, 0.2)
    expect = sum(W[k] * raw[k] * t[0] / t[k] for k in range(3))
    np.testing.assert_allclose(mnf.fuse_position(raw, t, p), expect, rtol=1e-14)


def test_quantise_rounds_half_to_even():
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 0.49])
    np.testing.assert_array_equal(mnf.quantise(x, 1.0), [0.0, 2.0, 2.0, -0.0, -2.0, 0.0])
    np.testing.assert_array_equal(mnf.quantise(np.array([0.3]), 0.0), [0.3])


def test_single_exposure_quantisation_bound():
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 4095, size=(64, 64))
    p = mnf.FuseParams(levels=4, sat=4095.0, delta=[3.0, 6.0, 12.0, 24.0])
    out = mnf.fuse_position(img[None], [1.0], p)
    bound = sum(p.delta) / 2
    err = np.abs(out - img)
    assert err.max() <= bound + 1e-9
    assert err.max() > 0.1 * bound  # the quantiser really acts


def test_quantisation_acts_on_the_finest_band_first():
    # delta only at l = 0 and far above every coefficient: the finest band
    # vanishes and the result is the expanded level-1 Gaussian image.
    rng = np.random.default_rng(8)
    img = rng.uniform(0, 4095, size=(32, 32))
    p = mnf.FuseParams(levels=3, sat=4095.0, delta=[1e9, 0.0, 0.0])
    out = mnf.fuse_position(img[None], [1.0], p)
    np.testing.assert_allclose(out, mnf.expand(mnf.reduce(img)), rtol=1e-12, atol=1e-9)


def test_multi_exposure_quantisation_bound():
    rng = np.random.default_rng(9)
    raw = rng.integers(0, 4096, size=(3, 32, 32)).astype(np.float64)
    t = [1.0, 10.0, 100.0]
    d = [2.0, 4.0, 8.0]
    p0 = mnf.FuseParams(levels=3, sat=4095.0)
    pq = mnf.FuseParams(levels=3, sat=4095.0, delta=d)
    diff = np.abs(mnf.fuse_position(raw, t, pq) - mnf.fuse_position(raw, t, p0))
    bound = sum(d[l] * t[0] / t[k] for k in range(3) for l in range(3)) / 2
    assert diff.max() <= bound + 1e-9


def test_per_exposure_collapse_equals_collapse_of_sum():
    rng = np.random.default_rng(11)
    raw = rng.integers(0, 4096, size=(4, 32, 32)).astype(np.float64)
    t = [1.0, 3.0, 9.0, 27.0]
    p = mnf.FuseParams(levels=3, sat=4095.0, delta=[1.0, 2.0, 4.0])
    out, _, parts = mnf.fuse_position(raw, t, p, return_parts=True)
    base = sum(pt["base"] for pt in parts)
    details = [sum(pt["details"][l] for pt in parts) for l in range(3)]
    np.testing.assert_allclose(mnf.collapse(base, details), out, rtol=1e-12, atol=1e-9)


def test_scale_equivariance():
    # scaling counts and full scale together leaves I_bar (and the weights)
    # unchanged and scales I_tilde, so the fusion output scales too.
    rng = np.random.default_rng(12)
    raw = rng.uniform(0, 4095, size=(3, 16, 16))
    t = [1.0, 5.0, 25.0]
    a = 7.5
    out1 = mnf.fuse_position(raw, t, mnf.FuseParams(levels=2, sat=4095.0))
    out2 = mnf.fuse_position(a * raw, t, mnf.FuseParams(levels=2, sat=a * 4095.0))
    np.testing.assert_allclose(out2, a * out1, rtol=1e-12, atol=1e-9)


def test_literal_mode_fuses_normalised_images():
    rng = np.random.default_rng(13)
    img = rng.uniform(0, 4095, size=(16, 16))
    raw = np.repeat(img[None], 2, axis=0)
    p = mnf.FuseParams(levels=2, sat=4095.0, radiometric=False)
    np.testing.assert_allclose(mnf.fuse_position(raw, [1.0, 1.0], p), img / 4095.0, rtol=1e-13)


def test_literal_mode_step_is_in_normalised_units():
    # Literal reading (radiometric = 0): the fused quantity is I_bar in [0, 1],
    # so a step of delta ADU is delta / (sat - dark) there (Eq. 8 applied to
    # the normalised images).  K = 1: the weight is 1, so every deviation comes
    # from quantisation and stays within sum_l delta_l / (2 (sat - dark)).
    # A step left in ADU (delta itself) would round every band coefficient of
    # a [0, 1] image to 0 and miss this bound by orders of magnitude; a step of
    # zero would leave no deviation at all.
    rng = np.random.default_rng(31)
    sat, dark = 4095.0, 15.0
    raw = np.clip(rng.gamma(2.0, 600.0, size=(1, 48, 40)) + dark, 0, sat)
    d = [3.0, 2.0, 1.5]
    pq = mnf.FuseParams(levels=3, sat=sat, dark=dark, delta=d, radiometric=False)
    p0 = mnf.FuseParams(levels=3, sat=sat, dark=dark, radiometric=False)
    assert mnf.step_size(pq, 1, [1.0], 0) == pytest.approx(2.0 / (sat - dark), rel=1e-15)
    out = mnf.fuse_position(raw, [1.0], pq)
    Ibar = np.clip((raw[0] - dark) / (sat - dark), 0.0, 1.0)
    np.testing.assert_allclose(mnf.fuse_position(raw, [1.0], p0), Ibar, rtol=0, atol=1e-12)
    dev = np.abs(out - Ibar)
    assert dev.max() <= sum(d) / (2 * (sat - dark)) + 1e-12
    assert dev.max() > 0.1 * min(d) / (sat - dark)


def test_literal_mode_step_ignores_exposure_times():
    # in the literal reading every exposure is quantised in the same units
    p = mnf.FuseParams(levels=2, sat=4095.0, dark=0.0, delta=[4.0, 2.0], radiometric=False)
    t = [1.0, 10.0, 100.0]
    for k in range(3):
        assert mnf.step_size(p, 0, t, k) == 4.0 / 4095.0
        assert mnf.step_size(p, 1, t, k) == 2.0 / 4095.0


# --- optional contrast factor (the paper's weight is contrast_exp = 0) ------

def test_contrast_of_a_single_bright_pixel():
    # by hand: a lone value v gives 4v at the pixel and v at its four
    # neighbours, zero elsewhere (interior pixel)
    g = np.zeros((8, 9))
    g[3, 4] = 0.5
    C = mnf.contrast(g)
    want = np.zeros((8, 9))
    want[3, 4] = 2.0
    for y, x in [(2, 4), (4, 4), (3, 3), (3, 5)]:
        want[y, x] = 0.5
    np.testing.assert_array_equal(C, want)


def test_contrast_reflects_without_repeating_the_edge():
    # reflect-101: a value one row in from the top edge is seen twice by the
    # edge pixel above it (its neighbours at rows -1 and 1 are both row 1),
    # so that edge pixel's contrast is 2v, not v (a repeated edge) or v + 0
    g = np.zeros((6, 7))
    g[1, 3] = 0.25
    C = mnf.contrast(g)
    assert C[0, 3] == 0.5
    assert C[1, 3] == 1.0 and C[2, 3] == 0.25 and C[1, 2] == 0.25 and C[1, 4] == 0.25
    assert C.sum() == 0.5 + 1.0 + 3 * 0.25


def test_contrast_of_a_ramp_is_zero_inside_and_twice_the_slope_at_the_edges():
    # I = a + b x: the second difference vanishes inside; at x = 0 the
    # reflected neighbour is x = 1, giving |2 (a + b) - 2 a| = 2 b, and
    # likewise at x = W - 1
    a, b = 0.2, 0.05
    g = np.tile(a + b * np.arange(10.0), (5, 1))
    C = mnf.contrast(g)
    np.testing.assert_allclose(C[:, 1:-1], 0.0, atol=1e-15)
    np.testing.assert_allclose(C[:, 0], 2 * b, rtol=1e-12)
    np.testing.assert_allclose(C[:, -1], 2 * b, rtol=1e-12)


def test_contrast_exponent_zero_is_the_paper_weight():
    rng = np.random.default_rng(7)
    raw = rng.integers(0, 4096, size=(2, 3, 16, 16)).astype(np.float64)
    W0 = mnf.weights(raw, mnf.FuseParams(sat=4095.0))
    Wc = mnf.weights(raw, mnf.FuseParams(sat=4095.0, contrast_exp=0.0))
    np.testing.assert_array_equal(W0, Wc)


def test_contrast_weights_at_one_pixel_by_hand():
    # K = 2 at the peak of exposure 1 (a lone pixel of I_bar = 0.6 on zero)
    # while exposure 0 is flat at I_bar = 0.3: W_1 / W_0 =
    # E(0.6) (4 * 0.6 + eps)^c / (E(0.3) eps^c), E(x) = exp(-(x - mu)^2 / (2 s^2))
    mu, s, c, sat = 0.5, 0.2, 1.5, 1000.0
    raw = np.zeros((1, 2, 5, 5))
    raw[0, 0] = 300.0
    raw[0, 1, 2, 2] = 600.0
    W = mnf.weights(raw, mnf.FuseParams(mu=mu, sigma=s, sat=sat, contrast_exp=c))[0]
    E = lambda x: math.exp(-(x - mu) ** 2 / (2 * s * s))
    r = E(0.6) * (2.4 + 1e-6) ** c / (E(0.3) * 1e-6 ** c)
    assert W[1, 2, 2] == pytest.approx(r / (1 + r), rel=1e-12)
    assert W[0, 2, 2] == pytest.approx(1 / (1 + r), rel=1e-12)
    # a neighbour of the peak: contrast 0.6 in exposure 1, still 0 in exposure 0
    # (I_bar of exposure 1 is 0 there)
    r1 = E(0.0) * (0.6 + 1e-6) ** c / (E(0.3) * 1e-6 ** c)
    assert W[1, 1, 2] == pytest.approx(r1 / (1 + r1), rel=1e-12)


def test_contrast_leaves_flat_brackets_at_the_paper_weight():
    # every exposure flat: every C_k = 0, the common factor eps^c cancels in
    # the normalisation, and the fused result is that of the paper's weight
    raw = np.stack([np.full((16, 16), v) for v in (200.0, 900.0, 3000.0)])
    t = [1.0, 4.0, 16.0]
    p0 = mnf.FuseParams(levels=2, sat=4095.0)
    pc = mnf.FuseParams(levels=2, sat=4095.0, contrast_exp=2.0)
    np.testing.assert_allclose(mnf.fuse_position(raw, t, pc), mnf.fuse_position(raw, t, p0), rtol=1e-12)
