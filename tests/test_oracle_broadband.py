"""Pins of the discrete-spectrum measurement (Eq. 4) resampling."""
import numpy as np
from scipy.ndimage import map_coordinates

from oracle import broadband


def test_unit_scale_is_identity():
    I = np.random.default_rng(0).random((2, 16, 16))
    assert np.array_equal(broadband.resample(I, 1.0), I)


def test_linear_ramp_is_interpolated_exactly():
    # bilinear interpolation reproduces a linear function inside the detector
    Nd, s = 32, 0.8
    y, x = np.mgrid[0:Nd, 0:Nd].astype(float)
    I = 3.0 + 0.5 * y - 0.25 * x
    out = broadband.resample(I, s) / s ** 2
    c = Nd // 2
    want = 3.0 + 0.5 * (c + (y - c) * s) - 0.25 * (c + (x - c) * s)
    assert np.abs(out - want).max() < 1e-12


def test_matches_library_bilinear_interpolation():
    rng = np.random.default_rng(1)
    I = rng.random((24, 24))
    for s in (0.7, 0.9, 1.3):
        c = 12
        u = c + (np.arange(24) - c) * s
        uu, vv = np.meshgrid(u, u, indexing="ij")
        lib = map_coordinates(I, [uu, vv], order=1, mode="constant", cval=0.0, prefilter=False)
        inside = (uu >= 0) & (uu <= 23) & (vv >= 0) & (vv <= 23)
        got = broadband.resample(I, s) / s ** 2
        assert np.abs(got - lib)[inside].max() < 1e-12


def test_magnified_pattern_keeps_its_total():
    # a compact centred blob: s^2 keeps the total (to interpolation error), the
    # width grows by 1 / s and the centre stays the centre
    Nd, c, w = 64, 32, 3.0
    y, x = np.mgrid[0:Nd, 0:Nd].astype(float)
    I = np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * w * w))
    for s in (0.8, 0.9):
        out = broadband.resample(I, s)
        assert abs(out.sum() / I.sum() - 1.0) < 1e-2  # bilinear error on a 3-px blob
        want = s * s * np.exp(-s * s * ((y - c) ** 2 + (x - c) ** 2) / (2 * w * w))
        assert np.abs(out - want).max() < 0.02 * want.max()
        assert np.unravel_index(np.argmax(out), out.shape) == (c, c)
    mix = broadband.broadband(I, [1.0, 0.8], [0.5, 0.5])
    assert abs(mix.sum() / I.sum() - 1.0) < 1e-2
