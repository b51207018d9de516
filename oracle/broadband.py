"""Oracle: the broadband measurement of Eq. 4 for discrete spectra.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64.

Eq. 4 sums the far-field intensities of every wavelength weighted by the
spectral density S(lambda).  Reading for discrete lines (the two harmonics of
the XUV source, Methods 3.2): an achromatic probe and object (P_lambda = P,
O_lambda = O), so the only change with wavelength is the detector sampling.
A detector pixel at distance k pixels from the zero frequency samples the
spatial frequency k p / (lambda z); relative to the reference wavelength
lambda_0 the pattern of lambda is the reference pattern magnified by
lambda / lambda_0, i.e. sampled at the scaled coordinate
    u = c + (k - c) s,   s = lambda_0 / lambda,   c = Nd / 2 (the centred zero frequency),
with the intensity multiplied by s^2 so that the pattern's total is kept.
    I_meas = sum_m w_m s_m^2 I_ref(c + (k - c) s_m)
Sampling between pixels is bilinear; pixels outside the detector contribute 0.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def resample(I: np.ndarray, s: float) -> np.ndarray:
    """s^2 * bilinear interpolation of the centred pattern(s) I [..][Nd][Nd]
    at c + (k - c) s along both axes (zero outside the detector)."""
    I = np.asarray(I, np.float64)
    Nd = I.shape[-1]
    c = Nd // 2
    u = c + (np.arange(Nd) - c) * s
    i0 = np.floor(u).astype(int)
    f = u - i0

    def taps(idx, frac):
        # (index, weight) pairs of the two neighbours, weight 0 outside the detector
        out = []
        for di, w in ((0, 1.0 - frac), (1, frac)):
            j = idx + di
            ok = (j >= 0) & (j < Nd)
            out.append((np.where(ok, j, 0), np.where(ok, w, 0.0)))
        return out

    ty, tx = taps(i0, f), taps(i0, f)
    res = np.zeros(I.shape)
    for jy, wy in ty:
        for jx, wx in tx:
            res += I[..., jy[:, None], jx[None, :]] * (wy[:, None] * wx[None, :])
    return res * s * s


def broadband(I_ref: np.ndarray, scales: Sequence[float], weights: Sequence[float]) -> np.ndarray:
    """Eq. 4 for discrete lines: sum_m w_m resample(I_ref, s_m)."""
    return sum(w * resample(I_ref, s) for s, w in zip(scales, weights))
