"""Oracle: the linear fusion baselines MNF is compared against, and the
image metrics of a fused pattern.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64.

The paper compares MNF with standard linear integration (SLI) of the
bracket — fusion that keeps the intensity proportional to |Psi|^2 — and with
a single exposure (Introduction; Results 2.2 and 2.3), without writing
either out.  Readings:

  SLI  at each pixel the frames below saturation are combined into the
       exposure-time-weighted rate sum_k m_k (I_k - dark) / sum_k m_k t_k,
       expressed in counts of the shortest exposure (times t_1), with
       m_k = [I_k < sat].  For independent Poisson frames this is the
       maximum-likelihood rate (read noise neglected).  A pixel saturated in
       every frame keeps the shortest frame's value.
  Raw  the shortest exposure alone, I_1 - dark.

Image metrics of a fused pattern F against the clean intensity C in the same
units (the simulation knows C):
  radiometric deviation  ||F - C|| / ||C||          (Results 2.2 quotes ~13 % for MNF)
  SNR                     10 log10(sum C^2 / sum (F - C)^2) dB   (Results 2.3)
  background variance     variance of F over the pixels with C < 1e-3 max C
                          (the structure-free region of Results 2.3)

Resolution of a reconstruction: the modulation transfer function (Results
2.3 quotes MTF values of the reconstructed phase up to the 0.5 cycles/pixel
Nyquist limit; its definition is in the unavailable supplement).  Reading:
on the largest centred square inside the illuminated region, after the
global complex factor of the reconstruction is fixed by matching the
square's mean to the truth's (gamma = mean O_true / mean O_rec, so the zero
frequency transfers with 1: a blur or noise would bias a least-squares
factor) and with each square's mean removed, the cross-spectral transfer per annulus of
radial frequency f (cycles/pixel, nbins equal bins up to 0.5)
    H(f) = |sum_{k in bin} R^(k) conj(T^(k))| / sum_{k in bin} |T^(k)|^2,
R^ and T^ the 2D DFTs of reconstruction and truth.  For a linear
shift-invariant blur this is the blur's transfer averaged over the bin with
weights |T^|^2; noise uncorrelated with the object averages out.  For a
phase object (|O| ~ 1), O - mean ~ i (phi - mean phi), so it is the
transfer of the phase map to first order.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def linear_integration(raw: np.ndarray, t: Sequence[float], sat: float, dark: float = 0.0) -> np.ndarray:
    """SLI of raw [J][K][H][W] (exposure times t ascending) -> [J][H][W]."""
    raw = np.asarray(raw, np.float64)
    tt = np.asarray(t, np.float64)[None, :, None, None]
    m = raw < sat
    num = np.sum(np.where(m, raw - dark, 0.0), axis=1)
    den = np.sum(np.where(m, tt, 0.0), axis=1)
    out = raw[:, 0] - dark
    ok = den > 0
    out[ok] = num[ok] / den[ok] * t[0]
    return out


def single_exposure(raw: np.ndarray, dark: float = 0.0) -> np.ndarray:
    """The shortest exposure of raw [J][K][H][W] -> [J][H][W]."""
    return np.asarray(raw, np.float64)[:, 0] - dark


def radiometric_deviation(F: np.ndarray, C: np.ndarray) -> float:
    return float(np.linalg.norm(F - C) / np.linalg.norm(C))


def snr_db(F: np.ndarray, C: np.ndarray) -> float:
    return float(10.0 * np.log10(np.sum(C * C) / np.sum((F - C) ** 2)))


def background_variance(F: np.ndarray, C: np.ndarray, frac: float = 1e-3) -> float:
    bg = C < frac * C.max()
    return float(np.var(F[bg]))


def inscribed_square(mask: np.ndarray):
    """(y0, x0, n): the largest square centred on the mask's bounding-box
    centre with every pixel inside the mask."""
    ys, xs = np.nonzero(mask)
    cy, cx = (ys.min() + ys.max() + 1) // 2, (xs.min() + xs.max() + 1) // 2
    h = 0
    while True:
        y0, x0, n = cy - (h + 1), cx - (h + 1), 2 * (h + 1)
        if y0 < 0 or x0 < 0 or y0 + n > mask.shape[0] or x0 + n > mask.shape[1]:
            break
        if not mask[y0:y0 + n, x0:x0 + n].all():
            break
        h += 1
    return cy - h, cx - h, 2 * h


def mtf(O_rec: np.ndarray, O_true: np.ndarray, mask: np.ndarray, nbins: int = 16):
    """(bin centres in cycles/pixel, H per bin) of the reading above."""
    O_rec = np.asarray(O_rec, np.complex128)
    O_true = np.asarray(O_true, np.complex128)
    y0, x0, n = inscribed_square(np.asarray(mask, bool))
    T = O_true[y0:y0 + n, x0:x0 + n]
    R = O_rec[y0:y0 + n, x0:x0 + n]
    R = R * (T.mean() / R.mean())
    Rh = np.fft.fft2(R - R.mean())
    Th = np.fft.fft2(T - T.mean())
    f = np.fft.fftfreq(n)
    fr = np.sqrt(f[:, None] ** 2 + f[None, :] ** 2)
    edges = np.linspace(0.0, 0.5, nbins + 1)
    H = np.full(nbins, np.nan)
    for b in range(nbins):
        sel = (fr >= edges[b]) & (fr < edges[b + 1]) if b < nbins - 1 else (fr >= edges[b]) & (fr <= 0.5)
        den = np.sum(np.abs(Th[sel]) ** 2)
        if den > 0:
            H[b] = abs(np.sum(Rh[sel] * np.conj(Th[sel]))) / den
    return 0.5 * (edges[:-1] + edges[1:]), H
