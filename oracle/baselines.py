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
