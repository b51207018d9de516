"""Oracle: Multi-Scale Non-linear Fusion (MNF) of an exposure bracket.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64 throughout.

Follows Methods 3.4 of the paper step by step, one position at a time and
one exposure at a time:

  3.4.1  normalised intensity in [0, 1] and the Gaussian well-exposedness
         weight (Eq. 5), normalised to sum to one over the exposures;
  3.4.2  Gaussian pyramids of every image and every weight map (Eq. 6) and
         the Laplacian pyramid of every image (Eq. 7);
  3.4.3  modulation of each exposure's Laplacian coefficients by its
         weight pyramid and per-level quantisation (Eq. 8);
  3.4.4  per-exposure recursive collapse (Eq. 9) and the sum over
         exposures (Eq. 10).

Readings of points the paper leaves open (each is also listed in the
design notes):
  * normalisation: I_bar = clip((I - dark) / (sat - dark), 0, 1);
  * the images that are decomposed are radiometrically scaled counts,
    I_tilde_k = (I_k - dark) * t_1 / t_k ("counts at the shortest
    exposure"); with radiometric=False the normalised I_bar_k is used;
  * w_G is the 5-tap binomial [1, 4, 6, 4, 1] / 16, separable;
  * borders: reflect-101 on the grid the filter runs on (scipy's
    ``mode='mirror'``); down-sampling keeps even indices; up-sampling
    inserts zeros and filters with 2 w_G per axis;
  * L levels means L band-pass levels l = 0..L-1 (l = 0 finest) plus the
    Gaussian base G_L;
  * the base is weighted but not quantised: R_L = G_L[W_k] G_L[I_tilde_k];
  * the collapse is recursive: R_{l-1} = U(R_l) + L_tilde_{l-1};
  * the quantisation step of exposure k at level l is
    delta_l * t_1 / t_k (delta_l in ADU of that exposure), a zero step
    disables quantisation; rounding is half-to-even;
  * optional contrast factor (Mertens-style; the paper's weight is Eq. 5
    alone, which contrast_exp = 0 gives exactly): the raw weight of
    exposure k is multiplied by (C_k + CONTRAST_EPS) ** contrast_exp, with
    C_k = |4-neighbour Laplacian of I_bar_k| on the level-0 grid
    (reflect-101 borders; along an axis of length one the neighbours are
    the pixel itself) and CONTRAST_EPS = 1e-6, so that flat regions,
    where every C_k is zero, keep the Eq. 5 weights.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np
from scipy.ndimage import correlate1d

# Binomial smoothing kernel w_G (Eq. 6 reading).
W_G = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0

# Offset added to the contrast before the exponent (flat regions keep the
# well-exposedness weights).
CONTRAST_EPS = 1e-6


@dataclasses.dataclass
class FuseParams:
    levels: int = 4
    mu: float = 0.5
    sigma: float = 0.2
    sat: float = 4095.0
    dark: float = 0.0
    delta: Sequence[float] = ()       # per-level step in ADU, l = 0 finest; empty => no quantisation
    radiometric: bool = True
    contrast_exp: float = 0.0         # 0: the paper's weight (Eq. 5 only)

    def delta_at(self, l: int) -> float:
        return float(self.delta[l]) if l < len(self.delta) else 0.0


# --- Section 3.4.1: exposure quality -----------------------------------------

def normalised_intensity(I: np.ndarray, sat: float, dark: float) -> np.ndarray:
    """I_bar in [0, 1]: dark-subtracted counts over the detector full scale."""
    return np.clip((np.asarray(I, np.float64) - dark) / (sat - dark), 0.0, 1.0)


def raw_weight(Ibar: np.ndarray, mu: float, sigma: float) -> np.ndarray:
    """Eq. 5: W = exp(-(I_bar - mu)^2 / (2 sigma^2))."""
    return np.exp(-((Ibar - mu) ** 2) / (2.0 * sigma * sigma))


def contrast(Ibar: np.ndarray) -> np.ndarray:
    """C = |I(y-1,x) + I(y+1,x) + I(y,x-1) + I(y,x+1) - 4 I(y,x)| of one
    normalised image, neighbours past the edge reflected without repeating
    the edge pixel (numpy's 'reflect', which repeats the pixel itself along
    an axis of length one)."""
    g = np.pad(np.asarray(Ibar, np.float64), 1, mode="reflect")
    return np.abs(g[:-2, 1:-1] + g[2:, 1:-1] + g[1:-1, :-2] + g[1:-1, 2:] - 4.0 * g[1:-1, 1:-1])


def normalised_weights(Ibars: np.ndarray, mu: float, sigma: float, contrast_exp: float = 0.0) -> np.ndarray:
    """Eq. 5 (times the optional contrast factor) followed by the
    normalisation sum_k W_k = 1 (per pixel); Ibars is [K][H][W]."""
    W = raw_weight(Ibars, mu, sigma)
    if contrast_exp > 0.0:
        C = np.stack([contrast(Ibars[k]) for k in range(Ibars.shape[0])])
        W = W * (C + CONTRAST_EPS) ** contrast_exp
    s = W.sum(axis=0)
    return W / np.maximum(s, 1e-30)


# --- Section 3.4.2: pyramids -------------------------------------------------

def reduce(g: np.ndarray) -> np.ndarray:
    """Eq. 6: G_{l+1} = D(G_l * w_G): separable binomial filter
    (reflect-101 borders), then keep even rows and columns."""
    f = correlate1d(g, W_G, axis=0, mode="mirror")
    f = correlate1d(f, W_G, axis=1, mode="mirror")
    return f[::2, ::2]


def expand(g: np.ndarray) -> np.ndarray:
    """U in Eq. 7: insert zeros to double each axis, then interpolate with
    2 w_G per axis (reflect-101 borders on the fine grid)."""
    h, w = g.shape
    z = np.zeros((2 * h, w))
    z[::2, :] = g
    z = correlate1d(z, 2.0 * W_G, axis=0, mode="mirror")
    y = np.zeros((2 * h, 2 * w))
    y[:, ::2] = z
    return correlate1d(y, 2.0 * W_G, axis=1, mode="mirror")


def gaussian_pyramid(g: np.ndarray, levels: int) -> List[np.ndarray]:
    """[G_0, ..., G_L] with G_0 = g (Eq. 6)."""
    pyr = [np.asarray(g, np.float64)]
    for _ in range(levels):
        pyr.append(reduce(pyr[-1]))
    return pyr


def laplacian_pyramid(G: List[np.ndarray]) -> List[np.ndarray]:
    """Eq. 7: L_l = G_l - U(G_{l+1}) for l < L."""
    return [G[l] - expand(G[l + 1]) for l in range(len(G) - 1)]


# --- Section 3.4.3: modulation and quantisation -----------------------------

def quantise(x: np.ndarray, step: float) -> np.ndarray:
    """Eq. 8: step * round(x / step), half-to-even; step 0 leaves x unchanged."""
    if step <= 0.0:
        return x
    return step * np.rint(x / step)


# --- Section 3.4.4: per-exposure collapse and accumulation ------------------

def collapse(base: np.ndarray, details: List[np.ndarray]) -> np.ndarray:
    """Eq. 9, recursive: R_{l-1} = U(R_l) + details[l-1], from R_L = base."""
    R = base
    for l in range(len(details), 0, -1):
        R = expand(R) + details[l - 1]
    return R


def exposure_images(raw: np.ndarray, t: Sequence[float], p: FuseParams):
    """(I_bar_k, I_tilde_k) for a bracket raw[K][H][W]."""
    raw = np.asarray(raw, np.float64)
    Ibar = normalised_intensity(raw, p.sat, p.dark)
    if p.radiometric:
        scale = np.array([t[0] / tk for tk in t], np.float64)[:, None, None]
        Itil = (raw - p.dark) * scale
    else:
        Itil = Ibar
    return Ibar, Itil


def step_size(p: FuseParams, l: int, t: Sequence[float], k: int) -> float:
    """Quantisation step of exposure k at level l in the units of I_tilde."""
    d = p.delta_at(l)
    if d <= 0.0:
        return 0.0
    if p.radiometric:
        return d * t[0] / t[k]
    return d / (p.sat - p.dark)


def fuse_position(raw: np.ndarray, t: Sequence[float], p: FuseParams,
                  return_parts: bool = False):
    """I_MNF for one scan position from its bracket raw[K][H][W] (Eqs. 5-10)."""
    K = raw.shape[0]
    Ibar, Itil = exposure_images(raw, t, p)
    W = normalised_weights(Ibar, p.mu, p.sigma, p.contrast_exp)
    total = np.zeros(raw.shape[1:])
    parts = []
    for k in range(K):
        GI = gaussian_pyramid(Itil[k], p.levels)
        GW = gaussian_pyramid(W[k], p.levels)
        LI = laplacian_pyramid(GI)
        details = [quantise(GW[l] * LI[l], step_size(p, l, t, k)) for l in range(p.levels)]
        base = GW[p.levels] * GI[p.levels]
        Rk = collapse(base, details)
        parts.append(dict(GI=GI, GW=GW, LI=LI, details=details, base=base, R0=Rk))
        total = total + Rk
    if return_parts:
        return total, W, parts
    return total


def fuse(raw: np.ndarray, t: Sequence[float], p: FuseParams) -> np.ndarray:
    """I_MNF for every position of raw[J][K][H][W] (float64 [J][H][W])."""
    return np.stack([fuse_position(raw[j], t, p) for j in range(raw.shape[0])])


def weights(raw: np.ndarray, p: FuseParams) -> np.ndarray:
    """Normalised weights [J][K][H][W] of every bracket (Eq. 5 + normalisation)."""
    Ibar = normalised_intensity(raw, p.sat, p.dark)
    return np.stack([normalised_weights(Ibar[j], p.mu, p.sigma, p.contrast_exp) for j in range(raw.shape[0])])
