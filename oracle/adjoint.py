"""Oracle: far-field loss on fused intensities and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64 throughout.

The paper frames reconstruction under the intensity model I ~ |F psi|^2
with Poisson statistics (Introduction; Methods 3.3, Eqs. 2-3).  The loss
summed over positions j and detector pixels q (no mean) is

  Poisson    l = |Psi|^2 - I ln(|Psi|^2 + eps)
  amplitude  l = (|Psi| - sqrt(I))^2

with Psi_j = F psi_j, psi_j = P O[p_j window] (zero-padded to Nd) and
I = max(I_MNF, 0) in FFT order.

Gradient convention: g = dL/dRe + i dL/dIm = 2 dL/dconj(z) (the convention
of PyTorch's complex autograd).  Chain rule, written out:
  g_Psi  = 2 (1 - I / (|Psi|^2 + eps)) Psi             (Poisson)
         = 2 (Psi - sqrt(I) Psi / |Psi|)   [Psi/|Psi| := 0 at 0]   (amplitude)
  g_psi  = F^-1 g_Psi     (F unitary, so its adjoint is its inverse), cropped
  gO[p_j + u] += conj(P(u)) g_psi(u),   gP(u) += conj(O_j(u)) g_psi(u).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from .fourier import fft2u, ifft2u, to_fft_order
from .ptycho import exit_wave


def fft_order_intensity(I_centred: np.ndarray) -> np.ndarray:
    return np.maximum(to_fft_order(np.asarray(I_centred, np.float64)), 0.0)


def loss(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray,
         kind: str = "poisson", eps: float = 1e-6) -> float:
    """Loss value summed over positions and pixels."""
    I = fft_order_intensity(I_centred)
    Nd = I.shape[-1]
    total = 0.0
    for j, p in enumerate(pos):
        Psi = fft2u(exit_wave(O, P, p, Nd))
        m2 = np.abs(Psi) ** 2
        if kind == "poisson":
            total += float(np.sum(m2 - I[j] * np.log(m2 + eps)))
        else:
            total += float(np.sum((np.sqrt(m2) - np.sqrt(I[j])) ** 2))
    return total


def loss_and_grad(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray,
                  kind: str = "poisson", eps: float = 1e-6,
                  upstream: float = 1.0) -> Tuple[float, np.ndarray, np.ndarray]:
    """(loss, gO, gP); the gradients are scaled by ``upstream``."""
    I = fft_order_intensity(I_centred)
    Nd = I.shape[-1]
    Nw = P.shape[0]
    gO = np.zeros(O.shape, np.complex128)
    gP = np.zeros(P.shape, np.complex128)
    total = 0.0
    for j, p in enumerate(pos):
        y, x = int(p[0]), int(p[1])
        Psi = fft2u(exit_wave(O, P, p, Nd))
        m2 = np.abs(Psi) ** 2
        if kind == "poisson":
            total += float(np.sum(m2 - I[j] * np.log(m2 + eps)))
            gPsi = 2.0 * (1.0 - I[j] / (m2 + eps)) * Psi
        else:
            m = np.sqrt(m2)
            total += float(np.sum((m - np.sqrt(I[j])) ** 2))
            unit = np.zeros_like(Psi)
            nz = m > 0
            unit[nz] = Psi[nz] / m[nz]
            gPsi = 2.0 * (Psi - np.sqrt(I[j]) * unit)
        gpsi = ifft2u(gPsi)[:Nw, :Nw] * upstream
        gO[y:y + Nw, x:x + Nw] += np.conj(P) * gpsi
        gP += np.conj(O[y:y + Nw, x:x + Nw]) * gpsi
    return total, gO, gP
