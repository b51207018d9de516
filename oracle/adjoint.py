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


# Relative increase of the loss over the reference that still counts as no
# increase (descend()).
DESCENT_TOL = 1e-6


def step_sizes(O: np.ndarray, P: np.ndarray, pos: np.ndarray) -> Tuple[float, float]:
    """Fixed gradient-descent step sizes (a reading; the paper fixes none):
    eta_O = 1 / (2 max_x sum_j |P(x - p_j)|^2) over the object grid and
    eta_P = 1 / (2 max_u sum_j |O_j(u)|^2) over the probe window, i.e. the
    inverse of the largest diagonal curvature of the amplitude loss in O
    (resp. P) with the other held fixed."""
    Nw = P.shape[0]
    illum = np.zeros(O.shape)
    cover = np.zeros(P.shape)
    for p in pos:
        y, x = int(p[0]), int(p[1])
        illum[y:y + Nw, x:x + Nw] += np.abs(P) ** 2
        cover += np.abs(O[y:y + Nw, x:x + Nw]) ** 2
    return 1.0 / (2.0 * illum.max()), 1.0 / (2.0 * cover.max())


def descend(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray, kind: str = "poisson",
            eps: float = 1e-6, n_steps: int = 1, eta_O: float = 0.0, eta_P: float = 0.0,
            update_probe: bool = True):
    """Full-batch gradient descent on the loss above with backtracking (a
    reading; the paper prescribes no descent schedule).  Pass s evaluates the
    loss L_s and both gradients at the current (O, P):
      * s = 0, or L_s <= L_ref + DESCENT_TOL |L_ref| with L_ref the loss of
        the last accepted pass: the pass is accepted, its point, gradients
        and loss become the reference, and O -= eta_O gO (and, with
        update_probe, P -= eta_P gP);
      * otherwise both step sizes are halved and the next point is the
        reference point minus the halved steps along its gradients.
    DESCENT_TOL bounds the float32 evaluation error of a loss: the Poisson
    loss carries a large data-only constant, so late improvements are small
    relative to it, and without the tolerance rounding noise could reject a
    good step.
    Step sizes <= 0 start from step_sizes() of the starting O and P.
    Returns (O, P, losses[n_steps], accepted[n_steps]); O and P are the last
    point formed (its loss not evaluated)."""
    O = np.array(O, np.complex128)
    P = np.array(P, np.complex128)
    eO, eP = step_sizes(O, P, pos)
    if eta_O > 0.0:
        eO = eta_O
    if eta_P > 0.0:
        eP = eta_P
    losses = np.zeros(n_steps)
    accepted = np.zeros(n_steps, bool)
    best = None  # the reference: (loss, O, P, gO, gP)
    for s in range(n_steps):
        losses[s], gO, gP = loss_and_grad(O, P, I_centred, pos, kind, eps)
        if best is None or losses[s] <= best[0] + DESCENT_TOL * abs(best[0]):
            accepted[s] = True
            best = (losses[s], O, P, gO, gP)
        else:
            eO, eP = eO / 2.0, eP / 2.0
        _, Ob, Pb, gOb, gPb = best
        O = Ob - eO * gOb
        P = Pb - eP * gPb if update_probe else Pb
    return O, P, losses, accepted
