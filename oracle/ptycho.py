"""Oracle: far-field ptychographic reconstruction from fused intensities.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64 throughout.

The paper feeds I_MNF to an iterative phase-retrieval engine (Introduction,
citing PIE and ePIE) over the forward model of Methods 3.3:
  Eq. 2  exit wave psi_j = P(r) O(r - r_j) (projection approximation),
  Eq. 3  far-field intensity |F psi_j|^2 (Fraunhofer, unitary F).
The engine is the mini-batched ePIE (Maiden & Rodenburg 2009) / rPIE
(Maiden, Johnson & Li 2017) update:

  for each mini-batch b of the iteration's position order, using O and P as
  they are at the start of the batch:
    psi_j   = P * O[p_j window]              (zero-padded to Nd if Nw < Nd)
    Psi_j   = F psi_j
    Psi'_j  = A_j Psi_j / |Psi_j|            (A_j where |Psi_j| = 0)
    psi'_j  = F^-1 Psi'_j                    (cropped to the Nw window)
    dpsi_j  = psi'_j - psi_j
    O[x]   += sum_j conj(P) dpsi_j / sum_j d_O          (over windows covering x)
    P      += sum_j conj(O_j) dpsi_j / sum_j d_P,j      (if the probe is updated)
  with
    rPIE: d_O = (1 - alpha) |P|^2 + alpha max|P|^2,
          d_P,j = (1 - beta) |O_j|^2 + beta max|O_j|^2
    ePIE: d_O = max|P|^2 / alpha,  d_P,j = max|O_j|^2 / beta.
  Object and probe updates are simultaneous (both use the batch-start
  state).  A batch of one position is exactly the published sequential
  algorithm.  Pixels no window covers keep their value.

Readings: A_j = sqrt(max(I_MNF, 0)) in FFT order (fused intensities are
detector-centred and may be slightly negative); scan positions are integer
top-left window corners (y, x) in O; the Fourier error of an iteration is
sum_j sum_q (|Psi_j| - A_j)^2 / sum_j sum_q A_j^2, accumulated with each
batch's start state.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

from .fourier import fft2u, ifft2u, to_fft_order


@dataclasses.dataclass
class PtychoParams:
    alg: str = "rpie"          # 'epie' | 'rpie'
    alpha: float = 0.1
    beta: float = 0.1
    batch: int = 1
    update_probe: bool = False
    probe_start_iter: int = 0


def amplitudes(I_centred: np.ndarray) -> np.ndarray:
    """A_j = sqrt(max(I, 0)) in FFT order, for I of shape [J][Nd][Nd]."""
    return np.sqrt(np.maximum(to_fft_order(np.asarray(I_centred, np.float64)), 0.0))


def exit_wave(O: np.ndarray, P: np.ndarray, p, Nd: int) -> np.ndarray:
    """Eq. 2 on an integer grid, zero-padded at the top-left into Nd x Nd."""
    Nw = P.shape[0]
    y, x = int(p[0]), int(p[1])
    psi = P * O[y:y + Nw, x:x + Nw]
    if Nd == Nw:
        return psi
    out = np.zeros((Nd, Nd), np.complex128)
    out[:Nw, :Nw] = psi
    return out


def forward_intensity(O: np.ndarray, P: np.ndarray, pos: np.ndarray, Nd: int) -> np.ndarray:
    """Eq. 3: detector-centred |F psi_j|^2 for every position, [J][Nd][Nd]."""
    out = np.empty((len(pos), Nd, Nd))
    for j, p in enumerate(pos):
        out[j] = np.fft.fftshift(np.abs(fft2u(exit_wave(O, P, p, Nd))) ** 2)
    return out


def modulus_projection(Psi: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Replace the modulus of Psi by A, keeping its phase (phase 0 where Psi = 0)."""
    mag = np.abs(Psi)
    out = A.astype(np.complex128)
    nz = mag > 0
    out[nz] = A[nz] * Psi[nz] / mag[nz]
    return out


def _den_object(P2: np.ndarray, maxP2: float, prm: PtychoParams) -> np.ndarray:
    if prm.alg == "epie":
        return np.full_like(P2, maxP2 / prm.alpha)
    return (1.0 - prm.alpha) * P2 + prm.alpha * maxP2


def _den_probe(O2: np.ndarray, maxO2: float, prm: PtychoParams) -> np.ndarray:
    if prm.alg == "epie":
        return np.full_like(O2, maxO2 / prm.beta)
    return (1.0 - prm.beta) * O2 + prm.beta * maxO2


def batch_update(O: np.ndarray, P: np.ndarray, A: np.ndarray, pos: np.ndarray,
                 idx: np.ndarray, prm: PtychoParams, update_probe: bool) -> Tuple[np.ndarray, np.ndarray, float]:
    """One mini-batch (positions ``idx``) from the batch-start state (O, P).

    Returns (O_new, P_new, sum over the batch of (|Psi| - A)^2)."""
    Nw = P.shape[0]
    Nd = A.shape[-1]
    P2 = np.abs(P) ** 2
    maxP2 = float(P2.max())
    numO = np.zeros_like(O)
    denO = np.zeros(O.shape)
    numP = np.zeros_like(P)
    denP = np.zeros(P.shape)
    err = 0.0
    for j in idx:
        y, x = int(pos[j, 0]), int(pos[j, 1])
        Oj = O[y:y + Nw, x:x + Nw]
        psi = exit_wave(O, P, pos[j], Nd)
        Psi = fft2u(psi)
        err += float(np.sum((np.abs(Psi) - A[j]) ** 2))
        psi_new = ifft2u(modulus_projection(Psi, A[j]))
        dpsi = psi_new[:Nw, :Nw] - psi[:Nw, :Nw]
        numO[y:y + Nw, x:x + Nw] += np.conj(P) * dpsi
        denO[y:y + Nw, x:x + Nw] += _den_object(P2, maxP2, prm)
        if update_probe:
            O2 = np.abs(Oj) ** 2
            numP += np.conj(Oj) * dpsi
            denP += _den_probe(O2, float(O2.max()), prm)
    O_new = O.copy()
    cov = denO > 0
    O_new[cov] += numO[cov] / denO[cov]
    P_new = P.copy()
    if update_probe:
        okp = denP > 0
        P_new[okp] += numP[okp] / denP[okp]
    return O_new, P_new, err


def iterate(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray,
            n_iter: int, prm: PtychoParams, order: Optional[np.ndarray] = None,
            it0: int = 0):
    """Run iterations it0 .. it0+n_iter-1.  ``order`` is [n_iter][J] (one
    permutation per iteration) or None for the identity order.

    Returns (O, P, err[n_iter]) with err the normalised Fourier error."""
    O = np.array(O, np.complex128)
    P = np.array(P, np.complex128)
    A = amplitudes(I_centred)
    J = len(pos)
    sumA2 = float(np.sum(A ** 2))
    errs = np.zeros(n_iter)
    for i in range(n_iter):
        it = it0 + i
        ordr = np.arange(J) if order is None else np.asarray(order[i])
        upd_p = bool(prm.update_probe) and it >= prm.probe_start_iter
        e = 0.0
        for b0 in range(0, J, prm.batch):
            O, P, eb = batch_update(O, P, A, pos, ordr[b0:b0 + prm.batch], prm, upd_p)
            e += eb
        errs[i] = e / sumA2 if sumA2 > 0 else 0.0
    return O, P, errs


def illumination_mask(P: np.ndarray, pos: np.ndarray, shape, frac: float = 0.1) -> np.ndarray:
    """Object pixels whose summed probe intensity reaches ``frac`` of its maximum."""
    Nw = P.shape[0]
    ill = np.zeros(shape)
    P2 = np.abs(P) ** 2
    for y, x in pos:
        ill[y:y + Nw, x:x + Nw] += P2
    return ill >= frac * ill.max()


def nrmse(O: np.ndarray, O_true: np.ndarray, mask: np.ndarray) -> float:
    """min over complex gamma of ||gamma O - O_true|| / ||O_true|| on the mask."""
    a = O[mask]
    b = O_true[mask]
    gamma = np.vdot(a, b) / np.vdot(a, a)
    return float(np.linalg.norm(gamma * a - b) / np.linalg.norm(b))


def window_values(patches: np.ndarray) -> np.ndarray:
    """Complex window values a e^{i phi} from (amplitude, phase) patches."""
    return patches[..., 0] * np.exp(1j * patches[..., 1])


def phase_sync(patches: np.ndarray, P: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """Unit phasors c_j that align overlapping window predictions z_j (each
    known only up to its own constant phase): the maximiser of
    sum_x |sum_j w_j(x) c_j z_j(x)|^2 over |c_j| = 1, relaxed to the leading
    eigenvector of the positive semidefinite matrix
        C_jk = sum_x w_j(x) w_k(x) conj(z_j(x)) z_k(x),  w_j = |P(x - p_j)|^2,
    each entry then projected to unit modulus (Singer's eigenvector method for
    angular synchronisation).  The common phase is fixed by making sum_j c_j
    real and positive.  A reading of the warm-start extension, which the
    paper does not contain."""
    Nw = P.shape[0]
    J = len(pos)
    w = np.abs(P) ** 2
    z = window_values(patches)
    C = np.zeros((J, J), complex)
    for j in range(J):
        for k in range(J):
            y0 = max(pos[j][0], pos[k][0])
            y1 = min(pos[j][0], pos[k][0]) + Nw
            x0 = max(pos[j][1], pos[k][1])
            x1 = min(pos[j][1], pos[k][1]) + Nw
            if y1 <= y0 or x1 <= x0:
                continue
            sj = (slice(y0 - pos[j][0], y1 - pos[j][0]), slice(x0 - pos[j][1], x1 - pos[j][1]))
            sk = (slice(y0 - pos[k][0], y1 - pos[k][0]), slice(x0 - pos[k][1], x1 - pos[k][1]))
            C[j, k] = np.sum(w[sj] * w[sk] * np.conj(z[j][sj]) * z[k][sk])
    vals, vecs = np.linalg.eigh(C)
    v = vecs[:, -1]
    c = np.where(np.abs(v) > 0, v / np.where(np.abs(v) > 0, np.abs(v), 1.0), 1.0)
    s = np.sum(c)
    if abs(s) > 0:
        c = c * np.conj(s) / abs(s)
    return c


def stitch(patches: np.ndarray, P: np.ndarray, pos: np.ndarray, shape,
           phasors: Optional[np.ndarray] = None) -> np.ndarray:
    """Starting object from per-window (amplitude, phase) predictions
    patches [J][Nw][Nw][2]: the |P|^2-weighted mean of c_j a e^{i phi} over
    the windows covering each pixel (c_j = 1 unless phasors are given), 1
    where the summed weight is zero.  This is the warm-start reading of an
    extension the paper does not specify."""
    Nw = P.shape[0]
    num = np.zeros(shape, complex)
    den = np.zeros(shape)
    w = np.abs(P) ** 2
    z = window_values(patches)
    for j, (y, x) in enumerate(pos):
        cj = 1.0 if phasors is None else phasors[j]
        num[y:y + Nw, x:x + Nw] += w * cj * z[j]
        den[y:y + Nw, x:x + Nw] += w
    out = np.ones(shape, complex)
    cov = den > 0
    out[cov] = num[cov] / den[cov]
    return out
