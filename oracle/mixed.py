"""Oracle: mixed-state (multi-mode) probes for partially coherent data.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64 throughout.

The paper's XUV source carries two harmonics (Methods 3.2), and Eq. 4 sums
their far-field intensities incoherently, which one coherent probe cannot
model.  The mixed-state model (Thibault & Menzel 2013) writes the measured
intensity as an incoherent sum over M probe modes sharing one object,
    I_j = sum_m |F(P_m O_j)|^2.
Reading (the paper does not reconstruct with modes): the mini-batched ePIE /
rPIE update of ``ptycho`` generalised to modes, all from the batch-start
state,
    psi_jm  = P_m O[p_j window],          Psi_jm = F psi_jm  (zero-padded to Nd)
    Psi'_jm = A_j Psi_jm / sqrt(sum_m |Psi_jm|^2)
              (where the sum is 0: A_j in mode 0, 0 in the others)
    dpsi_jm = F^-1 Psi'_jm - psi_jm      (cropped to the window)
    O[p_j window] += sum_j sum_m conj(P_m) dpsi_jm / sum_j d_O
    P_m           += sum_j conj(O_j) dpsi_jm / sum_j d_P,j
with d_O formed from the total probe intensity Q = sum_m |P_m|^2
(rPIE: (1 - alpha) Q + alpha max Q;  ePIE: max Q / alpha) and d_P,j as in
the single-mode engine.  The Fourier error is sum (sqrt(sum_m |Psi|^2) - A)^2
over the batch-start state.  The modes are not orthogonalised.  With M = 1
this is the single-mode engine.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .fourier import fft2u, ifft2u
from .ptycho import PtychoParams, _den_object, _den_probe, amplitudes


def _pad(psi: np.ndarray, Nd: int) -> np.ndarray:
    Nw = psi.shape[-1]
    if Nd == Nw:
        return psi
    out = np.zeros(psi.shape[:-2] + (Nd, Nd), np.complex128)
    out[..., :Nw, :Nw] = psi
    return out


def forward_intensity(O: np.ndarray, P: np.ndarray, pos: np.ndarray, Nd: int) -> np.ndarray:
    """Detector-centred sum_m |F(P_m O_j)|^2 for probes P [M][Nw][Nw], [J][Nd][Nd]."""
    P = np.asarray(P, np.complex128)
    Nw = P.shape[-1]
    out = np.empty((len(pos), Nd, Nd))
    for j, (y, x) in enumerate(np.asarray(pos, np.int64)):
        Psi = np.stack([fft2u(_pad(Pm * O[y:y + Nw, x:x + Nw], Nd)) for Pm in P])
        out[j] = np.fft.fftshift(np.sum(np.abs(Psi) ** 2, axis=0))
    return out


def project(Psi: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Scale every mode Psi[m] by A / sqrt(sum_m |Psi_m|^2) (mode 0 gets A where the sum is 0)."""
    tot = np.sqrt(np.sum(np.abs(Psi) ** 2, axis=0))
    out = np.zeros_like(Psi)
    nz = tot > 0
    for m in range(Psi.shape[0]):
        out[m][nz] = Psi[m][nz] * (A[nz] / tot[nz])
    out[0][~nz] = A[~nz]
    return out


def position_terms(O: np.ndarray, P: np.ndarray, A_j: np.ndarray, p):
    """For one position: (numO, numP[M], err) with numO = sum_m conj(P_m) dpsi_m
    on the window, numP[m] = conj(O_j) dpsi_m and err = sum (sqrt(sum_m |Psi_m|^2) - A)^2."""
    Nw = P.shape[-1]
    Nd = A_j.shape[-1]
    y, x = int(p[0]), int(p[1])
    Oj = O[y:y + Nw, x:x + Nw]
    psi = _pad(P * Oj[None], Nd)
    Psi = np.stack([fft2u(s) for s in psi])
    err = float(np.sum((np.sqrt(np.sum(np.abs(Psi) ** 2, axis=0)) - A_j) ** 2))
    Psi_new = project(Psi, A_j)
    dpsi = np.stack([ifft2u(s) for s in Psi_new])[:, :Nw, :Nw] - psi[:, :Nw, :Nw]
    numO = np.sum(np.conj(P) * dpsi, axis=0)
    numP = np.conj(Oj)[None] * dpsi
    return numO, numP, err


def batch_update(O: np.ndarray, P: np.ndarray, A: np.ndarray, pos: np.ndarray, idx, prm: PtychoParams,
                 update_probe: bool):
    """One mini-batch (positions ``idx``) from the batch-start state (O, P[M])."""
    Nw = P.shape[-1]
    Q = np.sum(np.abs(P) ** 2, axis=0)
    maxQ = float(Q.max())
    numO = np.zeros_like(O)
    denO = np.zeros(O.shape)
    numP = np.zeros_like(P)
    denP = np.zeros(P.shape[1:])
    err = 0.0
    for j in idx:
        y, x = int(pos[j, 0]), int(pos[j, 1])
        nO, nP, e = position_terms(O, P, A[j], pos[j])
        err += e
        numO[y:y + Nw, x:x + Nw] += nO
        denO[y:y + Nw, x:x + Nw] += _den_object(Q, maxQ, prm)
        if update_probe:
            O2 = np.abs(O[y:y + Nw, x:x + Nw]) ** 2
            numP += nP
            denP += _den_probe(O2, float(O2.max()), prm)
    O_new = O.copy()
    cov = denO > 0
    O_new[cov] += numO[cov] / denO[cov]
    P_new = P.copy()
    if update_probe:
        okp = denP > 0
        for m in range(P.shape[0]):
            P_new[m][okp] += numP[m][okp] / denP[okp]
    return O_new, P_new, err


def iterate(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray, n_iter: int,
            prm: PtychoParams, order: Optional[np.ndarray] = None, it0: int = 0):
    """Iterations it0 .. it0+n_iter-1 with probe modes P [M][Nw][Nw]; returns
    (O, P, normalised Fourier error per iteration)."""
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
