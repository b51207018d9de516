"""Oracle: real-valued (sub-pixel) scan positions for the far-field model and
the mini-batched ePIE / rPIE update.

TEST INFRASTRUCTURE ONLY (see the package docstring).  float64 throughout.

Eq. 2 evaluates the object at the probe coordinates shifted by the scan
position; the paper's positions (a Fermat spiral, Methods 3.3) are real
numbers, and the integer-grid engine in ``ptycho`` rounds them.  Here a
position r = p + d is split into the nearest integer corner
p = floor(r + 1/2) and a fraction d in [-1/2, 1/2) per axis.

Reading (the sub-pixel model).  The exit wave P(m) O(p + m + d) and the
same wave translated by d, P(m - d) O(p + m), have the same far-field
intensity (a translation only multiplies the spectrum by a phase ramp), so
the fraction is carried by the probe:
    psi_j = S_{d_j}[P] * O[p_j window],
    S_d[f] = F^-1[ F[f](k) exp(-2 pi i (k_y d_y + k_x d_x) / Nw) ],
a Fourier (band-limited) translation of f by +d over the Nw x Nw window,
with the discrete frequencies k in [-Nw/2, Nw/2) (the Nyquist bin taken as
-Nw/2).  S_d is unitary, S_d^-1 = S_d^H = S_{-d}.  Then, for each mini-batch
from the batch-start state:
    P_j     = S_{d_j}[P]
    dpsi_j  = psi'_j - psi_j           (Fourier-modulus projection as in ptycho)
    O[p_j window] += sum_j conj(P_j) dpsi_j / sum_j d_O
    P             += sum_j S_{-d_j}[conj(O_j) dpsi_j] / sum_j d_P,j
The numerators are minus the Wirtinger gradients of sum (|Psi| - A)^2 with
respect to conj(O) and conj(P) (the chain rule through the unitary S_d).
The step denominators d_O and d_P,j are those of the integer engine, formed
from the unshifted batch-start probe |P|^2 and the integer windows |O_j|^2:
they only scale the step, and a Fourier-translated intensity map can turn
negative.  With every d_j = 0 the iteration is the integer one.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

from .fourier import fft2u, ifft2u
from .ptycho import PtychoParams, _den_object, _den_probe, amplitudes, modulus_projection


def split_positions(pos: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Real positions [J][2] -> (integer corners p = floor(r + 1/2), fractions r - p)."""
    r = np.asarray(pos, np.float64)
    p = np.floor(r + 0.5)
    return p.astype(np.int64), r - p


def freqs(n: int) -> np.ndarray:
    """Discrete frequencies 0, 1, .., n/2 - 1, -n/2, .., -1 (integers)."""
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n)


def fourier_shift(f: np.ndarray, d) -> np.ndarray:
    """S_d[f]: band-limited translation of the square array f by +d = (d_y, d_x)
    over its own period (the result at m is f(m - d))."""
    n = f.shape[-1]
    k = freqs(n)
    ramp = np.exp(-2j * np.pi * (k[:, None] * d[0] + k[None, :] * d[1]) / n)
    return np.fft.ifft2(np.fft.fft2(f) * ramp)


def _pad(psi: np.ndarray, Nd: int) -> np.ndarray:
    Nw = psi.shape[0]
    if Nd == Nw:
        return psi
    out = np.zeros((Nd, Nd), np.complex128)
    out[:Nw, :Nw] = psi
    return out


def exit_wave(O: np.ndarray, P: np.ndarray, r, Nd: int) -> np.ndarray:
    """Eq. 2 at a real position r (y, x): S_d[P] * O[p window], zero-padded
    at the top-left into Nd x Nd."""
    Nw = P.shape[0]
    p, d = split_positions(np.asarray(r, np.float64)[None, :])
    y, x = int(p[0, 0]), int(p[0, 1])
    return _pad(fourier_shift(P, d[0]) * O[y:y + Nw, x:x + Nw], Nd)


def forward_intensity(O: np.ndarray, P: np.ndarray, pos: np.ndarray, Nd: int) -> np.ndarray:
    """Eq. 3 at real positions: detector-centred |F psi_j|^2, [J][Nd][Nd]."""
    out = np.empty((len(pos), Nd, Nd))
    for j, r in enumerate(np.asarray(pos, np.float64)):
        out[j] = np.fft.fftshift(np.abs(fft2u(exit_wave(O, P, r, Nd))) ** 2)
    return out


def position_terms(O: np.ndarray, P: np.ndarray, A_j: np.ndarray, r):
    """For one position: (numO, numP, err) with numO = conj(P_j) dpsi_j on the
    integer window, numP = S_{-d}[conj(O_j) dpsi_j] and err = sum (|Psi| - A)^2."""
    Nw = P.shape[0]
    Nd = A_j.shape[-1]
    p, d = split_positions(np.asarray(r, np.float64)[None, :])
    y, x = int(p[0, 0]), int(p[0, 1])
    Oj = O[y:y + Nw, x:x + Nw]
    Pj = fourier_shift(P, d[0])
    psi = _pad(Pj * Oj, Nd)
    Psi = fft2u(psi)
    err = float(np.sum((np.abs(Psi) - A_j) ** 2))
    dpsi = (ifft2u(modulus_projection(Psi, A_j)) - psi)[:Nw, :Nw]
    numO = np.conj(Pj) * dpsi
    numP = fourier_shift(np.conj(Oj) * dpsi, -d[0])
    return numO, numP, err


def batch_update(O: np.ndarray, P: np.ndarray, A: np.ndarray, pos: np.ndarray, idx: np.ndarray,
                 prm: PtychoParams, update_probe: bool):
    """One mini-batch (positions ``idx``) from the batch-start state (O, P)."""
    Nw = P.shape[0]
    p, _ = split_positions(pos)
    P2 = np.abs(P) ** 2
    maxP2 = float(P2.max())
    numO = np.zeros_like(O)
    denO = np.zeros(O.shape)
    numP = np.zeros_like(P)
    denP = np.zeros(P.shape)
    err = 0.0
    for j in idx:
        y, x = int(p[j, 0]), int(p[j, 1])
        nO, nP, e = position_terms(O, P, A[j], pos[j])
        err += e
        numO[y:y + Nw, x:x + Nw] += nO
        denO[y:y + Nw, x:x + Nw] += _den_object(P2, maxP2, prm)
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
        P_new[okp] += numP[okp] / denP[okp]
    return O_new, P_new, err


def iterate(O: np.ndarray, P: np.ndarray, I_centred: np.ndarray, pos: np.ndarray, n_iter: int,
            prm: PtychoParams, order: Optional[np.ndarray] = None, it0: int = 0):
    """Iterations it0 .. it0+n_iter-1 at real positions ``pos`` [J][2];
    returns (O, P, normalised Fourier error per iteration)."""
    O = np.array(O, np.complex128)
    P = np.array(P, np.complex128)
    pos = np.asarray(pos, np.float64)
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
