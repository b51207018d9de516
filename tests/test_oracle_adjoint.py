"""Pins of the loss-gradient oracle against central finite differences in
float64, against PyTorch complex autograd of an independently written
forward model, and at the noiseless truth.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import adjoint, ptycho
from paper_2608_01746_amd import synth


def _fd_problem(seed=0):
    # object 32^2, probe 16^2, 3 x 3 raster with step 8
    rng = np.random.default_rng(seed)
    O = synth.make_object(32, seed + 1)
    P = synth.make_probe(16, 6.0, np.pi) * (0.6 + 0.4 * rng.random((16, 16)))
    pos = synth.raster_positions(3, 8, 0)
    I = rng.uniform(0.0, 3.0, size=(len(pos), 16, 16))
    return O, P, pos, I


@pytest.mark.parametrize("kind", ["poisson", "amplitude"])
def test_gradient_matches_central_differences(kind):
    O, P, pos, I = _fd_problem()
    _, gO, gP = adjoint.loss_and_grad(O, P, I, pos, kind, 1e-6)
    h = 1e-6
    f = lambda O_, P_: adjoint.loss(O_, P_, I, pos, kind, 1e-6)
    fdO = np.zeros_like(O)
    for idx in np.ndindex(O.shape):
        for unit in (1.0, 1j):
            Op = O.copy(); Op[idx] += h * unit
            Om = O.copy(); Om[idx] -= h * unit
            fdO[idx] += unit * (f(Op, P) - f(Om, P)) / (2 * h)
    fdP = np.zeros_like(P)
    for idx in np.ndindex(P.shape):
        for unit in (1.0, 1j):
            Pp = P.copy(); Pp[idx] += h * unit
            Pm = P.copy(); Pm[idx] -= h * unit
            fdP[idx] += unit * (f(O, Pp) - f(O, Pm)) / (2 * h)
    assert np.linalg.norm(gO - fdO) / np.linalg.norm(fdO) < 1e-6
    assert np.linalg.norm(gP - fdP) / np.linalg.norm(fdP) < 1e-6


@pytest.mark.parametrize("kind", ["poisson", "amplitude"])
def test_gradient_matches_torch_autograd(kind):
    O, P, pos, I = _fd_problem(3)
    loss, gO, gP = adjoint.loss_and_grad(O, P, I, pos, kind, 1e-6, upstream=0.5)
    Ot = torch.tensor(O, dtype=torch.complex128, requires_grad=True)
    Pt = torch.tensor(P, dtype=torch.complex128, requires_grad=True)
    It = torch.fft.ifftshift(torch.tensor(I), dim=(-2, -1)).clamp_min(0)
    total = 0.0
    for j, (y, x) in enumerate(pos):
        Psi = torch.fft.fft2(Pt * Ot[y:y + 16, x:x + 16], norm="ortho")
        m2 = Psi.real ** 2 + Psi.imag ** 2
        if kind == "poisson":
            total = total + (m2 - It[j] * torch.log(m2 + 1e-6)).sum()
        else:
            total = total + ((m2.sqrt() - It[j].sqrt()) ** 2).sum()
    (0.5 * total).backward()
    assert abs(total.item() - loss) < 1e-10 * abs(loss)
    np.testing.assert_allclose(gO, Ot.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gP, Pt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_gradient_vanishes_at_noiseless_truth():
    O = synth.make_object(32, 5)
    P = synth.make_probe(16, 6.0, np.pi)
    pos = synth.raster_positions(3, 8, 0)
    I = ptycho.forward_intensity(O, P, pos, 16)
    _, gO, gP = adjoint.loss_and_grad(O, P, I, pos, "amplitude", 0.0)
    assert np.max(np.abs(gO)) < 1e-12 and np.max(np.abs(gP)) < 1e-12
    _, gO, gP = adjoint.loss_and_grad(O, P, I, pos, "poisson", 1e-30)
    assert np.max(np.abs(gO)) < 1e-12 and np.max(np.abs(gP)) < 1e-12


def test_gradient_with_padded_window_matches_differences():
    # Nw = 8 inside a 16^2 detector (zero-padded exit wave, cropped adjoint)
    rng = np.random.default_rng(11)
    O = synth.make_object(16, 12)
    P = synth.make_probe(8, 3.0, 1.0) * (0.5 + rng.random((8, 8)))
    pos = np.array([[0, 0], [4, 6], [8, 8]], np.int32)
    I = rng.uniform(0, 2, size=(3, 16, 16))
    _, gO, gP = adjoint.loss_and_grad(O, P, I, pos, "poisson", 1e-6)
    h = 1e-6
    f = lambda O_, P_: adjoint.loss(O_, P_, I, pos, "poisson", 1e-6)
    for idx in [(0, 0), (5, 9), (15, 15), (10, 3)]:
        d = np.zeros_like(O); d[idx] = h
        fd = (f(O + d, P) - f(O - d, P)) / (2 * h) + 1j * (f(O + 1j * d, P) - f(O - 1j * d, P)) / (2 * h)
        assert abs(fd - gO[idx]) <= 1e-6 * max(1.0, abs(fd))
    for idx in [(0, 0), (3, 4), (7, 7)]:
        d = np.zeros_like(P); d[idx] = h
        fd = (f(O, P + d) - f(O, P - d)) / (2 * h) + 1j * (f(O, P + 1j * d) - f(O, P - 1j * d)) / (2 * h)
        assert abs(fd - gP[idx]) <= 1e-6 * max(1.0, abs(fd))
