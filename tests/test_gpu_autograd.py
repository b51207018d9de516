"""The adjoint behind torch.autograd.Function: backward equals the library
gradient and the float64 oracle gradient, scales with the upstream factor,
and drives a few gradient-descent steps downhill."""
import numpy as np
import pytest
import torch

from oracle import adjoint, ptycho
from paper_2608_01746_amd import synth

from _cases import c64, f32, soft_probe

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api, autograd
    return api, autograd


def _problem(Nd=64, Nw=48, M=128, seed=3):
    rng = np.random.default_rng(seed)
    O_true = synth.make_object(M, seed)
    P = c64(soft_probe(synth.make_probe(Nw, Nw / 3, 1.0), seed))
    pos = synth.raster_positions(4, 24, 4)
    I = f32(ptycho.forward_intensity(O_true, P, pos, Nd))
    O = c64(O_true * (1 + 0.05 * rng.standard_normal(O_true.shape)))
    return O, P, pos, I


@pytest.mark.parametrize("kind", ["poisson", "amplitude"])
def test_backward_matches_oracle(mods, kind):
    api, ag = mods
    O, P, pos, I = _problem()
    Ot = torch.from_numpy(O.astype(np.complex64)).to(DEV).requires_grad_(True)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(DEV).requires_grad_(True)
    It = torch.from_numpy(I.astype(np.float32)).to(DEV)
    loss = ag.ptycho_loss(Ot, Pt, It, pos, kind, 1e-6, 8)
    (3.0 * loss).backward()
    lr, gOr, gPr = adjoint.loss_and_grad(O, P, I, pos, kind, 1e-6, upstream=3.0)
    assert abs(loss.item() - lr) <= 1e-5 * abs(lr) + 1e-3
    gO = Ot.grad.cpu().numpy()
    gP = Pt.grad.cpu().numpy()
    assert np.linalg.norm(gO - gOr) / np.linalg.norm(gOr) < 1e-5
    assert np.linalg.norm(gP - gPr) / np.linalg.norm(gPr) < 1e-5


def test_only_object_gradient_requested(mods):
    api, ag = mods
    O, P, pos, I = _problem(seed=4)
    Ot = torch.from_numpy(O.astype(np.complex64)).to(DEV).requires_grad_(True)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(DEV)
    loss = ag.ptycho_loss(Ot, Pt, torch.from_numpy(I.astype(np.float32)).to(DEV), pos)
    loss.backward()
    _, gO, _ = api.ptycho_grad(Ot.detach(), Pt, torch.from_numpy(I.astype(np.float32)).to(DEV), pos)
    assert torch.equal(Ot.grad, gO)


def test_gradient_descent_lowers_the_loss(mods):
    api, ag = mods
    O, P, pos, I = _problem(seed=5)
    Ot = torch.from_numpy(O.astype(np.complex64)).to(DEV).requires_grad_(True)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(DEV)
    It = torch.from_numpy(I.astype(np.float32)).to(DEV)
    # fixed step 1 / (2 max_x sum_j |P(x - p_j)|^2)
    cover = np.zeros(O.shape)
    for y, x in pos:
        cover[y:y + P.shape[0], x:x + P.shape[1]] += np.abs(P) ** 2
    eta = 1.0 / (2.0 * cover.max())
    losses = []
    for _ in range(5):
        loss = ag.ptycho_loss(Ot, Pt, It, pos, "amplitude", 0.0, 16)
        losses.append(loss.item())
        Ot.grad = None
        loss.backward()
        with torch.no_grad():
            Ot -= eta * Ot.grad
    assert all(b < a for a, b in zip(losses, losses[1:]))
