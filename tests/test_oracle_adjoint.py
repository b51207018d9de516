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


# --- gradient descent (full batch, backtracking) -----------------------------

def test_one_descent_step_is_the_modulus_projection():
    # unit probe covering the whole object at one position (Nw = Nd = M), the
    # amplitude loss: gO = 2 (psi - F^-1(sqrt(I) Psi / |Psi|)), the automatic
    # eta_O = 1 / (2 * 1) = 1/2, so one step lands exactly on the Fourier
    # modulus projection of the object (the error-reduction update)
    rng = np.random.default_rng(5)
    N = 16
    O0 = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    I_fft = rng.uniform(0.5, 2.0, size=(N, N)) ** 2
    I_centred = np.fft.fftshift(I_fft)[None]
    P = np.ones((N, N), complex)
    pos = np.zeros((1, 2), int)
    O1, P1, losses, acc = adjoint.descend(O0, P, I_centred, pos, "amplitude", 0.0, n_steps=1, update_probe=False)
    Psi = np.fft.fft2(O0, norm="ortho")
    want = np.fft.ifft2(np.sqrt(I_fft) * Psi / np.abs(Psi), norm="ortho")
    np.testing.assert_allclose(O1, want, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(P1, P)
    assert losses[0] == pytest.approx(float(np.sum((np.abs(Psi) - np.sqrt(I_fft)) ** 2)), rel=1e-12)


def test_step_sizes_by_hand():
    # |P|^2 = 4 everywhere, |O|^2 = 1/4 everywhere; three windows, two of them
    # at the same corner: the illumination peaks at 2 * 4 = 8 (eta_O = 1/16) and
    # every probe pixel sees 3 * 1/4 (eta_P = 2/3)
    P = np.full((4, 4), 2.0 + 0j)
    O = np.full((12, 12), 0.5j)
    pos = np.array([[0, 0], [0, 0], [6, 5]])
    eO, eP = adjoint.step_sizes(O, P, pos)
    assert eO == pytest.approx(1 / 16, rel=1e-15)
    assert eP == pytest.approx(2 / 3, rel=1e-15)
    # disjoint windows: eta_O = 1/8
    assert adjoint.step_sizes(O, P, np.array([[0, 0], [6, 5]]))[0] == pytest.approx(1 / 8, rel=1e-15)


def test_descent_lowers_the_amplitude_loss():
    # noiseless data from a true object, a perturbed start: every step is
    # accepted and lowers the loss, object and probe updated together
    rng = np.random.default_rng(8)
    M, Nw = 40, 16
    O_true = synth.make_object(M, 3)
    P = synth.make_probe(Nw, Nw / 4, 1.0)
    pos = np.array([[y, x] for y in range(0, M - Nw + 1, 6) for x in range(0, M - Nw + 1, 6)])
    I = ptycho.forward_intensity(O_true, P, pos, Nw)
    O0 = O_true * (1 + 0.1 * rng.standard_normal((M, M)))
    _, _, losses, acc = adjoint.descend(O0, P * 1.05, I, pos, "amplitude", 0.0, n_steps=6)
    assert acc.all() and np.all(np.diff(losses) < 0), losses
    assert losses[-1] < 0.5 * losses[0]


def test_descent_backtracks_by_hand():
    # one pixel (Nw = Nd = 1, the transform is the identity), amplitude loss
    # (|P O| - 1)^2 with gradients gO = conj(P) g, gP = conj(O) g,
    # g = 2 (psi - psi / |psi|), psi = P O, from O = 3, P = 1 (g = 4).
    O0 = np.array([[3.0 + 0j]])
    P0 = np.array([[1.0 + 0j]])
    I = np.array([[[1.0]]])
    pos = np.zeros((1, 2), int)
    # object only, eta_O = 2:
    #   pass 0: L = 4, accepted;       O = 3 - 2 * 4 = -5
    #   pass 1: L = 16 > 4, rejected;  eta_O = 1, O = 3 - 1 * 4 = -1
    #   pass 2: L = 0, accepted;       the gradient is 0, O stays -1
    O, P, losses, acc = adjoint.descend(O0, P0, I, pos, "amplitude", 0.0, n_steps=3, eta_O=2.0,
                                        update_probe=False)
    np.testing.assert_allclose(losses, [4.0, 16.0, 0.0], atol=1e-12)
    assert acc.tolist() == [True, False, True]
    np.testing.assert_allclose(O, [[-1.0]], atol=1e-12)
    np.testing.assert_array_equal(P, P0)
    # object and probe, eta_O = 2, eta_P = 1 (gP = 3 * 4 = 12):
    #   pass 0: L = 4, accepted;   O = -5, P = 1 - 12 = -11
    #   pass 1: psi = 55, L = 2916, rejected; O = 3 - 4 = -1, P = 1 - 6 = -5
    #   pass 2: psi = 5, L = 16 > 4, rejected; O = 3 - 2 = 1, P = 1 - 3 = -2
    O, P, losses, acc = adjoint.descend(O0, P0, I, pos, "amplitude", 0.0, n_steps=3, eta_O=2.0, eta_P=1.0)
    np.testing.assert_allclose(losses, [4.0, 2916.0, 16.0], atol=1e-9)
    assert acc.tolist() == [True, False, False]
    np.testing.assert_allclose(O, [[1.0]], atol=1e-12)
    np.testing.assert_allclose(P, [[-2.0]], atol=1e-12)


def test_descent_tolerates_increases_below_the_tolerance():
    # the one-pixel problem from O = 3 (L = 4, g = 4): a step to
    # O = -(3 + d) gives L = (2 + d)^2 = 4 (1 + d + d^2 / 4); it is accepted
    # for d = 5e-7 (an increase of 5e-7 relative, inside DESCENT_TOL = 1e-6)
    # and rejected for d = 4e-6
    O0 = np.array([[3.0 + 0j]])
    P0 = np.array([[1.0 + 0j]])
    I = np.array([[[1.0]]])
    pos = np.zeros((1, 2), int)
    assert adjoint.DESCENT_TOL == 1e-6
    for d, ok in [(5e-7, True), (4e-6, False)]:
        eta = (6.0 + d) / 4.0
        _, _, losses, acc = adjoint.descend(O0, P0, I, pos, "amplitude", 0.0, n_steps=2, eta_O=eta,
                                            update_probe=False)
        assert losses[1] == pytest.approx((2.0 + d) ** 2, rel=1e-12)
        assert acc.tolist() == [True, ok]
