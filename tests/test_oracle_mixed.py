"""Pins of the mixed-state oracle: the single-mode engine at M = 1, the
invariance of the model and the covariance of the update under unitary
mixing of the modes, the projection's exact total intensity, finite-
difference gradients of the loss, and a two-mode data set that one mode
cannot fit."""
import numpy as np
import pytest

from oracle import mixed, ptycho
from oracle.fourier import fft2u

RNG = np.random.default_rng(21)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def gauss_probe(n, shift, phase):
    yy, xx = np.mgrid[0:n, 0:n]
    return np.exp(-((yy - n / 2 - shift) ** 2 + (xx - n / 2) ** 2) / (n / 4) ** 2) * np.exp(1j * phase * yy / n)


def problem(M=2, Nw=16, Nd=16, J=9, seed=4):
    rng = np.random.default_rng(seed)
    Mo = 40
    O_true = np.exp(1j * rng.standard_normal((Mo, Mo)) * 0.5) * (1 + 0.2 * rng.standard_normal((Mo, Mo)))
    P = np.stack([gauss_probe(Nw, 1.5 * m, 2.0 + m) * (0.8 ** m) for m in range(M)])
    pos = np.stack(np.meshgrid(np.arange(3) * 9 + 2, np.arange(3) * 9 + 3, indexing="ij"), -1).reshape(-1, 2)[:J]
    I = mixed.forward_intensity(O_true, P, pos, Nd)
    return O_true, P, pos, I


def unitary(M, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((M, M)) +
                        1j * np.random.default_rng(seed + 1).standard_normal((M, M)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("alg,batch,Nd", [("epie", 1, 16), ("rpie", 4, 16), ("rpie", 3, 32)])
def test_one_mode_is_the_single_mode_engine(alg, batch, Nd):
    O_true, P, pos, I = problem(M=1, Nd=Nd)
    O0 = np.ones_like(O_true)
    prm = ptycho.PtychoParams(alg=alg, alpha=0.3, beta=0.4, batch=batch, update_probe=True)
    Oa, Pa, ea = mixed.iterate(O0, P * 0.9, I, pos, 2, prm)
    Ob, Pb, eb = ptycho.iterate(O0, P[0] * 0.9, I, pos, 2, prm)
    np.testing.assert_allclose(Oa, Ob, atol=1e-12)
    np.testing.assert_allclose(Pa[0], Pb, atol=1e-12)
    np.testing.assert_allclose(ea, eb, rtol=1e-12)


@pytest.mark.parametrize("M", [2, 3])
def test_intensity_is_invariant_under_unitary_mode_mixing(M):
    O_true, P, pos, _ = problem(M=M)
    U = unitary(M, M)
    Pu = np.einsum("mk,kyx->myx", U, P)
    np.testing.assert_allclose(mixed.forward_intensity(O_true, Pu, pos, 16),
                               mixed.forward_intensity(O_true, P, pos, 16), rtol=1e-11, atol=1e-13)
    # and it is the sum of the modes' single-mode intensities
    single = sum(ptycho.forward_intensity(O_true, P[m], pos, 16) for m in range(M))
    np.testing.assert_allclose(mixed.forward_intensity(O_true, P, pos, 16), single, rtol=1e-12)


@pytest.mark.parametrize("alg", ["epie", "rpie"])
def test_update_is_covariant_under_unitary_mode_mixing(alg):
    # mixing the starting modes by U gives the same object and the modes of
    # the unmixed run mixed by U
    M = 3
    O_true, P, pos, I = problem(M=M)
    O0 = np.ones_like(O_true) * (0.9 + 0.2j)
    P0 = P * 0.8 + 0.05 * crandn(*P.shape)
    U = unitary(M, 7)
    prm = ptycho.PtychoParams(alg=alg, alpha=0.3, beta=0.4, batch=3, update_probe=True)
    Oa, Pa, ea = mixed.iterate(O0, P0, I, pos, 2, prm)
    Ob, Pb, eb = mixed.iterate(O0, np.einsum("mk,kyx->myx", U, P0), I, pos, 2, prm)
    np.testing.assert_allclose(Ob, Oa, atol=1e-11)
    np.testing.assert_allclose(Pb, np.einsum("mk,kyx->myx", U, Pa), atol=1e-11)
    np.testing.assert_allclose(eb, ea, rtol=1e-11)


def test_projection_keeps_mode_ratios_and_sets_the_total():
    Psi = crandn(3, 8, 8)
    A = np.abs(crandn(8, 8))
    out = mixed.project(Psi, A)
    np.testing.assert_allclose(np.sum(np.abs(out) ** 2, axis=0), A ** 2, rtol=1e-12)
    ratio = out / Psi
    np.testing.assert_allclose(ratio.imag, 0, atol=1e-12)
    np.testing.assert_allclose(ratio[0].real, ratio[1].real, rtol=1e-12)
    assert np.all(ratio.real > 0)
    zero = np.zeros((2, 4, 4), complex)
    out0 = mixed.project(zero, np.full((4, 4), 2.0))
    assert np.all(out0[0] == 2.0) and np.all(out0[1] == 0)


def loss(O, P, A, p):
    Nw = P.shape[-1]
    y, x = p
    psi = mixed._pad(P * O[y:y + Nw, x:x + Nw][None], A.shape[-1])
    tot = np.sqrt(sum(np.abs(fft2u(s)) ** 2 for s in psi))
    return float(np.sum((tot - A) ** 2))


@pytest.mark.parametrize("Nd", [16, 32])
def test_numerators_are_minus_the_conjugate_gradients(Nd):
    O_true, P, pos, I = problem(M=2, Nd=Nd)
    A = ptycho.amplitudes(I)
    O = np.ones_like(O_true) + 0.1 * crandn(*O_true.shape)
    Pw = P + 0.05 * crandn(*P.shape)
    p = pos[4]
    numO, numP, _ = mixed.position_terms(O, Pw, A[4], p)
    h = 1e-6
    E = crandn(*Pw.shape)
    fd = (loss(O, Pw + h * E, A[4], p) - loss(O, Pw - h * E, A[4], p)) / (2 * h)
    assert abs(fd + 2 * np.real(np.vdot(numP, E))) < 1e-6 * abs(fd)
    Ew = crandn(16, 16)
    EO = np.zeros_like(O)
    EO[p[0]:p[0] + 16, p[1]:p[1] + 16] = Ew
    fd = (loss(O + h * EO, Pw, A[4], p) - loss(O - h * EO, Pw, A[4], p)) / (2 * h)
    assert abs(fd + 2 * np.real(np.vdot(numO, Ew))) < 1e-6 * abs(fd)


def test_two_mode_data_need_two_modes():
    # an even and an odd (first-order Hermite-Gauss-like) mode, 5 x 5 raster
    # with 4 px steps, known probe modes: after 60 ePIE iterations the two-mode
    # engine's error is well below that of one mode carrying the same total
    # intensity, whose error stalls
    rng = np.random.default_rng(4)
    O_true = np.exp(1j * rng.standard_normal((40, 40)) * 0.5) * (1 + 0.2 * rng.standard_normal((40, 40)))
    yy, xx = np.mgrid[0:16, 0:16]
    g = np.exp(-((yy - 8) ** 2 + (xx - 8) ** 2) / 16.0)
    P = np.stack([g * np.exp(2j * yy / 16), 0.7 * g * (yy - 8) / 4 * np.exp(1j * xx / 16)])
    pos = np.stack(np.meshgrid(np.arange(5) * 4 + 2, np.arange(5) * 4 + 3, indexing="ij"), -1).reshape(-1, 2)
    I = mixed.forward_intensity(O_true, P, pos, 16)
    O0 = np.ones_like(O_true)
    prm = ptycho.PtychoParams(alg="epie", alpha=1.0, beta=1.0, batch=1, update_probe=False)
    _, _, e2 = mixed.iterate(O0, P, I, pos, 60, prm)
    P1 = P[0] * np.sqrt(np.sum(np.abs(P) ** 2) / np.sum(np.abs(P[0]) ** 2))
    _, _, e1 = ptycho.iterate(O0, P1, I, pos, 60, prm)
    assert e2[-1] < 0.5 * e1[-1]
    assert e1[-1] > 0.9 * e1[-20]                 # one mode has stalled


def test_unit_probe_step_on_a_constant_modulus_window_projects_every_mode():
    # ePIE with beta = 1 and one position whose object window has |O| = c: the
    # probe step conj(O) dpsi_m / c^2 makes P_m,new O the projected wave of
    # every mode, so the position's error with the new probe and the old
    # object vanishes (a step counted once per mode would leave half of it)
    n, c = 16, 1.3
    m = np.arange(n)
    O = np.ones((30, 30), complex)
    O[5:21, 7:23] = c * np.exp(2j * np.pi * (m[:, None] + 3 * m[None, :]) / n)
    P = crandn(2, n, n)
    pos = np.array([[5, 7]])
    A = ptycho.amplitudes(mixed.forward_intensity(crandn(30, 30), P, pos, n))
    prm = ptycho.PtychoParams(alg="epie", alpha=1.0, beta=1.0, batch=1, update_probe=True)
    assert loss(O, P, A[0], (5, 7)) > 1.0
    _, P1, _ = mixed.batch_update(O, P, A, pos, [0], prm, True)
    assert loss(O, P1, A[0], (5, 7)) < 1e-20 * loss(O, P, A[0], (5, 7))
