"""Pins of the sub-pixel oracle against facts fixed outside it: translations
by whole pixels, the translation of a sampled plane wave, the group
properties of the Fourier translation, the shift invariance of the far-field
intensity for band-limited waves, the integer engine as the zero-fraction
case, finite-difference gradients, and exact projections for unit steps."""
import numpy as np
import pytest

from oracle import ptycho, subpixel
from oracle.fourier import fft2u

RNG = np.random.default_rng(11)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def test_split_positions_nearest_corner():
    r = np.array([[2.5, -0.5], [3.49, 7.0], [0.51, 10.25]])
    p, d = subpixel.split_positions(r)
    assert p.tolist() == [[3, 0], [3, 7], [1, 10]]
    np.testing.assert_allclose(d, [[-0.5, -0.5], [0.49, 0.0], [-0.49, 0.25]], atol=1e-12)
    assert np.all(d >= -0.5) and np.all(d < 0.5)


@pytest.mark.parametrize("d", [(3, -2), (0, 5), (-7, 1)])
def test_whole_pixel_translation_is_a_cyclic_roll(d):
    f = crandn(16, 16)
    np.testing.assert_allclose(subpixel.fourier_shift(f, d), np.roll(f, d, axis=(0, 1)), atol=1e-12)


@pytest.mark.parametrize("a,b", [(1, 2), (-3, 5), (-8, 0), (0, -8), (7, -8)])
def test_translation_of_a_sampled_plane_wave(a, b):
    # f(m) = exp(2 pi i (a m_y + b m_x) / n) translated by d is f(m - d) in closed
    # form; a or b = -n/2 fixes the reading of the Nyquist bin as -n/2
    n = 16
    m = np.arange(n)
    d = (0.3, -0.45)
    f = np.exp(2j * np.pi * (a * m[:, None] + b * m[None, :]) / n)
    want = np.exp(2j * np.pi * (a * (m[:, None] - d[0]) + b * (m[None, :] - d[1])) / n)
    np.testing.assert_allclose(subpixel.fourier_shift(f, d), want, atol=1e-12)


def test_translation_group_properties():
    f, g = crandn(32, 32), crandn(32, 32)
    a, b = (0.37, -0.21), (-0.12, 0.44)
    S = subpixel.fourier_shift
    np.testing.assert_allclose(S(S(f, a), b), S(f, (a[0] + b[0], a[1] + b[1])), atol=1e-12)
    np.testing.assert_allclose(S(S(f, a), (-a[0], -a[1])), f, atol=1e-12)
    assert np.isclose(np.linalg.norm(S(f, a)), np.linalg.norm(f))
    # adjoint of S_a is S_-a
    lhs = np.vdot(g, S(f, a))
    rhs = np.vdot(S(g, (-a[0], -a[1])), f)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def trig_poly(coef, n, y, x):
    """sum_k c_k exp(2 pi i (k_y y + k_x x) / n) at real coordinates."""
    out = np.zeros(np.broadcast(y, x).shape, np.complex128)
    for (ky, kx), c in coef.items():
        out = out + c * np.exp(2j * np.pi * (ky * y + kx * x) / n)
    return out


@pytest.mark.parametrize("r", [(10.3, 20.7), (5.5, 7.45), (12.0, 3.2), (8.49, 9.51)])
def test_intensity_matches_the_directly_evaluated_exit_wave(r):
    # band-limited object and probe (total bandwidth below n/2): the model's
    # translated probe times the integer window has the far-field intensity of
    # P(m) O(r + m) evaluated exactly at the real position
    n = 32
    rng = np.random.default_rng(5)
    co = {(ky, kx): complex(*rng.standard_normal(2)) for ky in range(-3, 4) for kx in range(-3, 4)}
    cp = {(ky, kx): complex(*rng.standard_normal(2)) for ky in range(-4, 5) for kx in range(-4, 5)}
    M = 64
    yy, xx = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    O = trig_poly(co, n, yy, xx)
    m = np.arange(n)
    P = trig_poly(cp, n, m[:, None], m[None, :])
    model = subpixel.forward_intensity(O, P, np.array([r]), n)[0]
    direct = P * trig_poly(co, n, r[0] + m[:, None], r[1] + m[None, :])
    want = np.fft.fftshift(np.abs(fft2u(direct)) ** 2)
    np.testing.assert_allclose(model, want, atol=1e-9 * want.max())


def small_problem(Nw=16, Nd=16, J=6, seed=3):
    rng = np.random.default_rng(seed)
    M = 40
    O = 1 + 0.3 * (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    yy, xx = np.meshgrid(np.arange(Nw), np.arange(Nw), indexing="ij")
    P = np.exp(-((yy - Nw / 2) ** 2 + (xx - Nw / 2) ** 2) / (Nw / 3) ** 2) * np.exp(0.4j * yy)
    pos = rng.uniform(1.0, M - Nw - 2.0, size=(J, 2))
    O_true = 1 + 0.3 * (rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)))
    I = subpixel.forward_intensity(O_true, P, pos, Nd)
    return O, P, pos, I


@pytest.mark.parametrize("alg,batch", [("epie", 1), ("rpie", 4)])
def test_zero_fractions_reduce_to_the_integer_engine(alg, batch):
    O, P, pos, I = small_problem()
    pos = np.round(pos)
    prm = ptycho.PtychoParams(alg=alg, alpha=0.3, beta=0.4, batch=batch, update_probe=True)
    Oa, Pa, ea = subpixel.iterate(O, P, I, pos, 2, prm)
    Ob, Pb, eb = ptycho.iterate(O, P, I, pos.astype(np.int64), 2, prm)
    np.testing.assert_allclose(Oa, Ob, atol=1e-12)
    np.testing.assert_allclose(Pa, Pb, atol=1e-12)
    np.testing.assert_allclose(ea, eb, rtol=1e-12)


def loss(O, P, A, r):
    Nw = P.shape[0]
    psi = subpixel.exit_wave(O, P, r, A.shape[-1])
    return float(np.sum((np.abs(fft2u(psi)) - A) ** 2))


@pytest.mark.parametrize("Nd", [16, 32])
def test_numerators_are_minus_the_conjugate_gradients(Nd):
    # dL along a direction E is 2 Re <g, E> with g = dL/d conj(z); the numerators are -g
    O, P, pos, I = small_problem(Nd=Nd)
    A = ptycho.amplitudes(I)
    r = pos[1]
    numO, numP, _ = subpixel.position_terms(O, P, A[1], r)
    p, _ = subpixel.split_positions(r[None, :])
    y, x = int(p[0, 0]), int(p[0, 1])
    h = 1e-6
    E = crandn(*P.shape)
    fd = (loss(O, P + h * E, A[1], r) - loss(O, P - h * E, A[1], r)) / (2 * h)
    assert abs(fd + 2 * np.real(np.vdot(numP, E))) < 1e-6 * abs(fd)
    Ew = crandn(*P.shape)
    EO = np.zeros_like(O)
    EO[y:y + 16, x:x + 16] = Ew
    fd = (loss(O + h * EO, P, A[1], r) - loss(O - h * EO, P, A[1], r)) / (2 * h)
    assert abs(fd + 2 * np.real(np.vdot(numO, Ew))) < 1e-6 * abs(fd)


def test_unit_steps_on_constant_modulus_fields_project_exactly():
    # |P_j| = c everywhere (a plane-wave probe stays one under translation): the
    # object step conj(P_j) dpsi / c^2 makes P_j O_new the projected wave, so the
    # position's error vanishes; likewise the probe step on a constant-modulus
    # object window.  A step built with the untranslated probe would not.
    n = 16
    m = np.arange(n)
    c = 1.7
    P = c * np.exp(2j * np.pi * (3 * m[:, None] - 2 * m[None, :]) / n)
    rng = np.random.default_rng(2)
    O = 1 + 0.4 * (rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32)))
    r = np.array([6.3, 9.8])
    A = ptycho.amplitudes(subpixel.forward_intensity(crandn(32, 32), P, r[None, :], n))[0]
    numO, _, e0 = subpixel.position_terms(O, P, A, r)
    assert e0 > 1.0
    O1 = O.copy()
    O1[6:22, 10:26] += numO / c ** 2
    assert loss(O1, P, A, r) < 1e-20 * e0
    Ow = c * np.exp(2j * np.pi * (m[:, None] + 5 * m[None, :]) / n)
    O2 = np.zeros((32, 32), complex)
    O2[6:22, 10:26] = Ow
    P1 = P + 0.3 * crandn(n, n)  # any probe: the step projects onto the measured modulus
    _, numP, e1 = subpixel.position_terms(O2, P1, A, r)
    assert loss(O2, P1 + numP / c ** 2, A, r) < 1e-20 * e1


def test_iterations_reduce_the_error_on_consistent_data():
    O, P, pos, I = small_problem(J=12)
    prm = ptycho.PtychoParams(alg="rpie", alpha=0.1, batch=4)
    _, _, err = subpixel.iterate(O, P, I, pos, 6, prm)
    assert err[-1] < 0.5 * err[0]
