"""Pins of the reconstruction oracle (Eqs. 2-3, mini-batched ePIE/rPIE)
against the published sequential algorithms, fixed points, projection
identities and noiseless convergence.  CPU only."""
import numpy as np
import pytest

from oracle import fourier, ptycho
from paper_2608_01746_amd import synth


def _tiny_geometry(M=48, Nw=16, r=5.0, n_side=6, step=5, offset=4, seed=1):
    O = synth.make_object(M, seed)
    P = synth.make_probe(Nw, r, np.pi)
    pos = synth.raster_positions(n_side, step, offset)
    assert pos.max() + Nw <= M
    return O, P, pos


def test_projection_identities():
    rng = np.random.default_rng(0)
    Psi = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    Psi[3, 4] = 0.0
    A = rng.uniform(0, 2, size=(16, 16))
    Q = ptycho.modulus_projection(Psi, A)
    np.testing.assert_allclose(np.abs(Q), A, atol=1e-14)
    np.testing.assert_allclose(ptycho.modulus_projection(Q, A), Q, atol=1e-14)
    assert Q[3, 4] == A[3, 4]
    m = np.abs(Psi) > 0
    np.testing.assert_allclose(np.angle(Q[m] * np.conj(Psi[m])), 0.0, atol=1e-12)


@pytest.mark.parametrize("alg,B,upd", [("epie", 1, False), ("rpie", 4, True), ("epie", 36, True)])
def test_truth_is_a_fixed_point(alg, B, upd):
    O, P, pos = _tiny_geometry()
    I = ptycho.forward_intensity(O, P, pos, 16)
    prm = ptycho.PtychoParams(alg=alg, alpha=0.3, beta=0.7, batch=B, update_probe=upd)
    O1, P1, err = ptycho.iterate(O, P, I, pos, 1, prm)
    assert np.max(np.abs(O1 - O)) < 1e-12
    assert np.max(np.abs(P1 - P)) < 1e-12
    assert err[0] < 1e-24


def test_rpie_alpha_one_equals_epie_alpha_one():
    O, P, pos = _tiny_geometry(seed=2)
    I = ptycho.forward_intensity(synth.make_object(48, 99), P, pos, 16)
    O0 = np.ones_like(O)
    a = ptycho.iterate(O0, P, I, pos, 2, ptycho.PtychoParams("epie", 1.0, 1.0, 3, True))
    b = ptycho.iterate(O0, P, I, pos, 2, ptycho.PtychoParams("rpie", 1.0, 1.0, 3, True))
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-14, atol=1e-14)


def _textbook_epie(O, P, A, pos, alpha, beta, update_probe):
    # Maiden & Rodenburg (2009), one position at a time, written directly.
    Nw = P.shape[0]
    O = O.copy()
    P = P.copy()
    for (y, x), Aj in zip(pos, A):
        Oj = O[y:y + Nw, x:x + Nw].copy()
        psi = P * Oj
        F = np.fft.fft2(psi, norm="ortho")
        F = Aj * np.exp(1j * np.angle(F))
        d = np.fft.ifft2(F, norm="ortho") - psi
        O[y:y + Nw, x:x + Nw] = Oj + alpha * np.conj(P) / np.max(np.abs(P) ** 2) * d
        if update_probe:
            P = P + beta * np.conj(Oj) / np.max(np.abs(Oj) ** 2) * d
    return O, P


def test_batch_of_one_is_textbook_epie():
    O_true, P, pos = _tiny_geometry(seed=3)
    I = ptycho.forward_intensity(O_true, P, pos, 16)
    A = ptycho.amplitudes(I)
    O0 = np.ones_like(O_true)
    P0 = P * np.exp(0.3j)
    Oa, Pa, _ = ptycho.iterate(O0, P0, I, pos, 1, ptycho.PtychoParams("epie", 0.8, 0.6, 1, True))
    Ob, Pb = _textbook_epie(O0, P0, A, pos, 0.8, 0.6, True)
    np.testing.assert_allclose(Oa, Ob, atol=1e-12)
    np.testing.assert_allclose(Pa, Pb, atol=1e-12)


def test_disjoint_batch_equals_sequential_object_update():
    O_true = synth.make_object(64, 4)
    P = synth.make_probe(16, 6.0, np.pi)
    pos = np.array([[0, 0], [0, 24], [24, 0], [40, 40]], np.int32)
    I = ptycho.forward_intensity(O_true, P, pos, 16)
    O0 = np.ones_like(O_true)
    prm_b = ptycho.PtychoParams("rpie", 0.2, 0.2, 4, False)
    prm_s = ptycho.PtychoParams("rpie", 0.2, 0.2, 1, False)
    Ob, _, eb = ptycho.iterate(O0, P, I, pos, 1, prm_b)
    Os, _, es = ptycho.iterate(O0, P, I, pos, 1, prm_s)
    np.testing.assert_allclose(Ob, Os, atol=1e-13)
    np.testing.assert_allclose(eb, es, rtol=1e-13)


def test_overlapping_updates_are_averaged():
    # two identical positions in one batch move O exactly as one would
    O_true = synth.make_object(32, 5)
    P = synth.make_probe(16, 6.0, 0.0)
    pos1 = np.array([[8, 8]], np.int32)
    pos2 = np.array([[8, 8], [8, 8]], np.int32)
    I1 = ptycho.forward_intensity(O_true, P, pos1, 16)
    I2 = np.concatenate([I1, I1])
    O0 = np.ones_like(O_true)
    prm = ptycho.PtychoParams("rpie", 0.5, 0.5, 2, False)
    a, _, _ = ptycho.iterate(O0, P, I1, pos1, 1, prm)
    b, _, _ = ptycho.iterate(O0, P, I2, pos2, 1, prm)
    np.testing.assert_allclose(a, b, atol=1e-14)


def test_zero_padded_window_placement_is_irrelevant():
    # |F| is invariant to where the window sits inside the padded frame
    O = synth.make_object(32, 6)
    P = synth.make_probe(8, 3.0, 1.0)
    psi = ptycho.exit_wave(O, P, (4, 4), 32)
    moved = np.roll(psi, (11, 7), axis=(0, 1))
    np.testing.assert_allclose(np.abs(fourier.fft2u(psi)), np.abs(fourier.fft2u(moved)), atol=1e-13)


def test_nrmse_properties():
    rng = np.random.default_rng(7)
    O = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    mask = np.ones(O.shape, bool)
    assert ptycho.nrmse(O * np.exp(0.7j) * 2.0, O, mask) < 1e-14
    noise = 1e-3 * (rng.standard_normal(O.shape) + 1j * rng.standard_normal(O.shape))
    v = ptycho.nrmse(O + noise, O, mask)
    assert 0.5e-3 < v < 2e-3


def test_error_metric_zero_at_truth_and_positive_elsewhere():
    O, P, pos = _tiny_geometry(seed=8)
    I = ptycho.forward_intensity(O, P, pos, 16)
    _, _, e0 = ptycho.iterate(O, P, I, pos, 1, ptycho.PtychoParams(batch=6))
    _, _, e1 = ptycho.iterate(np.ones_like(O), P, I, pos, 1, ptycho.PtychoParams(batch=6))
    assert e0[0] < 1e-25 and e1[0] > 1e-3


def test_noiseless_known_probe_converges():
    # noiseless data, known probe: rPIE drives the object NRMSE below 1e-6
    O_true, P, pos = _tiny_geometry(M=48, Nw=16, r=6.0, n_side=7, step=4, offset=4, seed=9)
    I = ptycho.forward_intensity(O_true, P, pos, 16)
    mask = ptycho.illumination_mask(P, pos, O_true.shape, 0.5)
    O = np.ones_like(O_true)
    prm = ptycho.PtychoParams("rpie", 0.05, 0.1, 1, False)
    v = 1.0
    for it in range(40):
        O, _, _ = ptycho.iterate(O, P, I, pos, 25, prm)
        v = ptycho.nrmse(O, O_true, mask)
        if v < 1e-6:
            break
    assert v < 1e-6, v


def test_batch_of_one_is_textbook_rpie_with_soft_probe():
    # Maiden, Johnson & Li (2017) regularised update, one position at a time;
    # a probe with a varying modulus makes alpha and beta matter.
    rng = np.random.default_rng(12)
    O_true, P, pos = _tiny_geometry(seed=12)
    P = P * (0.3 + 0.7 * rng.random(P.shape))
    I = ptycho.forward_intensity(O_true, P, pos, 16)
    A = ptycho.amplitudes(I)
    O = np.ones_like(O_true)
    Pc = P * np.exp(0.2j)
    a, b = 0.3, 0.6
    Oa, Pa, _ = ptycho.iterate(O, Pc, I, pos, 1, ptycho.PtychoParams("rpie", a, b, 1, True))
    Nw = 16
    for (y, x), Aj in zip(pos, A):
        Oj = O[y:y + Nw, x:x + Nw].copy()
        psi = Pc * Oj
        F = np.fft.fft2(psi, norm="ortho")
        d = np.fft.ifft2(Aj * np.exp(1j * np.angle(F)), norm="ortho") - psi
        P2, O2 = np.abs(Pc) ** 2, np.abs(Oj) ** 2
        O[y:y + Nw, x:x + Nw] = Oj + np.conj(Pc) * d / ((1 - a) * P2 + a * P2.max())
        Pc = Pc + np.conj(Oj) * d / ((1 - b) * O2 + b * O2.max())
    np.testing.assert_allclose(Oa, O, atol=1e-12)
    np.testing.assert_allclose(Pa, Pc, atol=1e-12)


def test_nrmse_closed_forms():
    # orthogonal estimate: nothing to align, error 1; half-and-half mixture: sqrt(1/2)
    T = np.zeros(8, complex)
    T[:4] = 1.0
    O = np.zeros(8, complex)
    O[4:] = 1.0
    m = np.ones(8, bool)
    assert abs(ptycho.nrmse(O, T, m) - 1.0) < 1e-15
    assert abs(ptycho.nrmse(T + O, T, m) - np.sqrt(0.5)) < 1e-15
    # the mask removes pixels entirely
    m2 = np.arange(8) < 4
    assert ptycho.nrmse(T + O, T, m2) < 1e-15


def test_stitch_reproduces_truth_and_fills_uncovered():
    O, P, pos = _tiny_geometry()
    Nw = P.shape[0]
    patches = np.stack([np.stack([np.abs(O[y:y + Nw, x:x + Nw]), np.angle(O[y:y + Nw, x:x + Nw])], -1)
                        for y, x in pos])
    S = ptycho.stitch(patches, P, pos, O.shape)
    cov = np.zeros(O.shape)
    for y, x in pos:
        cov[y:y + Nw, x:x + Nw] += np.abs(P) ** 2
    assert np.abs(S - O)[cov > 0].max() < 1e-12
    assert np.all(S[cov == 0] == 1.0)


def test_stitch_weighted_mean_by_hand():
    # two 2x2 windows overlapping in one column; probe intensities 1 and 4
    P = np.array([[1.0, 2.0], [1.0, 2.0]], complex)
    pos = np.array([[0, 0], [0, 1]])
    patches = np.zeros((2, 2, 2, 2))
    patches[0, ..., 0] = 2.0
    patches[1, ..., 0] = 1.0
    patches[1, ..., 1] = np.pi / 2
    S = ptycho.stitch(patches, P, pos, (2, 4))
    # column 0: window 0 only (u=0, w=1) -> 2; column 1: window 0 at u=1 (w=4, value 2)
    # and window 1 at u=0 (w=1, value i) -> (8 + i) / 5; column 2: window 1 only -> i; column 3: 1
    want = np.array([2.0, (8 + 1j) / 5, 1j, 1.0])
    assert np.abs(S - want[None, :]).max() < 1e-15


def test_phase_sync_recovers_window_offsets():
    # true patches, each rotated by its own random constant phase: the
    # synchronised stitch equals the object up to one global phase
    O, P, pos = _tiny_geometry()
    Nw = P.shape[0]
    rng = np.random.default_rng(3)
    off = rng.uniform(-np.pi, np.pi, len(pos))
    patches = np.stack([np.stack([np.abs(O[y:y + Nw, x:x + Nw]),
                                  np.angle(O[y:y + Nw, x:x + Nw] * np.exp(1j * off[j]))], -1)
                        for j, (y, x) in enumerate(pos)])
    mask = ptycho.illumination_mask(P, pos, O.shape)
    plain = ptycho.stitch(patches, P, pos, O.shape)
    assert ptycho.nrmse(plain, O, mask) > 0.3
    c = ptycho.phase_sync(patches, P, pos, O.shape)
    assert np.allclose(np.abs(c), 1.0)
    assert abs(np.angle(np.sum(c))) < 1e-12
    # c_j undoes the offsets up to one common phase
    rel = c * np.exp(1j * off)
    assert np.abs(rel / rel[0] - 1.0).max() < 1e-9
    synced = ptycho.stitch(patches, P, pos, O.shape, phasors=c)
    assert ptycho.nrmse(synced, O, mask) < 1e-9


def test_phase_sync_gram_is_hermitian_psd_by_brute_force():
    # two windows overlapping in a 1 x 2 strip, flat probe: C by hand
    P = np.ones((2, 2), complex)
    pos = np.array([[0, 0], [1, 0]])
    patches = np.zeros((2, 2, 2, 2))
    patches[..., 0] = 1.0
    patches[0, 1, :, 1] = [0.2, 0.4]     # window 0, row 1 (overlap)
    patches[1, 0, :, 1] = [0.7, 0.9]     # window 1, row 0 (overlap)
    c = ptycho.phase_sync(patches, P, pos, (3, 2))
    # C_01 = sum over the strip of e^{-i 0.2} e^{i 0.7} + e^{-i 0.4} e^{i 0.9} = 2 e^{i 0.5}
    # leading eigenvector of [[4, 2e^{i.5}], [2e^{-i.5}, 4]] is (e^{i.5}, 1)/sqrt 2
    want = np.array([np.exp(0.25j), np.exp(-0.25j)])
    assert np.abs(c - want).max() < 1e-12


def test_conditioning_record_reproduces():
    # the spreads recorded in tests/golden (written by make_conditioning.py from
    # the oracle) are what the oracle gives now; the GPU bars scale with them
    import json
    import os
    from _cases import SMALL_ONE_ITER_CASES, small_one_iter_spread
    rec = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "conditioning_spreads.json")))
    for alg, B, upd in SMALL_ONE_ITER_CASES:
        sO, sP = small_one_iter_spread(alg, B, upd)
        r = rec[f"{alg}-{B}-{upd}"]
        assert sO == pytest.approx(r["spread_object"], rel=1e-9)
        assert sP == pytest.approx(r["spread_probe"], rel=1e-9, abs=1e-15)


def test_illumination_mask_by_hand():
    # |P|^2 = [[1, 0], [0, 4]] at corners (0, 0) and (1, 1) of a 3 x 3 object:
    # summed intensity [[1, 0, 0], [0, 5, 0], [0, 0, 4]], maximum 5
    P = np.array([[1.0, 0.0], [0.0, 2.0j]])
    pos = np.array([[0, 0], [1, 1]])
    m = ptycho.illumination_mask(P, pos, (3, 3))          # threshold 0.5
    np.testing.assert_array_equal(m, np.eye(3, dtype=bool))
    m = ptycho.illumination_mask(P, pos, (3, 3), frac=0.3)  # threshold 1.5
    np.testing.assert_array_equal(m, np.diag([False, True, True]))
    m = ptycho.illumination_mask(P, pos, (3, 3), frac=0.9)  # threshold 4.5
    np.testing.assert_array_equal(m, np.diag([False, True, False]))
