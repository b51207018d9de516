"""Parity of the mixed-state (multi-mode probe) entry points with the float64
oracle, through the C ABI.

Bars as for the single-mode path: the forward model to relative L2 2e-6,
one or two float32 iterations from identical float32-representable inputs
to relative L2 1e-5.  One mode is the single-mode path, bit for bit."""
import numpy as np
import pytest
import torch

from oracle import mixed, ptycho
from paper_2608_01746_amd import synth

from _cases import c64, f32, soft_probe

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def tc64(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.complex64))).to(DEV)


def tf32(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(DEV)


def modes(Nw, M, seed):
    """M distinct probe modes: the synthetic probe and Hermite-Gauss-like
    odd/even variants of it with decreasing weights."""
    P = soft_probe(synth.make_probe(Nw, Nw / 4.0, 2.0), seed)
    yy, xx = (np.mgrid[0:Nw, 0:Nw] - Nw / 2.0) / (Nw / 4.0)
    shapes = [np.ones_like(yy), yy, xx, yy * xx]
    return np.stack([P * shapes[m] * 0.7 ** m for m in range(M)])


@pytest.mark.parametrize("Nd,Nw,Mo,M", [(16, 16, 40, 2), (64, 64, 96, 3), (128, 64, 120, 2), (256, 256, 288, 4),
                                        (192, 192, 224, 2), (512, 512, 544, 2)])
def test_forward_matches_oracle(api, Nd, Nw, Mo, M):
    O = c64(synth.make_object(Mo, Nd + M))
    P = c64(modes(Nw, M, 1))
    pos = np.random.default_rng(Nd).integers(0, Mo - Nw + 1, size=(5, 2)).astype(np.int32)
    ref = mixed.forward_intensity(O, P, pos, Nd)
    out = api.ptycho_forward_modes(tc64(O), tc64(P), pos, Nd).cpu().numpy()
    assert rel(out, ref) < 2e-6


def test_one_mode_is_the_single_mode_path(api):
    O, P, pos, I = scan(120, 64, 64, 12, 1, 5)
    order = synth.random_orders(len(pos), 2, 4)
    a = api.ptycho_forward_modes(tc64(O), tc64(P), pos, 64)
    b = api.ptycho_forward(tc64(O), tc64(P[0]), pos, 64)
    assert torch.equal(a, b)
    O1, P1 = tc64(np.ones_like(O)), tc64(P * 0.9)
    O2, P2 = tc64(np.ones_like(O)), tc64(P[0] * 0.9)
    e1 = api.ptycho_iterate_modes(O1, P1, tf32(I), pos, 2, alg="rpie", alpha=0.2, beta=0.3, batch=5,
                                  update_probe=True, order=order)
    e2 = api.ptycho_iterate(O2, P2, tf32(I), pos, 2, alg="rpie", alpha=0.2, beta=0.3, batch=5, update_probe=True,
                            order=order)
    assert torch.equal(O1, O2) and torch.equal(P1[0], P2) and torch.equal(e1, e2)


def scan(Mo, Nw, Nd, J, M, seed):
    O = synth.make_object(Mo, seed)
    P = modes(Nw, M, seed)
    pos = np.random.default_rng(seed).integers(0, Mo - Nw + 1, size=(J, 2)).astype(np.int32)
    I = f32(mixed.forward_intensity(O, P, pos, Nd))
    return O, P, pos, I


def run(api, O0, P0, I, pos, prm, order, n_iter, graph=False):
    Og, Pg = tc64(O0), tc64(P0)
    e = api.ptycho_iterate_modes(Og, Pg, tf32(I), pos, n_iter, alg=prm.alg, alpha=prm.alpha, beta=prm.beta,
                                 batch=prm.batch, update_probe=prm.update_probe,
                                 probe_start_iter=prm.probe_start_iter, order=order, graph=graph)
    return Og.cpu().numpy(), Pg.cpu().numpy(), e.cpu().numpy()


@pytest.mark.parametrize("Nd,Nw,Mo,J,M,alg,B,upd", [
    (64, 64, 128, 16, 2, "rpie", 4, True),
    (64, 64, 128, 13, 3, "epie", 1, True),       # sequential (batches of one position)
    (64, 64, 128, 13, 2, "rpie", 5, False),      # ragged last batch, fixed probe
    (128, 64, 160, 9, 4, "rpie", 4, True),       # exit waves padded into a larger detector
    (32, 32, 80, 25, 2, "rpie", 32, True),       # whole scan in one batch
    (256, 256, 360, 6, 2, "rpie", 4, True),
    (16, 16, 40, 7, 4, "epie", 3, True),
    (512, 512, 560, 3, 2, "rpie", 2, True),      # the largest detector
    (384, 384, 440, 4, 3, "rpie", 3, True),
])
def test_iterations_match_oracle(api, Nd, Nw, Mo, J, M, alg, B, upd):
    O, P, pos, I = scan(Mo, Nw, Nd, J, M, Nd + J)
    O0 = c64(synth.make_object(Mo, 77) * (0.9 + 0.1j))
    P0 = c64(P * np.exp(0.1j) * 0.9)
    prm = ptycho.PtychoParams(alg, 0.2, 0.3, B, upd)
    order = synth.random_orders(J, 2, 3)
    Og, Pg, eg = run(api, O0, P0, I, pos, prm, order, 2)
    Or, Pr, er = mixed.iterate(O0, P0, I, pos, 2, prm, order)
    assert rel(Og, Or) < 1e-5
    assert rel(Pg, Pr) < 1e-5
    np.testing.assert_allclose(eg, er, rtol=1e-5)


def test_probe_start_iteration_and_graph_replay(api):
    O, P, pos, I = scan(128, 64, 64, 12, 2, 9)
    O0 = c64(synth.make_object(128, 78))
    P0 = c64(P * 0.9)
    order = synth.random_orders(12, 3, 5)
    prm = ptycho.PtychoParams("rpie", 0.2, 0.3, 4, True, probe_start_iter=1)
    Og, Pg, eg = run(api, O0, P0, I, pos, prm, order, 3)
    Or, Pr, er = mixed.iterate(O0, P0, I, pos, 3, prm, order)
    assert rel(Og, Or) < 1e-5 and rel(Pg, Pr) < 1e-5
    O2, P2, e2 = run(api, O0, P0, I, pos, prm, order, 3, graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(O2, Og) and np.array_equal(P2, Pg) and np.array_equal(e2, eg)


def test_lab_size_two_modes_one_iteration(api):
    # 1024^2 object, two 256^2 probe modes, the lab raster (400 positions),
    # rPIE mini-batch 32 (64 mode slots per launch, ragged last batch), probe updated
    w = synth.lab_workload()
    O = w.object()
    P = modes(w.Nw, 2, 1)
    I = f32(mixed.forward_intensity(O, P, w.pos, w.Nd))
    O0 = c64(synth.make_object(w.M, 77) * (0.9 + 0.1j))
    P0 = c64(P * np.exp(0.2j) * 0.8)
    prm = ptycho.PtychoParams("rpie", 0.1, 0.1, 32, True)
    order = synth.random_orders(w.J, 1, 2)
    Og, Pg, eg = run(api, O0, P0, I, w.pos, prm, order, 1)
    Or, Pr, er = mixed.iterate(O0, P0, I, w.pos, 1, prm, order)
    assert rel(Og, Or) < 1e-5
    assert rel(Pg, Pr) < 1e-5
    assert abs(eg[0] - er[0]) <= 1e-5 * er[0]


def test_invalid_arguments(api):
    O = tc64(np.ones((80, 80)))
    I = tf32(np.ones((2, 32, 32)))
    pos = np.array([[1, 1], [2, 2]], np.int32)
    with pytest.raises(RuntimeError):  # five modes
        api.ptycho_iterate_modes(O, tc64(np.ones((5, 32, 32))), I, pos, 1)
    with pytest.raises(RuntimeError):  # batch x modes above 512
        api.ptycho_iterate_modes(O, tc64(np.ones((4, 32, 32))), I, pos, 1, batch=200)
