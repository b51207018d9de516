"""Many scans of uneven sizes in one call (ptycho_iterate_many): parity with
the float64 oracle per scan, bitwise agreement with one-scan calls, and the
graph-captured replay against direct launches."""
import numpy as np
import pytest
import torch

from oracle import ptycho
from paper_2608_01746_amd import synth, tune

from _cases import c64, f32, soft_probe, tiny_scan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def tc64(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.complex64))).to(DEV)


def tf32(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(DEV)


# (Nd, Nw, M, n_side, step) per scan: uneven sizes and position counts
SPECS = [(16, 16, 48, 5, 6), (64, 48, 120, 3, 30), (32, 32, 72, 4, 10), (64, 64, 140, 4, 24),
         (128, 128, 200, 2, 50), (32, 24, 50, 2, 20)]


def _scans(n_iter, seed=0):
    out = []
    for i, (Nd, Nw, M, n, step) in enumerate(SPECS):
        O, P, pos, I = tiny_scan(M, Nw, Nd, n, step, 2, seed=seed + 31 * i, jitter=1)
        out.append(dict(O0=c64(np.ones_like(O)), P0=c64(soft_probe(P, i) * np.exp(0.1j)), pos=pos, I=I,
                        order=synth.random_orders(len(pos), n_iter, seed + i)))
    return out


def _run_many(api, scans, n_iter, graph, **kw):
    ts = [dict(O=tc64(s["O0"]), P=tc64(s["P0"]), I=tf32(s["I"]), pos=s["pos"], order=s["order"]) for s in scans]
    errs = api.ptycho_iterate_many(ts, n_iter, graph=graph, **kw)
    torch.cuda.synchronize()
    return [(t["O"].cpu().numpy(), t["P"].cpu().numpy(), e.cpu().numpy()) for t, e in zip(ts, errs)]


KW = dict(alg="rpie", alpha=0.2, beta=0.3, batch=4, update_probe=True, probe_start_iter=1)


def test_many_scans_match_oracle(api):
    scans = _scans(2)
    res = _run_many(api, scans, 2, graph=False, **KW)
    prm = ptycho.PtychoParams("rpie", 0.2, 0.3, 4, True, 1)
    for s, (Og, Pg, eg) in zip(scans, res):
        Or, Pr, er = ptycho.iterate(s["O0"], s["P0"], s["I"], s["pos"], 2, prm, s["order"])
        assert rel(Og, Or) < 1e-5
        assert rel(Pg, Pr) < 1e-5
        np.testing.assert_allclose(eg, er, rtol=1e-5)


def test_many_scans_equal_single_scan_calls(api):
    scans = _scans(3, seed=5)
    res = _run_many(api, scans, 3, graph=False, **KW)
    for s, (Og, Pg, eg) in zip(scans, res):
        O, P = tc64(s["O0"]), tc64(s["P0"])
        e = api.ptycho_iterate(O, P, tf32(s["I"]), s["pos"], 3, order=s["order"], **KW)
        assert np.array_equal(O.cpu().numpy(), Og)
        assert np.array_equal(P.cpu().numpy(), Pg)
        assert np.array_equal(e.cpu().numpy(), eg)


def test_graph_replay_equals_direct_launches(api):
    scans = _scans(3, seed=9)
    a = _run_many(api, scans, 3, graph=False, **KW)
    b = _run_many(api, scans, 3, graph=True, **KW)
    # a second graph call (re-capture, previous graph released)
    c = _run_many(api, scans, 3, graph=True, **KW)
    for x, y, z in zip(a, b, c):
        for u, v, w in zip(x, y, z):
            assert np.array_equal(u, v) and np.array_equal(u, w)


def test_cached_multi_class_graph_replays_equal_direct_launches(api):
    # four size classes, each on a stream of its own inside the captured
    # graph: the same tensors (reset between calls) give the cached graph on
    # every call after the first; eager work between the replays; every
    # replay equal to the direct launches bit for bit
    scans = _scans(3, seed=4)
    want = _run_many(api, scans, 3, graph=False, **KW)
    ts = [dict(O=tc64(s["O0"]), P=tc64(s["P0"]), I=tf32(s["I"]), pos=s["pos"], order=s["order"]) for s in scans]
    assert len({s["I"].shape[-1] for s in scans}) >= 4
    for rep in range(4):
        for t, s in zip(ts, scans):
            t["O"].copy_(torch.from_numpy(s["O0"]).to(DEV))
            t["P"].copy_(torch.from_numpy(s["P0"]).to(DEV))
        errs = api.ptycho_iterate_many(ts, 3, graph=True, **KW)
        junk = torch.randn(1 << 16, device=DEV).sum()  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for (Ow, Pw, ew), t, e in zip(want, ts, errs):
            assert np.array_equal(t["O"].cpu().numpy(), Ow), rep
            assert np.array_equal(t["P"].cpu().numpy(), Pw), rep
            assert np.array_equal(e.cpu().numpy(), ew), rep


def test_single_scan_graph_matches_direct(api):
    O, P, pos, I = tiny_scan(300, 128, 128, 4, 50, 2, seed=6)
    order = synth.random_orders(len(pos), 4, 1)
    out = []
    for graph in (False, True):
        Og, Pg = tc64(np.ones_like(O)), tc64(P * 0.8)
        e = api.ptycho_iterate(Og, Pg, tf32(I), pos, 4, alg="rpie", batch=5, update_probe=True, order=order,
                               graph=graph)
        out.append((Og.cpu(), Pg.cpu(), e.cpu()))
    for u, v in zip(*out):
        assert torch.equal(u, v)


def test_multiscan_workload_sample_full_size(api):
    # three scans of the uneven-size workload at their real sizes, one iteration
    chosen = []
    seen = set()
    for w in synth.multiscan_workloads(64):
        if w.Nd not in seen and w.J <= 260:
            seen.add(w.Nd)
            chosen.append(w)
        if len(chosen) == 3:
            break
    assert len(chosen) == 3
    scans = []
    for w in chosen:
        O = w.object()
        P = c64(soft_probe(w.probe(), 3))
        I = f32(ptycho.forward_intensity(O, P, w.pos, w.Nd))
        scans.append(dict(O0=c64(np.ones_like(O)), P0=P, pos=w.pos, I=I, order=synth.random_orders(w.J, 1, w.seed)))
    res = _run_many(api, scans, 1, graph=True, alg="rpie", alpha=0.1, beta=0.1, batch=32, update_probe=True)
    prm = ptycho.PtychoParams("rpie", 0.1, 0.1, 32, True)
    for s, (Og, Pg, eg) in zip(scans, res):
        Or, Pr, er = ptycho.iterate(s["O0"], s["P0"], s["I"], s["pos"], 1, prm, s["order"])
        assert rel(Og, Or) < 1e-5
        assert rel(Pg, Pr) < 1e-5
        assert abs(eg[0] - er[0]) <= 1e-5 * er[0]


def test_many_rejects_bad_scan(api):
    s = _scans(1)
    ts = [dict(O=tc64(x["O0"]), P=tc64(x["P0"]), I=tf32(x["I"]), pos=x["pos"]) for x in s]
    ts[2]["pos"] = np.array(ts[2]["pos"]) + 1000
    with pytest.raises(api.MnfError, match="scan 2"):
        api.ptycho_iterate_many(ts, 1)


def test_cached_graph_replays_and_recaptures(api):
    # the same call three times on the same buffers (the second and third
    # replay the cached graph), then another order (a new capture); every
    # result equals direct launches, and each call's errors reach its own
    # output tensor
    O, P, pos, I = tiny_scan(300, 128, 128, 4, 50, 2, seed=7)
    It = tf32(I)
    kw = dict(alg="rpie", batch=5, update_probe=True, probe_start_iter=1)
    Og, Pg = tc64(np.ones_like(O)), tc64(P * 0.8)
    for seed in (1, 1, 1, 2):
        order = synth.random_orders(len(pos), 3, seed)
        Og.copy_(tc64(np.ones_like(O)))
        Pg.copy_(tc64(P * 0.8))
        eg = api.ptycho_iterate(Og, Pg, It, pos, 3, order=order, graph=True, **kw)
        Od, Pd = tc64(np.ones_like(O)), tc64(P * 0.8)
        ed = api.ptycho_iterate(Od, Pd, It, pos, 3, order=order, **kw)
        assert torch.equal(Og, Od) and torch.equal(Pg, Pd) and torch.equal(eg, ed), seed


@pytest.mark.parametrize("Nd,Nw,M,B,n_side,step", [(256, 256, 520, 8, 3, 120), (64, 48, 300, 7, 6, 40),
                                                   (128, 100, 400, 5, 5, 60), (512, 512, 900, 4, 2, 300)])
def test_three_launch_path_equals_four_launch_path(api, Nd, Nw, M, B, n_side, step):
    # one scan at integer positions takes the fused object-update / exit-wave
    # pass (three launches per mini-batch); launch-shape bit 2 keeps four.
    # The sums run in the same order, so the results are bit-identical,
    # including ragged last mini-batches, probe updates from iteration 1 and
    # iteration boundaries inside the fused pass
    O, P, pos, I = tiny_scan(M, Nw, Nd, n_side, step, 2, seed=Nd + 1, jitter=1)
    order = synth.random_orders(len(pos), 3, 4)
    res = []
    for v in (0, 4):
        tune.set_variant(Nd, v)
        Og, Pg = tc64(np.ones_like(O)), tc64(P * 0.9)
        e = api.ptycho_iterate(Og, Pg, tf32(I), pos, 3, alg="rpie", alpha=0.3, beta=0.2, batch=B,
                               update_probe=True, probe_start_iter=1, order=order)
        res.append((Og.cpu(), Pg.cpu(), e.cpu()))
    tune.set_variant(Nd, 0)
    for a, b in zip(*res):
        assert torch.equal(a, b)


@pytest.mark.parametrize("alg,Nd,Nw,M,n_side,step,upd", [("epie", 64, 64, 192, 6, 20, True),
                                                          ("rpie", 64, 48, 160, 5, 20, True),
                                                          ("rpie", 32, 32, 96, 5, 12, False),
                                                          ("epie", 16, 12, 48, 5, 6, True)])
def test_single_workgroup_run_equals_multi_pass(api, alg, Nd, Nw, M, n_side, step, upd):
    # mini-batches of one on patterns of at most 64^2 run as a whole in one
    # workgroup; launch-shape bit 3 keeps the four passes per position.  The
    # two agree to float32 rounding (bit for bit at 16^2; at 32^2 and 64^2 the
    # transforms round a few values differently) and both match the float64
    # oracle at the one-iteration bar.
    O, P, pos, I = tiny_scan(M, Nw, Nd, n_side, step, 2, seed=Nd + Nw, jitter=1)
    order = synth.random_orders(len(pos), 3, 8)
    P0 = c64(soft_probe(P, 3) * np.exp(0.2j))
    res = []
    for v in (0, 8):
        tune.set_variant(Nd, v)
        Og, Pg = tc64(np.ones_like(O)), tc64(P0)
        e = api.ptycho_iterate(Og, Pg, tf32(I), pos, 3, alg=alg, alpha=0.3, beta=0.3, batch=1,
                               update_probe=upd, probe_start_iter=1, order=order)
        res.append((Og.cpu(), Pg.cpu(), e.cpu()))
    tune.set_variant(Nd, 0)
    (Oa, Pa, ea), (Ob, Pb, eb) = res
    if Nd == 16:
        assert torch.equal(Oa, Ob) and torch.equal(Pa, Pb)
    assert rel(Oa.numpy(), Ob.numpy()) < 1e-5 and rel(Pa.numpy(), Pb.numpy()) < 1e-5
    torch.testing.assert_close(ea, eb, rtol=1e-6, atol=0)
    Or, Pr, er = ptycho.iterate(c64(np.ones_like(O)), P0, I, pos, 3, ptycho.PtychoParams(alg, 0.3, 0.3, 1, upd, 1),
                                order)
    assert rel(Oa.numpy(), Or) < 1e-5 and rel(Pa.numpy(), Pr) < 1e-5
    np.testing.assert_allclose(ea.numpy(), er, rtol=1e-5)


def test_single_workgroup_run_reports_errors_and_graph(api):
    # err_out and graph capture through the single-workgroup path
    O, P, pos, I = tiny_scan(96, 32, 32, 5, 12, 2, seed=3)
    order = synth.random_orders(len(pos), 4, 2)
    out = []
    for graph in (False, True, True):
        Og, Pg = tc64(np.ones_like(O)), tc64(P * 0.9)
        e = api.ptycho_iterate(Og, Pg, tf32(I), pos, 4, alg="epie", batch=1, update_probe=True, order=order,
                               graph=graph)
        out.append((Og.cpu(), Pg.cpu(), e.cpu()))
    for o in out[1:]:
        assert all(torch.equal(a, b) for a, b in zip(out[0], o))
    assert torch.all(out[0][2][1:] < out[0][2][:-1])  # the error falls on noiseless data
