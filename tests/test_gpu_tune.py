"""Launch-shape variants: every variant reproduces the default results, and
the tuner picks and caches a variant per detector size."""
import json

import numpy as np
import pytest
import torch

from paper_2608_01746_amd import synth

from _cases import c64, soft_probe, tiny_scan

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api, tune
    return api, tune


def _run(api, O, P, I, pos, order):
    Og = torch.from_numpy(np.asarray(O, np.complex64)).to(DEV)
    Pg = torch.from_numpy(np.asarray(P, np.complex64)).to(DEV)
    e = api.ptycho_iterate(Og, Pg, torch.from_numpy(np.asarray(I, np.float32)).to(DEV), pos, 2, alg="rpie",
                           alpha=0.2, beta=0.3, batch=5, update_probe=True, order=order)
    loss, gO, gP = api.ptycho_grad(Og, Pg, torch.from_numpy(np.asarray(I, np.float32)).to(DEV), pos, "poisson",
                                   1e-6, 4)
    If = api.ptycho_forward(Og, Pg, pos, I.shape[-1])
    return [x.cpu().numpy() for x in (Og, Pg, e, loss, gO, gP, If)]


@pytest.mark.parametrize("Nd,Nw,M", [(16, 16, 48), (64, 48, 120), (192, 192, 260), (256, 256, 340)])
def test_variants_agree(mods, Nd, Nw, M):
    api, tune = mods
    O, P, pos, I = tiny_scan(M, Nw, Nd, 3, (M - Nw - 4) // 2, 2, seed=Nd)
    P = c64(soft_probe(P, 1))
    order = synth.random_orders(len(pos), 2, 0)
    res = []
    for v in range(8):  # row shape, column shape, three or four launches per mini-batch
        tune.set_variant(Nd, v)
        res.append(_run(api, np.ones_like(O), P, I, pos, order))
    tune.set_variant(Nd, 0)
    for r in res[1:]:
        for k, (a, b) in enumerate(zip(res[0], r)):
            if k in (2, 3):   # float64 sums whose partial grouping depends on the column shape
                np.testing.assert_allclose(a, b, rtol=1e-12)
            else:
                assert np.array_equal(a, b), k


def test_autotune_picks_and_caches(mods, tmp_path):
    api, tune = mods
    path = str(tmp_path / "tune.json")
    out = tune.autotune([64, 256], batch=8, reps=3, path=path)
    assert set(out) == {64, 256}
    for N, e in out.items():
        assert 0 <= e["variant"] <= 7
        assert len(e["times_us"]) == 8 and min(e["times_us"]) > 0
        # the default is kept unless another variant is at least 3 % faster
        t = e["times_us"]
        assert e["variant"] == 0 or t[e["variant"]] < 0.97 * t[0]
        assert tune.get_variant(N) == e["variant"]
    data = json.load(open(path))
    assert len(data) == 2
    # cached: applied without timing
    tune.set_variant(64, 0)
    again = tune.autotune([64], batch=8, reps=3, path=path)
    assert again[64]["variant"] == out[64]["variant"] == tune.get_variant(64)
    tune.set_variant(64, 0)
    tune.set_variant(256, 0)
