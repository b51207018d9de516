"""What the learned warm start gains over the method without it.

The U-Net is trained on the GPU by the library's own forward, backward and
Adam kernels on patterns simulated by the library (forward model, detector
exposures, MNF fusion), with window phases labelled relative to each
window's mean phase; its predictions are stitched with the windows' phases
aligned, and the start is judged by object NRMSE against the ground truth
on unseen objects.  On MNF-fused noisy patterns the plain iterations
from a flat start stall at the floor the data allow; the network's stitched
start lies below that floor before any iteration."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import warmstart as ws
    S = ws.setup()
    tr = ws.simulate(S, range(5000, 5200), "fused", DEV, relative=True)
    params = ws.init_params(ws.WIDTHS, 0, DEV)
    steps = 2000
    info = ws.train(S, tr, params, steps=steps, seed=0)
    del tr
    torch.cuda.empty_cache()
    assert info["steps"] == steps
    return ws, S, params, info


def test_training_reduces_the_loss(trained):
    ws, S, params, info = trained
    h = info["history"]
    assert np.isfinite(h[-1][1])
    assert h[-1][1] < 0.9 * h[0][1], h
    assert torch.isfinite(params).all()


def test_warm_start_beats_plain_iterations_on_fused_data(trained):
    ws, S, params, _ = trained
    te = ws.simulate(S, range(9000, 9003), "fused", DEV)
    res = ws.time_to_threshold(S, te, params, tau=1e-2, max_plain=50, max_warm=5, sync=True)
    flat = np.median([r["plain_curve"][0] for r in res])
    plain50 = np.median([r["plain_curve"][-1] for r in res])
    plain_best = np.median([min(r["plain_curve"]) for r in res])
    warm0 = np.median([r["warm_curve"][0] for r in res])
    print(f"flat {flat:.4f} plain@50 {plain50:.4f} plain best {plain_best:.4f} warm start {warm0:.4f}")
    # the stitched network prediction is closer to the truth than 50 plain
    # iterations get, and much closer than the flat start
    assert warm0 < plain50
    assert warm0 < 0.6 * flat
    for r in res:
        assert r["t_start"] > 0 and r["t_iter"] > 0


def test_warm_start_on_noise_free_data_is_a_better_start(trained):
    ws, S, params, _ = trained
    te = ws.simulate(S, range(9000, 9003), "clean", DEV)
    res = ws.time_to_threshold(S, te, params, tau=1e-2, max_plain=80, max_warm=80, sync=True)
    print("noise-free: " + "; ".join(f"start {r['warm_curve'][0]:.4f} flat {r['plain_curve'][0]:.4f} "
                                      f"n_warm {r['n_warm']} n_plain {r['n_plain']}" for r in res))
    for r in res:
        # a closer start than flat, and the iterations still converge from it.
        # After this short training (128 k samples) the start's NRMSE, relative
        # to the flat start's, measured 0.55-0.79 over runs that differ only in
        # float summation order and kernel versions (starts 0.21-0.30 against a
        # flat 0.38-0.41), so the bound is 0.85.  Such a start does not reach
        # 1e-2 sooner than the flat one (40-50 against 17-37 iterations in one
        # run: the short-trained network's error converges slowly); the full
        # 480 s training of the benchmark (start 0.13-0.14) does, in median
        # (22.5 against 32 iterations), which the benchmark reports
        assert r["warm_curve"][0] < 0.85 * r["plain_curve"][0]
        assert r["n_warm"] is not None
