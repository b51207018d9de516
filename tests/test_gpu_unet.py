"""BF16 MFMA convolution kernels and the warm-start network against the
float64 oracle.  Inputs and weights are rounded to bf16 first, so every
product is exact and float32 accumulation is the only difference for a
single layer (relative error <= 1e-5 for float32 outputs; bf16 outputs are
compared to within one bf16 rounding).  Through the whole network the
activations are stored in bf16 between layers, which bounds agreement at a
few 1e-3 relative."""
import numpy as np
import pytest
import torch

from oracle import unet

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TAPS = {"conv3": 9, "down": 4, "up": 4, "conv1": 1}
FWD = {"conv3": unet.conv3, "down": unet.conv_down, "up": unet.conv_up, "conv1": unet.conv1}
BWD = {"conv3": unet.conv3_backward, "down": unet.conv_down_backward, "up": unet.conv_up_backward,
       "conv1": unet.conv1_backward}


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_01746_amd import api as _api
    return _api


def bf(a):
    """Round to bf16 (as a torch tensor on the GPU) and return (tensor, float64 values)."""
    t = torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.to(DEV), t.to(torch.float64).numpy()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


CASES = [("conv3", 2, 16, 1, 32), ("conv3", 2, 16, 48, 72), ("conv3", 1, 24, 64, 16), ("down", 2, 16, 32, 64),
         ("down", 3, 8, 24, 40), ("up", 2, 8, 64, 32), ("up", 1, 4, 16, 24), ("conv1", 2, 16, 128, 2),
         ("conv1", 1, 8, 40, 72)]


@pytest.mark.parametrize("mode,n,H,Ci,Co", CASES)
def test_conv_forward(api, mode, n, H, Ci, Co):
    rng = np.random.default_rng(Ci * Co + H)
    xt, x = bf(rng.standard_normal((n, H, H, Ci)))
    Wt, W = bf(rng.standard_normal((TAPS[mode], Ci, Co)) / np.sqrt(Ci * TAPS[mode]))
    b = rng.standard_normal(Co)
    y = api.conv2d(mode, xt, Wt.float(), torch.from_numpy(b.astype(np.float32)).to(DEV), relu=False)
    ref = FWD[mode](x, W, b.astype(np.float32).astype(np.float64))
    assert rel(y.cpu().numpy(), ref) < 1e-5
    yr = api.conv2d(mode, xt, Wt.float(), None, relu=True)
    np.testing.assert_allclose(yr.cpu().numpy(), np.maximum(FWD[mode](x, W, 0.0), 0), rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("mode,n,H,Ci,Co", CASES)
@pytest.mark.parametrize("masked", [False, True])
def test_conv_gradients(api, mode, n, H, Ci, Co, masked):
    rng = np.random.default_rng(Ci + 7 * Co + H)
    xt, x = bf(rng.standard_normal((n, H, H, Ci)))
    Wt, W = bf(rng.standard_normal((TAPS[mode], Ci, Co)) / np.sqrt(Ci * TAPS[mode]))
    Ho = {"conv3": H, "down": H // 2, "up": 2 * H, "conv1": H}[mode]
    dyt, dy = bf(rng.standard_normal((n, Ho, Ho, Co)))
    actt, act = bf(rng.standard_normal((n, Ho, Ho, Co)))
    dz = dy * (act > 0) if masked else dy
    dx, dW, db = api.conv2d_grad(mode, xt, Wt.float(), dyt, actt if masked else None)
    rdx, rdW, rdb = BWD[mode](x, W, dz)
    assert rel(dW.cpu().numpy(), rdW) < 1e-5
    assert rel(db.cpu().numpy(), rdb) < 1e-5
    # dx is stored in bf16: within one rounding (2^-8 relative) of the float64 value
    d = dx.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(d - rdx) <= 2.0 ** -8 * np.abs(rdx) + 1e-6 * np.abs(rdx).max())


# 3x3 shapes that take the direct tiled kernel (input channels a multiple of 32,
# 64- or 32-pixel-wide tiles), forward and masked input gradient; a partial
# output-channel tile in the last case
TILED = [("conv3", 2, 64, 32, 64), ("conv3", 2, 32, 64, 96), ("conv3", 1, 128, 96, 40), ("conv3", 2, 64, 32, 32),
         ("conv3", 1, 64, 64, 24)]


@pytest.mark.parametrize("mode,n,H,Ci,Co", TILED)
def test_tiled_conv3_forward(api, mode, n, H, Ci, Co):
    test_conv_forward(api, mode, n, H, Ci, Co)


@pytest.mark.parametrize("mode,n,H,Ci,Co", TILED[:2] + TILED[3:])
def test_tiled_conv3_gradients(api, mode, n, H, Ci, Co):
    test_conv_gradients(api, mode, n, H, Ci, Co, True)


# 3x3 weight gradients through the all-taps tiled kernel: 32- and 64-channel
# output tiles, 64-pixel rows and pairs of 32-pixel rows, two input-channel
# tiles (the bias from the first only), masked and unmasked
WGRAD_TILED = [("conv3", 1, 64, 32, 32), ("conv3", 1, 32, 32, 64), ("conv3", 2, 32, 64, 96),
               ("conv3", 2, 128, 64, 32), ("conv3", 1, 64, 96, 128),
               # 2x2 stride-2 layers through the all-taps kernel (output 64 or 32 wide)
               ("down", 1, 128, 32, 64), ("down", 2, 64, 64, 32), ("down", 1, 128, 64, 96)]


@pytest.mark.parametrize("mode,n,H,Ci,Co", WGRAD_TILED)
@pytest.mark.parametrize("masked", [False, True])
def test_tiled_weight_gradients(api, mode, n, H, Ci, Co, masked):
    test_conv_gradients(api, mode, n, H, Ci, Co, masked)


# large layers (the full network's sizes at batch 4)
LARGE = [("down", 4, 256, 32, 256), ("conv1", 4, 128, 64, 256), ("conv3", 4, 128, 32, 256)]


@pytest.mark.parametrize("mode,n,H,Ci,Co", LARGE)
def test_large_layer_forward(api, mode, n, H, Ci, Co):
    test_conv_forward(api, mode, n, H, Ci, Co)


@pytest.mark.parametrize("mode,n,H,Ci,Co", [("conv1", 4, 128, 256, 64), ("conv3", 4, 128, 256, 8)])
def test_large_layer_gradients(api, mode, n, H, Ci, Co):
    test_conv_gradients(api, mode, n, H, Ci, Co, True)


WID = (8, 16, 16, 24)


def _net_problem(H=32, n=3, seed=0):
    rng = np.random.default_rng(seed)
    p = unet.init_params(WID, seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
        p[k] = torch.from_numpy(p[k].astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    I = rng.gamma(0.5, 50.0, size=(n, H, H))
    scale = 1.0 / np.log1p(I.max())
    target = rng.standard_normal((n, H // 4, H // 4, 2)) * 0.5
    return p, I, scale, target


def _flat(p):
    names = [nm for L in unet.layer_specs(WID) for nm in (L[0] + ".W", L[0] + ".b")]
    return np.concatenate([p[k].ravel() for k in names]), names


def test_network_forward_and_gradient(api):
    p, I, scale, target = _net_problem()
    flat, names = _flat(p)
    assert flat.size == api.unet_param_count(32, WID)
    params = torch.from_numpy(flat.astype(np.float32)).to(DEV)
    It = torch.from_numpy(I.astype(np.float32)).to(DEV)
    out = api.unet_forward(params, It, scale, 32, WID).cpu().numpy()
    x = np.log1p(I.astype(np.float32).astype(np.float64)) * np.float32(scale)
    x = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()[..., None]
    ref, acts = unet.forward(p, x, WID)
    assert rel(out, ref) < 2e-2
    grads = torch.zeros_like(params)
    tt = torch.from_numpy(target.astype(np.float32)).to(DEV)
    loss = api.unet_train_step(params, None, None, 1, 0.0, It, scale, tt, 32, WID, grads=grads)
    L, dout = unet.mse_loss(ref, target)
    assert abs(loss.item() - L) < 2e-2 * L
    g = unet.backward(p, acts, dout, WID)
    gref, _ = _flat(g)
    gg = grads.cpu().numpy()
    assert rel(gg, gref) < 3e-2
    # every layer's weight gradient points the same way
    off = 0
    for k in names:
        n_ = g[k].size
        a, r = gg[off:off + n_], g[k].ravel()
        off += n_
        if np.linalg.norm(r) > 0:
            assert a @ r / (np.linalg.norm(a) * np.linalg.norm(r)) > 0.99, k


def test_adam_steps_reduce_the_loss(api):
    p, I, scale, target = _net_problem(seed=1)
    flat, _ = _flat(p)
    params = torch.from_numpy(flat.astype(np.float32)).to(DEV)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    It = torch.from_numpy(I.astype(np.float32)).to(DEV)
    tt = torch.from_numpy(target.astype(np.float32)).to(DEV)
    losses = [api.unet_train_step(params, m, v, s, 3e-3, It, scale, tt, 32, WID).item() for s in range(1, 31)]
    assert losses[-1] < 0.5 * losses[0]


def test_full_size_network_forward_matches_oracle(api):
    # the warm-start network at its real size (256^2 input, widths 32..256),
    # one sample, bf16-representable weights and input: only the float32
    # accumulation order and the bf16 rounding of activations between layers
    # differ from the float64 oracle (the same bar as the small network)
    W = (32, 64, 128, 256)
    rng = np.random.default_rng(7)
    p = unet.init_params(W, 11)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.05
        p[k] = torch.from_numpy(p[k].astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    names = [nm for L in unet.layer_specs(W) for nm in (L[0] + ".W", L[0] + ".b")]
    flat = np.concatenate([p[k].ravel() for k in names])
    assert flat.size == api.unet_param_count(256, W)
    I = rng.gamma(0.5, 50.0, size=(1, 256, 256))
    scale = 1.0 / np.log1p(I.max())
    out = api.unet_forward(torch.from_numpy(flat.astype(np.float32)).to(DEV),
                           torch.from_numpy(I.astype(np.float32)).to(DEV), scale, 256, W).cpu().numpy()
    x = np.log1p(I.astype(np.float32).astype(np.float64)) * np.float32(scale)
    x = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()[..., None]
    ref, _ = unet.forward(p, x, W)
    assert out.shape == ref.shape == (1, 64, 64, 2)
    assert rel(out, ref) < 2e-2


def test_full_size_network_runs(api):
    # the warm-start network at its real size: 256^2 input, widths 32..256
    W = (32, 64, 128, 256)
    n_par = api.unet_param_count(256, W)
    rng = np.random.default_rng(3)
    params = torch.from_numpy((rng.standard_normal(n_par) * 0.02).astype(np.float32)).to(DEV)
    I = torch.from_numpy(rng.gamma(0.5, 50.0, size=(4, 256, 256)).astype(np.float32)).to(DEV)
    out = api.unet_forward(params, I, 0.1, 256, W)
    assert out.shape == (4, 64, 64, 2) and torch.isfinite(out).all()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = api.unet_train_step(params, m, v, 1, 1e-3, I, 0.1, torch.zeros_like(out), 256, W)
    assert np.isfinite(loss.item())
