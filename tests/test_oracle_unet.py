"""Pins of the warm-start network oracle: every layer against brute force
or PyTorch's CPU convolutions, the transposition identity between the
strided and transposed convolutions, and finite differences of the whole
network.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet

W4 = (4, 6, 6, 8)


def _brute_conv3(x, W, b):
    n, H, Wd, ci = x.shape
    out = np.zeros((n, H, Wd, W.shape[2]))
    for i in range(n):
        for y in range(H):
            for xx in range(Wd):
                for ky in range(3):
                    for kx in range(3):
                        yy, xs = y + ky - 1, xx + kx - 1
                        if 0 <= yy < H and 0 <= xs < Wd:
                            out[i, y, xx] += x[i, yy, xs] @ W[ky * 3 + kx]
    return out + b


def test_conv3_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    W = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(unet.conv3(x, W, b), _brute_conv3(x, W, b), atol=1e-12)


def _torch_w(W, R):
    # W[tap][ci][co] -> torch [co][ci][ky][kx]
    taps, ci, co = W.shape
    return torch.tensor(W.reshape(R, R, ci, co).transpose(3, 2, 0, 1).copy())


def test_layers_match_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 8, 8, 3))
    t = torch.tensor(x.transpose(0, 3, 1, 2).copy())
    W3, W2, W1 = rng.standard_normal((9, 3, 5)), rng.standard_normal((4, 3, 5)), rng.standard_normal((1, 3, 5))
    b = rng.standard_normal(5)
    tb = torch.tensor(b)
    ref3 = F.conv2d(t, _torch_w(W3, 3), tb, padding=1).numpy().transpose(0, 2, 3, 1)
    ref2 = F.conv2d(t, _torch_w(W2, 2), tb, stride=2).numpy().transpose(0, 2, 3, 1)
    ref1 = F.conv2d(t, _torch_w(W1, 1), tb).numpy().transpose(0, 2, 3, 1)
    np.testing.assert_allclose(unet.conv3(x, W3, b), ref3, atol=1e-12)
    np.testing.assert_allclose(unet.conv_down(x, W2, b), ref2, atol=1e-12)
    np.testing.assert_allclose(unet.conv1(x, W1, b), ref1, atol=1e-12)
    # transposed convolution: torch weight layout [ci][co][ky][kx]
    Wu = rng.standard_normal((4, 3, 5))
    tw = torch.tensor(Wu.reshape(2, 2, 3, 5).transpose(2, 3, 0, 1).copy())
    refu = F.conv_transpose2d(t, tw, tb, stride=2).numpy().transpose(0, 2, 3, 1)
    np.testing.assert_allclose(unet.conv_up(x, Wu, b), refu, atol=1e-12)


def test_up_is_the_transpose_of_down():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 8, 8, 3))
    y = rng.standard_normal((1, 4, 4, 5))
    W = rng.standard_normal((4, 3, 5))
    Wt = W.transpose(0, 2, 1)
    lhs = np.sum(unet.conv_down(x, W, np.zeros(5)) * y)
    rhs = np.sum(x * unet.conv_up(y, Wt, np.zeros(3)))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_output_shape_and_relu():
    p = unet.init_params(W4, 0)
    x = np.random.default_rng(3).random((2, 16, 16, 1))
    out, acts = unet.forward(p, x, W4)
    assert out.shape == (2, 4, 4, 2)
    assert acts["cat"].shape == (2, 4, 4, 12)
    assert all((acts[k] >= 0).all() for k in acts if k not in ("x", "head", "cat"))


def test_network_gradient_matches_finite_differences():
    p = unet.init_params(W4, 5)
    for k in p:
        if k.endswith(".b"):
            p[k] = np.random.default_rng(len(k)).standard_normal(p[k].shape) * 0.1
    rng = np.random.default_rng(6)
    x = rng.random((2, 16, 16, 1))
    target = rng.standard_normal((2, 4, 4, 2))

    def loss(pp):
        out, _ = unet.forward(pp, x, W4)
        return unet.mse_loss(out, target)[0]

    out, acts = unet.forward(p, x, W4)
    _, dout = unet.mse_loss(out, target)
    g = unet.backward(p, acts, dout, W4)
    h = 1e-6
    rng2 = np.random.default_rng(7)
    for name in p:
        flat = p[name].ravel()
        idxs = rng2.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idxs:
            pp = {k: v.copy() for k, v in p.items()}
            pp[name].ravel()[i] += h
            lp = loss(pp)
            pp[name].ravel()[i] -= 2 * h
            lm = loss(pp)
            fd = (lp - lm) / (2 * h)
            an = g[name].ravel()[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i, fd, an)


def test_network_matches_torch_autograd():
    p = unet.init_params(W4, 8)
    rng = np.random.default_rng(9)
    x = rng.random((2, 16, 16, 1))
    target = rng.standard_normal((2, 4, 4, 2))
    out, acts = unet.forward(p, x, W4)
    L, dout = unet.mse_loss(out, target)
    g = unet.backward(p, acts, dout, W4)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}

    def conv(h, name, kind):
        W, b = tp[name + ".W"], tp[name + ".b"]
        taps, ci, co = W.shape
        if kind == "up":
            tw = W.reshape(2, 2, ci, co).permute(2, 3, 0, 1)
            return F.conv_transpose2d(h, tw, b, stride=2)
        R = {9: 3, 4: 2, 1: 1}[taps]
        tw = W.reshape(R, R, ci, co).permute(3, 2, 0, 1)
        return F.conv2d(h, tw, b, stride=2 if kind == "down" else 1, padding=1 if kind == "conv3" else 0)

    h = torch.tensor(x.transpose(0, 3, 1, 2).copy())
    saved = {}
    for name, kind, _, _ in unet.layer_specs(W4):
        if name == "u2a":
            h = torch.cat([h, saved["e2b"]], dim=1)
        h = conv(h, name, kind)
        if name != "head":
            h = torch.relu(h)
        saved[name] = h
    tl = ((h - torch.tensor(target.transpose(0, 3, 1, 2).copy())) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - L) < 1e-12
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-12)
