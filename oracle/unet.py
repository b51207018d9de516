"""Oracle: the warm-start network, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A four-level U-Net maps a log-scaled fused pattern [n][H][H][1] (channels
last) to the amplitude and phase of the illuminated object patch
[n][H/4][H/4][2]:

  encoder level l (l = 0..3, size H / 2^l, width c_l):
      two 3x3 convolutions (stride 1, zero padding 1) + ReLU
  between levels: 2x2 convolution with stride 2 + ReLU
  decoder: 2x2 transposed convolution with stride 2 from level 3 to level 2
      (+ ReLU), concatenated with the level-2 encoder output (up first),
      two 3x3 convolutions (width c_2) + ReLU, 1x1 convolution to 2 outputs.

Weights are stored tap-major, W[tap][c_in][c_out] with tap = ky * R + kx,
plus a bias per output channel.  For the transposed convolution the tap is
the output pixel's parity: out[2y+dy, 2x+dx] = sum_ci in[y, x, ci] W[2dy+dx][ci].
The loss is the mean squared error over every output element.  Everything
here is written from these definitions; the tests check it against brute
force, the transposition identity between the strided and transposed
convolutions, finite differences and PyTorch's CPU convolutions.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

Params = Dict[str, np.ndarray]


# ------------------------------------------------------------------ layers

def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 convolution, stride 1, zero padding 1: x [n,H,W,Ci], W [9,Ci,Co]."""
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((n, H, Wd, W.shape[2]))
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[ky * 3 + kx]
    return out + b


def conv3_backward(x, W, dy):
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            win = xp[:, ky:ky + H, kx:kx + Wd, :]
            dW[ky * 3 + kx] = np.einsum("nhwc,nhwo->co", win, dy)
            dxp[:, ky:ky + H, kx:kx + Wd, :] += dy @ W[ky * 3 + kx].T
    return dxp[:, 1:-1, 1:-1, :], dW, dy.sum(axis=(0, 1, 2))


def conv_down(x, W, b):
    """2x2 convolution with stride 2: out[y, x] = sum_{dy,dx} in[2y+dy, 2x+dx] W[2dy+dx]."""
    out = 0.0
    for dy in range(2):
        for dx in range(2):
            out = out + x[:, dy::2, dx::2, :] @ W[2 * dy + dx]
    return out + b


def conv_down_backward(x, W, dy_):
    dx_ = np.zeros_like(x)
    dW = np.zeros_like(W)
    for dy in range(2):
        for dx in range(2):
            dW[2 * dy + dx] = np.einsum("nhwc,nhwo->co", x[:, dy::2, dx::2, :], dy_)
            dx_[:, dy::2, dx::2, :] = dy_ @ W[2 * dy + dx].T
    return dx_, dW, dy_.sum(axis=(0, 1, 2))


def conv_up(x, W, b):
    """2x2 transposed convolution with stride 2: out[2y+dy, 2x+dx] = in[y, x] W[2dy+dx]."""
    n, H, Wd, _ = x.shape
    out = np.zeros((n, 2 * H, 2 * Wd, W.shape[2]))
    for dy in range(2):
        for dx in range(2):
            out[:, dy::2, dx::2, :] = x @ W[2 * dy + dx]
    return out + b


def conv_up_backward(x, W, dy_):
    dx_ = np.zeros_like(x)
    dW = np.zeros_like(W)
    for dy in range(2):
        for dx in range(2):
            g = dy_[:, dy::2, dx::2, :]
            dW[2 * dy + dx] = np.einsum("nhwc,nhwo->co", x, g)
            dx_ += g @ W[2 * dy + dx].T
    return dx_, dW, dy_.sum(axis=(0, 1, 2))


def conv1(x, W, b):
    return x @ W[0] + b


def conv1_backward(x, W, dy):
    return dy @ W[0].T, np.einsum("nhwc,nhwo->co", x, dy)[None], dy.sum(axis=(0, 1, 2))


def relu(z):
    return np.maximum(z, 0.0)


# ----------------------------------------------------------------- network

def layer_specs(widths: Sequence[int]) -> List[Tuple[str, str, int, int]]:
    """(name, kind, c_in, c_out) in execution order."""
    c0, c1, c2, c3 = widths
    return [
        ("e0a", "conv3", 1, c0), ("e0b", "conv3", c0, c0), ("d0", "down", c0, c1),
        ("e1a", "conv3", c1, c1), ("e1b", "conv3", c1, c1), ("d1", "down", c1, c2),
        ("e2a", "conv3", c2, c2), ("e2b", "conv3", c2, c2), ("d2", "down", c2, c3),
        ("e3a", "conv3", c3, c3), ("e3b", "conv3", c3, c3), ("up", "up", c3, c2),
        ("u2a", "conv3", 2 * c2, c2), ("u2b", "conv3", c2, c2), ("head", "conv1", c2, 2),
    ]


TAPS = {"conv3": 9, "down": 4, "up": 4, "conv1": 1}


def init_params(widths: Sequence[int], seed: int) -> Params:
    """He-normal weights (fan-in = taps x c_in), zero biases."""
    rng = np.random.default_rng(seed)
    p: Params = {}
    for name, kind, ci, co in layer_specs(widths):
        taps = TAPS[kind]
        fan_in = taps * ci if kind != "up" else ci
        p[name + ".W"] = rng.standard_normal((taps, ci, co)) * np.sqrt(2.0 / fan_in)
        p[name + ".b"] = np.zeros(co)
    return p


_FWD = {"conv3": conv3, "down": conv_down, "up": conv_up, "conv1": conv1}
_BWD = {"conv3": conv3_backward, "down": conv_down_backward, "up": conv_up_backward, "conv1": conv1_backward}


def forward(p: Params, x: np.ndarray, widths: Sequence[int]):
    """Output [n][H/4][H/4][2] and the activations needed by backward."""
    acts = {"x": x}
    h = x
    for name, kind, _, _ in layer_specs(widths):
        if name == "u2a":
            h = np.concatenate([h, acts["e2b"]], axis=-1)
            acts["cat"] = h
        z = _FWD[kind](h, p[name + ".W"], p[name + ".b"])
        h = z if name == "head" else relu(z)
        acts[name] = h
    return h, acts


def backward(p: Params, acts, dout: np.ndarray, widths: Sequence[int]) -> Params:
    """Gradients of sum(dout * output) with respect to every parameter."""
    specs = layer_specs(widths)
    inputs = {}
    prev = "x"
    for name, _, _, _ in specs:
        inputs[name] = "cat" if name == "u2a" else prev
        prev = name
    grads: Params = {}
    g = {"head": dout}
    for name, kind, ci, co in reversed(specs):
        dh = g[name]
        dz = dh if name == "head" else dh * (acts[name] > 0)
        dx, dW, db = _BWD[kind](acts[inputs[name]], p[name + ".W"], dz)
        grads[name + ".W"] = dW
        grads[name + ".b"] = db
        if name == "u2a":
            # the concatenation: up first, then the level-2 encoder output (skip)
            c = acts["up"].shape[-1]
            g["up"] = dx[..., :c]
            g["e2b"] = dx[..., c:]
        elif inputs[name] != "x":
            g[inputs[name]] = g.get(inputs[name], 0.0) + dx
    return grads


def mse_loss(out: np.ndarray, target: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean squared error and its gradient with respect to out."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def log_input(I: np.ndarray, I_max: float) -> np.ndarray:
    """Network input: ln(1 + max(I, 0)) / ln(1 + I_max), channels last."""
    return (np.log1p(np.maximum(I, 0.0)) / np.log1p(I_max))[..., None]
