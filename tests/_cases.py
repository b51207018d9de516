"""Seeded test inputs built from the synthetic generators and the CPU oracle
(never from the HIP path)."""
from __future__ import annotations

import functools

import numpy as np

from oracle import mnf, ptycho
from paper_2608_01746_amd import synth


def c64(a: np.ndarray) -> np.ndarray:
    """Round to complex64 and back, so both sides start from identical values."""
    return np.asarray(a, np.complex64).astype(np.complex128)


def f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, np.float32).astype(np.float64)


def soft_probe(P: np.ndarray, seed: int) -> np.ndarray:
    """Probe with a smoothly varying modulus (so rPIE's alpha/beta matter)."""
    rng = np.random.default_rng(seed)
    n = P.shape[0]
    y, x = np.mgrid[0:n, 0:n] / n
    return P * (0.4 + 0.6 * (0.5 + 0.5 * np.cos(2 * np.pi * (y + 0.3 * x) + rng.uniform(0, 6))))


def fuse_params(w: synth.Workload, quantise: bool = True) -> mnf.FuseParams:
    d = synth.default_deltas(w.levels, w.sigma_read) if quantise else ()
    return mnf.FuseParams(levels=w.levels, sat=float(w.sat), delta=d)


@functools.lru_cache(maxsize=None)
def small_case(quantise: bool = True):
    """The small workload: 192^2 object, 64^2 probe, 100 positions, 3 exposures,
    4-level fusion.  Returns dict with truth, raw stack and oracle-fused I."""
    w = synth.small_workload()
    O = w.object()
    P = w.probe()
    clean = ptycho.forward_intensity(O, P, w.pos, w.Nd)
    s = synth.flux_scale(clean.max(), w.sat)
    raw = synth.expose(clean, w.t, w.sat, w.sigma_read, seed=101, scale=s)
    I = mnf.fuse(raw, w.t, fuse_params(w, quantise))
    return dict(w=w, O=O, P=P, scale=s, raw=raw, I=f32(I), clean=clean)


def tiny_scan(M, Nw, Nd, n_side, step, offset, seed, jitter=0):
    """Noiseless small scan: truth, probe, positions and detector-centred I."""
    O = synth.make_object(M, seed)
    P = synth.make_probe(Nw, Nw / 4.0, np.pi)
    pos = synth.raster_positions(n_side, step, offset, jitter=jitter, seed=seed)
    assert pos.min() >= 0 and pos.max() + Nw <= M
    I = ptycho.forward_intensity(O, P, pos, Nd)
    return O, P, pos, f32(I)


def oracle_spread(run, I, trials=2, seed=0):
    """How far float32-level rounding of the intensity input alone moves the
    float64 oracle: max relative deviation of each output of run(I) when I is
    perturbed by a relative 2^-24 Gaussian.  Sequential single-position
    updates with large steps amplify rounding, so a float32 path can only be
    held to a multiple of this."""
    base = run(I)
    rng = np.random.default_rng(seed)
    dev = [0.0] * len(base)
    for _ in range(trials):
        out = run(I * (1.0 + 2.0 ** -24 * rng.standard_normal(I.shape)))
        dev = [max(d, float(np.linalg.norm(o - b) / np.linalg.norm(b))) for d, o, b in zip(dev, out, base)]
    return base, dev


# one-iteration cases on the small workload: (alg, batch, probe updated)
SMALL_ONE_ITER_CASES = [("epie", 1, True), ("rpie", 1, False), ("rpie", 7, True), ("epie", 100, True)]


def small_one_iter_setup(alg: str, B: int, upd: bool):
    """Start state, parameters and order of a one-iteration small-workload case:
    a generic smooth start (a flat object puts the exit wave's far field on the
    probe's exact diffraction zeros, where the phase is ill-conditioned) and
    alpha = beta = 0.3 (with beta = 0.6 a sequential probe update amplifies
    float32-level input rounding ~1300-fold in the float64 oracle itself)."""
    c = small_case()
    w = c["w"]
    O0 = c64(synth.make_object(w.M, 77) * (0.9 + 0.1j))
    P0 = c64(soft_probe(c["P"] * np.sqrt(c["scale"]), 1) * np.exp(0.2j))
    prm = ptycho.PtychoParams(alg, 0.3, 0.3, B, upd)
    order = synth.random_orders(w.J, 1, 11)
    return c, O0, P0, prm, order


def small_one_iter_spread(alg: str, B: int, upd: bool):
    """The oracle's spread (object, probe) for one one-iteration case."""
    c, O0, P0, prm, order = small_one_iter_setup(alg, B, upd)
    w = c["w"]
    _, (sO, sP, _) = oracle_spread(lambda I: ptycho.iterate(O0, P0, I, w.pos, 1, prm, order), c["I"])
    return sO, sP
