"""Learned warm start for the reconstruction: simulate training patterns
with the library's forward model, detector model and fusion, train the
U-Net with the library's training kernels, and compare the time the
iterations need to reach an object error threshold from the network's
starting object and from a flat one.

Every computation runs in libmnfpty's kernels (forward model, exposures,
fusion, network training and inference, stitching, iterations, NRMSE).
Objects, probes and positions come from the seeded generators; window
labels (amplitude and phase of the true object) are cut from those
generated objects on the host.  PyTorch only holds device memory, gathers
mini-batches and records events.

Workload: the small plain-method geometry (192^2 object, 64^2 probe of
radius 16 with phase pi, 10 x 10 raster step 8, exposures 1/10/100 at
12 bits, read noise 2, 4-level fusion) with the exit wave zero-padded into
a 256^2 detector; known probe; rPIE with mini-batch 10.  The network maps
ln(1 + I) / ln(1 + sat) of a 256^2 pattern to the 64^2 window's amplitude
and phase.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import api, synth

WIDTHS = (32, 64, 128, 256)
H = 256


@dataclasses.dataclass
class Setup:
    w: synth.Workload
    P: np.ndarray            # probe of unit flux (complex128)
    log_scale: float
    levels: int
    deltas: List[float]

    @property
    def pos(self) -> np.ndarray:
        return self.w.pos


def setup() -> Setup:
    w = synth.warmstart_workload(0)
    return Setup(w, w.probe(), 1.0 / math.log1p(float(w.sat)), w.levels,
                 synth.default_deltas(w.levels, w.sigma_read))


def layer_shapes(widths: Sequence[int]):
    """(taps, c_in, c_out) per layer in the library's parameter order."""
    c0, c1, c2, c3 = widths
    return [(9, 1, c0), (9, c0, c0), (4, c0, c1), (9, c1, c1), (9, c1, c1), (4, c1, c2),
            (9, c2, c2), (9, c2, c2), (4, c2, c3), (9, c3, c3), (9, c3, c3), (4, c3, c2),
            (9, 2 * c2, c2), (9, c2, c2), (1, c2, 2)]


def layer_flops(H: int, widths: Sequence[int]):
    """Multiply-add flops (2 per MAC) of every layer's forward pass for one sample."""
    out_px = [H, H, H // 2, H // 2, H // 2, H // 4, H // 4, H // 4, H // 8, H // 8, H // 8, H // 4, H // 4,
              H // 4, H // 4]
    fl = []
    for i, (taps, ci, co) in enumerate(layer_shapes(widths)):
        per_px = ci * co if i == 11 else taps * ci * co   # the transposed layer: one tap per output pixel
        fl.append(2 * out_px[i] ** 2 * per_px)
    return fl


def train_flops_per_sample(H: int, widths: Sequence[int]) -> int:
    """Forward + input gradient (all layers but the first) + weight gradient."""
    fl = layer_flops(H, widths)
    return 3 * sum(fl) - fl[0]


def init_params(widths: Sequence[int], seed: int, device="cuda:0") -> torch.Tensor:
    """He-normal weights (fan-in = taps x c_in; c_in for the transposed layer), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (taps, ci, co) in enumerate(layer_shapes(widths)):
        fan_in = ci if i == 11 else taps * ci
        parts.append(rng.standard_normal(taps * ci * co) * math.sqrt(2.0 / fan_in))
        parts.append(np.zeros(co))
    flat = np.concatenate(parts).astype(np.float32)
    if flat.size != api.unet_param_count(H, widths):
        raise RuntimeError("parameter layout does not match the library")
    return torch.from_numpy(flat).to(device)


def window_labels(O: np.ndarray, pos: np.ndarray, Nw: int, weight: Optional[np.ndarray] = None) -> np.ndarray:
    """Amplitude and phase of the true object in every scan window: [J][Nw][Nw][2] float32.
    With `weight` (|P|^2), each window's phase is taken relative to the phase of
    its weighted sum, the part a single far-field pattern cannot determine."""
    out = np.empty((len(pos), Nw, Nw, 2), np.float32)
    for j, (y, x) in enumerate(pos):
        win = O[y:y + Nw, x:x + Nw]
        if weight is not None:
            win = win * np.exp(-1j * np.angle(np.sum(weight * win)))
        out[j, ..., 0] = np.abs(win)
        out[j, ..., 1] = np.angle(win)
    return out


def simulate(S: Setup, seeds: Sequence[int], kind: str = "fused", device="cuda:0",
             labels: bool = True, relative: bool = False) -> Dict[str, object]:
    """Patterns of every scan position of the objects drawn with `seeds`.

    kind 'fused': the detector model (Poisson + read noise, 12-bit clip,
    exposures 1/10/100, flux putting the brightest pixel of the shortest
    exposure at half scale) followed by MNF fusion, in counts of the
    shortest exposure.  kind 'clean': the noise-free intensity at the same
    flux (what the fusion returns for an unsaturated, noise-free bracket).
    Returns I [n][256][256] (device), targets [n][64][64][2] (device), the
    true objects and the flux of each object.  With `relative`, window phases
    are labelled relative to each window's weighted mean phase."""
    w = S.w
    J = len(S.pos)
    n = J * len(seeds)
    I = torch.empty((n, w.Nd, w.Nd), dtype=torch.float32, device=device)
    tgt = torch.empty((n, w.Nw, w.Nw, 2), dtype=torch.float32, device=device) if labels else None
    P = torch.from_numpy(S.P.astype(np.complex64)).to(device)
    objs, scales = [], []
    for i, sd in enumerate(seeds):
        O = synth.make_object(w.M, int(sd))
        objs.append(O)
        Od = torch.from_numpy(O.astype(np.complex64)).to(device)
        clean = api.ptycho_forward(Od, P, S.pos, w.Nd)
        s = synth.flux_scale(float(clean.max().item()), w.sat)
        scales.append(s)
        sl = slice(i * J, (i + 1) * J)
        if kind == "clean":
            I[sl] = clean * s
        elif kind == "fused":
            raw = api.detector_expose(clean, w.t, s, w.sat, w.sigma_read, seed=1_000_003 * int(sd) + 17)
            api.fuse_exposures(raw, w.t, S.levels, sat=float(w.sat), delta=S.deltas, out=I[sl])
        else:
            raise ValueError(kind)
        if labels:
            wt = np.abs(S.P) ** 2 if relative else None
            tgt[sl] = torch.from_numpy(window_labels(O, S.pos, w.Nw, wt)).to(device)
    torch.cuda.synchronize(device)
    return dict(I=I, target=tgt, objects=objs, scales=scales, kind=kind)


def train(S: Setup, data, params: torch.Tensor, epochs: float = 1.0, batch: int = 64, lr: float = 1e-3,
          seed: int = 0, time_budget: Optional[float] = None, log=None,
          steps: Optional[int] = None) -> Dict[str, object]:
    """Adam on the mean-squared error of (amplitude, phase); stops after
    `steps` mini-batches (else `epochs` passes) or `time_budget` seconds.
    The learning rate drops tenfold for the last fifth of the steps (of the
    steps the time budget allows, estimated after 100 steps).  Returns the
    loss history and the training rate."""
    I, tgt = data["I"], data["target"]
    n = I.shape[0]
    dev = I.device
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = n // batch
    total = int(steps) if steps is not None else int(epochs * steps_per_epoch)
    hist = []
    t0 = time.perf_counter()
    step = 0
    loss_sum = torch.zeros((), dtype=torch.float64, device=dev)
    decay_at = int(0.8 * total)
    while step < total:
        perm = torch.randperm(n, generator=gen).to(dev)
        for b in range(steps_per_epoch):
            if step >= total:
                break
            idx = perm[b * batch:(b + 1) * batch]
            step += 1
            if time_budget is not None and step == 101:
                torch.cuda.synchronize(dev)
                per = (time.perf_counter() - t0) / 100
                decay_at = int(0.8 * min(total, int(time_budget / per)))
            cur_lr = lr if step <= decay_at else 0.1 * lr
            loss = api.unet_train_step(params, m, v, step, cur_lr, I.index_select(0, idx), S.log_scale,
                                       tgt.index_select(0, idx), H, WIDTHS)
            loss_sum += loss
            if step % 100 == 0:
                hist.append((step, float(loss_sum.item()) / 100))
                loss_sum.zero_()
                if log:
                    log(f"step {step} loss {hist[-1][1]:.5f} {time.perf_counter() - t0:.1f}s")
                if time_budget is not None and time.perf_counter() - t0 > time_budget:
                    total = step
                    break
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    return dict(history=hist, steps=step, seconds=dt, samples_per_s=step * batch / dt)


def predict(S: Setup, params: torch.Tensor, I: torch.Tensor, chunk: int = 100) -> torch.Tensor:
    out = torch.empty((I.shape[0], S.w.Nw, S.w.Nw, 2), dtype=torch.float32, device=I.device)
    for c0 in range(0, I.shape[0], chunk):
        api.unet_forward(params, I[c0:c0 + chunk], S.log_scale, H, WIDTHS, out=out[c0:c0 + chunk])
    return out


def _elapsed(fn, device) -> float:
    st = torch.cuda.current_stream(device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def covering_subset(pos: np.ndarray, min_dist: float) -> np.ndarray:
    """Indices of scan windows chosen by farthest-point sampling: start from the
    window farthest from the scan's centroid, repeatedly add the window farthest
    from those chosen, stop when every window lies within `min_dist` of a chosen
    one.  The corners and edges of the scan are taken first, so the network can
    run on these patterns only while the stitch still covers the scanned area
    with overlapping windows.  Returned in scan order."""
    p = np.asarray(pos, float)
    first = int(np.argmax(np.hypot(*(p - p.mean(axis=0)).T)))
    keep = [first]
    d = np.hypot(*(p - p[first]).T)
    while True:
        j = int(np.argmax(d))
        if d[j] < min_dist:
            break
        keep.append(j)
        d = np.minimum(d, np.hypot(*(p - p[j]).T))
    return np.sort(np.asarray(keep, np.int64))


def time_to_threshold(S: Setup, data, params: Optional[torch.Tensor], tau: float = 1e-2,
                      max_plain: int = 200, max_warm: int = 50, alpha: float = 0.1,
                      sync: bool = False, subset: Optional[np.ndarray] = None) -> List[Dict[str, object]]:
    """For every object of `data`: NRMSE per iteration from a flat start and
    from the network's stitched start, the iteration count at which each
    first reaches tau, and the timed cost of reaching it:
      plain: n_plain iterations;  warm: inference + stitching + n_warm iterations,
    each timed as one event-bracketed run on the stream.  With `subset`
    (window indices), the network runs on those patterns only."""
    w = S.w
    dev = data["I"].device
    J = len(S.pos)
    mask_np = _illumination_mask(S.P, S.pos, (w.M, w.M))
    mask = torch.from_numpy(mask_np.astype(np.uint8)).to(dev)
    res = []
    for i, (O_true, s) in enumerate(zip(data["objects"], data["scales"])):
        I = data["I"][i * J:(i + 1) * J]
        Pk = torch.from_numpy((math.sqrt(s) * S.P).astype(np.complex64)).to(dev)
        Ot = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
        kw = dict(alg="rpie", alpha=alpha, batch=w.batch, update_probe=False, err=False)

        def curve(O0, n_max):
            O = O0.clone()
            vals = [api.nrmse(O, Ot, mask).item()]
            for it in range(n_max):
                api.ptycho_iterate(O, Pk, I, S.pos, 1, it0=it, **kw)
                vals.append(api.nrmse(O, Ot, mask).item())
                if vals[-1] <= tau:
                    break
            return vals

        def first(vals):
            for k, v in enumerate(vals):
                if v <= tau:
                    return k
            return None

        flat = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
        plain = curve(flat, max_plain)
        n_plain = first(plain)
        r = dict(plain_curve=plain, n_plain=n_plain)
        # seconds per iteration: a 10-iteration run from the flat start
        Ox = flat.clone()
        r["t_iter"] = _elapsed(lambda: api.ptycho_iterate(Ox, Pk, I, S.pos, 10, **kw), dev) / 10
        if params is not None:
            sub = np.arange(J) if subset is None else np.asarray(subset)
            I_sub = I if subset is None else I.index_select(0, torch.from_numpy(sub).to(dev)).contiguous()
            pos_sub = S.pos[sub]
            patches = torch.empty((len(sub), w.Nw, w.Nw, 2), dtype=torch.float32, device=dev)
            P_unit = Pk / math.sqrt(s)

            def warm_start(out):
                api.unet_forward(params, I_sub, S.log_scale, H, WIDTHS, out=patches)
                api.ptycho_stitch(patches, P_unit, pos_sub, (w.M, w.M), sync=sync, out=out)

            O0 = torch.empty((w.M, w.M), dtype=torch.complex64, device=dev)
            warm_start(O0)
            warm = curve(O0, max_warm)
            n_warm = first(warm)
            r.update(warm_curve=warm, n_warm=n_warm, nrmse_init=warm[0])
            r["t_start"] = _elapsed(lambda: warm_start(O0), dev)
            if n_warm is not None:
                Ow = torch.empty_like(O0)

                def warm_run():
                    warm_start(Ow)
                    if n_warm:
                        api.ptycho_iterate(Ow, Pk, I, S.pos, n_warm, **kw)

                r["t_warm"] = _elapsed(warm_run, dev)
        if n_plain is not None:
            Op = flat.clone()
            r["t_plain"] = _elapsed(lambda: api.ptycho_iterate(Op, Pk, I, S.pos, n_plain, **kw), dev)
        res.append(r)
    return res


def _illumination_mask(P: np.ndarray, pos: np.ndarray, shape, frac: float = 0.1) -> np.ndarray:
    """Object pixels whose summed probe intensity reaches `frac` of its maximum
    (the region the NRMSE is taken over)."""
    Nw = P.shape[0]
    ill = np.zeros(shape)
    P2 = np.abs(P) ** 2
    for y, x in pos:
        ill[y:y + Nw, x:x + Nw] += P2
    return ill >= frac * ill.max()
