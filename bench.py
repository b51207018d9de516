"""Benchmark: scan-position updates per second of the full HDR-fused
ptychography job on one MI355X.

Workload (lab scale): 1024^2 complex object, 256^2 probe window (aperture
radius 64 px, defocus phase), 20 x 20 raster with 32 px pitch and +-2 px
jitter (400 positions), 5 exposures (1x to 1e4x, 16-bit, read noise 3),
6-level fusion, rPIE with mini-batch 32 for 200 iterations, probe updated
from iteration 5.  A step is the whole job: fusion of the 400 x 5 exposure
stack, then 200 rPIE iterations with the per-iteration Fourier error.
value = 400 * 200 / (seconds per step).

The synthetic exposure stack is simulated once before timing (the library's
forward model on the GPU, Poisson + Gaussian detector noise on the host).

--workload multiscan times the uneven-size workload instead: 64 independent
scans (N in {128,192,256,384,512}, 50-1000 Fermat-spiral positions each,
30,537 positions in all), rPIE mini-batch 32, 20 iterations, every scan
advanced by one ptycho_iterate_many call captured in a hipGraph.  Its
intensities come straight from the forward model (no noise or fusion), which
does not change the reconstruction's work.

--workload warmstart measures the second half of the headline metric:
time to object NRMSE 1e-2 from the U-Net's stitched start versus a flat
start (t_plain / t_warm), after training the network on 50,000 simulated
fused patterns (training time reported separately, excluded).  Its roofline
entry is the network's forward pass in TFLOP/s against the bf16 MFMA peak.

--workload subpixel runs the lab job at 400 real (unrounded) Fermat-spiral
positions with the same density, through the Fourier-translated-probe entry
points (translation passes added to every mini-batch); traffic is null there
(the stored counters describe the integer-position kernels).
--workload small runs the small configuration: 192^2 object, 64^2 probe
(r = 16), 10 x 10 raster of pitch 8 (100 positions), 3 exposures (1, 10, 100;
12 bit, read noise 2), 4-level fusion, 50 ePIE iterations with mini-batches
of one, probe refined from iteration 5 (one workgroup runs the whole call).
--workload grad times the loss gradient (the adjoint) on the 2048^2 /
512^2 / 1000-position gradient workload in position-gradients/s.
--workload unet times the network's training step and inference alone.
--workload broadband runs two-harmonic (Eq. 4) data through fusion and the
monochromatic reconstruction.
--workload batch-sweep times the lab-scale reconstruction at mini-batches
8..256 (per-launch durations of every pass), and --workload fusion-compare
compares MNF with linear integration and the shortest frame on the small
workload at three flux levels (image metrics and the object NRMSE that 50
ePIE iterations reach on each).

Roofline: achieved = (algorithmic bytes per position update, 20 N^2 + 16 N^2 / B)
x (positions one launch of the dominant kernel processes) / (its mean launch
duration, HIP events on the launch stream over the timed region, around
every k-th launch of that kernel, k <= 64 leaving at least 64 timed launches:
an event pair costs the queue a few microseconds, which timing every launch
would add to the step).  traffic =
counter-measured bytes per launch of that kernel from profiles/, or null when
the kernel sources changed since the counters were taken.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic HBM bytes per position update of an N x N pattern with
# mini-batch B: amplitude read 4 N^2, object patch read + write 16 N^2, probe
# read + write 16 N^2 amortised over the batch
def algo_bytes_per_update(N: int, B: int) -> float:
    return 20.0 * N * N + 16.0 * N * N / B


HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["fft.hpp", "kernels_common.hpp", "pattern_kernels.hpp", "shift_kernels.hpp", "update_kernels.hpp",
                  "objrow_kernels.hpp", "small_kernels.hpp", "descent_kernels.hpp", "tables.hpp", "ptycho.hip"]


def kernel_source_hash() -> str:
    """Hash of the reconstruction kernels' sources, their launch code and the
    compiler flags."""
    from paper_2608_01746_amd import build as _build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_01746_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(_build.HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


RECON_PASSES = ("rows_fwd", "cols_modulus", "rows_inv", "object_update")


def measured_traffic_all():
    """Counter-measured bytes per launch (fetch x 2.0 + write x 1.0) of every
    reconstruction pass from profiles/lab256_counters.txt, if taken with the
    current kernel sources; {} otherwise."""
    path = os.path.join(ROOT, "profiles", "lab256_counters.txt")
    if not os.path.exists(path):
        return {}
    src_hash, rows = None, {}
    for line in open(path):
        parts = line.split()
        if len(parts) >= 2 and parts[0] == "source_hash":
            src_hash = parts[1]
        elif len(parts) == 3 and parts[0] in RECON_PASSES:
            rows[parts[0]] = (2.0 * float(parts[1]) + float(parts[2])) * 1024.0
    return rows if src_hash == kernel_source_hash() else {}


def measured_traffic(kernel: str):
    return measured_traffic_all().get(kernel)


def host_cpu():
    """(model name, usable host cores) of this machine."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def batch_update_all_cores(O, P, A, pos, idx, alpha, beta, update_probe, workers):
    """The float64 rPIE mini-batch update of the oracle (same formulas, same
    batch-start semantics), written batched so that every host core works:
    the batch's exit waves are transformed together by scipy.fft with
    `workers` threads.  A CPU throughput reference for the benchmark only;
    its agreement with the oracle is tested."""
    import numpy as np
    import scipy.fft as sfft

    Nw, Nd = P.shape[0], A.shape[-1]
    idx = np.asarray(idx)
    Oj = np.stack([O[y:y + Nw, x:x + Nw] for y, x in pos[idx]])
    psi = np.zeros((len(idx), Nd, Nd), np.complex128)
    psi[:, :Nw, :Nw] = P * Oj
    Psi = sfft.fft2(psi, norm="ortho", workers=workers)
    mag = np.abs(Psi)
    Aj = A[idx]
    err = float(np.sum((mag - Aj) ** 2))
    nz = mag > 0
    Psi_p = np.where(nz, Aj * Psi / np.where(nz, mag, 1.0), Aj)
    dpsi = sfft.ifft2(Psi_p, norm="ortho", workers=workers)[:, :Nw, :Nw] - psi[:, :Nw, :Nw]
    P2 = np.abs(P) ** 2
    numO = np.zeros_like(O)
    denO = np.zeros(O.shape)
    dO = (1.0 - alpha) * P2 + alpha * float(P2.max())
    for k, (y, x) in enumerate(pos[idx]):
        numO[y:y + Nw, x:x + Nw] += np.conj(P) * dpsi[k]
        denO[y:y + Nw, x:x + Nw] += dO
    O_new = O.copy()
    cov = denO > 0
    O_new[cov] += numO[cov] / denO[cov]
    P_new = P.copy()
    if update_probe:
        O2 = np.abs(Oj) ** 2
        numP = np.sum(np.conj(Oj) * dpsi, axis=0)
        denP = np.sum((1.0 - beta) * O2 + beta * O2.max(axis=(1, 2), keepdims=True), axis=0)
        okp = denP > 0
        P_new[okp] += numP[okp] / denP[okp]
    return O_new, P_new, err


def cpu_baseline(w, O_true, P, clean, scale, seconds: float, sub: bool = False, alg: str = "rpie",
                 step: float = 0.1):
    """The float64 oracle on the host: rPIE mini-batches of the same workload
    (at real positions with the sub-pixel oracle when `sub`), repeated for
    about `seconds`; returns position updates per second."""
    import numpy as np
    from oracle import ptycho, subpixel

    I = clean * scale  # noiseless intensities at the fused scale (same shapes as the job)
    A = ptycho.amplitudes(I)
    O = np.ones_like(O_true)
    Pk = P * math.sqrt(scale)
    prm = ptycho.PtychoParams(alg, step, step, w.batch, True)
    order = np.random.default_rng(0).permutation(w.J)
    n = 0
    t0 = time.perf_counter()
    b = 0
    while time.perf_counter() - t0 < seconds:
        idx = order[(b * w.batch) % w.J:][:w.batch]
        upd = subpixel.batch_update if sub else ptycho.batch_update
        O, Pk, _ = upd(O, Pk, A, w.pos.astype(np.float64) if sub else w.pos, idx, prm, True)
        n += len(idx)
        b += 1
    dt = time.perf_counter() - t0
    return n / dt, n, dt


def cpu_baseline_all_cores(w, O_true, P, clean, scale, seconds: float):
    """The batched float64 update on every usable host core (FFTs threaded),
    repeated for about `seconds`; returns (position updates/s, n, s, cores)."""
    import numpy as np
    from oracle import ptycho

    _, cores = host_cpu()
    workers = min(cores, 16)
    A = ptycho.amplitudes(clean * scale)
    O = np.ones_like(O_true)
    Pk = P * math.sqrt(scale)
    order = np.random.default_rng(0).permutation(w.J)
    n, b = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        idx = order[(b * w.batch) % w.J:][:w.batch]
        O, Pk, _ = batch_update_all_cores(O, Pk, A, w.pos, idx, 0.1, 0.1, True, workers)
        n += len(idx)
        b += 1
    dt = time.perf_counter() - t0
    return n / dt, n, dt, workers


# In a timed region the dominant kernel's launch durations come from HIP
# events recorded around every k-th launch of it (the first included): each
# timed launch costs the queue a few microseconds of event work, which
# bracketing every launch would add to the step time.  k is at most
# TIMING_PERIOD and leaves at least 64 timed launches.
TIMING_PERIOD = 64


def timing_period(expected_launches):
    return max(1, min(TIMING_PERIOD, int(expected_launches) // 64))


def profile_dominant(api, run_step, classes):
    """Time one step with events around every launch of `classes`; return the
    dominant class and the per-class (launches, ms)."""
    import torch
    api.profile(classes)
    api.profile_reset()
    run_step()
    torch.cuda.synchronize()
    ranks = api.profile_read()
    api.profile([])
    dominant = max((k for k in ranks if k in ("rows_fwd", "cols_modulus", "rows_inv", "object_update", "small_run")),
                   key=lambda k: ranks[k][1])
    return dominant, ranks


def roofline(dominant, nlaunch, kms, positions_per_launch, N, B, counters=True, updates_per_step=None,
             ms_per_step=None, timed_every=1):
    """`counters`: the stored counter readings describe this launch (the
    integer-position lab workload).  With the step's updates and duration the
    entry also carries pipeline_frac: the whole step's algorithmic bytes per
    second (every pass, fusion and launch gaps included) against the HBM peak;
    traffic_ratio: the reconstruction passes' counter-measured bytes per
    mini-batch against the algorithmic bytes of that mini-batch."""
    avg_us = kms / nlaunch * 1e3
    bytes_launch = algo_bytes_per_update(N, B) * positions_per_launch
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    traffic = measured_traffic(dominant) if counters else None
    out = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(traffic),
           "avg_launch_us": round(avg_us, 2), "launches": nlaunch, "timed_every": timed_every,
           "algorithmic_bytes_per_launch": round(bytes_launch)}
    if updates_per_step and ms_per_step:
        gbs = algo_bytes_per_update(N, B) * updates_per_step / (ms_per_step * 1e-3) / 1e9
        out["pipeline_achieved"] = round(gbs, 1)
        out["pipeline_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    allt = measured_traffic_all() if counters else {}
    out["traffic_ratio"] = (round(sum(allt.values()) / bytes_launch, 3)
                            if len(allt) == len(RECON_PASSES) else None)
    return out


PASSES = ["rows_fwd", "cols_modulus", "rows_inv", "object_update", "fuse"]
SUB_PASSES = PASSES + ["shift", "probe_update"]
SMALL_PASSES = PASSES + ["small_run"]


def tune_sizes(sizes, batch):
    """Pick the launch-shape variant per detector size (timed once, cached)."""
    from paper_2608_01746_amd import tune
    out = tune.autotune(sizes, batch=batch, reps=5)
    return {str(N): e["variant"] for N, e in out.items()}


def run_lab(args, api, synth, dev):
    import numpy as np
    import torch

    sub = args.workload == "subpixel"
    small = args.workload == "small"
    w = synth.lab_subpixel_workload() if sub else (synth.small_workload() if small else synth.lab_workload())
    # the small workload runs textbook ePIE (unit steps); the lab ones rPIE 0.1
    alg, step_a = ("epie", 1.0) if small else ("rpie", 0.1)
    forward = api.ptycho_forward_subpixel if sub else api.ptycho_forward
    iterate = api.ptycho_iterate_subpixel if sub else api.ptycho_iterate
    n_iter = args.iters
    tuned = tune_sizes([w.Nd], w.batch) if args.tune and not small else None
    if getattr(args, "three_launch", False):
        from paper_2608_01746_amd import tune
        tune.set_variant(w.Nd, tune.get_variant(w.Nd) | 4)
        tuned = {str(w.Nd): tune.get_variant(w.Nd)}
    O_true = w.object()
    P = w.probe()
    Ot = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(dev)
    clean_t = forward(Ot, Pt, w.pos, w.Nd)
    torch.cuda.synchronize()
    clean = clean_t.cpu().numpy().astype(np.float64)
    del Ot, Pt, clean_t
    scale = synth.flux_scale(clean.max(), w.sat)
    print(f"# simulating {w.J} x {len(w.t)} exposures of {w.Nd}^2", file=sys.stderr, flush=True)
    raw = torch.from_numpy(synth.expose(clean, w.t, w.sat, w.sigma_read, 2002, scale)).to(dev)
    delta = synth.default_deltas(w.levels, w.sigma_read)
    order = synth.random_orders(w.J, n_iter, 2)
    energy = scale * float(np.sum(np.abs(P) ** 2)) * 0.75 ** 2
    O0 = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
    P0 = torch.from_numpy(synth.flat_probe_guess(w.Nw, w.radius, energy).astype(np.complex64)).to(dev)
    O = torch.empty_like(O0)
    Pw = torch.empty_like(P0)
    fused = torch.empty((w.J, w.Nd, w.Nd), dtype=torch.float32, device=dev)
    state = {}
    graph = False

    def step():
        O.copy_(O0)
        Pw.copy_(P0)
        api.fuse_exposures(raw, w.t, w.levels, sat=float(w.sat), delta=delta, out=fused)
        state["err"] = iterate(O, Pw, fused, w.pos, n_iter, alg=alg, alpha=step_a, beta=step_a,
                               batch=w.batch, update_probe=True, probe_start_iter=5, order=order, graph=graph)

    dominant, ranks = profile_dominant(api, step, SUB_PASSES if sub else (SMALL_PASSES if small else PASSES))
    graph = args.graph
    print("# per-class ms (warm-up step): " +
          ", ".join(f"{k} {v[1]:.2f} ({v[0]})" for k, v in ranks.items()), file=sys.stderr, flush=True)
    for _ in range(args.warmup - 1):
        step()
    # timed region: events bracket a sample of the dominant kernel's launches
    # (all of them for the single-workgroup run: one launch per call)
    every = 1 if dominant == "small_run" else timing_period(ranks[dominant][0] * args.steps)
    api.profile([dominant], every=every)
    api.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = api.profile_read()
    api.profile([])
    # inside a captured graph no per-launch events are recorded: take them
    # from the direct-launch warm-up step instead
    nlaunch, kms = ranks[dominant] if graph else prof[dominant]
    dt = (t1 - t0) / args.steps
    value = w.J * n_iter / dt
    # positions one launch of the dominant kernel processes (the whole run for
    # the single-workgroup kernel of the small workload)
    per_launch = w.J * n_iter * args.steps / nlaunch if dominant == "small_run" else w.J / math.ceil(w.J / w.batch)
    if small:
        metric = "scan-position updates/s at 64^2 FP32 (small ePIE, mini-batch 1, fusion included)"
        wl = ("small-64: 192^2 object, 64^2 probe, 100 positions, 3 exposures, 4-level fusion, ePIE B=1, "
              "%d iterations" % n_iter)
    elif sub:
        metric = ("scan-position updates/s at 256^2 FP32 (lab-scale rPIE at real Fermat-spiral positions, "
                  "Fourier-translated probes, mini-batch 32, fusion included)")
        wl = ("lab-256-subpixel: 1024^2 object, 256^2 probe, 400 real Fermat-spiral positions, 5 exposures, "
              "6-level fusion, rPIE B=32, %d iterations" % n_iter)
    else:
        metric = "scan-position updates/s at 256^2 FP32 (lab-scale rPIE, mini-batch 32, fusion included)"
        wl = ("lab-256: 1024^2 object, 256^2 probe, 400 positions, 5 exposures, "
              "6-level fusion, rPIE B=32, %d iterations" % n_iter)
    out = {
        "metric": metric,
        "value": round(value, 1),
        "unit": "position-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded object/probe, simulated Poisson+Gaussian exposures)",
        "config": {"workload": wl, "positions": w.J, "pattern": w.Nd, "batch": w.batch, "iterations": n_iter,
                   "exposures": len(w.t), "levels": w.levels},
        "roofline": roofline(dominant, nlaunch, kms, per_launch, w.Nd, w.batch, counters=not (sub or small),
                             updates_per_step=w.J * n_iter, ms_per_step=dt * 1e3,
                             timed_every=1 if graph else every),
        "per_class_ms_one_step": {k: round(v[1], 3) for k, v in ranks.items()},
        "launch_variants": tuned,
        "graph": graph,
        "final_fourier_error": float(state["err"][-1].item()),
    }
    if not args.no_cpu:
        v, n, sec = cpu_baseline(w, O_true, P, clean, scale, args.cpu_seconds, sub, alg, step_a)
        model, _ = host_cpu()
        out["cpu_baseline"] = {"value": round(v, 3), "unit": "position-updates/s", "cores": 1,
                               "kind": "oracle", "host": model,
                               "sample": f"{n} {alg} position updates (mini-batches of {w.batch}) of the "
                                         f"same workload in float64 NumPy, {sec:.1f} s"}
        if not (sub or small):
            v2, n2, sec2, cores = cpu_baseline_all_cores(w, O_true, P, clean, scale, args.cpu_seconds)
            out["cpu_baseline_all_cores"] = {
                "value": round(v2, 3), "unit": "position-updates/s", "cores": cores,
                "kind": "batched float64 update, scipy.fft over all usable host cores", "host": model,
                "sample": f"{n2} rPIE position updates (mini-batches of {w.batch}) of the same workload, "
                          f"{sec2:.1f} s"}
    return out


def run_grad(args, api, synth, dev):
    """Gradient-descent reconstruction (the adjoint of Eqs. 2-3 under the
    Poisson model) on the gradient workload: 2048^2 object, 512^2 probe,
    1000 Fermat-spiral positions, MNF-fused data from exposures simulated on
    the GPU (5 exposures, 16 bit, read noise 3, 6 levels).  A step is one
    full-batch descent step: the Poisson loss and the object and probe
    gradients over every position (exit waves recomputed in batches of 32),
    then the backtracking step of ptycho_descend, from a flat object and the
    known probe (both updated).  The warm-up computes the initial step sizes; the
    timed call resumes with the step sizes the warm-up ended with.
    value = positions / s; the loss of every step and the final object NRMSE
    are reported."""
    import numpy as np
    import torch

    w = synth.gradient_workload()
    O_true = w.object()
    P = w.probe()
    Ot = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
    Pt = torch.from_numpy(P.astype(np.complex64)).to(dev)
    clean = api.ptycho_forward(Ot, Pt, w.pos, w.Nd)
    s = synth.flux_scale(float(clean.max().item()), w.sat)
    print(f"# simulating {w.J} x {len(w.t)} exposures of {w.Nd}^2 on the GPU", file=sys.stderr, flush=True)
    raw = api.detector_expose(clean, w.t, s, w.sat, w.sigma_read, seed=4004)
    del clean
    fused = api.fuse_exposures(raw, w.t, w.levels, sat=float(w.sat), delta=synth.default_deltas(w.levels, w.sigma_read))
    del raw
    torch.cuda.synchronize()
    O_start = np.ones((w.M, w.M), np.complex64)  # flat start, as the iterative engines
    O0 = torch.from_numpy(O_start).to(dev)
    Pk = torch.from_numpy((np.sqrt(s) * P).astype(np.complex64)).to(dev)
    Ot_scaled = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(_illum_mask(P, w.pos, (w.M, w.M)).astype(np.uint8)).to(dev)
    nrmse0 = api.nrmse(O0, Ot_scaled, mask).item()

    # step sizes from the start and a profiled first step, then the rest of
    # the warm-up
    classes = ["rows_fwd", "grad_cols", "rows_inv", "grad_scatter", "small"]
    api.profile(classes)
    api.profile_reset()
    loss_w, eta = api.ptycho_descend(O0, Pk, fused, w.pos, 1, "poisson", 1e-6, w.batch)
    torch.cuda.synchronize()
    ranks = api.profile_read()
    api.profile([])
    eta_O, eta_P = (float(x) for x in eta.cpu().tolist())
    eta_start = (eta_O, eta_P)
    losses = [loss_w]
    if args.warmup > 1:
        loss_w, eta = api.ptycho_descend(O0, Pk, fused, w.pos, args.warmup - 1, "poisson", 1e-6, w.batch,
                                         eta_O=eta_O, eta_P=eta_P)
        losses.append(loss_w)
        eta_O, eta_P = (float(x) for x in eta.cpu().tolist())
    dominant = max(classes[:4], key=lambda k: ranks[k][1])
    every = timing_period(ranks[dominant][0] * args.steps)
    api.profile([dominant], every=every)
    api.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss_t, eta = api.ptycho_descend(O0, Pk, fused, w.pos, args.steps, "poisson", 1e-6, w.batch, eta_O=eta_O,
                                     eta_P=eta_P)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = api.profile_read()
    api.profile([])
    losses.append(loss_t)
    loss_hist = torch.cat(losses).cpu().tolist()
    nrmse1 = api.nrmse(O0, Ot_scaled, mask).item()
    api.check_status(dev)
    nlaunch, kms = prof[dominant]
    dt = (t1 - t0) / args.steps
    N, B = w.Nd, w.batch
    per_launch = w.J / math.ceil(w.J / B)
    # algorithmic bytes per position gradient: intensity 4 N^2, object window
    # read 8 N^2, object-gradient window write 8 N^2, probe read and probe
    # gradient write 16 N^2 amortised over the batch
    bytes_pos = 20.0 * N * N + 16.0 * N * N / B
    avg_us = kms / nlaunch * 1e3
    achieved = bytes_pos * per_launch / (avg_us * 1e-6) / 1e9
    # the step itself: O and gO read, O written (object grid), the same for P
    bytes_step = 24.0 * (w.M * w.M + N * N)
    pipe = (bytes_pos * w.J + bytes_step) / dt / 1e9
    out = {
        "metric": "position-gradients/s at 512^2 FP32 (gradient-descent reconstruction: Poisson loss, object and "
                  "probe gradients and the step, batches of 32)",
        "value": round(w.J / dt, 1), "unit": "position-gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded object/probe, exposures simulated on the GPU, MNF-fused)",
        "config": {"workload": "grad-512: 2048^2 object, 512^2 probe, 1000 Fermat-spiral positions, 5 exposures, "
                               "6-level fusion, Poisson loss, recompute batches of 32, full-batch descent with "
                               "backtracking"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_us": round(avg_us, 2), "launches": nlaunch, "timed_every": every,
                     "algorithmic_bytes_per_launch": round(bytes_pos * per_launch),
                     "pipeline_achieved": round(pipe, 1), "pipeline_frac": round(pipe / HBM_PEAK_GBS, 4)},
        "per_class_ms_one_step": {k: round(v[1], 3) for k, v in ranks.items()},
        "step_sizes": {"start": list(eta_start), "end": [float(x) for x in eta.cpu().tolist()]},
        "loss_per_step": [float(f"{x:.6e}") for x in loss_hist],
        "nrmse_start": round(nrmse0, 5), "nrmse_end": round(nrmse1, 5),
        "note": "MNF-fused patterns of this detector model hold every reconstruction (rPIE included) near object "
                "NRMSE 0.2 (radiometric deviation of the fusion); on the noise-free patterns the same descent "
                "from the same start reaches 0.005 after 200 steps",
    }
    if not args.no_cpu:
        from oracle import adjoint
        O_np, P_np = O_start.astype(np.complex128), (np.sqrt(s) * P).astype(np.complex128)
        I_np = fused.cpu().numpy().astype(np.float64)
        n, t_start = 0, time.perf_counter()
        while time.perf_counter() - t_start < args.cpu_seconds and n < w.J:
            adjoint.loss_and_grad(O_np, P_np, I_np[n:n + 1], w.pos[n:n + 1], "poisson", 1e-6)
            n += 1
        sec = time.perf_counter() - t_start
        out["cpu_baseline"] = {"value": round(n / sec, 3), "unit": "position-gradients/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{n} positions' Poisson loss and gradients in float64 NumPy, {sec:.1f} s "
                                         "(the step itself, one pass over the arrays, not included)"}
    return out


def run_multiscan(args, api, synth, dev):
    import numpy as np
    import torch

    ws = synth.multiscan_workloads(64)
    n_iter = args.iters
    tuned = tune_sizes(sorted({w.Nd for w in ws}), 32) if args.tune else None
    scans = []
    for w in ws:
        # each scan's exposure bracket (3-5 exposures, 16 bit, read noise 3)
        # simulated once on the GPU; every step fuses it before iterating
        O_true = torch.from_numpy(w.object().astype(np.complex64)).to(dev)
        P = w.probe()
        Pt = torch.from_numpy(P.astype(np.complex64)).to(dev)
        clean = api.ptycho_forward(O_true, Pt, w.pos, w.Nd)
        flux = synth.flux_scale(float(clean.max().item()), w.sat)
        raw = api.detector_expose(clean, w.t, flux, w.sat, w.sigma_read, seed=w.seed)
        del clean
        energy = flux * float(np.sum(np.abs(P) ** 2)) * 0.75 ** 2
        P0 = torch.from_numpy(synth.flat_probe_guess(w.Nw, w.radius, energy).astype(np.complex64)).to(dev)
        O0 = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
        I = torch.empty((w.J, w.Nd, w.Nd), dtype=torch.float32, device=dev)
        scans.append(dict(O0=O0, P0=P0, O=torch.empty_like(O0), P=torch.empty_like(P0), I=I, pos=w.pos,
                          order=synth.random_orders(w.J, n_iter, w.seed), raw=raw, w=w,
                          deltas=synth.default_deltas(w.levels, w.sigma_read)))
        del O_true, Pt
    torch.cuda.synchronize()
    total_J = sum(w.J for w in ws)
    raw_gb = sum(sc["raw"].numel() * 2 for sc in scans) / 1e9
    print(f"# {len(ws)} scans, {total_J} positions, {raw_gb:.1f} GB of exposures", file=sys.stderr, flush=True)
    state = {}

    def fuse_all():
        for sc in scans:
            w = sc["w"]
            api.fuse_exposures(sc["raw"], w.t, w.levels, sat=float(w.sat), delta=sc["deltas"], out=sc["I"])

    def step(graph=True):
        fuse_all()
        for sc in scans:
            sc["O"].copy_(sc["O0"])
            sc["P"].copy_(sc["P0"])
        state["err"] = api.ptycho_iterate_many(scans, n_iter, alg="rpie", alpha=0.1, beta=0.1, batch=32,
                                               update_probe=True, probe_start_iter=5, graph=graph)

    dominant, ranks = profile_dominant(api, lambda: step(False), PASSES)
    print("# per-class ms (direct-launch step): " +
          ", ".join(f"{k} {v[1]:.2f} ({v[0]})" for k, v in ranks.items()), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    value = total_J * n_iter / dt
    # the fusion's share of a step, timed alone
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    fuse_all()
    torch.cuda.synchronize()
    fuse_ms = (time.perf_counter() - f0) * 1e3
    nlaunch, kms = ranks[dominant]
    # positions per launch of the dominant pass, averaged over the step
    per_launch = total_J * n_iter / nlaunch
    Nbar = math.sqrt(sum(w.J * w.Nd ** 2 for w in ws) / total_J)
    return {
        "metric": "scan-position updates/s, 64 uneven scans in one graph-captured call (fusion included)",
        "value": round(value, 1),
        "unit": "position-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded objects/probes, exposures simulated on the GPU, MNF-fused every step)",
        "config": {"workload": "multiscan: 64 scans, N in {128,192,256,384,512}, 50-1000 Fermat-spiral "
                               "positions, 3-5 exposures, 4-level fusion, rPIE B=32, %d iterations" % n_iter,
                   "scans": len(ws), "positions": total_J, "iterations": n_iter,
                   "exposure_gb": round(raw_gb, 2)},
        "fusion_ms_per_step": round(fuse_ms, 3),
        # the stored counters describe the lab-256 launches, not these
        "roofline": dict(roofline(dominant, nlaunch, kms, per_launch, Nbar, 32, counters=False),
                         note="per-launch events from one step with direct launches; N = rms pattern size"),
        "per_class_ms_direct_step": {k: round(v[1], 3) for k, v in ranks.items()},
        "launch_variants": tuned,
    }


def run_batch_sweep(args, api, synth, dev):
    """Launch latency versus work: the lab-scale scan reconstructed with
    mini-batches of 8..256 (same kernels), per-launch duration of every pass
    from HIP events and the iteration rate.  One JSON object per batch size
    under "sweep"; the headline value is the configured batch's rate."""
    import numpy as np
    import torch

    w = synth.lab_workload()
    O_true = torch.from_numpy(w.object().astype(np.complex64)).to(dev)
    P = torch.from_numpy(w.probe().astype(np.complex64)).to(dev)
    I = api.ptycho_forward(O_true, P, w.pos, w.Nd)
    rows = []
    for B in (8, 16, 32, 64, 128, 256):
        O = torch.ones_like(O_true)
        Pw = P.clone()
        api.ptycho_iterate(O, Pw, I, w.pos, 2, batch=B, update_probe=True)
        api.profile(PASSES[:4])
        api.profile_reset()
        api.ptycho_iterate(O, Pw, I, w.pos, 5, batch=B, update_probe=True)
        torch.cuda.synchronize()
        prof = api.profile_read()
        api.profile([])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.ptycho_iterate(O, Pw, I, w.pos, args.iters, batch=B, update_probe=True)
        e1.record()
        e1.synchronize()
        it_ms = e0.elapsed_time(e1) / args.iters
        rows.append({"batch": B, "ms_per_iteration": round(it_ms, 4), "updates_per_s": round(w.J / it_ms * 1e3),
                     "us_per_launch": {k: round(v[1] / v[0] * 1e3, 2) for k, v in prof.items()}})
        print(f"# B={B}: {rows[-1]}", file=sys.stderr, flush=True)
    ref = next(r for r in rows if r["batch"] == w.batch)
    return {"metric": "scan-position updates/s at 256^2 FP32 versus mini-batch size (reconstruction only)",
            "value": ref["updates_per_s"], "unit": "position-updates/s", "n_gpus": 1, "steps": args.iters,
            "warmup": 2, "ms_per_step": ref["ms_per_iteration"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic (noiseless forward-model intensities)",
            "config": {"workload": "lab-256 geometry, rPIE with probe update, mini-batch 8..256"},
            "sweep": rows}


def _mtf(O_rec, O_true, mask, nbins=16):
    """Modulation transfer of a reconstruction (host evaluation of a result):
    on the largest centred square inside the illuminated mask, the
    reconstruction's global factor matched by the squares' means, means
    removed, H(f) = |sum R^ conj(T^)| / sum |T^|^2 over annuli of radial
    frequency (cycles/pixel, nbins equal bins up to 0.5).  Returns H."""
    import numpy as np
    ys, xs = np.nonzero(mask)
    cy, cx = (ys.min() + ys.max() + 1) // 2, (xs.min() + xs.max() + 1) // 2
    h = 0
    while (cy - h - 1 >= 0 and cx - h - 1 >= 0 and cy + h + 1 <= mask.shape[0] and cx + h + 1 <= mask.shape[1]
           and mask[cy - h - 1:cy + h + 1, cx - h - 1:cx + h + 1].all()):
        h += 1
    T = np.asarray(O_true[cy - h:cy + h, cx - h:cx + h], np.complex128)
    R = np.asarray(O_rec[cy - h:cy + h, cx - h:cx + h], np.complex128)
    R = R * (T.mean() / R.mean())
    Rh, Th = np.fft.fft2(R - R.mean()).ravel(), np.fft.fft2(T - T.mean()).ravel()
    f = np.fft.fftfreq(2 * h)
    fr = np.hypot(f[:, None], f[None, :]).ravel()
    keep = fr <= 0.5
    b = np.minimum((fr[keep] / 0.5 * nbins).astype(int), nbins - 1)
    cross = np.bincount(b, (Rh[keep] * np.conj(Th[keep])).real, nbins) + \
        1j * np.bincount(b, (Rh[keep] * np.conj(Th[keep])).imag, nbins)
    power = np.bincount(b, np.abs(Th[keep]) ** 2, nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.abs(cross) / power


def run_fusion_compare(args, api, synth, dev):
    """MNF against the linear baselines on the small workload's simulated
    data at three flux levels: image metrics of each fused stack against the
    clean intensity, and the object NRMSE reached by 50 sequential ePIE
    iterations (known probe) on each.  Value: MNF's median final NRMSE at the
    default flux.  Every step runs on the GPU (forward model, exposures,
    fusions, iterations, NRMSE); the image metrics are host sums."""
    import numpy as np
    import torch

    w = synth.small_workload()
    P = w.probe()
    mask_np = None
    deltas = synth.default_deltas(w.levels, w.sigma_read)
    # MNF with the default parameters and a stability sweep around them (no
    # quantisation, eight-fold steps, weight width 0.1 / 0.3, weight centre
    # 0.4 / 0.6); the two linear baselines
    mnf_variants = {"mnf": {}, "mnf_delta0": {"delta": ()}, "mnf_delta8": {"delta": [8 * d for d in deltas]},
                    "mnf_sigma0.1": {"sigma": 0.1}, "mnf_sigma0.3": {"sigma": 0.3},
                    "mnf_mu0.4": {"mu": 0.4}, "mnf_mu0.6": {"mu": 0.6}}
    methods = tuple(mnf_variants) + ("linear", "shortest")
    rows = []
    # the configured 1/10/100 bracket at three flux levels, and the paper's own
    # 1/2/4 s ratio (Results 2.3) at two
    settings = [((1.0, 10.0, 100.0), 1.0), ((1.0, 10.0, 100.0), 0.1), ((1.0, 10.0, 100.0), 0.01),
                ((1.0, 2.0, 4.0), 1.0), ((1.0, 2.0, 4.0), 0.1)]
    for tb, f in settings:
        w.t = list(tb)
        per = {m: {"dev": [], "snr": [], "bgvar": [], "nrmse": [], "nrmse_best": [], "mtf_nyquist": [],
                   "mtf50": []} for m in methods}
        for seed in range(1, 5):
            O_true = w.object() if seed == 1 else synth.make_object(w.M, seed)
            Ot = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
            Pt = torch.from_numpy(P.astype(np.complex64)).to(dev)
            clean = api.ptycho_forward(Ot, Pt, w.pos, w.Nd)
            s = synth.flux_scale(float(clean.max().item()), w.sat) * f
            raw = api.detector_expose(clean, w.t, s, w.sat, w.sigma_read, seed=7919 * seed + int(1000 * f))
            C = (clean * s).cpu().numpy().astype(np.float64)
            if mask_np is None:
                mask_np = _illum_mask(P, w.pos, (w.M, w.M))
                mask = torch.from_numpy(mask_np.astype(np.uint8)).to(dev)
            Pk = torch.from_numpy((np.sqrt(s) * P).astype(np.complex64)).to(dev)
            for m in methods:
                if m in mnf_variants:
                    kw = {"delta": deltas, **mnf_variants[m]}
                    I = api.fuse_exposures(raw, w.t, w.levels, sat=float(w.sat), **kw)
                else:
                    I = api.fuse_linear(raw, w.t, float(w.sat), mode=m)
                F = I.cpu().numpy().astype(np.float64)
                per[m]["dev"].append(float(np.linalg.norm(F - C) / np.linalg.norm(C)))
                per[m]["snr"].append(float(10 * np.log10(np.sum(C * C) / np.sum((F - C) ** 2))))
                per[m]["bgvar"].append(float(np.var(F[C < 1e-3 * C.max()])))
                O = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
                best = 1e9
                for it in range(50):
                    api.ptycho_iterate(O, Pk, I, w.pos, 1, alg="epie", alpha=1.0, beta=1.0, batch=1, it0=it,
                                       err=False)
                    best = min(best, api.nrmse(O, Ot, mask).item())
                per[m]["nrmse"].append(api.nrmse(O, Ot, mask).item())
                per[m]["nrmse_best"].append(best)
                H = _mtf(O.cpu().numpy(), O_true, mask_np)
                per[m]["mtf_nyquist"].append(float(H[-1]))
                below = np.nonzero(H < 0.5)[0]
                per[m]["mtf50"].append(float((below[0] + 0.5) / (2 * len(H))) if len(below) else 0.5)
        med = lambda xs: round(float(np.median(xs)), 4)
        rows.append({"bracket": list(tb), "flux": f, **{m: {k: med(v) for k, v in per[m].items()} for m in methods}})
        print(f"# t={tb} flux x{f}: " + "  ".join(f"{m} nrmse {rows[-1][m]['nrmse']} dev {rows[-1][m]['dev']} "
                                            f"snr {rows[-1][m]['snr']}" for m in methods), file=sys.stderr, flush=True)
    return {"metric": "object NRMSE after 50 ePIE iterations on MNF-fused data (small workload, 4 objects)",
            "value": rows[0]["mnf"]["nrmse"], "unit": "NRMSE", "n_gpus": 1, "steps": 4, "warmup": 0,
            "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic (seeded objects 1-4, Philox detector noise)",
            "config": {"workload": "small-64: 192^2 object, 64^2 probe r=16 known, 100 positions, brackets "
                                   "1/10/100 and 1/2/4, 12-bit, read noise 2, 4-level MNF; linear integration "
                                   "and shortest frame as baselines; flux as a multiple of half-scale in the "
                                   "shortest frame"},
            "comparison": rows,
            "metrics": "dev = ||F - C||/||C||; snr = 10 log10(sum C^2 / sum (F - C)^2) dB; bgvar = variance of F "
                       "where C < 1e-3 max C; nrmse / nrmse_best = final / best over 50 iterations; "
                       "mtf_nyquist = transfer of the final object in the last of 16 radial bins (0.47-0.5 "
                       "cycles/px), mtf50 = centre of the first bin below 0.5 (0.5 if none); medians"}


def run_broadband(args, api, synth, dev):
    """Discrete-spectrum data (Eq. 4) through the monochromatic engine: the
    warm-start geometry (64^2 probe in a 256^2 detector, 100 positions, known
    probe) measured with one line (the reference) or with the XUV source's two
    harmonics (9th and 11th of 515 nm, reference the 11th, weights 0.5/0.5),
    noise-free or through the 12-bit detector and MNF / linear fusion, then
    rPIE (mini-batch 10) for 100 iterations at the reference wavelength.
    On the noise-free data it also runs 200 rPIE iterations with the probe
    updated from iteration 10, once with one probe and once with two
    mixed-state modes (the second started as a weak odd copy of the probe).
    Reports the object NRMSE reached (median of four objects)."""
    import numpy as np
    import torch

    w = synth.warmstart_workload(0)
    P = w.probe()
    deltas = synth.default_deltas(w.levels, w.sigma_read)
    mask = None
    lines = {"one line": ([1.0], [1.0]), "two harmonics": ([1.0, 9.0 / 11.0], [0.5, 0.5])}
    rows = []
    for name, (scales, weights) in lines.items():
        res = {k: [] for k in ("clean", "mnf", "linear", "clean_probe_1mode", "clean_probe_2modes",
                               "err_1mode", "err_2modes")}
        for seed in range(1, 5):
            O_true = synth.make_object(w.M, seed)
            Ot = torch.from_numpy(O_true.astype(np.complex64)).to(dev)
            Pt = torch.from_numpy(P.astype(np.complex64)).to(dev)
            clean = api.broadband_forward(Ot, Pt, w.pos, w.Nd, scales, weights)
            s = synth.flux_scale(float(clean.max().item()), w.sat)
            raw = api.detector_expose(clean, w.t, s, w.sat, w.sigma_read, seed=104729 * seed + len(scales))
            if mask is None:
                mask_np = _illum_mask(P, w.pos, (w.M, w.M))
                mask = torch.from_numpy(mask_np.astype(np.uint8)).to(dev)
            Pk = torch.from_numpy((np.sqrt(s) * P).astype(np.complex64)).to(dev)
            data = {"clean": clean * s,
                    "mnf": api.fuse_exposures(raw, w.t, w.levels, sat=float(w.sat), delta=deltas),
                    "linear": api.fuse_linear(raw, w.t, float(w.sat))}
            for k, I in data.items():
                O = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
                api.ptycho_iterate(O, Pk, I.contiguous(), w.pos, 100, alg="rpie", alpha=0.1, batch=10, err=False)
                res[k].append(api.nrmse(O, Ot, mask).item())
            # probe refinement with one mode and with two mixed-state modes
            yy = (np.arange(w.Nw)[:, None] - w.Nw / 2.0) / (w.Nw / 4.0)
            P2 = np.stack([np.sqrt(s * 0.9) * P, np.sqrt(s * 0.1) * P * yy]).astype(np.complex64)
            for k, Pm in (("1mode", P2[:1]), ("2modes", P2)):
                O = torch.ones((w.M, w.M), dtype=torch.complex64, device=dev)
                Pt2 = torch.from_numpy(np.ascontiguousarray(Pm)).to(dev)
                e = api.ptycho_iterate_modes(O, Pt2, data["clean"].contiguous(), w.pos, 200, alg="rpie", alpha=0.1,
                                             beta=0.1, batch=10, update_probe=True, probe_start_iter=10)
                res["clean_probe_" + k].append(api.nrmse(O, Ot, mask).item())
                res["err_" + k].append(float(e[-1].item()))
        rows.append({"spectrum": name, "scales": scales, "weights": weights,
                     **{k: round(float(np.median(v)), 4) for k, v in res.items()}})
        print(f"# {name}: {rows[-1]}", file=sys.stderr, flush=True)
    return {"metric": "object NRMSE after 100 rPIE iterations, discrete-spectrum data (4 objects, median)",
            "note": "clean_probe_1mode / clean_probe_2modes: object NRMSE after 200 rPIE iterations on the noise-free "
                    "data with the probe updated from iteration 10, one probe or two mixed-state modes; err_*: "
                    "their final normalised Fourier errors",
            "value": rows[-1]["mnf"], "unit": "NRMSE", "n_gpus": 1, "steps": 4, "warmup": 0, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded objects 1-4, Philox detector noise)",
            "config": {"workload": "192^2 object, 64^2 probe r=16 known, 100 positions, 256^2 detector, "
                                   "t=1/10/100 12-bit, read noise 2; lines 515/11 and 515/9 nm, reference 515/11"},
            "comparison": rows}


def _illum_mask(P, pos, shape, frac=0.1):
    import numpy as np
    Nw = P.shape[0]
    ill = np.zeros(shape)
    P2 = np.abs(P) ** 2
    for y, x in pos:
        ill[y:y + Nw, x:x + Nw] += P2
    return ill >= frac * ill.max()


def run_unet(args, api, synth, dev):
    """The warm-start network's kernels alone: Adam training steps at batch 64
    and inference over 100 patterns, 256^2 inputs, widths 32/64/128/256, timed
    with events; value = training samples/s, roofline = training TFLOP/s
    (forward + input gradient + weight gradient flops of the layer shapes)
    against the dense bf16 MFMA peak."""
    import torch

    from paper_2608_01746_amd import warmstart as ws

    S = ws.setup()
    data = ws.simulate(S, range(5000, 5004), "fused", dev, relative=True)
    params = ws.init_params(ws.WIDTHS, 0, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    I, T = data["I"][:64].contiguous(), data["target"][:64].contiguous()
    for step in range(1, 4):
        api.unet_train_step(params, m, v, step, 1e-3, I, S.log_scale, T, ws.H, ws.WIDTHS)
    n_steps = max(args.steps, 10)

    def train():
        for k in range(n_steps):
            api.unet_train_step(params, m, v, 4 + k, 1e-3, I, S.log_scale, T, ws.H, ws.WIDTHS)

    t_train = ws._elapsed(train, dev) / n_steps
    I100 = data["I"][:100].contiguous()
    out = torch.empty((100, S.w.Nw, S.w.Nw, 2), dtype=torch.float32, device=dev)
    api.unet_forward(params, I100, S.log_scale, ws.H, ws.WIDTHS, out=out)
    t_inf = ws._elapsed(lambda: [api.unet_forward(params, I100, S.log_scale, ws.H, ws.WIDTHS, out=out)
                                 for _ in range(n_steps)], dev) / n_steps
    tf_train = 64 * ws.train_flops_per_sample(ws.H, ws.WIDTHS) / t_train / 1e12
    tf_inf = 100 * sum(ws.layer_flops(ws.H, ws.WIDTHS)) / t_inf / 1e12
    return {"metric": "U-Net training samples/s (256^2 inputs, batch 64, Adam)", "value": round(64 / t_train, 1),
            "unit": "samples/s", "n_gpus": 1, "steps": n_steps, "warmup": 3, "ms_per_step": round(t_train * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 (f32 accumulate, f32 master weights)", "data": "synthetic (simulated fused patterns)",
            "config": {"workload": "U-Net 32/64/128/256, 256^2 log-fused input -> 64^2 x 2 output, batch 64"},
            "roofline": {"bound": "mfma", "kernel": "whole training step", "achieved": round(tf_train, 1),
                         "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf_train / 2500.0, 4), "traffic": None},
            "inference": {"patterns": 100, "ms": round(t_inf * 1e3, 3), "tflops": round(tf_inf, 1),
                          "frac": round(tf_inf / 2500.0, 4)}}


def run_warmstart(args, api, synth, dev):
    """Learned warm start on the small geometry with a 256^2 detector: train
    the U-Net (excluded from the timed comparison), then for ten test objects
    time reaching object NRMSE 1e-2 from the network's stitched start and from
    a flat start.  The threshold is taken on noise-free patterns (see the
    note in the output); on MNF-fused noisy patterns the NRMSE reached after
    the same iteration budgets is reported beside it."""
    import numpy as np
    import torch

    from paper_2608_01746_amd import warmstart as ws

    S = ws.setup()
    params = ws.init_params(ws.WIDTHS, 0, dev)
    train_info = None
    if args.params_in:
        params.copy_(torch.from_numpy(np.load(args.params_in)).to(dev))
    else:
        tr = ws.simulate(S, range(5000, 5000 + args.train_objects), "fused", dev, relative=True)
        print(f"# training on {tr['I'].shape[0]} fused patterns for up to {args.train_seconds:.0f} s",
              file=sys.stderr, flush=True)
        train_info = ws.train(S, tr, params, epochs=args.epochs, time_budget=args.train_seconds,
                              log=lambda m: print("# " + m, file=sys.stderr, flush=True)
                              if m.split()[1].endswith("000") else None)
        del tr
        torch.cuda.empty_cache()
    if args.params_out:
        np.save(args.params_out, params.cpu().numpy())
    # inference throughput of the dominant kernels (one launch sequence per 100 patterns)
    te_clean = ws.simulate(S, range(9000, 9010), "clean", dev)
    I100 = te_clean["I"][:100]
    out = torch.empty((100, S.w.Nw, S.w.Nw, 2), dtype=torch.float32, device=dev)
    for _ in range(2):
        api.unet_forward(params, I100, S.log_scale, ws.H, ws.WIDTHS, out=out)
    t_inf = min(ws._elapsed(lambda: api.unet_forward(params, I100, S.log_scale, ws.H, ws.WIDTHS, out=out), dev)
                for _ in range(5))
    fwd_flops = sum(ws.layer_flops(ws.H, ws.WIDTHS))
    infer_tfs = 100 * fwd_flops / t_inf / 1e12
    # the network runs on a covering subset of the scan (farthest-point
    # sampling, corners at least --warm-spacing px apart); 0 = every window
    subset = ws.covering_subset(S.pos, args.warm_spacing) if args.warm_spacing > 0 else None
    res_c = ws.time_to_threshold(S, te_clean, params, tau=1e-2, max_plain=200, max_warm=50, sync=True,
                                 subset=subset)
    res_all = ws.time_to_threshold(S, te_clean, params, tau=1e-2, max_plain=200, max_warm=50, sync=True) \
        if subset is not None else res_c
    te_f = ws.simulate(S, range(9000, 9010), "fused", dev)
    res_f = ws.time_to_threshold(S, te_f, params, tau=1e-2, max_plain=200, max_warm=50, sync=True, subset=subset)
    def ratio_of(res):
        ok = [r for r in res if r.get("t_warm") is not None and r.get("t_plain") is not None]
        return ok, ((sum(r["t_plain"] for r in ok) / sum(r["t_warm"] for r in ok)) if ok else None)

    both, ratio = ratio_of(res_c)
    _, ratio_all = ratio_of(res_all)
    med = lambda xs: float(np.median(xs)) if xs else None
    per_obj = [{"n_plain": r["n_plain"], "n_warm": r.get("n_warm"), "nrmse_start": round(r["nrmse_init"], 4),
                "t_plain_ms": None if r.get("t_plain") is None else round(r["t_plain"] * 1e3, 3),
                "t_warm_ms": None if r.get("t_warm") is None else round(r["t_warm"] * 1e3, 3)} for r in res_c]
    fused = {"nrmse_flat_start": round(med([r["plain_curve"][0] for r in res_f]), 4),
             "nrmse_warm_start": round(med([r["warm_curve"][0] for r in res_f]), 4),
             "nrmse_plain_200": round(med([r["plain_curve"][-1] for r in res_f]), 4),
             "nrmse_plain_best": round(med([min(r["plain_curve"]) for r in res_f]), 4),
             "nrmse_warm_50": round(med([r["warm_curve"][-1] for r in res_f]), 4)}
    t_iter = med([r["t_iter"] for r in res_c])
    out_json = {
        "metric": "time-to-NRMSE 1e-2, warm vs plain (t_plain / t_warm)",
        "value": None if ratio is None else round(ratio, 3),
        "unit": "x",
        "n_gpus": 1,
        "steps": len(res_c),
        "warmup": 1,
        "ms_per_step": None if not both else round(1e3 * sum(r["t_warm"] for r in both) / len(both), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 network (f32 accumulate), f32 iterations",
        "data": "synthetic (seeded objects 5000.. for training, 9000..9009 for test)",
        "config": {"workload": "warm-start: 192^2 object, 64^2 probe r=16 known, 100 raster positions, "
                               "256^2 detector, rPIE B=10; U-Net 32/64/128/256 on 256^2 log patterns, "
                               "window-relative phase labels, phase-aligned stitching, network on a "
                               "covering subset of the windows",
                   "threshold": 1e-2, "max_plain": 200, "max_warm": 50,
                   "objects_reaching_in_both": len(both)},
        "roofline": {"bound": "mfma", "kernel": "U-Net forward (100 patterns)", "achieved": round(infer_tfs, 1),
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": round(infer_tfs / 2500.0, 4), "traffic": None,
                     "flops_per_launch_sequence": 100 * fwd_flops, "seconds": round(t_inf, 6)},
        "t_iter_ms": round(t_iter * 1e3, 4),
        "t_start_ms": round(med([r["t_start"] for r in res_c]) * 1e3, 3),
        "n_plain_median": med([r["n_plain"] for r in res_c if r["n_plain"] is not None]),
        "n_warm_median": med([r["n_warm"] for r in res_c if r.get("n_warm") is not None]),
        "network_windows": len(S.pos) if subset is None else int(len(subset)),
        "every_window": {"value": None if ratio_all is None else round(ratio_all, 3),
                         "nrmse_start_median": round(med([r["nrmse_init"] for r in res_all]), 4),
                         "n_warm_median": med([r["n_warm"] for r in res_all if r.get("n_warm") is not None]),
                         "t_start_ms": round(med([r["t_start"] for r in res_all]) * 1e3, 3)},
        "per_object": per_obj,
        "fused_noisy_patterns": fused,
        "note": "MNF-fused patterns of this detector model hold every reconstruction at NRMSE ~0.2 (fusion "
                "deviation), so the 1e-2 threshold is timed on the noise-free patterns the fusion returns in "
                "the unsaturated, noise-free limit; the network is trained on fused noisy patterns only. "
                "t_warm = network inference + aligned stitching + n_warm iterations, one event-timed run; "
                "t_plain = n_plain iterations from a flat start, one event-timed run",
    }
    if train_info is not None:
        tf = train_info["samples_per_s"] * ws.train_flops_per_sample(ws.H, ws.WIDTHS) / 1e12
        out_json["training"] = {"samples": train_info["steps"] * 64, "seconds": round(train_info["seconds"], 1),
                                "samples_per_s": round(train_info["samples_per_s"], 1),
                                "tflops": round(tf, 1), "final_loss": train_info["history"][-1][1]
                                if train_info["history"] else None}
    if not args.no_cpu:
        out_json["cpu_baseline"] = warm_cpu_baseline(S, te_clean, args.cpu_seconds)
    return out_json


def warm_cpu_baseline(S, data, seconds):
    """The float64 oracle's plain rPIE on the first test object: seconds per
    iteration over a bounded number of iterations, scaled to that object's
    iteration count to NRMSE 1e-2."""
    import numpy as np

    from oracle import ptycho as optycho
    w = S.w
    J = len(S.pos)
    I = data["I"][:J].cpu().numpy().astype(np.float64)
    s = data["scales"][0]
    O_true = data["objects"][0]
    mask = optycho.illumination_mask(S.P, S.pos, O_true.shape)
    prm = optycho.PtychoParams(alg="rpie", alpha=0.1, batch=w.batch, update_probe=False)
    O = np.ones_like(O_true)
    P = np.sqrt(s) * S.P
    t0 = time.perf_counter()
    it = 0
    reached = None
    while time.perf_counter() - t0 < seconds and it < 200:
        O, _, _ = optycho.iterate(O, P, I, S.pos, 1, prm, it0=it)
        it += 1
        if optycho.nrmse(O, O_true, mask) <= 1e-2:
            reached = it
            break
    dt = (time.perf_counter() - t0) / it
    return {"value": round(dt * (reached if reached else it), 3), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"plain rPIE to NRMSE 1e-2 on test object 9000 in float64 NumPy: {it} iterations "
                      f"({'reached' if reached else 'not reached'}), {dt * 1e3:.0f} ms each"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=None, help="iterations per step (200 lab, 20 multiscan)")
    ap.add_argument("--workload", choices=["lab", "subpixel", "small", "multiscan", "grad", "warmstart", "batch-sweep",
                                           "fusion-compare", "unet", "broadband"], default="lab")
    ap.add_argument("--train-seconds", type=float, default=240.0, help="warm start: training time budget")
    ap.add_argument("--train-objects", type=int, default=500, help="warm start: training objects x 100 patterns")
    ap.add_argument("--epochs", type=float, default=100.0, help="warm start: epoch cap")
    ap.add_argument("--params-in", default=None, help="warm start: load trained parameters (.npy) instead")
    ap.add_argument("--params-out", default=None, help="warm start: save the trained parameters (.npy)")
    ap.add_argument("--warm-spacing", type=float, default=10.0,
                    help="warm start: minimum corner distance (px) of the windows the network runs on; 0 = all")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="keep the default launch shapes instead of the tuned ones")
    ap.add_argument("--graph", action="store_true", help="lab: capture each step's iterations in a hipGraph")
    ap.add_argument("--three-launch", action="store_true",
                    help="lab: three launches per mini-batch (object update fused with the next exit waves)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 256 MiB device copy (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        return 2
    if args.iters is None:
        args.iters = {"lab": 200, "subpixel": 200, "small": 50}.get(args.workload, 20)

    import torch

    from paper_2608_01746_amd import api, synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    run = {"lab": run_lab, "subpixel": run_lab, "small": run_lab, "multiscan": run_multiscan, "grad": run_grad, "warmstart": run_warmstart,
           "batch-sweep": run_batch_sweep, "fusion-compare": run_fusion_compare, "unet": run_unet,
           "broadband": run_broadband}[args.workload]
    out = run(args, api, synth, dev)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
