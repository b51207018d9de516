"""Seeded synthetic inputs for the HDR-fused ptychography path.

This module draws objects, probes, scan positions, position orders and
detector noise.  It holds none of the method's arithmetic: it never fuses,
transforms or reconstructs anything.  The clean far-field intensities that
the noise model needs are computed by the caller (the test suite uses the
CPU reference, the benchmark uses the library's forward-model entry point)
and passed in.

Workload recipes (sizes, value ranges, overlap, exposure ladders) follow the
paper's acquisition description: a bracket of K exposures per scan position
(Results 2.1, Eq. 1), spiral or raster scans at roughly 80 % overlap
(Methods 3.1), detector saturation and read noise (Results 2.3, Eq. 4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy.ndimage import gaussian_filter

# ---------------------------------------------------------------------------
# Objects and probes
# ---------------------------------------------------------------------------


def make_object(M: int, seed: int, Mx: Optional[int] = None, smooth: float = 3.0) -> np.ndarray:
    """Complex128 object: amplitude in [0.5, 1], phase in [-pi/2, pi/2].

    Two standard-normal fields are smoothed with a periodic Gaussian
    (sigma = ``smooth`` px) and min-max scaled to [0, 1] (a, b); the object
    is (0.5 + 0.5 a) * exp(i pi (b - 0.5)).
    """
    Mx = M if Mx is None else Mx
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((2, M, Mx))
    out = []
    for k in range(2):
        g = gaussian_filter(f[k], smooth, mode="wrap")
        g = (g - g.min()) / (g.max() - g.min())
        out.append(g)
    a, b = out
    return (0.5 + 0.5 * a) * np.exp(1j * np.pi * (b - 0.5))


def make_probe(Nw: int, radius: float, phase_max: float) -> np.ndarray:
    """Hard circular aperture of ``radius`` px centred at ((Nw-1)/2, (Nw-1)/2)
    carrying a quadratic (defocus-like) phase phase_max * (rho / radius)^2."""
    y, x = np.mgrid[0:Nw, 0:Nw].astype(np.float64)
    c = (Nw - 1) / 2.0
    rho = np.hypot(y - c, x - c)
    ap = (rho <= radius).astype(np.float64)
    return ap * np.exp(1j * phase_max * (rho / radius) ** 2)


def flat_probe_guess(Nw: int, radius: float, energy: float) -> np.ndarray:
    """Blind-mode starting probe: the aperture with a flat phase, scaled so
    that sum |P|^2 equals ``energy``."""
    p = make_probe(Nw, radius, 0.0)
    return p * math.sqrt(energy / np.sum(np.abs(p) ** 2))


# ---------------------------------------------------------------------------
# Scan positions (integer top-left corners (y, x) of each window in O)
# ---------------------------------------------------------------------------


def raster_positions(n_side: int, step: int, offset: int, jitter: int = 0,
                     seed: int = 0) -> np.ndarray:
    """n_side x n_side raster with ``step`` px pitch starting at ``offset``,
    plus an integer jitter uniform in [-jitter, jitter] per coordinate."""
    iy, ix = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    pos = np.stack([offset + step * iy.ravel(), offset + step * ix.ravel()], axis=1)
    if jitter:
        rng = np.random.default_rng(seed)
        pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    return pos.astype(np.int32)


def fermat_positions(J: int, c: float, centre: float) -> np.ndarray:
    """Fermat spiral (golden-angle) scan: p_n = centre + c sqrt(n) (cos n g, sin n g),
    g = pi (3 - sqrt 5), rounded to the nearest integer."""
    n = np.arange(J, dtype=np.float64)
    g = math.pi * (3.0 - math.sqrt(5.0))
    r = c * np.sqrt(n)
    y = np.rint(centre + r * np.sin(n * g))
    x = np.rint(centre + r * np.cos(n * g))
    return np.stack([y, x], axis=1).astype(np.int32)


def fermat_positions_real(J: int, c: float, centre: float) -> np.ndarray:
    """The Fermat spiral of fermat_positions without rounding, float32 [J][2]."""
    n = np.arange(J, dtype=np.float64)
    g = math.pi * (3.0 - math.sqrt(5.0))
    r = c * np.sqrt(n)
    return np.stack([centre + r * np.sin(n * g), centre + r * np.cos(n * g)], axis=1).astype(np.float32)


def random_orders(J: int, n_iter: int, seed: int) -> np.ndarray:
    """One position permutation per iteration, int32 [n_iter][J]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(J) for _ in range(n_iter)]).astype(np.int32)


# ---------------------------------------------------------------------------
# Detector model: exposures of a clean intensity
# ---------------------------------------------------------------------------


def flux_scale(clean_max: float, sat: float) -> float:
    """Counts per unit |Psi|^2 at t = 1 so that the brightest clean pixel of
    the shortest exposure sits at half the full scale."""
    return (sat / 2.0) / float(clean_max)


def expose(clean: np.ndarray, t: Sequence[float], sat: int, sigma_read: float,
           seed: int, scale: float) -> np.ndarray:
    """uint16 exposure stack [J][K][H][W] from clean intensities [J][H][W].

    counts_k = clip(rint(Poisson(scale * t_k * clean) + N(0, sigma_read^2)), 0, sat)
    """
    rng = np.random.default_rng(seed)
    J = clean.shape[0]
    K = len(t)
    out = np.empty((J, K) + clean.shape[1:], dtype=np.uint16)
    for j in range(J):
        lam_base = np.maximum(clean[j].astype(np.float64), 0.0) * scale
        for k in range(K):
            lam = lam_base * float(t[k])
            c = rng.poisson(np.minimum(lam, 1e15)).astype(np.float64)
            if sigma_read > 0:
                c += rng.normal(0.0, sigma_read, size=c.shape)
            out[j, k] = np.clip(np.rint(c), 0, sat).astype(np.uint16)
    return out


def default_deltas(levels: int, sigma_read: float) -> List[float]:
    """Per-band quantisation steps in ADU: sigma_read at the coarsest band
    (l = L-1), halving for each finer band."""
    return [sigma_read * 2.0 ** (l - (levels - 1)) for l in range(levels)]


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Workload:
    name: str
    M: int                  # object side (square)
    Nw: int                 # probe window side
    Nd: int                 # detector side
    radius: float
    phase_max: float
    pos: np.ndarray         # int32 [J][2]
    t: List[float]
    sat: int
    sigma_read: float
    levels: int
    seed: int
    batch: int
    n_iter: int
    alg: str                # 'epie' | 'rpie'

    @property
    def J(self) -> int:
        return int(self.pos.shape[0])

    def object(self) -> np.ndarray:
        return make_object(self.M, self.seed)

    def probe(self) -> np.ndarray:
        return make_probe(self.Nw, self.radius, self.phase_max)


def small_workload() -> Workload:
    """192^2 object, 64^2 probe (r = 16, phase pi), 10 x 10 raster step 8,
    exposures 1/10/100 at 12 bits, read noise 2, 4-level fusion, ePIE B = 1."""
    return Workload("small-64", 192, 64, 64, 16.0, math.pi,
                    raster_positions(10, 8, 28), [1.0, 10.0, 100.0], 4095, 2.0,
                    4, 1, 1, 50, "epie")


def lab_workload() -> Workload:
    """1024^2 object, 256^2 probe (r = 64, defocus 3 pi), 20 x 20 raster step 32
    with +-2 px jitter, exposures 1..1e4 at 16 bits, read noise 3, 6-level
    fusion, rPIE with mini-batch 32, 200 iterations."""
    return Workload("lab-256", 1024, 256, 256, 64.0, 3 * math.pi,
                    raster_positions(20, 32, 80, jitter=2, seed=2),
                    [1.0, 10.0, 100.0, 1e3, 1e4], 65535, 3.0, 6, 2, 32, 200, "rpie")


def lab_subpixel_workload() -> Workload:
    """lab-256 at real positions: 400 unrounded Fermat-spiral positions with
    the raster's density (one position per 32^2 px, c = 32 / sqrt(pi))
    around the object centre; everything else as lab-256."""
    w = lab_workload()
    pos = fermat_positions_real(400, 32.0 / math.sqrt(math.pi), (1024 - 256) / 2.0)
    return dataclasses.replace(w, name="lab-256-subpixel", pos=pos)


def gradient_workload() -> Workload:
    """2048^2 object, 512^2 probe (r = 128, defocus), 1000-position Fermat
    spiral (c = 24), 5 exposures at 16 bits, 6-level fusion."""
    return Workload("grad-512", 2048, 512, 512, 128.0, 3 * math.pi,
                    fermat_positions(1000, 24.0, (2048 - 512) / 2.0),
                    [1.0, 10.0, 100.0, 1e3, 1e4], 65535, 3.0, 6, 4, 32, 1, "rpie")


def roundup(x: float, m: int) -> int:
    return int(math.ceil(x / m) * m)


def multiscan_workloads(n_scans: int = 64, base_seed: int = 3000) -> List[Workload]:
    """Independent scans of uneven sizes: N uniform in {128,192,256,384,512},
    J uniform in [50, 1000] on a Fermat spiral with c = N/20, K uniform in {3,4,5}."""
    out = []
    for s in range(n_scans):
        rng = np.random.default_rng(base_seed + s)
        N = int(rng.choice([128, 192, 256, 384, 512]))
        J = int(rng.integers(50, 1001))
        K = int(rng.integers(3, 6))
        c = N / 20.0
        M = roundup(N + 2 * c * math.sqrt(J) + 2, 16)
        pos = fermat_positions(J, c, (M - N) / 2.0)
        out.append(Workload(f"scan{s}-{N}", M, N, N, N / 4.0, 3 * math.pi, pos,
                            [10.0 ** k for k in range(K)], 65535, 3.0, 4,
                            base_seed + s, 32, 20, "rpie"))
    return out


def warmstart_workload(seed: int) -> Workload:
    """Small-workload geometry with the 64^2 exit wave zero-padded into a
    256^2 detector (4x oversampling); rPIE with mini-batch 10."""
    w = small_workload()
    return Workload(f"warm-{seed}", 192, 64, 256, 16.0, math.pi, w.pos, w.t, w.sat,
                    w.sigma_read, 4, seed, 10, 200, "rpie")
