"""Python binding of libmnfpty: argument marshalling from torch tensors
(device memory, streams) to the C ABI.  Every computation runs in the
library's HIP kernels; this module only checks shapes, dtypes and devices,
passes pointers and raises on error codes."""
from __future__ import annotations

import ctypes
import threading
from typing import Optional, Sequence

import numpy as np
import torch

from . import lib as _L


class MnfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_L.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_ctx_lock = threading.Lock()
_contexts = {}


def _ctx(device: torch.device) -> ctypes.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    with _ctx_lock:
        c = _contexts.get(idx)
        if c is None:
            lib = _L.load()
            c = ctypes.c_void_p()
            rc = lib.mnf_create(ctypes.byref(c), idx)
            if rc != 0:
                raise MnfError(rc, f"mnf_create({idx}) failed: {lib.mnf_last_error(None).decode()}")
            _contexts[idx] = c
        return c


def _check(rc: int, ctx) -> None:
    if rc != 0:
        msg = _L.load().mnf_last_error(ctx)
        raise MnfError(rc, msg.decode() if msg else "")


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype, ndim: int) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if t.dim() != ndim or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {ndim}-D tensor, got shape {tuple(t.shape)}")


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _host_i32(a, shape_tail, name) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    if arr.shape[1:] != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [*]{list(shape_tail)}, got {arr.shape}")
    return arr


def _host_f32(a, shape_tail, name) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if arr.ndim != 1 + len(shape_tail) or arr.shape[1:] != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [*]{list(shape_tail)}, got {arr.shape}")
    return arr


def _f32p(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _i32p(arr: Optional[np.ndarray]):
    if arr is None:
        return None
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def supported_sizes():
    lib = _L.load()
    buf = (ctypes.c_int32 * 32)()
    n = lib.mnf_supported_sizes(buf, 32)
    return [buf[i] for i in range(n)]


# ------------------------------------------------------------------ fusion

def fuse_exposures(raw: torch.Tensor, t: Sequence[float], levels: int, mu: float = 0.5,
                   sigma: float = 0.2, sat: float = 65535.0, dark: float = 0.0,
                   delta: Sequence[float] = (), radiometric: bool = True,
                   return_weights: bool = False, out: Optional[torch.Tensor] = None,
                   contrast_exp: float = 0.0):
    """MNF fusion of raw[J][K][H][W] (uint16 counts) -> fused float32 [J][H][W].
    contrast_exp > 0 adds the optional Laplacian-contrast factor to the weights
    (0, the default, is the paper's weight)."""
    _dev(raw, "raw", (torch.uint16, torch.int16), 4)
    J, K, H, W = raw.shape
    if len(t) != K:
        raise ValueError("one exposure time per exposure")
    if len(delta) > 16:
        raise ValueError("at most 16 quantisation steps")
    if out is None:
        out = torch.empty((J, H, W), dtype=torch.float32, device=raw.device)
    else:
        _dev(out, "out", torch.float32, 3)
    wts = torch.empty((J, K, H, W), dtype=torch.float32, device=raw.device) if return_weights else None
    prm = _L.FuseParamsC()
    prm.levels, prm.mu, prm.sigma, prm.sat, prm.dark = int(levels), mu, sigma, sat, dark
    for i, d in enumerate(delta):
        prm.delta[i] = float(d)
    prm.radiometric = 1 if radiometric else 0
    prm.contrast_exp = float(contrast_exp)
    tt = (ctypes.c_float * K)(*[float(x) for x in t])
    ctx = _ctx(raw.device)
    rc = _L.load().fuse_exposures(ctx, _ptr(raw), tt, J, K, H, W, ctypes.byref(prm), _ptr(out), _ptr(wts),
                                  _stream(raw.device))
    _check(rc, ctx)
    return (out, wts) if return_weights else out


def fuse_linear(raw: torch.Tensor, t: Sequence[float], sat: float, dark: float = 0.0, mode: str = "linear",
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Linear baselines of raw[J][K][H][W]: 'linear' (rate over unsaturated frames, in counts of
    the shortest exposure) or 'shortest' (the shortest frame alone) -> float32 [J][H][W]."""
    _dev(raw, "raw", (torch.uint16, torch.int16), 4)
    J, K, H, W = raw.shape
    if len(t) != K:
        raise ValueError("one exposure time per exposure")
    if out is None:
        out = torch.empty((J, H, W), dtype=torch.float32, device=raw.device)
    else:
        _dev(out, "out", torch.float32, 3)
    tt = (ctypes.c_float * K)(*[float(x) for x in t])
    ctx = _ctx(raw.device)
    rc = _L.load().fuse_linear(ctx, _ptr(raw), tt, J, K, H, W, float(sat), float(dark),
                               {"linear": 0, "shortest": 1}[mode], _ptr(out), _stream(raw.device))
    _check(rc, ctx)
    return out


# ----------------------------------------------------------- forward model

def ptycho_forward(O: torch.Tensor, P: torch.Tensor, pos, Nd: int,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Detector-centred |F(P O_j)|^2 for every window corner in pos [J][2]."""
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 2)
    posa = _host_i32(pos, (2,), "pos")
    J = posa.shape[0]
    if out is None:
        out = torch.empty((J, Nd, Nd), dtype=torch.float32, device=O.device)
    else:
        _dev(out, "out", torch.float32, 3)
    ctx = _ctx(O.device)
    rc = _L.load().ptycho_forward(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), P.shape[0], Nd,
                                  _i32p(posa), J, _ptr(out), _stream(O.device))
    _check(rc, ctx)
    return out


def ptycho_forward_subpixel(O: torch.Tensor, P: torch.Tensor, pos, Nd: int,
                            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """As ptycho_forward at real positions pos [J][2] (float32): the fraction of
    each position translates the probe in Fourier space."""
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 2)
    posa = _host_f32(pos, (2,), "pos")
    J = posa.shape[0]
    if out is None:
        out = torch.empty((J, Nd, Nd), dtype=torch.float32, device=O.device)
    else:
        _dev(out, "out", torch.float32, 3)
    ctx = _ctx(O.device)
    rc = _L.load().ptycho_forward_subpixel(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), P.shape[0], Nd,
                                           _f32p(posa), J, _ptr(out), _stream(O.device))
    _check(rc, ctx)
    return out


def ptycho_forward_modes(O: torch.Tensor, P: torch.Tensor, pos, Nd: int,
                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Detector-centred sum_m |F(P_m O_j)|^2 for probe modes P [M][Nw][Nw]."""
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 3)
    if P.shape[1] != P.shape[2]:
        raise ValueError("probe modes must be [M][Nw][Nw]")
    posa = _host_i32(pos, (2,), "pos")
    J = posa.shape[0]
    if out is None:
        out = torch.empty((J, Nd, Nd), dtype=torch.float32, device=O.device)
    else:
        _dev(out, "out", torch.float32, 3)
    ctx = _ctx(O.device)
    rc = _L.load().ptycho_forward_modes(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), P.shape[0], P.shape[1], Nd,
                                        _i32p(posa), J, _ptr(out), _stream(O.device))
    _check(rc, ctx)
    return out


# ----------------------------------------------------------- reconstruction

ALGS = {"epie": 0, "rpie": 1}


def ptycho_iterate(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, n_iter: int,
                   alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1, batch: int = 1,
                   update_probe: bool = False, probe_start_iter: int = 0, order=None, it0: int = 0,
                   err: bool = True, graph: bool = False) -> Optional[torch.Tensor]:
    """Run n_iter mini-batched ePIE/rPIE iterations, updating O and P in place.
    Returns the float64 error per iteration (device tensor) if err."""
    return _iterate("ptycho_iterate", _host_i32(pos, (2,), "pos"), _i32p, O, P, I, n_iter, alg, alpha, beta,
                    batch, update_probe, probe_start_iter, order, it0, err, graph)


def ptycho_iterate_noalloc(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, n_iter: int,
                           alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1, batch: int = 1,
                           update_probe: bool = False, probe_start_iter: int = 0, order=None, it0: int = 0,
                           err: bool = True) -> Optional[torch.Tensor]:
    """ptycho_iterate through the entry point that allocates no device memory
    (its scratch is the library's static 48 MiB array).  The returned error
    tensor, when requested, is allocated here by torch, not by the library."""
    return _iterate("ptycho_iterate_noalloc", _host_i32(pos, (2,), "pos"), _i32p, O, P, I, n_iter, alg, alpha,
                    beta, batch, update_probe, probe_start_iter, order, it0, err, False)


def ptycho_iterate_subpixel(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, n_iter: int,
                            alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1, batch: int = 1,
                            update_probe: bool = False, probe_start_iter: int = 0, order=None, it0: int = 0,
                            err: bool = True, graph: bool = False) -> Optional[torch.Tensor]:
    """ptycho_iterate at real positions pos [J][2] (float32): translated
    probes in the exit waves and object numerators, probe numerators
    translated back."""
    return _iterate("ptycho_iterate_subpixel", _host_f32(pos, (2,), "pos"), _f32p, O, P, I, n_iter, alg, alpha,
                    beta, batch, update_probe, probe_start_iter, order, it0, err, graph)


def ptycho_iterate_modes(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, n_iter: int,
                         alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1, batch: int = 1,
                         update_probe: bool = False, probe_start_iter: int = 0, order=None, it0: int = 0,
                         err: bool = True, graph: bool = False) -> Optional[torch.Tensor]:
    """ptycho_iterate with mixed-state probe modes P [M][Nw][Nw] (updated in
    place with O)."""
    return _iterate("ptycho_iterate_modes", _host_i32(pos, (2,), "pos"), _i32p, O, P, I, n_iter, alg, alpha,
                    beta, batch, update_probe, probe_start_iter, order, it0, err, graph, modes=True)


def _iterate(entry, posa, posp, O, P, I, n_iter, alg, alpha, beta, batch, update_probe, probe_start_iter, order,
             it0, err, graph, modes=False):
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 3 if modes else 2)
    if modes and P.shape[1] != P.shape[2]:
        raise ValueError("probe modes must be [M][Nw][Nw]")
    _dev(I, "I", torch.float32, 3)
    J = posa.shape[0]
    if I.shape[0] != J or I.shape[1] != I.shape[2]:
        raise ValueError("I must be [J][Nd][Nd]")
    orda = None
    if order is not None:
        orda = _host_i32(order, (J,), "order")
        if orda.shape[0] != n_iter:
            raise ValueError("order must have one row per iteration")
    prm = _L.PtychoParamsC(ALGS[alg], alpha, beta, batch, 1 if update_probe else 0, probe_start_iter, it0,
                           1 if graph else 0)
    e = torch.empty(max(n_iter, 1), dtype=torch.float64, device=O.device) if err else None
    ctx = _ctx(O.device)
    psize = (P.shape[0], P.shape[1]) if modes else (P.shape[0],)
    rc = getattr(_L.load(), entry)(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), *psize, _ptr(I),
                                   I.shape[1], posp(posa), J, _i32p(orda), n_iter, ctypes.byref(prm),
                                   _ptr(e), _stream(O.device))
    _check(rc, ctx)
    return e[:n_iter] if err else None


def ptycho_iterate_many(scans, n_iter: int, alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1,
                        batch: int = 32, update_probe: bool = False, probe_start_iter: int = 0, it0: int = 0,
                        err: bool = True, graph: bool = True):
    """Iterate many independent scans in one call.  `scans` is a list of dicts
    with keys O, P, I (tensors), pos (host [J][2]) and optionally order
    ([n_iter][J]).  O and P are updated in place; returns the per-scan error
    tensors (float64 [n_iter]) if err."""
    if not scans:
        raise ValueError("no scans")
    arr = (_L.PtychoScanC * len(scans))()
    keep = []
    errs = []
    dev = scans[0]["O"].device
    for k, sc in enumerate(scans):
        O, P, I = sc["O"], sc["P"], sc["I"]
        _dev(O, "O", torch.complex64, 2)
        _dev(P, "P", torch.complex64, 2)
        _dev(I, "I", torch.float32, 3)
        if O.device != dev or P.device != dev or I.device != dev:
            raise ValueError("all scans must live on one device")
        posa = _host_i32(sc["pos"], (2,), "pos")
        J = posa.shape[0]
        orda = None
        if sc.get("order") is not None:
            orda = _host_i32(sc["order"], (J,), "order")
            if orda.shape[0] != n_iter:
                raise ValueError("order must have one row per iteration")
        e = torch.empty(max(n_iter, 1), dtype=torch.float64, device=dev) if err else None
        errs.append(e[:n_iter] if err else None)
        keep += [posa, orda]
        arr[k] = _L.PtychoScanC(O.data_ptr(), O.shape[0], O.shape[1], P.data_ptr(), P.shape[0], I.data_ptr(),
                                I.shape[1], _i32p(posa), J, _i32p(orda), e.data_ptr() if err else None)
    prm = _L.PtychoParamsC(ALGS[alg], alpha, beta, batch, 1 if update_probe else 0, probe_start_iter, it0,
                           1 if graph else 0)
    ctx = _ctx(dev)
    rc = _L.load().ptycho_iterate_many(ctx, arr, len(scans), n_iter, ctypes.byref(prm), _stream(dev))
    _check(rc, ctx)
    return errs if err else None


PLAN_INFO_KEYS = ("launches", "slots", "groups", "object_tiles", "max_launch_slots", "pattern_scratch_bytes",
                  "size_classes")


def plan_info(scans, n_iter: int, alg: str = "rpie", alpha: float = 0.1, beta: float = 0.1, batch: int = 32,
              update_probe: bool = False, probe_start_iter: int = 0, context_device=None) -> dict:
    """Validate and plan a ptycho_iterate_many call on the host, with no device
    work (no GPU needed).  `scans` is a list of dicts with the shapes
    My, Mx, Nw, Nd, the host positions pos [J][2] and optionally order
    [n_iter][J]; the library is handed placeholder device addresses, which
    the planner never dereferences.  Raises MnfError as the call itself
    would (same checks and codes).  context_device: take the launch shapes
    set on that device's context instead of the defaults."""
    if not scans:
        raise ValueError("no scans")
    arr = (_L.PtychoScanC * len(scans))()
    keep = []
    for k, sc in enumerate(scans):
        posa = _host_i32(sc["pos"], (2,), "pos")
        J = posa.shape[0]
        orda = _host_i32(sc["order"], (J,), "order") if sc.get("order") is not None else None
        if J == 0:
            raise ValueError("a scan needs at least one position")
        if orda is not None and orda.shape[0] != n_iter:
            raise ValueError("order must have one row per iteration")
        keep += [posa, orda]
        arr[k] = _L.PtychoScanC(8, int(sc["My"]), int(sc["Mx"]), 8, int(sc["Nw"]), 8, int(sc["Nd"]), _i32p(posa),
                                J, _i32p(orda), None)
    prm = _L.PtychoParamsC(ALGS[alg], alpha, beta, batch, 1 if update_probe else 0, probe_start_iter, 0, 0)
    ctx = _ctx(torch.device(context_device)) if context_device is not None else None
    info = (ctypes.c_int64 * len(PLAN_INFO_KEYS))()
    rc = _L.load().ptycho_plan_info(ctx, arr, len(scans), int(n_iter), ctypes.byref(prm), info, len(info))
    _check(rc, ctx)
    return dict(zip(PLAN_INFO_KEYS, list(info)))


# ------------------------------------------------------------------ adjoint

LOSSES = {"poisson": 0, "amplitude": 1}


def ptycho_grad(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, kind: str = "poisson",
                eps: float = 1e-6, batch: int = 32, upstream=None, need_gO: bool = True,
                need_gP: bool = True):
    """(loss float64 device scalar, gO or None, gP or None).  `upstream` scales
    the gradients: None (1), a float, or a float64 device scalar tensor that
    the kernels read in place (no device-to-host copy)."""
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 2)
    _dev(I, "I", torch.float32, 3)
    posa = _host_i32(pos, (2,), "pos")
    J = posa.shape[0]
    loss = torch.empty((), dtype=torch.float64, device=O.device)
    gO = torch.empty_like(O) if need_gO else None
    gP = torch.empty_like(P) if need_gP else None
    if upstream is not None and not isinstance(upstream, torch.Tensor):
        upstream = torch.tensor(float(upstream), dtype=torch.float64, device=O.device)
    if upstream is not None:
        if upstream.device != O.device or upstream.dtype != torch.float64 or upstream.numel() != 1:
            raise ValueError("upstream must be a float64 scalar on the device of O")
        upstream = upstream.contiguous()
    ctx = _ctx(O.device)
    rc = _L.load().ptycho_grad(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), P.shape[0], _ptr(I),
                               I.shape[1], _i32p(posa), J, LOSSES[kind], eps, batch, _ptr(upstream),
                               _ptr(loss), _ptr(gO), _ptr(gP), _stream(O.device))
    _check(rc, ctx)
    return loss, gO, gP


def ptycho_descend(O: torch.Tensor, P: torch.Tensor, I: torch.Tensor, pos, n_steps: int, kind: str = "poisson",
                   eps: float = 1e-6, batch: int = 32, eta_O: float = 0.0, eta_P: float = 0.0,
                   update_probe: bool = True):
    """Gradient descent with backtracking on the ptycho_grad loss, O and P
    updated in place.  Returns (losses float64 [n_steps] on the device, the
    loss of each pass; eta float64 [2] on the device, the step sizes at the
    end, halvings included).  Step sizes of 0 start from the curvature bound
    of the starting O and P."""
    _dev(O, "O", torch.complex64, 2)
    _dev(P, "P", torch.complex64, 2)
    _dev(I, "I", torch.float32, 3)
    posa = _host_i32(pos, (2,), "pos")
    J = posa.shape[0]
    losses = torch.empty((max(int(n_steps), 0),), dtype=torch.float64, device=O.device)
    eta = torch.empty((2,), dtype=torch.float64, device=O.device)
    ctx = _ctx(O.device)
    rc = _L.load().ptycho_descend(ctx, _ptr(O), O.shape[0], O.shape[1], _ptr(P), P.shape[0], _ptr(I), I.shape[1],
                                  _i32p(posa), J, LOSSES[kind], eps, batch, int(n_steps), float(eta_O), float(eta_P),
                                  1 if update_probe else 0, _ptr(losses) if n_steps > 0 else None, _ptr(eta),
                                  _stream(O.device))
    _check(rc, ctx)
    return losses, eta


def status(device="cuda:0") -> int:
    """Wait for the device's current stream and return the numerical status
    recorded since the last call (0, MNF_ENONFINITE or MNF_EDIVERGED); the
    record is cleared."""
    dev = torch.device(device)
    ctx = _ctx(dev)
    rc = _L.load().mnf_status(ctx, _stream(dev))
    if rc not in (0, _L.MNF_ENONFINITE, _L.MNF_EDIVERGED):
        _check(rc, ctx)
    return rc


def check_status(device="cuda:0") -> None:
    """Raise MnfError if a non-finite value or divergence was recorded."""
    dev = torch.device(device)
    ctx = _ctx(dev)
    _check(_L.load().mnf_status(ctx, _stream(dev)), ctx)


# ------------------------------------------------------------ launch timing

def profile(classes, device="cuda:0", every: int = 1) -> None:
    """Time the launches of the named kernel classes with HIP events (empty /
    None disables): every launch, or with `every` > 1 the first and then
    every `every`-th launch of each class (profile_read then reports the
    timed launches only)."""
    mask = 0
    for c in classes or ():
        mask |= 1 << _L.KERNEL_CLASSES.index(c)
    dev = torch.device(device)
    ctx = _ctx(dev)
    if every == 1:
        _check(_L.load().mnf_profile(ctx, mask), ctx)
    else:
        _check(_L.load().mnf_profile_sampled(ctx, mask, int(every)), ctx)


def profile_reset(device="cuda:0") -> None:
    ctx = _ctx(torch.device(device))
    _check(_L.load().mnf_profile_reset(ctx), ctx)


def profile_read(device="cuda:0") -> dict:
    """{class: (launches, total_ms)} for every class with launches."""
    ctx = _ctx(torch.device(device))
    out = {}
    for i, name in enumerate(_L.KERNEL_CLASSES):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        _check(_L.load().mnf_profile_read(ctx, i, ctypes.byref(n), ctypes.byref(ms)), ctx)
        if n.value:
            out[name] = (int(n.value), float(ms.value))
    return out


# ------------------------------------------------------------ warm start

def unet_shape(H: int, widths):
    s = _L.UnetShapeC()
    s.H = int(H)
    for i, w in enumerate(widths):
        s.widths[i] = int(w)
    return s


def unet_param_count(H: int, widths) -> int:
    return int(_L.load().unet_param_count(ctypes.byref(unet_shape(H, widths))))


def unet_forward(params: torch.Tensor, I: torch.Tensor, log_scale: float, H: int, widths,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Network output [n][H/4][H/4][2] (amplitude, phase) for fused patterns I [n][H][H]."""
    _dev(params, "params", torch.float32, 1)
    _dev(I, "I", torch.float32, 3)
    n = I.shape[0]
    if out is None:
        out = torch.empty((n, H // 4, H // 4, 2), dtype=torch.float32, device=I.device)
    shp = unet_shape(H, widths)
    ctx = _ctx(I.device)
    rc = _L.load().unet_forward(ctx, ctypes.byref(shp), _ptr(params), _ptr(I), float(log_scale), n, _ptr(out),
                                _stream(I.device))
    _check(rc, ctx)
    return out


def unet_train_step(params: torch.Tensor, adam_m: Optional[torch.Tensor], adam_v: Optional[torch.Tensor],
                    step: int, lr: float, I: torch.Tensor, log_scale: float, target: torch.Tensor, H: int, widths,
                    grads: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One Adam step (or only gradients when adam_m/adam_v are None); returns the float64 loss."""
    _dev(params, "params", torch.float32, 1)
    _dev(I, "I", torch.float32, 3)
    _dev(target, "target", torch.float32, 4)
    n = I.shape[0]
    loss = torch.empty((), dtype=torch.float64, device=I.device)
    shp = unet_shape(H, widths)
    ctx = _ctx(I.device)
    rc = _L.load().unet_train_step(ctx, ctypes.byref(shp), _ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                   float(lr), _ptr(I), float(log_scale), _ptr(target), n, _ptr(loss), _ptr(grads),
                                   _ptr(out), _stream(I.device))
    _check(rc, ctx)
    return loss


CONV_MODES = {"conv3": 0, "down": 1, "up": 2, "conv1": 3}


def conv2d(mode: str, x: torch.Tensor, W: torch.Tensor, b: Optional[torch.Tensor], relu: bool = False):
    """One convolution layer: x bf16 [n][H][H][Ci], W float [taps][Ci][Co] -> float [n][Ho][Ho][Co]."""
    _dev(x, "x", torch.bfloat16, 4)
    _dev(W, "W", torch.float32, 3)
    n, H, _, Ci = x.shape
    Co = W.shape[2]
    Ho = {"conv3": H, "down": H // 2, "up": 2 * H, "conv1": H}[mode]
    y = torch.empty((n, Ho, Ho, Co), dtype=torch.float32, device=x.device)
    ctx = _ctx(x.device)
    rc = _L.load().mnf_conv2d(ctx, CONV_MODES[mode], _ptr(x), n, H, Ci, _ptr(W), _ptr(b), Co, 1 if relu else 0,
                              _ptr(y), _stream(x.device))
    _check(rc, ctx)
    return y


def conv2d_grad(mode: str, x: torch.Tensor, W: torch.Tensor, dy: torch.Tensor, act: Optional[torch.Tensor] = None):
    """(dx bf16, dW float, db float) of one layer; dy is masked by act > 0 when act is given."""
    _dev(x, "x", torch.bfloat16, 4)
    _dev(W, "W", torch.float32, 3)
    _dev(dy, "dy", torch.bfloat16, 4)
    n, H, _, Ci = x.shape
    Co = W.shape[2]
    dx = torch.empty_like(x)
    dW = torch.empty_like(W)
    db = torch.empty(Co, dtype=torch.float32, device=x.device)
    ctx = _ctx(x.device)
    rc = _L.load().mnf_conv2d_grad(ctx, CONV_MODES[mode], _ptr(x), n, H, Ci, _ptr(W), Co, _ptr(dy), _ptr(act),
                                   _ptr(dx), _ptr(dW), _ptr(db), _stream(x.device))
    _check(rc, ctx)
    return dx, dW, db


def detector_expose(clean: torch.Tensor, t: Sequence[float], scale: float, sat: float, sigma_read: float,
                    seed: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """uint16 exposure stack [J][K][H][W] of clean intensities [J][H][W] (Philox-keyed by seed)."""
    _dev(clean, "clean", torch.float32, 3)
    J, H, W = clean.shape
    K = len(t)
    if out is None:
        out = torch.empty((J, K, H, W), dtype=torch.uint16, device=clean.device)
    else:
        _dev(out, "out", torch.uint16, 4)
        if tuple(out.shape) != (J, K, H, W):
            raise ValueError("out must have shape [J][K][H][W]")
    tt = (ctypes.c_float * max(K, 1))(*[float(x) for x in t])
    ctx = _ctx(clean.device)
    rc = _L.load().detector_expose(ctx, _ptr(clean), J, H, W, tt, K, float(scale), float(sat), float(sigma_read),
                                   int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out), _stream(clean.device))
    _check(rc, ctx)
    return out


def ptycho_stitch(patches: torch.Tensor, P: torch.Tensor, pos, shape, sync: bool = False,
                  out: Optional[torch.Tensor] = None):
    """Probe-intensity-weighted starting object [My][Mx] from patches [J][Nw][Nw][2] (amplitude, phase);
    with sync, each window's constant phase is first aligned with its neighbours."""
    _dev(patches, "patches", torch.float32, 4)
    _dev(P, "P", torch.complex64, 2)
    posa = _host_i32(pos, (2,), "pos")
    J, Nw = patches.shape[0], patches.shape[1]
    if patches.shape[1:] != (Nw, Nw, 2) or tuple(P.shape) != (Nw, Nw) or posa.shape[0] != J:
        raise ValueError("patches must be [J][Nw][Nw][2] with P [Nw][Nw] and J positions")
    My, Mx = shape
    if out is None:
        out = torch.empty((My, Mx), dtype=torch.complex64, device=patches.device)
    else:
        _dev(out, "out", torch.complex64, 2)
    ctx = _ctx(patches.device)
    rc = _L.load().ptycho_stitch(ctx, _ptr(patches), _ptr(P), Nw, _i32p(posa), J, 1 if sync else 0, _ptr(out),
                                 My, Mx, _stream(patches.device))
    _check(rc, ctx)
    return out


def nrmse(O: torch.Tensor, O_true: torch.Tensor, mask: Optional[torch.Tensor] = None,
          out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """float64 device scalar min_gamma ||gamma O - O_true|| / ||O_true|| over the mask."""
    if not (O.is_cuda and O_true.is_cuda and O.dtype == torch.complex64 and O_true.dtype == torch.complex64):
        raise ValueError("O and O_true must be complex64 CUDA tensors")
    if O.shape != O_true.shape or not O.is_contiguous() or not O_true.is_contiguous():
        raise ValueError("O and O_true must be contiguous and of one shape")
    if mask is not None and (mask.dtype not in (torch.uint8, torch.bool) or mask.shape != O.shape
                             or not mask.is_contiguous() or not mask.is_cuda):
        raise ValueError("mask must be a contiguous uint8/bool CUDA tensor of O's shape")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=O.device)
    ctx = _ctx(O.device)
    rc = _L.load().mnf_nrmse(ctx, _ptr(O), _ptr(O_true), _ptr(mask), O.numel(), _ptr(out), _stream(O.device))
    _check(rc, ctx)
    return out


def detector_resample(I: torch.Tensor, scale: float, weight: float = 1.0, out: Optional[torch.Tensor] = None,
                      accumulate: bool = False) -> torch.Tensor:
    """weight * scale^2 * I(c + (k - c) scale), bilinear, of detector-centred patterns I [J][Nd][Nd]."""
    _dev(I, "I", torch.float32, 3)
    J, Nd, _ = I.shape
    if out is None:
        out = torch.empty_like(I)
        accumulate = False
    else:
        _dev(out, "out", torch.float32, 3)
        if out.shape != I.shape:
            raise ValueError("out must have I's shape")
    ctx = _ctx(I.device)
    rc = _L.load().detector_resample(ctx, _ptr(I), J, Nd, float(scale), float(weight), 1 if accumulate else 0,
                                     _ptr(out), _stream(I.device))
    _check(rc, ctx)
    return out


def broadband_forward(O: torch.Tensor, P: torch.Tensor, pos, Nd: int, scales: Sequence[float],
                      weights: Sequence[float]) -> torch.Tensor:
    """Discrete-spectrum far-field intensities (Eq. 4) of an achromatic probe and
    object: sum_m w_m s_m^2 I_ref(c + (k - c) s_m), with I_ref the reference-wavelength
    pattern of ptycho_forward and s_m = lambda_0 / lambda_m."""
    if len(scales) != len(weights) or not scales:
        raise ValueError("one weight per spectral line")
    ref = ptycho_forward(O, P, pos, Nd)
    out = torch.empty_like(ref)
    for m, (s, w) in enumerate(zip(scales, weights)):
        detector_resample(ref, s, w, out=out, accumulate=m > 0)
    return out
