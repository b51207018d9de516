"""Launch-shape tuning with an on-disk cache.

The library compiles every pattern pass in two launch shapes, giving four
variants per detector size (see mnf_autotune in include/mnfpty.h).  This
module times them once per (GPU architecture, detector size, mini-batch)
through the C ABI, stores the winner in a JSON cache and applies cached
choices to the library context.  The algorithm and the mini-batch never
change."""
from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, Iterable, Optional

import torch

from . import api as _api
from . import lib as _L


def cache_path() -> str:
    return os.environ.get("MNF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mnfpty", "tune.json"))


def _arch(device: torch.device) -> str:
    return getattr(torch.cuda.get_device_properties(device), "gcnArchName", "unknown").split(":")[0]


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(sizes: Iterable[int], batch: int = 32, reps: int = 10, device="cuda:0",
             path: Optional[str] = None, force: bool = False) -> Dict[int, dict]:
    """Pick a variant for every detector size in `sizes` (timing only the
    ones missing from the cache unless force) and apply it.  Returns
    {N: {"variant": v, "times_us": [...] or None}}."""
    dev = torch.device(device)
    path = path or cache_path()
    data = _load(path)
    arch = _arch(dev)
    ctx = _api._ctx(dev)
    lib = _L.load()
    out = {}
    changed = False
    for N in sizes:
        key = f"{arch}:{int(N)}:{int(batch)}"
        entry = data.get(key)
        if entry is None or force:
            times = (ctypes.c_double * 8)()
            v = lib.mnf_autotune(ctx, int(N), int(batch), int(reps), times,
                                 ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
            _api._check(v if v < 0 else 0, ctx)
            entry = {"variant": int(v), "times_us": [round(t, 3) for t in times]}
            data[key] = entry
            changed = True
        else:
            _api._check(lib.mnf_set_variant(ctx, int(N), int(entry["variant"])), ctx)
        out[int(N)] = entry
    if changed:
        _save(path, data)
    return out


def set_variant(N: int, variant: int, device="cuda:0") -> None:
    dev = torch.device(device)
    ctx = _api._ctx(dev)
    _api._check(_L.load().mnf_set_variant(ctx, int(N), int(variant)), ctx)


def get_variant(N: int, device="cuda:0") -> int:
    dev = torch.device(device)
    ctx = _api._ctx(dev)
    v = _L.load().mnf_get_variant(ctx, int(N))
    _api._check(v if v < 0 else 0, ctx)
    return int(v)
