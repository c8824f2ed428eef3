"""Far-field tile-shape autotuner.

Times every candidate shape (targets per thread x number of source chunks)
of the far-field kernel on the context's own workload with HIP events
(ehd_time_far), keeps the fastest in the context, and caches the choice in a
JSON file keyed by device architecture, workload signature and precision.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

TPT_CANDIDATES = (1, 2)
CHUNK_CANDIDATES = (1, 4, 16)


def default_cache_path() -> str:
    return os.environ.get("EHD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ehdbim_tune.json"))


def signature(ctx, p, q_far, grid_mode: int, far_prec: int) -> str:
    prop = torch.cuda.get_device_properties(ctx.device)
    arch = getattr(prop, "gcnArchName", prop.name)
    h = hashlib.sha1()
    h.update(repr((list(map(int, p)), list(map(int, q_far)), int(grid_mode))).encode())
    return f"{arch}|{prop.multi_processor_count}|T{ctx.ntargets}|{h.hexdigest()[:16]}|prec{far_prec}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune_far(ctx, p, q_far, grid_mode: int, far_prec: int, reps: int = 1,
                 cache_path: str | None = None, use_cache: bool = True):
    """Pick and set the fastest far-field tile shape; returns
    (targets_per_thread, nchunk, {shape: ms}, from_cache)."""
    path = cache_path or default_cache_path()
    key = signature(ctx, p, q_far, grid_mode, far_prec)
    cache = _load(path) if use_cache else {}
    if key in cache:
        tpt, nch = cache[key]["best"]
        ctx.set_far_config(tpt, nch)
        return tpt, nch, cache[key]["timings"], True
    timings = {}
    for tpt in TPT_CANDIDATES:
        for nch in CHUNK_CANDIDATES:
            try:
                ms = ctx.time_far(far_prec, tpt, nch, reps)
            except RuntimeError:
                continue      # shape not valid for this workload (e.g. more chunks than tiles)
            timings[f"{tpt}x{nch}"] = ms
    best = min(timings, key=timings.get)
    tpt, nch = (int(v) for v in best.split("x"))
    ctx.set_far_config(tpt, nch)
    if use_cache:
        cache = _load(path)
        cache[key] = {"best": [tpt, nch], "timings": timings}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return tpt, nch, timings, False
