"""Far-field tile-shape and self-interaction prefetch autotuners.

Times every candidate shape (targets per thread x number of source chunks)
of the far-field kernel on the context's own workload, for the kinds the
caller evaluates, with HIP events (ehd_time_far: the kernel launched alone;
the share that overlap mode forks beside the self-interaction uses the same
shape).  Each shape is timed `reps` times (once when a launch takes longer
than LONG_MS) and ranked by its median.  The
fastest is kept in the context and cached in a JSON file keyed by device
architecture, library build, workload signature, kinds and precision, so a
rebuilt library never reuses a stale choice.

The self-interaction autotuner does the same for the Legendre prefetch
batch of each degree class present (ehd_time_self over the batches the
library builds for the class), keyed by device, library build, class, the
(p, q_self) mix of the class's drops and their number.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics

import torch

TPT_CANDIDATES = (1, 2)
# Counts just under the maximum matter on large workloads: the last round of
# blocks is partly empty for some counts and full for others (about 1%).
CHUNK_CANDIDATES = (1, 4, 8, 12, 14, 15, 16)
LONG_MS = 100.0
_LIB_HASH = {}


def default_cache_path() -> str:
    return os.environ.get("EHD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ehdbim_tune.json"))


def library_hash() -> str:
    """Content hash of the loaded HIP library (the build the timings are for)."""
    from . import ehdbim
    path = ehdbim.LIB_PATH
    if path not in _LIB_HASH:
        h = hashlib.sha1()
        with open(path, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _LIB_HASH[path] = h.hexdigest()[:16]
    return _LIB_HASH[path]


def signature(ctx, p, q_far, grid_mode: int, far_prec: int, kinds: int) -> str:
    prop = torch.cuda.get_device_properties(ctx.device)
    arch = getattr(prop, "gcnArchName", prop.name)
    h = hashlib.sha1()
    h.update(repr((list(map(int, p)), list(map(int, q_far)), int(grid_mode))).encode())
    return (f"{arch}|{prop.multi_processor_count}|lib{library_hash()}|T{ctx.ntargets}|{h.hexdigest()[:16]}"
            f"|prec{far_prec}|kinds{kinds}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune_far(ctx, p, q_far, grid_mode: int, far_prec: int, kinds: int = 31, reps: int = 3,
                 cache_path: str | None = None, use_cache: bool = True):
    """Pick and set the fastest far-field tile shape for `kinds`; returns
    (targets_per_thread, nchunk, {shape: median ms}, from_cache)."""
    path = cache_path or default_cache_path()
    key = signature(ctx, p, q_far, grid_mode, far_prec, kinds)
    cache = _load(path) if use_cache else {}
    if key in cache:
        tpt, nch = cache[key]["best"]
        ctx.set_far_config(tpt, nch)
        return tpt, nch, cache[key]["timings"], True
    timings = {}
    for tpt in TPT_CANDIDATES:
        for nch in CHUNK_CANDIDATES:
            try:
                ms = [ctx.time_far(far_prec, tpt, nch, 1, kinds=kinds)]
                # long launches (hundreds of ms) vary little: one timing
                while len(ms) < reps and ms[0] < LONG_MS:
                    ms.append(ctx.time_far(far_prec, tpt, nch, 1, kinds=kinds))
            except RuntimeError:
                continue      # shape not valid for this workload (e.g. more chunks than tiles)
            timings[f"{tpt}x{nch}"] = statistics.median(ms)
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


def self_signature(ctx, cls: int, pq, grid_mode: int) -> str:
    prop = torch.cuda.get_device_properties(ctx.device)
    arch = getattr(prop, "gcnArchName", prop.name)
    # the number of drops in the class too: its timings are reported, and a
    # class of a few drops runs in a handful of waves per CU
    return (f"{arch}|{prop.multi_processor_count}|lib{library_hash()}|self{cls}|"
            f"{sorted(set(pq))}|n{len(pq)}|grid{int(grid_mode)}")


def autotune_self(ctx, p, q_self, grid_mode: int, fcoef, sigcoef, reps: int = 3,
                  cache_path: str | None = None, use_cache: bool = True):
    """Pick and set the fastest Legendre prefetch batch of every degree class
    that has drops; returns ({class pmax: batch}, {class pmax: {batch: median
    ms}}, from_cache) (from_cache: every class came from the cache)."""
    from . import ehdbim
    path = cache_path or default_cache_path()
    cache = _load(path) if use_cache else {}
    best, timings, cached, new = {}, {}, True, {}
    lo = 0
    for cls, pmax in enumerate(ehdbim.DEGREE_CLASSES):
        pq = [(int(a), int(b)) for a, b in zip(p, q_self) if lo < int(a) <= pmax]
        lo = pmax
        if not pq:
            continue
        key = self_signature(ctx, cls, pq, grid_mode)
        if key in cache:
            pf = int(cache[key]["best"])
            ctx.set_self_config(cls, pf)
            best[pmax], timings[pmax] = pf, cache[key]["timings"]
            continue
        cached = False
        t = {}
        for pf in ehdbim.self_config_candidates(cls):
            ms = [ctx.time_self(cls, pf, fcoef, sigcoef, 1)]
            while len(ms) < reps and ms[0] < LONG_MS:
                ms.append(ctx.time_self(cls, pf, fcoef, sigcoef, 1))
            t[str(pf)] = statistics.median(ms)
        pf = int(min(t, key=t.get))
        ctx.set_self_config(cls, pf)
        best[pmax], timings[pmax] = pf, t
        new[key] = {"best": pf, "timings": t}
    if use_cache and new:
        cache = _load(path)
        cache.update(new)
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return best, timings, cached and bool(best)
