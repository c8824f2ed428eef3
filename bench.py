"""Benchmark: layer-potential target evaluations per second on one MI355X.

One step = one call of ehd_layer_potentials over the whole workload: the
singular self-interaction of every target (FP64, rotated-pole rule) plus the
far-field direct sums over every other drop, the four potentials of the
metric (S, D, S_L, L: 8 values per target).  Inputs are resident in HBM
before the timed region.

Default: the 256-drop suspension at p = 32 (q = 2p), timed twice: all in
FP64 (the paper's precision; this is `value`) and with the FP32 compensated
far field (the `fp32_far` object, with its measured error per output against
the FP64 path at every target and against the FP64 oracle on 16 drops).

Prints one JSON line (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6        # vector and matrix
PEAK_FP32_VECTOR_TFLOPS = 157.3
# FP32 without packed instructions: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FAR_FLOPS_PER_INTERACTION = 53   # S 18, D 19, S_L 2, L 3, xh/r^2/powers 11 (K* would add 5)
SELF_KERNEL_FLOPS_PER_NODE = 75


def _nlon(P: int, grid_mode: int) -> int:
    return 2 * P + 2 if grid_mode == 0 else 2 * P


def self_flops_per_drop(p: int, q: int, grid_mode: int) -> float:
    """Dense algorithmic FP64 work of the singular self-interaction of one
    drop (the scope table's count): complex rotation of 7 fields, Legendre
    sums (7 fields + 3 theta derivatives), longitude sums of 13 grid
    quantities as a dense DFT, kernel evaluation per rotated node."""
    nlon_p, nlon_q = _nlon(p, grid_mode), _nlon(q, grid_mode)
    T = (p + 1) * nlon_p
    rot = 4 * 7 * T * sum((n + 1) * (2 * n + 1) for n in range(p + 1))
    leg = 4 * (q + 1) * ((p + 1) * (p + 2) // 2) * 10 * T
    dft = 2 * nlon_q * (2 * p + 1) * (q + 1) * 13 * T
    ker = SELF_KERNEL_FLOPS_PER_NODE * T * (q + 1) * nlon_q
    return float(rot + leg + dft + ker)


def self_exec_flops_per_drop(p: int, q: int, grid_mode: int) -> float:
    """FP64 work of the singular self-interaction as the kernel's route does
    it (no padding counted):
      rotation, real form: per field and degree n, the phase e^{i m phi_t}
        (6 flops per m) and two real (n+1) x (n+1) products (4 (n+1)^2);
      Legendre sums: as in the dense count;
      longitude sums, quarter-period split: per latitude and quantity,
        rows l = 0..floor(H/2) (H = nlon_q / 2) of 2p+1 terms, 2 flops each,
        plus 12 flops per row to form the four images;
      kernel: 75 flops per rotated node."""
    nlon_p, nlon_q = _nlon(p, grid_mode), _nlon(q, grid_mode)
    T = (p + 1) * nlon_p
    rot = 7 * T * sum(4 * (n + 1) ** 2 + 6 * (n + 1) for n in range(p + 1))
    leg = 4 * (q + 1) * ((p + 1) * (p + 2) // 2) * 10 * T
    rows = nlon_q // 4 + 1
    dft = 13 * (q + 1) * T * rows * (2 * (2 * p + 1) + 12)
    ker = SELF_KERNEL_FLOPS_PER_NODE * T * (q + 1) * nlon_q
    return float(rot + leg + dft + ker)


# HBM bytes per launch of each (workload, far precision, kernel) from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs summarised in profiles/
# (counters scaled by what they read for a plain device copy of known size),
# valid only for the kernel source they were taken with.
TRAFFIC_SOURCE_SHA256 = "60810dad5ec8cec55a8307727e9bb7747487add5813133afb8f5c1052345e121"
# (workload, "fp64" | "fp32c", kernel name[, far-field tile shape]) -> bytes per
# launch of all its items; a far-field kernel's traffic depends on its tile
# shape (per-chunk partial sums, source re-reads per block of targets)
TRAFFIC_BYTES = {
    ("large_256_p32", "fp32c", "k_far32", "1x12"): 9.241e+09,
    ("large_256_p32", "fp32c", "k_far32", "1x14"): 9.513e+09,
    ("large_256_p32", "fp32c", "k_far32", "1x15"): 9.478e+09,
    ("large_256_p32", "fp32c", "k_far32", "1x16"): 1.091e+10,
    ("large_256_p32", "fp32c", "k_far32", "2x12"): 5.428e+09,
    ("large_256_p32", "fp32c", "k_far32", "2x14"): 5.514e+09,
    ("large_256_p32", "fp32c", "k_far32", "2x15"): 5.564e+09,
    ("large_256_p32", "fp32c", "k_far32", "2x16"): 5.648e+09,
    ("large_256_p32", "fp64", "k_far64", "1x12"): 6.26e+10,
    ("large_256_p32", "fp64", "k_far64", "1x14"): 8.783e+10,
    ("large_256_p32", "fp64", "k_far64", "1x15"): 7.441e+10,
    ("large_256_p32", "fp64", "k_far64", "1x16"): 9.977e+10,
    ("large_256_p32", "fp64", "k_far64", "2x12"): 1.695e+10,
    ("large_256_p32", "fp64", "k_far64", "2x14"): 1.902e+10,
    ("large_256_p32", "fp64", "k_far64", "2x15"): 1.94e+10,
    ("large_256_p32", "fp64", "k_far64", "2x16"): 2.234e+10,
    ("batched_64_mixed_p", "fp32c", "k_far32", "1x12"): 4.735e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "1x14"): 4.518e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "1x15"): 4.571e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "1x16"): 4.661e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "2x12"): 5.844e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "2x14"): 5.558e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "2x15"): 5.453e+08,
    ("batched_64_mixed_p", "fp32c", "k_far32", "2x16"): 5.381e+08,
    ("batched_64_mixed_p", "fp64", "k_far64", "1x12"): 5.991e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "1x14"): 4.871e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "1x15"): 3.977e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "1x16"): 3.348e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "2x12"): 2.147e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "2x14"): 2.085e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "2x15"): 1.887e+09,
    ("batched_64_mixed_p", "fp64", "k_far64", "2x16"): 1.746e+09,
    ("large_256_p32", "fp64", "k_self<32>"): 1.815e9,
    ("large_256_p32", "fp32c", "k_self<32>"): 1.815e9,
}
for _pmax, _b in ((48, 6.773e8), (32, 1.202e8), (24, 2.543e7), (16, 7.398e6)):
    for _prec in ("fp64", "fp32c"):
        TRAFFIC_BYTES[("batched_64_mixed_p", _prec, f"k_self<{_pmax}>")] = _b


def kernel_source_sha256() -> str:
    """SHA-256 of the device code of the library source (the text above its
    host-side section), on which the counted bytes depend."""
    import hashlib
    path = os.path.join(ROOT, "paper_1811_10270_amd", "csrc", "ehdbim.hip")
    with open(path, "rb") as fh:
        text = fh.read()
    cut = text.find(b"\n// Host side\n")
    return hashlib.sha256(text[:cut] if cut > 0 else text).hexdigest()


def measured_traffic(kernel: str, workload: str, far_prec: int, far_tile: str):
    if kernel_source_sha256() != TRAFFIC_SOURCE_SHA256:
        return None
    key = (workload, "fp64" if far_prec == 0 else "fp32c", kernel.split(" ")[0])
    if key[2].startswith("k_far"):
        key += (far_tile,)
    return TRAFFIC_BYTES.get(key)


def far_interactions(s) -> float:
    tot = 0.0
    nt = []
    ns = []
    for d in range(s.ndrops):
        p, qf = int(s.p[d]), int(s.q_far[d])
        nlp = 2 * p + 2 if s.grid_mode == 0 else 2 * p
        nlq = 2 * qf + 2 if s.grid_mode == 0 else 2 * qf
        nt.append((p + 1) * nlp)
        ns.append((qf + 1) * nlq)
    S = sum(ns)
    for d in range(s.ndrops):
        tot += nt[d] * (S - ns[d])
    return tot


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, nsample: int, seed: int = 0, one_core_targets: int = 4):
    """The oracle as it stands, timed on the host on a bounded sample of the
    workload: the singular self-interaction of `nsample` random targets, the
    far-field source records of every drop (built once per evaluation) and
    the far sums at the same targets.  The rate is that of a whole
    evaluation, extrapolated per target from the sample: T / (T (t_self +
    t_far) + t_sources).  The one-core rate takes one_core_targets of the
    same targets (evenly spaced in the sample) and the source records of two
    drops, scaled to all drops by their nodes x coefficients."""
    import numpy as np
    import oracle
    td, tn = oracle.all_targets(s)
    T = len(td)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(T, size=min(nsample, T), replace=False))
    nthr = oracle.num_threads()

    from paper_1811_10270_amd.workloads import subset as W_subset
    t0 = time.perf_counter()
    far_all = oracle.FarSources(s)
    t_src = time.perf_counter() - t0

    def timed(threads, sel, src_drops=None):
        """Per-target self and far times on `threads` threads, and the time
        to build the source records of src_drops (None: skipped)."""
        oracle.set_threads(threads)
        try:
            t0 = time.perf_counter()
            oracle.self_(s, td[sel], tn[sel])
            t1 = time.perf_counter()
            t_sub = 0.0
            if src_drops is not None:
                fs = oracle.FarSources(W_subset(s, src_drops))
                t_sub = time.perf_counter() - t1
                fs.close()
            x0, n0 = oracle.targets(s, td[sel], tn[sel])
            t3 = time.perf_counter()
            far_all.eval(x0, n0, td[sel])
            t4 = time.perf_counter()
        finally:
            oracle.set_threads(nthr)
        return (t1 - t0) / len(sel), t_sub, (t4 - t3) / len(sel)

    t_self, _, t_far = timed(nthr, idx)
    rate = T / (T * (t_self + t_far) + t_src)
    # one core: a few targets, and the source records of two drops scaled
    # to all drops by nodes x coefficients
    sub = [0, s.ndrops - 1] if s.ndrops > 1 else [0]
    cost = [(int(s.q_far[d]) + 1) * (2 * int(s.q_far[d]) + 2) * (int(s.p[d]) + 1) * (int(s.p[d]) + 2)
            for d in range(s.ndrops)]
    pick = idx[np.linspace(0, len(idx) - 1, min(one_core_targets, len(idx))).astype(int)]
    s1_self, s1_src_sub, s1_far = timed(1, pick, sub)
    s1_src = s1_src_sub * sum(cost) / sum(cost[d] for d in sub)
    rate1 = T / (T * (s1_self + s1_far) + s1_src)
    far_all.close()
    return {
        "value": rate,
        "unit": "target-evals/s",
        "cores": nthr,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "sample": f"{len(idx)} random targets of {T} (seed {seed}) of the same workload, self + far over all "
                  f"{s.ndrops} drops, FP64, {nthr} threads: self {t_self * 1e3:.1f} ms and far "
                  f"{t_far * 1e3:.2f} ms per target, far source records {t_src:.1f} s per evaluation; "
                  f"rate extrapolated to all {T} targets",
        "one_core": {"value": rate1, "unit": "target-evals/s", "cores": 1,
                     "sample": f"{len(pick)} of the same targets (evenly spaced): self "
                               f"{s1_self:.2f} s and far {s1_far * 1e3:.1f} ms per target; source records of "
                               f"drops {sub} ({s1_src_sub:.2f} s) scaled to all drops ({s1_src:.1f} s)"},
    }


COMP_NAMES = ("S_x", "S_y", "S_z", "D_x", "D_y", "D_z", "S_L", "L", "K*")
GOLDEN_FAR = {"large_256_p32": os.path.join(ROOT, "tests", "golden", "large_256_p32_far16.npz")}


def input_checksums(s):
    """Sums and weighted sums of the input coefficients (as stored with the
    oracle's values, to detect a change of the generator's draws)."""
    import numpy as np
    out = []
    for a in (s.xcoef, s.fcoef, s.sigcoef):
        w = np.arange(1, a.size + 1, dtype=np.float64) / a.size
        out += [float(a.sum()), float((a * w).sum())]
    return np.array(out)


def normwise(got, ref):
    """Per output row: max |got - ref| / max |ref| over the targets."""
    import numpy as np
    den = np.abs(ref).max(axis=-1)
    den = np.where(den == 0, 1.0, den)
    return np.abs(got - ref).max(axis=-1) / den


def time_evaluation(args, torch, E, ctx, s, far_prec, kinds, f, sig, out, u=None):
    """Warm-up, then args.steps timed evaluations with HIP-event stage and
    class times; per-kernel work and rates; the far part of one more
    (untimed, split) evaluation for the error report."""
    K = args.steps
    if args.far_tile:
        shapes = args.far_tile.lower().split(",")
        shape = shapes[1] if far_prec == E.FAR_FP32C and len(shapes) > 1 else shapes[0]
        tpt, nch = (int(v) for v in shape.split("x"))
        ctx.set_far_config(tpt, nch)
    tile = {"targets_per_thread": ctx.far_config()[0], "source_chunks": ctx.far_config()[1], "autotuned": False}
    if not args.no_autotune and not args.far_tile:
        from paper_1811_10270_amd import autotune
        tpt, nch, timings, cached = autotune.autotune_far(ctx, s.p, s.q_far, s.grid_mode, far_prec, kinds=kinds)
        tile = {"targets_per_thread": tpt, "source_chunks": nch, "autotuned": True, "from_cache": cached,
                "timings_ms": timings}
    log("far tile", tile)
    ctx.set_graph(bool(args.graph))
    for _ in range(args.warmup):
        ctx.layer_potentials(f, u, sig, kinds, far_prec, out)
    ctx.sync()
    torch.cuda.synchronize()
    ctx.set_timing(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.layer_potentials(f, u, sig, kinds, far_prec, out)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"far_prec {far_prec}: {K} steps in {dt:.3f} s")
    timing_pass = "timed region"
    if args.graph:
        # a replayed graph records no per-kernel events: time the same
        # launch sequence once more without the graph
        ctx.set_graph(False)
        ctx.set_timing(K)
        for _ in range(K):
            ctx.layer_potentials(f, u, sig, kinds, far_prec, out)
        ctx.sync()
        timing_pass = "separate pass of the same launches without the graph"
    stages = [ctx.stage_times(i) for i in range(K)]
    avg = [sum(st[k] for st in stages) / K for k in range(4)]
    cls_times = [ctx.self_class_times(i) for i in range(K)]

    T = ctx.ntargets
    tpt_, nch_ = ctx.far_config()
    # the library's overlap plan: classes beside a forked far-field share
    beside, forked = ctx.overlap_plan(kinds, far_prec) if args.overlap else (0, 0)
    overlap = forked > 0
    kernels = []
    for c, pmax in enumerate(E.DEGREE_CLASSES):
        ms = sum(ct[c] for ct in cls_times) / K
        lo = E.DEGREE_CLASSES[c - 1] if c else 0
        sel = [d for d in range(s.ndrops) if lo < int(s.p[d]) <= pmax]
        fl = sum(self_exec_flops_per_drop(int(s.p[d]), int(s.q_self[d]), s.grid_mode) for d in sel)
        dense = sum(self_flops_per_drop(int(s.p[d]), int(s.q_self[d]), s.grid_mode) for d in sel)
        if ms > 0 and fl > 0:
            # shared: a forked far-field share runs beside the class
            shared = overlap and bool(beside >> c & 1)
            kernels.append({"kernel": f"k_self<{pmax}> (singular self-interaction, p <= {pmax}, FP64)",
                            "bound": "alu", "algorithmic_flops": fl, "dense_flops": dense, "avg_ms": ms,
                            "achieved": fl / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS, "shared": shared})
    if u is not None:
        # a separate u takes a second self-interaction pass per class (x, u),
        # whose class events overwrite the first pass's: the self stage time
        # holds both, the class rows would not
        kernels = []
    far_flops = far_interactions(s) * FAR_FLOPS_PER_INTERACTION
    # the far field runs alone in the timed region unless a share of it is
    # forked beside the self-interaction
    far_alone = not overlap
    name = "k_far32" if far_prec == E.FAR_FP32C else "k_far64"
    far_ms = avg[2] if far_alone else None
    far_src = timing_pass
    if far_ms is None and far_flops > 0:
        # time the far kernel alone with HIP events (ehd_time_far), same tile
        far_ms = ctx.time_far(far_prec, tpt_, nch_, reps=3, kinds=kinds)
        far_src = "launched alone (ehd_time_far, 3 launches)"
    if far_flops > 0:
        peak = PEAK_FP32_VECTOR_TFLOPS if far_prec == E.FAR_FP32C else PEAK_FP64_TFLOPS
        ach = far_flops / (far_ms * 1e-3) / 1e12
        k = {"kernel": name + " (far-field direct sums)", "bound": "alu", "algorithmic_flops": far_flops,
             "avg_ms": far_ms, "achieved": ach, "peak": peak, "shared": not far_alone, "timed": far_src}
        if far_prec == E.FAR_FP32C:
            k["peak_unpacked"] = PEAK_FP32_UNPACKED_TFLOPS
            k["frac_unpacked"] = ach / PEAK_FP32_UNPACKED_TFLOPS
        kernels.append(k)
    for k in kernels:
        k["unit"] = "TFLOP/s"
        k["frac"] = k["achieved"] / k["peak"]
        k["traffic"] = (measured_traffic(k["kernel"], args.workload, far_prec, f"{tpt_}x{nch_}")
                        if not k["shared"] else None)
    roof = None
    alone = [k for k in kernels if not k["shared"]]
    if alone:
        dom = max(alone, key=lambda k: k["avg_ms"])
        roof = {key: dom[key] for key in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "algorithmic_flops", "avg_ms")}
        for key in ("dense_flops", "peak_unpacked", "frac_unpacked"):
            if key in dom:
                roof[key] = dom[key]
        roof["per_unit"] = ("53 flops per target-source interaction" if dom["kernel"].startswith("k_far")
                            else "executed self-interaction flops per drop (rotation, Legendre, quarter-period "
                                 "longitude sums, 75 per rotated node)")
    ctx.set_timing(0)
    # far part of one split evaluation (errors)
    so = torch.empty_like(out)
    fo = torch.empty_like(out)
    ctx.layer_potentials(f, u, sig, kinds, far_prec, so, fo)
    ctx.sync()
    return {"dt": dt, "ms_per_step": dt / K * 1e3, "value": T * K / dt, "stage_ms": dict(zip(E.STAGES, avg)),
            "kernels": kernels, "roofline": roof, "far_tile": tile, "far": fo.cpu().numpy(),
            "kernel_times": timing_pass,
            "overlap_plan": {"classes_beside_far": [p for c, p in enumerate(E.DEGREE_CLASSES) if beside >> c & 1],
                             "far_items_forked": forked}}


def bench_eval(args, torch, E, W, dev):
    """The layer-potential evaluation (the metric)."""
    import numpy as np
    s = W.WORKLOADS[args.workload](args.grid_mode)
    if args.separate_u:
        s = W.with_separate_u(s)
    kinds = E.METRIC_KINDS
    rows = E.rows_for_kinds(kinds)
    precs = {"both": [E.FAR_FP64, E.FAR_FP32C], "fp64": [E.FAR_FP64], "fp32c": [E.FAR_FP32C]}[args.far_prec]
    log(f"workload {args.workload}: {s.ndrops} drops, far precisions {precs}")
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if args.overlap:
        ctx.set_overlap(True)
    T = ctx.ntargets
    f = torch.from_numpy(s.fcoef).to(dev)
    sig = torch.from_numpy(s.sigcoef).to(dev)
    u = torch.from_numpy(s.ucoef).to(dev) if args.separate_u else None
    out = torch.empty(len(rows), T, dtype=torch.float64, device=dev)
    # the self-interaction's Legendre prefetch batch per degree class (one
    # choice for both far-field precisions: the self-interaction is the same)
    self_tile = {str(pm): ctx.self_config(c) for c, pm in enumerate(E.DEGREE_CLASSES)}
    self_tile = {"prefetch": self_tile, "autotuned": False}
    if not args.no_autotune:
        from paper_1811_10270_amd import autotune
        best, timings, cached = autotune.autotune_self(ctx, s.p, s.q_self, s.grid_mode, f, sig)
        self_tile = {"prefetch": {str(k): v for k, v in best.items()}, "autotuned": True, "from_cache": cached,
                     "timings_ms": {str(k): v for k, v in timings.items()}}
    log("self prefetch", self_tile)
    runs = {prec: time_evaluation(args, torch, E, ctx, s, prec, kinds, f, sig, out, u) for prec in precs}
    # one lone far-field launch per listed tile shape, after the timed steps
    # (for counter runs: each shape's dispatch has a grid size of its own)
    for prec in precs:
        for tpt, nch in args.count_shapes:
            ctx.time_far(prec, tpt, nch, 1, kinds=kinds)
    ctx.close()

    golden = None
    path = GOLDEN_FAR.get(args.workload)
    # the stored oracle far field is for D on f (no separate u)
    if path and os.path.exists(path) and s.grid_mode == 0 and not args.separate_u:
        g = np.load(path)
        if np.allclose(g["checksums"], input_checksums(s), rtol=1e-14, atol=0):
            golden = g

    def errors(run):
        e = {}
        if E.FAR_FP64 in runs and run is not runs[E.FAR_FP64]:
            err = normwise(run["far"], runs[E.FAR_FP64]["far"])
            e["vs_fp64_path_all_targets"] = {COMP_NAMES[c]: float(v) for c, v in zip(rows, err)}
        if golden is not None:
            idx = golden["far_idx"]
            err = normwise(run["far"][:, idx], golden["far"][list(rows)])
            e["vs_oracle_16_drops"] = {COMP_NAMES[c]: float(v) for c, v in zip(rows, err)}
            e["oracle_targets"] = int(len(idx))
        return e

    def q_desc(qs):
        ratio = {int(q) / int(p) for p, q in zip(s.p, qs)}
        return f"{ratio.pop():g}p" if len(ratio) == 1 else sorted({(int(p), int(q)) for p, q in zip(s.p, qs)})

    main_prec = precs[0]
    r = runs[main_prec]
    res = {
        "metric": "layer-potential target evals/sec (singular+far) FP64 vs FP32 at stated rel err",
        "value": r["value"],
        "unit": "target-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == E.FAR_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "overlap": bool(args.overlap and s.ndrops > 1), "ndrops": s.ndrops,
                   "p": sorted(set(int(x) for x in s.p)), "targets": T,
                   "q_self": q_desc(s.q_self), "q_far": q_desc(s.q_far),
                   "grid": "paper (2p+2 longitudes)" if s.grid_mode == 0 else "2p longitudes",
                   "kinds": "S,D,S_L,L", "double_layer_density": "separate u" if args.separate_u else "f",
                   "far_prec": "fp64" if main_prec == E.FAR_FP64 else "fp32c",
                   "far_interactions": far_interactions(s), "far_tile": r["far_tile"],
                   "overlap_plan": r["overlap_plan"], "self_tile": self_tile, "graph": bool(args.graph)},
        "stage_ms": r["stage_ms"],
        "roofline": r["roofline"],
        "kernels": r["kernels"],
        "kernel_times": r["kernel_times"],
    }
    if golden is not None or len(runs) > 1:
        res["far_error"] = errors(r)
    if len(runs) > 1:
        r32 = runs[E.FAR_FP32C]
        res["fp32_far"] = {"value": r32["value"], "unit": "target-evals/s", "ms_per_step": r32["ms_per_step"],
                           "dtype": "f64+f32", "far_tile": r32["far_tile"], "overlap_plan": r32["overlap_plan"],
                           "stage_ms": r32["stage_ms"],
                           "roofline": r32["roofline"], "kernels": r32["kernels"],
                           "far_error": errors(r32),
                           "error_bound_stated": 1e-6}
    if args.count_shapes:
        res["counted_far_shapes"] = [f"{t}x{c}" for t, c in args.count_shapes]
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = {"read": n * 8, "written": n * 8}
        del a, b
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(s, args.cpu_sample)
    print(json.dumps(res), flush=True)
    return 0


def bench_solve(args, torch, E, W, dev):
    """Galerkin GMRES solves (tol 1e-12 true relative residual, restart 30)
    from a zero initial guess; also one mat-vec (evaluation + projection)
    timed alone."""
    s = W.WORKLOADS[args.workload](args.grid_mode)
    far_prec = E.FAR_FP32C if args.far_prec == "fp32c" else E.FAR_FP64
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if args.overlap:
        ctx.set_overlap(True)
    nc = ctx.num_coefs()
    T = ctx.ntargets
    f = torch.from_numpy(s.fcoef).to(dev)
    nf = 1 if args.solve == "en" else 3
    x = torch.zeros(nf * nc, dtype=torch.float64, device=dev)
    grid = torch.empty(nf, T, dtype=torch.float64, device=dev)
    proj = torch.empty(nf * nc, dtype=torch.float64, device=dev)

    tol = 1e-12 if far_prec == E.FAR_FP64 else 1e-6

    def solve():
        x.zero_()
        if args.solve == "en":
            return ctx.solve_En(0.5, 1.0, 0.0, x, far_prec=far_prec, tol=tol)
        return ctx.solve_velocity(2.0, f, x, far_prec=far_prec, tol=tol)

    def matvec():
        if args.solve == "en":
            ctx.layer_potentials(None, None, x, E.LAP_DLADJ, far_prec, grid)
        else:
            ctx.layer_potentials(None, x, None, E.STOKES_DL, far_prec, grid)
        ctx.analyze(nf, grid, proj)

    for _ in range(max(args.warmup, 1)):
        its, rr = solve()
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        its, rr = solve()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    for _ in range(3):
        matvec()
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(10):
        matvec()
    ctx.sync()
    mv = (time.perf_counter() - t0) / 10
    ctx.close()
    res = {
        "metric": "Galerkin GMRES solve (" + ("E_n, adjoint double layer" if args.solve == "en"
                                               else "velocity, Stokes double layer") + "), tol %g" % tol,
        "value": 1.0 / dt, "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": max(args.warmup, 1),
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if far_prec == E.FAR_FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": args.workload, "overlap": args.overlap, "ndrops": s.ndrops, "p": sorted(set(int(v) for v in s.p)),
                   "targets": T, "unknowns": nf * nc, "far_prec": "fp64" if far_prec == E.FAR_FP64 else "fp32c",
                   "R" if args.solve == "en" else "lambda": 0.5 if args.solve == "en" else 2.0},
        "iterations": its, "relres": rr, "matvec_ms": mv * 1e3,
        "matvec_share": its * mv / dt,
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_step(args, torch, E, W, dev):
    """One explicit step per timed iteration, each from zero initial guesses."""
    s = W.WORKLOADS[args.workload](args.grid_mode)
    far_prec = E.FAR_FP32C if args.far_prec == "fp32c" else E.FAR_FP64
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if args.overlap:
        ctx.set_overlap(True)
    nc = ctx.num_coefs()
    en = torch.zeros(nc, dtype=torch.float64, device=dev)
    u = torch.zeros(3 * nc, dtype=torch.float64, device=dev)
    xn = torch.zeros(3 * nc, dtype=torch.float64, device=dev)

    # the FP32 far field perturbs the operator at the 1e-7 level: GMRES stops there
    tol = 1e-12 if far_prec == E.FAR_FP64 else 1e-6

    def step():
        en.zero_()
        u.zero_()
        return ctx.explicit_step(2.0, 0.5, 2.0, 0.3, 1.0, 0.0, 0.01, en, u, xn, far_prec=far_prec, tol=tol)

    for _ in range(max(args.warmup, 1)):
        its = step()
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        its = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    ctx.close()
    res = {
        "metric": "explicit time step (E_n GMRES + forces + velocity GMRES + x update), tol %g" % tol,
        "value": 1.0 / dt, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": max(args.warmup, 1),
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if far_prec == E.FAR_FP64 else "f64+f32", "data": "synthetic",
        "config": {"workload": args.workload, "overlap": args.overlap, "ndrops": s.ndrops, "p": sorted(set(int(v) for v in s.p)),
                   "targets": ctx.ntargets, "lambda": 2.0, "R": 0.5, "Q": 2.0, "CaE": 0.3, "E_u": 1.0,
                   "eos": "clean", "dt": 0.01,
                   "far_prec": "fp64" if far_prec == E.FAR_FP64 else "fp32c"},
        "gmres_iterations": {"E_n": its[0], "velocity": its[1]},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_near(args, torch, E, W, dev):
    """Evaluation of two unit spheres (p = 32, q_far = 3p) whose surfaces are
    args.near_gap apart, all kinds in FP64, with and without the nearly
    singular correction (targets closer than 3 pi/(q_far + 1), check points
    on a degree-min(10p, 400) grid from three of its spacings, m = 8)."""
    s = W.two_drops(32, seed=2, gap=args.near_gap)
    f = torch.from_numpy(s.fcoef).to(dev)
    sg = torch.from_numpy(s.sigcoef).to(dev)
    qf, qc = int(s.q_far[0]), min(E.MAX_Q_CHECK, 10 * 32)
    delta, sc = 3 * math.pi / (qf + 1), 3 * math.pi / (qc + 1)
    res = {}
    for near in (False, True):
        ctx = E.Context(0)
        ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
        if args.overlap:
            ctx.set_overlap(True)
        t0 = time.perf_counter()
        if near:
            ctx.set_near(delta, sc, 8, qc)
        setup = time.perf_counter() - t0
        out = torch.empty(9, ctx.ntargets, dtype=torch.float64, device=dev)
        for _ in range(max(args.warmup, 1)):
            ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP64, out)
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP64, out)
        ctx.sync()
        res[near] = ((time.perf_counter() - t0) / args.steps, ctx.near_pairs(), setup, ctx.ntargets)
        ctx.close()
    (t_plain, _, _, T), (t_near, pairs, setup, _) = res[False], res[True]
    out = {
        "metric": "layer-potential target evals/sec with the nearly singular correction (FP64)",
        "value": T / t_near, "unit": "target-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": t_near * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "two_drops_p32_gap%g" % args.near_gap, "targets": T, "q_far": qf, "q_check": qc,
                   "delta": delta, "s_check": sc, "m": 8, "kinds": "S,D,S_L,L,K*"},
        "near_pairs": pairs, "ms_without_correction": t_plain * 1e3, "setup_ms": setup * 1e3,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_evolve(args, torch, E, W, dev):
    """Steps of Algorithm 1 (ehd_evolve_step: two E_n solves, two velocity
    solves, the implicit surfactant solve, surface terms, midpoint and IMEX
    updates) from the workload's drops with a non-uniform surfactant."""
    import numpy as np
    s = W.WORKLOADS[args.workload](args.grid_mode)
    far_prec = E.FAR_FP32C if args.far_prec == "fp32c" else E.FAR_FP64
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if args.overlap:
        ctx.set_overlap(True)
    nc = ctx.num_coefs()
    rng = np.random.default_rng(7)
    g = np.zeros(nc)
    off = 0
    for p in (int(v) for v in s.p):
        g[off] = math.sqrt(4 * math.pi)
        for n in range(1, p + 1):
            for m in range(n + 1):
                k = off + 2 * (n * (n + 1) // 2 + m)
                g[k] = 0.05 * rng.standard_normal() / n ** 2
                if m:
                    g[k + 1] = 0.05 * rng.standard_normal() / n ** 2
        off += (p + 1) * (p + 2)
    gd = torch.from_numpy(g).to(dev)
    xn = torch.empty(3 * nc, dtype=torch.float64, device=dev)
    gn = torch.empty(nc, dtype=torch.float64, device=dev)
    tol = 1e-10 if far_prec == E.FAR_FP64 else 1e-6
    prm = dict(lam=2.0, R=0.5, Q=2.0, CaE=0.3, Eu=1.0, Eq=0.0, eos="linear", beta=0.5, Pe=10.0, dt=0.01)
    sp = E.Context.step_params(prm["lam"], prm["R"], prm["Q"], prm["CaE"], prm["Eu"], prm["Eq"], eos=E.EOS_LINEAR,
                               beta=prm["beta"], far_prec=far_prec, tol=tol)
    for _ in range(max(args.warmup, 1)):
        rep = ctx.evolve_step(sp, 1.0 / prm["Pe"], prm["dt"], gd, xn, gn)
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        rep = ctx.evolve_step(sp, 1.0 / prm["Pe"], prm["dt"], gd, xn, gn)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    ctx.close()
    res = {
        "metric": "time steps of Algorithm 1 (midpoint drops + IMEX-RK2 surfactant), tol %g" % tol,
        "value": 1.0 / dt, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": max(args.warmup, 1),
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if far_prec == E.FAR_FP64 else "f64+f32", "data": "synthetic",
        "config": dict({"workload": args.workload, "overlap": args.overlap, "ndrops": s.ndrops, "p": sorted(set(int(v) for v in s.p)),
                        "targets": ctx.ntargets,
                        "far_prec": "fp64" if far_prec == E.FAR_FP64 else "fp32c"}, **prm),
        "gmres_iterations": {"E_n": [rep["iters"][0], rep["iters"][2]], "velocity": [rep["iters"][1], rep["iters"][3]],
                             "surfactant": rep["iters_gamma"]},
        "error_estimates": {"drop": rep["err_drop"], "surfactant": rep["err_surf"]},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_learned(args, torch, E, W, dev):
    """Learned initial guess for the implicit surfactant-diffusion solve:
    generate the training solves with the library's preconditioned GMRES,
    train the 3 x 512 perceptron with the library's kernels, then count
    GMRES iterations to a 1e-10 true residual on held-out drops from zero
    (the preconditioned solve alone), from M^{-1} b and from the learned
    guess."""
    import numpy as np
    from paper_1811_10270_amd import learned_guess as L
    p, kind = args.learned_p, args.learned_kind
    t0 = time.perf_counter()
    tr = L.solve_all(L.draw(args.learned_train, p, seed=1, kind=kind))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m = L.train(tr)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    te = L.solve_all(L.draw(args.steps, p, seed=2, kind=kind))
    g = L.predict(m, te)
    r = L.compare(te, g, tol=1e-10)
    # mean iterations per decade of kappa = dt / (2 Pe)
    by_kappa = {}
    for lo in (5e-7, 5e-6, 5e-5):
        sel = (te.kappa >= lo) & (te.kappa < 10 * lo)
        if sel.any():
            by_kappa[f"[{lo:g}, {10 * lo:g})"] = {
                "solves": int(sel.sum()), "plain": float(r["iters_plain"][sel].mean()),
                "precond_rhs": float(r["iters_precond"][sel].mean()),
                "learned": float(r["iters_learned"][sel].mean()),
                "relres_median_precond_rhs": float(np.median(r["precond_relres"][sel])),
                "relres_median_learned": float(np.median(r["guess_relres"][sel]))}
    res = {
        "metric": "GMRES iterations to 1e-10 true residual, implicit surfactant solve, learned initial guess",
        "value": float(r["iters_learned"].mean()), "unit": "iterations", "n_gpus": 1, "steps": args.steps,
        "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 solve, f32 network", "data": "synthetic",
        "config": {"workload": f"learned_guess_{kind}_p{p}", "p": p, "train_solves": args.learned_train,
                   "test_solves": args.steps, "network": "3x512 ReLU", "epochs": 60,
                   "kappa": "dt/(2 Pe), Pe log-uniform [10,1000], dt uniform [1e-3,1e-2]"},
        "iters_plain_preconditioned": float(r["iters_plain"].mean()),
        "iters_from_precond_rhs": float(r["iters_precond"].mean()),
        "iters_learned": float(r["iters_learned"].mean()),
        "relres_median": {"precond_rhs": float(np.median(r["precond_relres"])),
                          "learned": float(np.median(r["guess_relres"]))},
        "guess_used_frac": float(r["guess_used"].mean()),
        "by_kappa": by_kappa,
        "train_loss": [float(m.history[0]), float(m.history[-1])],
        "active_outputs": int((m.gain > 0.5).sum()), "outputs": int(m.gain.size),
        "generate_s": t1 - t0, "train_s": t2 - t1,
    }
    print(json.dumps(res), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    choices=["batched_64_mixed_p", "large_256_p32", "two_drops_p32",
                             "single_drop_p16"],
                    help="default: large_256_p32 for the evaluation, two_drops_p32 for --solve, --step, "
                         "--evolve")
    ap.add_argument("--far-prec", default=None, choices=["fp32c", "fp64", "both"],
                    help="far-field precision (default: both for the evaluation, FP64 giving `value` and "
                         "the FP32 compensated far field the `fp32_far` object; fp64 for --solve)")
    ap.add_argument("--grid-mode", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=320)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--separate-u", action="store_true",
                    help="the double layer takes its own density u instead of f (a second self-interaction pass "
                         "per degree class; the far field reads u's records either way)")
    ap.add_argument("--graph", action="store_true", default=None,
                    help="replay the evaluation as a recorded HIP graph (default for "
                         "batched_64_mixed_p; per-kernel times then come from a second pass of the "
                         "same launches without the graph)")
    ap.add_argument("--no-graph", dest="graph", action="store_false")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--far-tile", default=None, metavar="TPTxCHUNKS[,TPTxCHUNKS]",
                    help="far-field tile shape (targets per thread x source chunks) instead of the autotuner's, "
                         "e.g. 2x16; a second shape after a comma is the FP32 path's when both precisions "
                         "run (profiling runs repeat the timed run's shapes)")
    ap.add_argument("--solve", choices=["en", "velocity"], default=None,
                    help="time the Galerkin GMRES solve (E_n with R = 0.5, E_u = 1; velocity with "
                         "lambda = 2 for the workload's f) instead of the evaluation; default workload "
                         "two_drops_p32, FP64 far field")
    ap.add_argument("--step", action="store_true",
                    help="time one explicit step of the method (E_n solve, forces, velocity solve, "
                         "position update) on two_drops_p32 with lambda = 2, R = 0.5, Q = 2, uniform "
                         "field E_u = 1, Ca_E = 0.3, clean drops, dt = 0.01")
    ap.add_argument("--serial", action="store_true",
                    help="self-interaction, then far field, on one stream (every kernel alone); by default "
                         "(overlap mode) the far field may run, whole or in part, on a second stream beside the "
                         "degree classes that leave room for it (the library's overlap plan, reported in the line)")
    ap.add_argument("--near", action="store_true",
                    help="time the evaluation of two p = 32 spheres --near-gap apart with and without the "
                         "nearly singular correction")
    ap.add_argument("--near-gap", type=float, default=0.01)
    ap.add_argument("--evolve", action="store_true",
                    help="time steps of Algorithm 1 (ehd_evolve_step) on two_drops_p32 with a linear-law "
                         "surfactant, Pe = 10, lambda = 2, R = 0.5, Q = 2, Ca_E = 0.3, E_u = 1, dt = 0.01")
    ap.add_argument("--learned", action="store_true",
                    help="train the learned initial guess of the implicit surfactant solve and count "
                         "GMRES iterations to 1e-10 with and without it (--steps = test solves)")
    ap.add_argument("--learned-p", type=int, default=32)
    ap.add_argument("--learned-kind", choices=["ehd", "iid"], default="ehd")
    ap.add_argument("--learned-train", type=int, default=10000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a MIB-mebibyte device buffer once (a plain "
                         "copy kernel of known size, to scale hardware byte counters)")
    ap.add_argument("--count-shapes", default="", metavar="TPTxCHUNKS[,...]",
                    help="after the timed steps, launch the far-field kernel once alone in each of these "
                         "tile shapes, per far-field precision (for hardware-counter runs)")
    args = ap.parse_args(argv)
    try:
        args.count_shapes = [tuple(int(v) for v in t.lower().split("x")) for t in args.count_shapes.split(",") if t]
        if any(len(t) != 2 for t in args.count_shapes):
            raise ValueError
    except ValueError:
        ap.error("--count-shapes takes TPTxCHUNKS[,TPTxCHUNKS...]")

    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        return 2

    import torch
    from paper_1811_10270_amd import ehdbim as E
    from paper_1811_10270_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        return 1
    dev = torch.device("cuda", 0)
    other = args.solve or args.step or args.evolve
    if args.workload is None:
        args.workload = "two_drops_p32" if other else "large_256_p32"
    if args.far_prec is None:
        args.far_prec = "fp64" if other else "both"
    if args.far_prec == "both" and other:
        args.far_prec = "fp64"
    if args.graph is None:
        args.graph = args.workload == "batched_64_mixed_p"
    args.overlap = not args.serial
    if args.learned:
        return bench_learned(args, torch, E, W, dev)
    if args.evolve:
        return bench_evolve(args, torch, E, W, dev)
    if args.near:
        return bench_near(args, torch, E, W, dev)
    if args.step:
        return bench_step(args, torch, E, W, dev)
    if args.solve:
        return bench_solve(args, torch, E, W, dev)
    return bench_eval(args, torch, E, W, dev)

if __name__ == "__main__":
    sys.exit(main())
