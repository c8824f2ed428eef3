"""Benchmark: layer-potential target evaluations per second on one MI355X.

One step = one call of ehd_layer_potentials over the whole workload: the
singular self-interaction of every target (FP64, rotated-pole rule) plus the
far-field direct sums over every other drop (FP32 with compensated
accumulation by default), the four potentials of the metric (S, D, S_L, L:
8 values per target).  Inputs are resident in HBM before the timed region.

Prints one JSON line.
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


def self_flops_per_drop(p: int, q: int, grid_mode: int) -> float:
    """Algorithmic FP64 work of the singular self-interaction of one drop:
    rotation of 7 fields, Legendre sums (7 fields + 3 theta derivatives),
    longitude sums of 13 grid quantities, kernel evaluation per rotated node."""
    nlon_p = 2 * p + 2 if grid_mode == 0 else 2 * p
    nlon_q = 2 * q + 2 if grid_mode == 0 else 2 * q
    T = (p + 1) * nlon_p
    rot = 4 * 7 * T * sum((n + 1) * (2 * n + 1) for n in range(p + 1))
    leg = 4 * (q + 1) * ((p + 1) * (p + 2) // 2) * 10 * T
    dft = 2 * nlon_q * (2 * p + 1) * (q + 1) * 13 * T
    ker = SELF_KERNEL_FLOPS_PER_NODE * T * (q + 1) * nlon_q
    return float(rot + leg + dft + ker)


# HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs
# recorded in profiles/hbm_traffic_batched_64_mixed_p.md (counters scaled by a
# 1 GiB copy), valid only for the kernel source they were taken with.
TRAFFIC_SOURCE_SHA256 = "4647d00ccf0c4d100f64afeb9ea8e37e22121ddc95bb82654628be165c9caef3"
TRAFFIC_WORKLOAD = "batched_64_mixed_p"
TRAFFIC_BYTES = {"k_self<48>": 6.527e+08, "k_self<32>": 1.201e+08, "k_self<24>": 2.54e+07,
                 "k_self<16>": 7.373e+06, "k_far32": 7.964e+08}


def measured_traffic(kernel: str, workload: str):
    import hashlib
    path = os.path.join(ROOT, "paper_1811_10270_amd", "csrc", "ehdbim.hip")
    with open(path, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != TRAFFIC_SOURCE_SHA256 or workload != TRAFFIC_WORKLOAD:
            return None
    return TRAFFIC_BYTES.get(kernel.split(" ")[0])


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


def cpu_baseline(s, nsample: int, seed: int = 0):
    """The oracle timed on a bounded random sample of the workload's targets:
    self (singular rule) + far (all other drops) for each sampled target."""
    import numpy as np
    import oracle
    td, tn = oracle.all_targets(s)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(td), size=min(nsample, len(td)), replace=False))
    t0 = time.perf_counter()
    oracle.self_(s, td[idx], tn[idx])
    t1 = time.perf_counter()
    oracle.far(s, td[idx], tn[idx])
    t2 = time.perf_counter()
    return {
        "value": len(idx) / (t2 - t0),
        "unit": "target-evals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{len(idx)} random targets of {len(td)} (seed {seed}), self + far over all "
                  f"{s.ndrops} drops, FP64; self {t1 - t0:.1f} s, far {t2 - t1:.1f} s",
    }


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
                             "single_drop_p16"])
    ap.add_argument("--far-prec", default=None, choices=["fp32c", "fp64"],
                    help="far-field precision (default: fp32c for the evaluation, fp64 for --solve)")
    ap.add_argument("--grid-mode", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=320)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="replay the evaluation as a recorded HIP graph (stage times then hold "
                         "the whole evaluation in the first stage)")
    ap.add_argument("--no-autotune", action="store_true")
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
                         "the far field runs, whole or in part, on a second stream beside the self-interaction")
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
    args = ap.parse_args(argv)

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
    if args.workload is None:
        args.workload = "two_drops_p32" if (args.solve or args.step or args.evolve) else "batched_64_mixed_p"
    if args.far_prec is None:
        args.far_prec = "fp64" if (args.solve or args.step or args.evolve) else "fp32c"
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
    s = W.WORKLOADS[args.workload](args.grid_mode)
    far_prec = E.FAR_FP32C if args.far_prec == "fp32c" else E.FAR_FP64
    kinds = E.METRIC_KINDS

    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if args.overlap:
        ctx.set_overlap(True)
    T = ctx.ntargets
    tile = {"targets_per_thread": ctx.far_config()[0], "source_chunks": ctx.far_config()[1],
            "autotuned": False}
    if not args.no_autotune:
        from paper_1811_10270_amd import autotune
        tpt, nch, timings, cached = autotune.autotune_far(ctx, s.p, s.q_far, s.grid_mode, far_prec)
        tile = {"targets_per_thread": tpt, "source_chunks": nch, "autotuned": True,
                "from_cache": cached}
    if args.graph:
        ctx.set_graph(True)
    f = torch.from_numpy(s.fcoef).to(dev)
    sig = torch.from_numpy(s.sigcoef).to(dev)
    out = torch.empty(len(E.rows_for_kinds(kinds)), T, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        ctx.layer_potentials(f, None, sig, kinds, far_prec, out)
    ctx.sync()
    torch.cuda.synchronize()

    K = args.steps
    ctx.set_timing(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.layer_potentials(f, None, sig, kinds, far_prec, out)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    stages = [ctx.stage_times(i) for i in range(K)]
    avg = [sum(st[k] for st in stages) / K for k in range(4)]
    cls_times = [ctx.self_class_times(i) for i in range(K)] if not args.graph else None

    # per-kernel rooflines; the dominant kernel's goes to "roofline" (none if
    # every kernel shares the device).  Kernels that run beside the forked
    # far field are "shared": their times are wall times, not theirs alone;
    # the far field itself then has no time of its own.
    self_flops = sum(self_flops_per_drop(int(s.p[d]), int(s.q_self[d]), s.grid_mode)
                     for d in range(s.ndrops))
    far_flops = far_interactions(s) * FAR_FLOPS_PER_INTERACTION
    kernels = []
    # the library's overlap regimes: a far field of at most two work items
    # per CU forks whole (every class shares the device), a larger one after
    # the p <= 48 class
    tpt_, nch_ = ctx.far_config()
    items = -(-T // (256 * tpt_)) * nch_
    whole = items <= 2 * torch.cuda.get_device_properties(0).multi_processor_count
    if s.ndrops < 2:
        args.overlap = False   # the library keeps the serial order for one drop
    if cls_times is not None:
        for c, pmax in enumerate(E.DEGREE_CLASSES):
            ms = sum(ct[c] for ct in cls_times) / K
            lo = E.DEGREE_CLASSES[c - 1] if c else 0
            fl = sum(self_flops_per_drop(int(s.p[d]), int(s.q_self[d]), s.grid_mode)
                     for d in range(s.ndrops) if lo < int(s.p[d]) <= pmax)
            if ms > 0 and fl > 0:
                kernels.append({"kernel": f"k_self<{pmax}> (singular self-interaction, p <= {pmax}, FP64)",
                                "bound": "alu", "algorithmic_flops": fl, "avg_ms": ms,
                                "achieved": fl / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                                "shared": bool(args.overlap and (whole or pmax < 48))})
        far_peak = PEAK_FP32_UNPACKED_TFLOPS if far_prec == E.FAR_FP32C else PEAK_FP64_TFLOPS
        far_ms = None if args.overlap else avg[2]
        kernels.append({"kernel": ("k_far32" if far_prec == E.FAR_FP32C else "k_far64")
                        + " (far-field direct sums)", "bound": "alu", "algorithmic_flops": far_flops,
                        "avg_ms": far_ms, "achieved": far_flops / (far_ms * 1e-3) / 1e12 if far_ms else None,
                        "peak": far_peak, "shared": bool(args.overlap)})
        for k in kernels:
            k["unit"] = "TFLOP/s"
            k["frac"] = k["achieved"] / k["peak"] if k["achieved"] is not None else None
            # per-launch counter bytes; the far field's two overlap launches have none
            k["traffic"] = None if (k["shared"] and k["avg_ms"] is None) else measured_traffic(k["kernel"], args.workload)
    roof = None
    alone = [k for k in kernels if not k["shared"]]
    if alone:
        dom = max(alone, key=lambda k: k["avg_ms"])
        roof = {"kernel": dom["kernel"], "bound": dom["bound"], "achieved": dom["achieved"],
                "peak": dom["peak"], "unit": "TFLOP/s", "frac": dom["frac"], "traffic": dom["traffic"],
                "algorithmic_flops": dom["algorithmic_flops"], "avg_ms": dom["avg_ms"]}

    res = {
        "metric": "layer-potential target evals/sec (singular+far) FP64 self + "
                  + ("FP32 far" if far_prec == E.FAR_FP32C else "FP64 far"),
        "value": T * K / dt,
        "unit": "target-evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if far_prec == E.FAR_FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "overlap": args.overlap, "ndrops": s.ndrops,
                   "p": sorted(set(int(x) for x in s.p)), "targets": T,
                   "q_self": "2p", "q_far": "2p", "grid": "paper (2p+2 longitudes)"
                   if s.grid_mode == 0 else "2p longitudes",
                   "kinds": "S,D,S_L,L", "far_prec": args.far_prec,
                   "far_interactions": far_interactions(s), "far_tile": tile,
                   "graph": bool(args.graph)},
        "stage_ms": dict(zip(E.STAGES, avg)),
        "self_tflops": None if args.overlap else self_flops / (avg[1] * 1e-3) / 1e12,
        "far_tflops": None if args.overlap else far_flops / (avg[2] * 1e-3) / 1e12,
        "roofline": roof,
        "kernels": kernels,
    }
    ctx.close()
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
        res["cpu_baseline"] = cpu_baseline(s, args.cpu_sample)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
