"""GPU: graph-mode replays and far-field tile shapes (batching row).

Graph replays must equal eager evaluations bit for bit (every kernel is
deterministic: fixed reduction orders, no atomics), also when the device
buffers are rewritten between replays and eager work runs in between; every
far-field tile shape must give the FP64 far field to rounding."""
import numpy as np
import pytest

from paper_1811_10270_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_10270_amd import ehdbim
    ehdbim.load()
    return ehdbim


def _setup(E, s):
    import torch
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    f = torch.from_numpy(s.fcoef).to(dev)
    sg = torch.from_numpy(s.sigcoef).to(dev)
    return ctx, f, sg, dev


def test_graph_replays_match_eager(E):
    import torch
    s = W.subset(W.batched_suspension(seed=3), list(range(10)))
    ctx, f, sg, dev = _setup(E, s)
    T = ctx.ntargets
    so = torch.zeros(9, T, dtype=torch.float64, device=dev)
    fo = torch.zeros_like(so)
    ref_s, ref_f = [], []
    for scale in (1.0, -0.5, 2.0):
        f.mul_(scale)
        sg.mul_(scale)
        ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP32C, so, fo)
        ctx.sync()
        ref_s.append(so.clone())
        ref_f.append(fo.clone())
        f.div_(scale)
        sg.div_(scale)
    ctx.set_graph(True)
    for rep in range(2):
        for k, scale in enumerate((1.0, -0.5, 2.0)):
            f.mul_(scale)
            sg.mul_(scale)
            so.zero_()
            fo.zero_()
            ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP32C, so, fo)
            ctx.sync()
            assert torch.equal(so, ref_s[k]) and torch.equal(fo, ref_f[k]), (rep, k)
            f.div_(scale)
            sg.div_(scale)
            # eager work of the program between replays
            torch.cuda.synchronize()
            _ = (so * 2.0).sum().item()
    # changing arguments records a new graph
    ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP32C, so[:8], fo[:8])
    ctx.sync()
    assert torch.equal(so[:8], ref_s[0][:8])
    ctx.set_graph(False)
    ctx.close()


def test_overlap_mode_matches_serial(E):
    """Far field on its own stream, concurrent with the self-interaction:
    the same bits as the serial evaluation, eagerly and in graph replays."""
    import torch
    for s in (W.subset(W.batched_suspension(seed=3), list(range(10))), W.two_drops(16, seed=4, gap=0.2),
              W.single_drop(16, seed=1)):
        ctx, f, sg, dev = _setup(E, s)
        T = ctx.ntargets
        ref = torch.zeros(9, T, dtype=torch.float64, device=dev)
        ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP32C, ref)
        ctx.sync()
        ctx.set_overlap(True)
        out = torch.zeros_like(ref)
        for graph in (False, True):
            ctx.set_graph(graph)
            for _ in range(3):
                out.zero_()
                ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP32C, out)
                ctx.sync()
                assert torch.equal(out, ref), graph
                _ = (out * 2.0).sum().item()          # eager work between replays
        ctx.set_graph(False)
        ctx.set_overlap(False)
        ctx.close()


def test_overlap_split_over_tile_shapes(E):
    """Overlap mode splits the far field's (target block, chunk) items into
    a looping part on the second stream and an ordinary launch: every tile
    shape, in both precisions, gives the serial evaluation's bits, with and
    without a p <= 48 class before the fork."""
    import torch
    for s in (W.subset(W.batched_suspension(seed=3), list(range(12))), W.two_drops(24, seed=5, gap=0.3)):
        ctx, f, sg, dev = _setup(E, s)
        T = ctx.ntargets
        for prec in (E.FAR_FP32C, E.FAR_FP64):
            for tpt, nch in ((1, 1), (1, 7), (2, 3), (2, 16)):
                ctx.set_far_config(tpt, nch)
                outs = []
                for ov in (False, True):
                    ctx.set_overlap(ov)
                    so = torch.zeros(9, T, dtype=torch.float64, device=dev)
                    fo = torch.zeros_like(so)
                    ctx.layer_potentials(f, None, sg, E.ALL_KINDS, prec, so, fo)
                    ctx.sync()
                    outs.append((so, fo))
                assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]), (prec, tpt, nch)
        ctx.set_overlap(False)
        ctx.close()


def test_overlap_with_separate_u(E):
    """A separate double-layer density takes a second self-interaction pass
    per degree class; in overlap mode both passes of the p <= 48 class run
    before the fork and both passes of the others after it.  Same bits as
    the serial order, every kind set that needs u, both precisions."""
    import torch
    s = W.with_separate_u(W.subset(W.batched_suspension(seed=3), list(range(12))))
    ctx, f, sg, dev = _setup(E, s)
    u = torch.from_numpy(s.ucoef).to(dev)
    T = ctx.ntargets
    for prec in (E.FAR_FP32C, E.FAR_FP64):
        for kinds in (E.ALL_KINDS, E.STOKES_DL, E.STOKES_DL | E.LAP_SL, E.STOKES_SL | E.STOKES_DL):
            outs = []
            for ov in (False, True):
                ctx.set_overlap(ov)
                rows = len(E.rows_for_kinds(kinds))
                so = torch.zeros(rows, T, dtype=torch.float64, device=dev)
                fo = torch.zeros_like(so)
                ctx.layer_potentials(f, u, sg, kinds, prec, so, fo)
                ctx.sync()
                outs.append((so, fo))
            assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]), (prec, kinds)
    ctx.set_overlap(False)
    ctx.close()


def test_overlap_fp64_single_kinds_and_solve(E):
    """Regression: the FP64 far field running beside the self-interaction
    slows some of its waves; the self kernel must not depend on its waves'
    relative timing (every kind alone, FP64 far field, bitwise), and a GMRES
    solve in overlap mode converges as the serial one does."""
    import torch
    s = W.two_drops(32, seed=2)
    ctx, f, sg, dev = _setup(E, s)
    T = ctx.ntargets
    for kinds in (E.LAP_DLADJ, E.LAP_SL, E.LAP_DL, E.STOKES_DL, E.STOKES_SL, E.ALL_KINDS):
        outs = []
        for ov in (False, True, True, True):
            ctx.set_overlap(ov)
            so = torch.zeros(9, T, dtype=torch.float64, device=dev)
            fo = torch.zeros_like(so)
            ctx.layer_potentials(f, None, sg, kinds, E.FAR_FP64, so, fo)
            ctx.sync()
            outs.append((so, fo))
        for so, fo in outs[1:]:
            assert torch.equal(so, outs[0][0]) and torch.equal(fo, outs[0][1]), kinds
    res = {}
    for ov in (False, True):
        ctx.set_overlap(ov)
        en = torch.zeros(ctx.num_coefs(), dtype=torch.float64, device=dev)
        res[ov] = ctx.solve_En(0.5, 1.0, 0.0, en, tol=1e-12) + (en.cpu(),)
    ctx.set_overlap(False)
    ctx.close()
    assert res[True][0] == res[False][0] and res[True][1] <= 1e-12
    assert torch.equal(res[True][2], res[False][2])


def test_far_tile_shapes_agree_and_autotune(E, tmp_path):
    import torch
    from paper_1811_10270_amd import autotune
    s = W.subset(W.batched_suspension(seed=3), list(range(12)))
    ctx, f, sg, dev = _setup(E, s)
    T = ctx.ntargets
    so = torch.zeros(9, T, dtype=torch.float64, device=dev)
    fo = torch.zeros_like(so)
    ref = None
    for tpt in (1, 2):
        for nch in (1, 3, 16):
            ctx.set_far_config(tpt, nch)
            ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP64, so, fo)
            ctx.sync()
            got = fo.cpu().numpy()
            if ref is None:
                ref = got
            else:
                err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
                assert np.all(err < 1e-13), (tpt, nch, err)
    with pytest.raises(E.EhdError):
        ctx.set_far_config(3, 1)
    cache = str(tmp_path / "tune.json")
    tpt, nch, timings, cached = autotune.autotune_far(ctx, s.p, s.q_far, s.grid_mode, E.FAR_FP32C,
                                                      cache_path=cache)
    assert not cached and len(timings) >= 4 and (tpt, nch) == ctx.far_config()
    tpt2, nch2, _, cached2 = autotune.autotune_far(ctx, s.p, s.q_far, s.grid_mode, E.FAR_FP32C,
                                                   cache_path=cache)
    assert cached2 and (tpt2, nch2) == (tpt, nch)
    ctx.layer_potentials(f, None, sg, E.ALL_KINDS, E.FAR_FP32C, so, fo)
    ctx.sync()
    err = np.abs(fo.cpu().numpy() - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert np.all(err < 1e-6), err
    ctx.close()


def test_self_class_times(E):
    """Per-degree-class kernel times: recorded for the classes present,
    zero for absent ones, and together within the self stage's time."""
    import torch
    s = W.batched_suspension(seed=3)
    # two drops of degree 16 and two of degree 32: classes 24 and 48 stay empty
    keep = ([d for d in range(s.ndrops) if int(s.p[d]) == 16][:2]
            + [d for d in range(s.ndrops) if int(s.p[d]) == 32][:2])
    sub = W.subset(s, keep)
    ctx, f, sg, dev = _setup(E, sub)
    out = torch.zeros(8, ctx.ntargets, dtype=torch.float64, device=dev)
    ctx.set_timing(2)
    for _ in range(2):
        ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP32C, out)
    ctx.sync()
    for slot in range(2):
        ms = ctx.self_class_times(slot)
        st = ctx.stage_times(slot)
        present = {pm for pm in E.DEGREE_CLASSES for d in range(sub.ndrops)
                   if (E.DEGREE_CLASSES[E.DEGREE_CLASSES.index(pm) - 1] if pm != 16 else 0)
                   < int(sub.p[d]) <= pm}
        for c, pm in enumerate(E.DEGREE_CLASSES):
            assert (ms[c] > 0) == (pm in present), (pm, ms)
        assert sum(ms) <= st[1] * 1.02 + 0.05
    ctx.close()


def test_bench_graph_configuration_batched(E):
    """The benchmark's configuration of the 64-drop mixed-degree workload:
    overlap mode, the far-field tile the autotuner picks for the metric's
    kinds, and the evaluation recorded as one HIP graph and replayed.  Every
    replay, with eager work and synchronisations between them, gives the
    eager result bit for bit, in both far-field precisions."""
    import torch
    from paper_1811_10270_amd import autotune
    s = W.batched_suspension(seed=3)
    ctx, f, sg, dev = _setup(E, s)
    ctx.set_overlap(True)
    out = torch.zeros(8, ctx.ntargets, dtype=torch.float64, device=dev)
    for prec in (E.FAR_FP32C, E.FAR_FP64):
        autotune.autotune_far(ctx, s.p, s.q_far, s.grid_mode, prec, kinds=E.METRIC_KINDS, use_cache=False)
        ctx.set_graph(False)
        ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, prec, out)
        ctx.sync()
        ref = out.clone()
        ctx.set_graph(True)
        for rep in range(3):
            out.fill_(7.0)
            ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, prec, out)
            ctx.sync()
            assert torch.equal(out, ref), (prec, rep)
            _ = (out * 2.0).sum().item()          # eager work between replays
            torch.cuda.synchronize()
        ctx.set_graph(False)
    ctx.close()


def test_overlap_plan(E):
    """The overlap plan the library reports: serial order outside overlap
    mode, for one drop and for the FP64 far field of a large workload; a
    tiny far field forks whole; the FP32 far field of the 64-drop workload
    never forks beside the p <= 48 class, forks exactly when some class
    runs beside it, and the evaluation it plans gives the serial bits."""
    import torch
    big = W.batched_suspension(seed=3)
    ctx, f, sg, dev = _setup(E, big)
    assert ctx.overlap_plan(E.ALL_KINDS, E.FAR_FP32C) == (0, 0)
    ctx.set_overlap(True)
    assert ctx.overlap_plan(E.METRIC_KINDS, E.FAR_FP64) == (0, 0)
    present = 0
    for c, pmax in enumerate(E.DEGREE_CLASSES):
        lo = E.DEGREE_CLASSES[c - 1] if c else 0
        present |= int(any(lo < int(p) <= pmax for p in big.p)) << c
    for kinds, with_u in ((E.METRIC_KINDS, False), (E.ALL_KINDS, True), (E.LAP_SL, False)):
        beside, forked = ctx.overlap_plan(kinds, E.FAR_FP32C, with_u)
        assert not beside & 8 and beside & ~present == 0, (kinds, beside)
        assert (forked > 0) == (beside != 0), (kinds, beside, forked)
    T = ctx.ntargets
    outs = []
    for ov in (False, True):
        ctx.set_overlap(ov)
        so = torch.zeros(8, T, dtype=torch.float64, device=dev)
        fo = torch.zeros_like(so)
        ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP32C, so, fo)
        ctx.sync()
        outs.append((so, fo))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    ctx.set_overlap(False)
    ctx.close()
    for s, whole in ((W.single_drop(16, seed=1), False), (W.two_drops(16, seed=4, gap=0.2), True)):
        ctx, f, sg, dev = _setup(E, s)
        ctx.set_overlap(True)
        ctx.set_far_config(2, 1)
        for prec in (E.FAR_FP32C, E.FAR_FP64):
            beside, forked = ctx.overlap_plan(E.METRIC_KINDS, prec)
            assert (forked > 0) == whole and beside == (1 if whole else 0), (s.ndrops, prec, beside, forked)
        ctx.set_overlap(False)
        ctx.close()


def test_self_prefetch_autotuner(E, tmp_path):
    """Every Legendre prefetch batch built for a degree class gives the same
    bits (only the load schedule differs); ehd_time_self times a class; the
    autotuner picks one of the candidates per class present, sets it, and a
    second call takes it from its cache; a batch not built is refused."""
    import torch
    from paper_1811_10270_amd import autotune
    s = W.subset(W.batched_suspension(seed=3), list(range(12)))
    ctx, f, sg, dev = _setup(E, s)
    T = ctx.ntargets
    present = [c for c, pm in enumerate(E.DEGREE_CLASSES)
               if any((E.DEGREE_CLASSES[c - 1] if c else 0) < int(p) <= pm for p in s.p)]
    assert len(present) >= 3
    ref = torch.zeros(8, T, dtype=torch.float64, device=dev)
    ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP64, ref)
    ctx.sync()
    for c in present:
        for pf in E.self_config_candidates(c):
            ctx.set_self_config(c, pf)
            assert ctx.self_config(c) == pf
            out = torch.zeros_like(ref)
            ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP64, out)
            ctx.sync()
            assert torch.equal(out, ref), (c, pf)
            assert ctx.time_self(c, pf, f, sg, 1) > 0.0
        ctx.set_self_config(c, 0)
    with pytest.raises(RuntimeError):
        ctx.set_self_config(present[0], 7)
    cache = str(tmp_path / "tune.json")
    best, timings, cached = autotune.autotune_self(ctx, s.p, s.q_self, s.grid_mode, f, sg, cache_path=cache)
    assert not cached and sorted(best) == sorted(E.DEGREE_CLASSES[c] for c in present)
    for c in present:
        pm = E.DEGREE_CLASSES[c]
        assert best[pm] in E.self_config_candidates(c) and ctx.self_config(c) == best[pm]
        assert min(timings[pm], key=timings[pm].get) == str(best[pm])
    ctx2, f2, sg2, _ = _setup(E, s)
    best2, _, cached2 = autotune.autotune_self(ctx2, s.p, s.q_self, s.grid_mode, f2, sg2, cache_path=cache)
    assert cached2 and best2 == best
    # overlap mode and graph replays with the tuned batches: the same bits
    ctx.set_overlap(True)
    ctx.set_graph(True)
    for _ in range(2):
        out = torch.zeros_like(ref)
        ctx.layer_potentials(f, None, sg, E.METRIC_KINDS, E.FAR_FP64, out)
        ctx.sync()
        assert torch.equal(out, ref)
    ctx.set_graph(False)
    ctx.set_overlap(False)
    ctx.close()
    ctx2.close()
