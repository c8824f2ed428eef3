"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bar: FP64 results within 1e-10 relative (normwise per output component:
max |gpu - oracle| / max |oracle| over the targets compared).  The FP32
compensated far field is held to 1e-6 against the oracle, per output
(FP32_FAR_BOUND).  Full-size workloads compare against oracle values stored
by tests/golden/make_golden.py (calls only the oracle and the seeded
generator).
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1811_10270_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_FAR_BOUND = 1e-6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name, s):
    """A stored oracle fixture, checked to belong to the inputs `s`."""
    sys.path.insert(0, GOLDEN)
    try:
        from make_golden import input_checksums
    finally:
        sys.path.pop(0)
    g = np.load(os.path.join(GOLDEN, name + ".npz"))
    np.testing.assert_allclose(g["checksums"], input_checksums(s), rtol=1e-14, atol=0,
                               err_msg="fixture does not match the generator's inputs")
    return g


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_10270_amd import ehdbim
    ehdbim.load()
    return ehdbim


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(got, ref):
    den = np.abs(ref).max(axis=-1)
    den = np.where(den == 0, 1.0, den)
    return np.abs(got - ref).max(axis=-1) / den


def run(E, s, kinds=31, far_prec=0, split=True, bench_config=False):
    """One evaluation; bench_config: overlap mode and the autotuned far-field
    tile shape, the launch configuration bench.py times."""
    say(f"[gpu] {s.name}: ndrops={s.ndrops} p={sorted(set(s.p.tolist()))} kinds={kinds} "
        f"far_prec={far_prec} grid_mode={s.grid_mode} bench_config={bench_config}")
    return E.evaluate(s, kinds=kinds, far_prec=far_prec, split=split, overlap=bench_config, autotune=bench_config)


def sample(s, per_drop, seed=0):
    rng = np.random.default_rng(seed)
    td, tn = oracle.all_targets(s)
    off = s.target_offsets()
    idx = []
    for d in range(s.ndrops):
        n = off[d + 1] - off[d]
        k = min(per_drop, n)
        pick = rng.choice(n, size=k, replace=False)
        # always include the first and last node (poles' neighbourhoods)
        pick = np.unique(np.concatenate([pick, [0, n - 1]]))
        idx.append(off[d] + pick)
    idx = np.concatenate(idx)
    return idx, td[idx], tn[idx]


# ---------------------------------------------------------------------------
def test_target_geometry_and_synthesis(E):
    import torch
    s = W.batched_suspension(seed=3)
    s = W.subset(s, [0, 1, 2, 3, 4, 5])
    ctx = E.Context(0)
    dev = torch.device("cuda", 0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    T = ctx.ntargets
    x = torch.zeros(3, T, dtype=torch.float64, device=dev)
    n = torch.zeros_like(x)
    ctx.target_geometry(x, n)
    g = torch.zeros(1, T, dtype=torch.float64, device=dev)
    ctx.synthesize(1, torch.from_numpy(s.sigcoef).to(dev), g)
    c = torch.zeros(s.sigcoef.shape[0], dtype=torch.float64, device=dev)
    ctx.analyze(1, g, c)
    ctx.sync()
    td, tn = oracle.all_targets(s)
    xr, nr = oracle.targets(s, td, tn)
    assert np.abs(x.cpu().numpy() - xr).max() < 1e-12
    assert np.abs(n.cpu().numpy() - nr).max() < 1e-12
    # synthesis against the oracle, drop by drop
    off = s.target_offsets()
    coff = W.drop_offsets(s.p.astype(np.int64))
    gg = g.cpu().numpy()[0]
    for d in range(s.ndrops):
        p = int(s.p[d])
        ref = oracle.synth_grid(p, s.sigcoef[coff[d]:coff[d + 1]], p, s.grid_mode).ravel()
        assert np.abs(gg[off[d]:off[d + 1]] - ref).max() < 1e-12
    # exact round trip on the paper's grid
    cc = c.cpu().numpy()
    for d in range(s.ndrops):
        blk = s.sigcoef[coff[d]:coff[d + 1]].copy()
        p = int(s.p[d])
        for nn in range(p + 1):
            blk[2 * (nn * (nn + 1) // 2) + 1] = 0.0
        assert np.abs(cc[coff[d]:coff[d + 1]] - blk).max() < 1e-12
    ctx.close()


def test_self_single_drop_full(E):
    """Single drop p=16 (shape 1 + 0.1 Y20 + random), q=32, every target."""
    s = W.single_drop(16, seed=1)
    so, fo = run(E, s)
    td, tn = oracle.all_targets(s)
    ref = oracle.self_(s, td, tn)
    err = normwise(so.numpy(), ref)
    say("self p16 normwise err", err)
    assert np.all(err < FP64_TOL), err
    assert np.abs(fo.numpy()).max() == 0.0      # one drop: no far field


def test_self_grid_mode_2p_and_separate_u(E):
    s = W.with_separate_u(W.single_drop(12, seed=4, grid_mode=1))
    s.q_self[:] = 30
    so, _ = run(E, s)
    td, tn = oracle.all_targets(s)
    ref = oracle.self_(s, td, tn)
    err = normwise(so.numpy(), ref)
    say("self p12 mode-2p separate-u err", err)
    assert np.all(err < FP64_TOL), err


@pytest.mark.parametrize("p", [1, 2, 3])
def test_self_tiny_degrees(E, p):
    s = W.single_drop(p, seed=7, eps_y20=0.0, amp=0.02)
    s.q_self[:] = 4 * p + 1
    s.q_far[:] = p
    so, _ = run(E, s)
    td, tn = oracle.all_targets(s)
    ref = oracle.self_(s, td, tn)
    err = normwise(so.numpy(), ref)
    assert np.all(err < FP64_TOL), err


@pytest.mark.parametrize("q", [48, 127])
def test_self_max_degree_and_grid_extremes(E, q):
    """p = 48, the largest degree, on the smallest (q = p: two row tiles of
    longitude sums) and the largest (q = 127, 256 longitudes: eight row
    tiles, one per wave) rotated grids; sampled targets, both poles'
    neighbourhoods included.  One degree more is refused."""
    import torch
    s = W.single_drop(48, seed=3)
    s.q_self[:] = q
    s.q_far[:] = q
    if q == 127:
        ctx = E.Context(0)
        with pytest.raises(E.EhdError) as ei:
            ctx.set_drops(s.p, s.q_self + 1, s.q_far, s.grid_mode,
                          torch.from_numpy(s.xcoef).to(torch.device("cuda", 0)))
        assert ei.value.code == E.EHD_E_SHAPE
        ctx.close()
    so, _ = run(E, s)
    idx, td, tn = sample(s, 6, seed=4)
    ref = oracle.self_(s, td, tn)
    err = normwise(so.numpy()[:, idx], ref)
    say(f"self p48 q{q} err", err)
    assert np.all(err < FP64_TOL), err


def test_far_largest_grid(E):
    """The far field on the largest source grid (q_far = 160, 51,842 nodes
    per drop) at every target of two p = 8 drops: FP64 against the oracle,
    the compensated FP32 sums within their bound."""
    s = W.two_drops(8, seed=6, gap=0.2)
    s.q_far[:] = 160
    _, fo = run(E, s, far_prec=0)
    _, fo32 = run(E, s, far_prec=1)
    td, tn = oracle.all_targets(s)
    ref = oracle.far(s, td, tn)
    err, err32 = normwise(fo.numpy(), ref), normwise(fo32.numpy(), ref)
    say("far q_far 160 err fp64", err, "fp32", err32)
    assert np.all(err < FP64_TOL) and np.all(err32 < FP32_FAR_BOUND), (err, err32)


def test_far_fp64_two_drops(E):
    """Two p=12 spheres at gap 0.1, far grid q = 3p (near-contact pair)."""
    s = W.two_drops(12, seed=2, q_far_mult=3)
    so, fo = run(E, s)
    td, tn = oracle.all_targets(s)
    ref = oracle.far(s, td, tn)
    err = normwise(fo.numpy(), ref)
    say("far fp64 two drops err", err)
    assert np.all(err < FP64_TOL), err


def test_far_fp32_two_drops_bound(E):
    s = W.two_drops(12, seed=2, q_far_mult=3)
    _, fo = run(E, s, far_prec=1)
    td, tn = oracle.all_targets(s)
    ref = oracle.far(s, td, tn)
    err = normwise(fo.numpy(), ref)
    say("far fp32 two drops err", err)
    assert np.all(err < FP32_FAR_BOUND), err


def test_mixed_degrees_subset_all_kinds(E):
    """Six drops of the batched suspension (p in {16,24,32,48}), sampled
    targets, self and far separately, FP64."""
    s0 = W.batched_suspension(seed=3)
    pick = [int(np.where(s0.p == pp)[0][0]) for pp in (16, 24, 32, 48)]
    s = W.subset(s0, pick + [int(np.where(s0.p == 16)[0][1]), int(np.where(s0.p == 48)[0][1])])
    so, fo = run(E, s)
    idx, td, tn = sample(s, 12, seed=1)
    rs = oracle.self_(s, td, tn)
    rf = oracle.far(s, td, tn)
    es = normwise(so.numpy()[:, idx], rs)
    ef = normwise(fo.numpy()[:, idx], rf)
    say("subset self err", es, "far err", ef)
    assert np.all(es < FP64_TOL) and np.all(ef < FP64_TOL), (es, ef)


def test_kinds_rows_and_summed_output(E):
    s = W.two_drops(8, seed=5)
    so_all, fo_all = run(E, s, kinds=31)
    kinds = E.STOKES_DL | E.LAP_SL
    rows = E.rows_for_kinds(kinds)
    so, fo = run(E, s, kinds=kinds)
    assert so.shape[0] == len(rows) == 4
    np.testing.assert_array_equal(so.numpy(), so_all.numpy()[rows])
    np.testing.assert_array_equal(fo.numpy(), fo_all.numpy()[rows])
    tot, none = run(E, s, kinds=31, split=False)
    assert none is None
    np.testing.assert_allclose(tot.numpy(), so_all.numpy() + fo_all.numpy(), rtol=0, atol=1e-14)


def test_argument_errors(E):
    import torch
    ctx = E.Context(0)
    dev = torch.device("cuda", 0)
    x = torch.zeros(3 * 20, dtype=torch.float64, device=dev)
    with pytest.raises(E.EhdError) as ei:        # no drops
        ctx.set_drops([], [], [], 0, x)
    assert ei.value.code == E.EHD_E_ARG
    with pytest.raises(E.EhdError) as ei:
        ctx.set_drops([0], [4], [4], 0, x)
    assert ei.value.code == E.EHD_E_SHAPE
    with pytest.raises(E.EhdError) as ei:
        ctx.set_drops([60], [120], [120], 0, torch.zeros(3 * 61 * 62, dtype=torch.float64, device=dev))
    assert ei.value.code == E.EHD_E_SHAPE
    out = torch.zeros(9, 10, dtype=torch.float64, device=dev)
    with pytest.raises(E.EhdError) as ei:
        ctx.layer_potentials(x, None, x, 31, 0, out)
    assert ei.value.code == E.EHD_E_STATE
    s = W.single_drop(3, seed=1)
    ctx.set_drops(s.p, s.q_self, s.q_far, 0, torch.from_numpy(s.xcoef).to(dev))
    f = torch.from_numpy(s.fcoef).to(dev)
    sg = torch.from_numpy(s.sigcoef).to(dev)
    for bad_kinds in (0, 32, 64):
        with pytest.raises(E.EhdError):
            ctx.layer_potentials(f, None, sg, bad_kinds, 0, out)
    with pytest.raises(E.EhdError):
        ctx.layer_potentials(f, None, sg, 31, 7, out)
    with pytest.raises(E.EhdError):
        ctx.layer_potentials(f, None, None, E.LAP_SL, 0, out)
    ctx.close()


def test_full_batched_suspension_sampled(E):
    """The full 64-drop batched suspension, FP64 and FP32 far field, in the
    benchmark's launch configuration, sampled targets against the oracle
    (self and far separately)."""
    s = W.batched_suspension(seed=3)
    so, fo = run(E, s, kinds=31, far_prec=0, bench_config=True)
    _, fo32 = run(E, s, kinds=31, far_prec=1, bench_config=True)
    rng = np.random.default_rng(2)
    td_all, tn_all = oracle.all_targets(s)
    idx = np.sort(rng.choice(len(td_all), size=48, replace=False))
    rf = oracle.far(s, td_all[idx], tn_all[idx])
    ef = normwise(fo.numpy()[:, idx], rf)
    ef32 = normwise(fo32.numpy()[:, idx], rf)
    say("batched far fp64 err", ef)
    say("batched far fp32 err", ef32)
    assert np.all(ef < FP64_TOL), ef
    assert np.all(ef32 < FP32_FAR_BOUND), ef32
    sidx = idx[::6]
    rs = oracle.self_(s, td_all[sidx], tn_all[sidx])
    es = normwise(so.numpy()[:, sidx], rs)
    say("batched self err", es)
    assert np.all(es < FP64_TOL), es


@pytest.mark.parametrize("name", ["two_drops_p32", "batched_64_mixed_p", "large_256_p32"])
def test_fp32_far_field_bound_full_size(E, name):
    """FP32 compensated far field against the FP64 far field at every target
    of the full workload (the FP64 far field itself is pinned to the oracle
    on sampled targets below and above): normwise error <= 1e-6 per output."""
    s = W.WORKLOADS[name](0)
    _, f64 = run(E, s, kinds=31, far_prec=0)
    _, f32 = run(E, s, kinds=31, far_prec=1, bench_config=True)
    err = normwise(f32.numpy(), f64.numpy())
    say(name, "fp32 far normwise err", err)
    assert np.all(err < 1e-6), err


def test_large_suspension_16_drops_against_oracle(E):
    """256 drops at p = 32 (q = 2p) in the benchmark's launch configuration:
    the far field at EVERY node of 16 drops (34,848 targets, all 255 other
    drops as sources) against the stored oracle values, FP64 to 1e-10 and
    the FP32 compensated far field to 1e-6 per output; the singular
    self-interaction at 352 stored sampled nodes of those drops to 1e-10."""
    s = W.large_suspension(seed=5)
    g = golden("large_256_p32_far16", s)
    idx, sidx = g["far_idx"], g["self_idx"]
    so, fo = run(E, s, kinds=31, far_prec=0, bench_config=True)
    ef = normwise(fo.numpy()[:, idx], g["far"])
    es = normwise(so.numpy()[:, sidx], g["self"])
    say("large 16-drop far fp64 err", ef)
    say("large sampled self err", es)
    _, fo32 = run(E, s, kinds=31, far_prec=1, bench_config=True)
    ef32 = normwise(fo32.numpy()[:, idx], g["far"])
    say("large 16-drop far fp32 err", ef32)
    assert np.all(ef < FP64_TOL) and np.all(es < FP64_TOL), (ef, es)
    assert np.all(ef32 < FP32_FAR_BOUND), ef32


def test_whole_p48_drop_self_against_oracle(E):
    """One p = 48 drop at q_self = 96: every one of its 4,802 nodes (every
    latitude's rotation table) against the stored oracle values."""
    b = W.batched_suspension(seed=3)
    d48 = int(np.nonzero(b.p == 48)[0][0])
    s = W.subset(b, [d48])
    g = golden("p48_q96_drop_self", s)
    assert int(g["drop"]) == d48
    so, _ = run(E, s, kinds=31, far_prec=0)
    es = normwise(so.numpy(), g["self"])
    say("whole p48 drop self err", es)
    assert np.all(es < FP64_TOL), es


def test_two_drops_near_contact_q96(E):
    """Two p=32 spheres at gap 0.1, far grid q = 96 (3x), every target of
    drop 0's first latitude rows and a sample of the rest against the oracle."""
    s = W.two_drops(32, seed=2)
    so, fo = run(E, s, kinds=31, far_prec=0)
    idx = np.concatenate([np.arange(0, 200), np.arange(2178, 2178 + 100)])
    td, tn = oracle.all_targets(s)
    rf = oracle.far(s, td[idx], tn[idx])
    ef = normwise(fo.numpy()[:, idx], rf)
    rs = oracle.self_(s, td[idx[::25]], tn[idx[::25]])
    es = normwise(so.numpy()[:, idx[::25]], rs)
    say("two drops q96 far err", ef, "self err", es)
    assert np.all(ef < FP64_TOL) and np.all(es < FP64_TOL), (ef, es)
