"""GPU: the nearly singular correction (Sec. 2.1, interpolation approach)
against the oracle's line interpolation on two close drops, and against the
exterior unit-sphere closed forms through the whole evaluation."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from oracle import near as N
from paper_1811_10270_amd import workloads as W
from test_oracle_pins import field, make_susp, sphere_x, tri, y_entry

pytestmark = pytest.mark.gpu


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


def two_spheres(p, gap, r2=1.0, seed=5, q_far=None):
    """Unit sphere at the origin and a sphere of radius r2 above it along a
    tilted axis, surfaces `gap` apart; random decaying densities."""
    axis = np.array([0.3, -0.2, 0.93])
    axis /= np.linalg.norm(axis)
    x = np.concatenate([sphere_x(p), sphere_x(p, R=r2, centre=tuple((1.0 + gap + r2) * axis))])
    rng = np.random.default_rng(seed)
    nc2 = (p + 1) * (p + 2)

    def dens(nf):
        out = np.zeros(2 * nf * nc2)
        for blk in range(2 * nf):
            for n in range(p + 1):
                for m in range(n + 1):
                    k = blk * nc2 + 2 * tri(n, m)
                    out[k] = rng.standard_normal() / (n + 1) ** 2
                    if m:
                        out[k + 1] = rng.standard_normal() / (n + 1) ** 2
        return out
    f, u, sg = dens(3), dens(3), dens(1)
    pa = np.array([p, p], np.int32)
    qf = 2 * pa if q_far is None else np.array([q_far, q_far], np.int32)
    return W.Suspension("near", pa, 2 * pa, qf, 0, x, f, sg, u, np.zeros((2, 3)), np.ones(2))


def gpu_eval(E, s, near=None):
    import torch
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    if near:
        ctx.set_near(*near)
    npairs = ctx.near_pairs()
    T = ctx.ntargets
    out = torch.empty(9, T, dtype=torch.float64, device=dev)
    ctx.layer_potentials(torch.from_numpy(s.fcoef).to(dev), torch.from_numpy(s.ucoef).to(dev),
                         torch.from_numpy(s.sigcoef).to(dev), E.ALL_KINDS, E.FAR_FP64, out)
    x0 = torch.empty(3, T, dtype=torch.float64, device=dev)
    n0 = torch.empty(3, T, dtype=torch.float64, device=dev)
    ctx.target_geometry(x0, n0)
    res = out.cpu().numpy(), x0.cpu().numpy(), n0.cpu().numpy(), npairs
    ctx.close()
    return res


def test_near_correction_matches_oracle(E):
    p, gap, delta, m, qc = 8, 0.02, 0.12, 6, 80
    sc = 3 * math.pi / (qc + 1)
    s = two_spheres(p, gap)
    plain, x0, n0, _ = gpu_eval(E, s)
    corr, _, _, npairs = gpu_eval(E, s, (delta, sc, m, qc))
    changed = np.flatnonzero(np.abs(corr - plain).max(axis=0) > 0)
    say("near pairs", npairs, "changed targets", len(changed))
    assert npairs > 0 and len(changed) > 0
    td, tn = oracle.all_targets(s)
    rng = np.random.default_rng(1)
    sample = rng.choice(changed, size=min(6, len(changed)), replace=False)
    ref = oracle.self_(s, td[sample], tn[sample]) + oracle.far(s, td[sample], tn[sample])
    for i, t in enumerate(sample):
        j = 1 - int(td[t])
        c, pl, info = N.near_value(s, j, x0[:, t], n0[:, t], sc, m, q_check=qc)
        assert info["dist"] < delta
        ref[:, i] += c - pl
    err = np.abs(corr[:, sample] - ref).max() / np.abs(ref).max()
    say("near correction vs oracle, rel err", err)
    assert err < 1e-10
    far = np.setdiff1d(np.arange(corr.shape[1]), changed)
    assert np.array_equal(corr[:, far], plain[:, far])          # other targets untouched


def test_near_correction_exterior_sphere_closed_form(E):
    """A unit sphere with sigma = Re Y_31 and a small sphere (radius 0.3,
    no densities) 0.004 above it: at the small sphere's nodes the evaluation
    is the unit sphere's exterior field, S_L = Y(d)/(7 r^4), L = 3 Y(d)/(7 r^4).
    Far sums on degree-5p grids (accurate beyond about 0.15), targets closer
    than delta = 0.16 corrected with check points on a degree-200 grid."""
    p, n, m = 12, 3, 1
    s = two_spheres(p, 0.004, r2=0.3, q_far=5 * p)
    nc2 = (p + 1) * (p + 2)
    s.sigcoef[:] = 0.0
    s.sigcoef[:nc2] = field(p, y_entry(n, m))
    s.fcoef[:] = 0.0
    s.ucoef[:] = 0.0
    plain, x0, _, _ = gpu_eval(E, s)
    corr, _, _, npairs = gpu_eval(E, s, (0.16, 3 * math.pi / 201, 8, 200))
    T1 = (p + 1) * (2 * p + 2)
    pts = x0[:, T1:]                                 # the small sphere's nodes
    r = np.linalg.norm(pts, axis=0)
    th, ph = np.arccos(pts[2] / r), np.arctan2(pts[1], pts[0])
    y = np.real(sph_harm_y(n, m, th, ph))
    ex = np.stack([y / ((2 * n + 1) * r ** (n + 1)), n * y / ((2 * n + 1) * r ** (n + 1))])
    e_corr = np.abs(corr[6:8, T1:] - ex).max() / np.abs(ex).max()
    e_plain = np.abs(plain[6:8, T1:] - ex).max() / np.abs(ex).max()
    say("closed form: pairs", npairs, "corrected err", e_corr, "plain err", e_plain, "min gap", (r - 1).min())
    assert npairs > 0
    assert e_corr < 1e-6 and e_plain > 1e-3


def test_near_correction_in_graph_mode(E):
    """The correction's kernels are part of the recorded evaluation: several
    replays, with eager work and synchronisations between them, each equal
    the eager result."""
    import torch
    p, qc = 8, 80
    s = two_spheres(p, 0.02)
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    ctx.set_near(0.12, 3 * math.pi / (qc + 1), 6, qc)
    f, u, sg = (torch.from_numpy(a).to(dev) for a in (s.fcoef, s.ucoef, s.sigcoef))
    T = ctx.ntargets
    eager = torch.empty(9, T, dtype=torch.float64, device=dev)
    ctx.layer_potentials(f, u, sg, E.ALL_KINDS, E.FAR_FP64, eager)
    ctx.sync()
    ref = eager.cpu().numpy()
    ctx.set_graph(True)
    out = torch.empty(9, T, dtype=torch.float64, device=dev)
    scratch = torch.randn(512, 512, dtype=torch.float64, device=dev)
    for _ in range(4):                     # the first call records, the others replay
        out.fill_(0.0)
        ctx.layer_potentials(f, u, sg, E.ALL_KINDS, E.FAR_FP64, out)
        ctx.sync()
        assert np.array_equal(out.cpu().numpy(), ref)
        scratch = torch.tanh(scratch @ scratch.T * 1e-3)          # unrelated eager work between replays
        torch.cuda.synchronize()
    ctx.close()


def test_near_correction_in_overlap_mode(E):
    """With the far field beside the self-interaction (the benchmark's
    default), the corrected outputs equal the serial ones bit for bit, in
    both far-field precisions, eagerly and in graph replays."""
    import torch
    p, qc = 8, 80
    s = two_spheres(p, 0.02)
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    ctx.set_near(0.12, 3 * math.pi / (qc + 1), 6, qc)
    assert ctx.near_pairs() > 0
    f, u, sg = (torch.from_numpy(a).to(dev) for a in (s.fcoef, s.ucoef, s.sigcoef))
    T = ctx.ntargets
    for prec in (E.FAR_FP64, E.FAR_FP32C):
        ref = torch.empty(9, T, dtype=torch.float64, device=dev)
        ctx.layer_potentials(f, u, sg, E.ALL_KINDS, prec, ref)
        ctx.sync()
        ctx.set_overlap(True)
        for graph in (False, True):
            ctx.set_graph(graph)
            for _ in range(2):
                out = torch.full_like(ref, 7.0)
                ctx.layer_potentials(f, u, sg, E.ALL_KINDS, prec, out)
                ctx.sync()
                assert torch.equal(out, ref), (prec, graph)
        ctx.set_graph(False)
        ctx.set_overlap(False)
    ctx.close()


def test_time_step_with_the_correction(E):
    """Algorithm 1 with the correction on: every shape of the step (the
    half-step one included) gets its own pairs, the corrected step differs
    from the plain one by a small amount, and overlap mode gives the same
    bits as the serial order."""
    import torch
    p, qc = 8, 80
    s = two_spheres(p, 0.02)
    dev = torch.device("cuda", 0)
    sp = E.Context.step_params(2.0, 0.5, 2.0, 0.3, 1.0, 0.0, tol=1e-12)
    gamma = torch.from_numpy(np.ascontiguousarray(s.sigcoef)).to(dev)
    res = {}
    for near in (False, True):
        for ov in (False, True):
            ctx = E.Context(0)
            ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
            if near:
                ctx.set_near(0.12, 3 * math.pi / (qc + 1), 6, qc)
                assert ctx.near_pairs() > 0
            ctx.set_overlap(ov)
            nc = ctx.num_coefs()
            xn = torch.empty(3 * nc, dtype=torch.float64, device=dev)
            gn = torch.empty(nc, dtype=torch.float64, device=dev)
            rep = ctx.evolve_step(sp, 0.1, 0.01, gamma, xn, gn)
            if near:
                assert ctx.near_pairs() > 0          # the context is back at x^n, pairs rebuilt
            res[(near, ov)] = (xn.cpu().numpy(), gn.cpu().numpy(), rep["iters"])
            ctx.close()
    for near in (False, True):
        assert np.array_equal(res[(near, False)][0], res[(near, True)][0]), near
        assert np.array_equal(res[(near, False)][1], res[(near, True)][1]), near
    d = np.abs(res[(True, False)][0] - res[(False, False)][0]).max()
    print("corrected vs plain step: max coefficient difference", d, "iterations", res[(True, False)][2],
          res[(False, False)][2], flush=True)
    assert 0.0 < d < 1e-2, d


def three_spheres(p, gap, seed=6):
    """Three unit spheres at the corners of a triangle in the plane z = 0
    (surfaces `gap` apart), turned so that a node of the first sphere's grid
    lies on the bisector between the other two: targets near two drops."""
    d = 2.0 + gap
    a1, a2 = math.radians(-10.0), math.radians(50.0)
    centres = [(0.0, 0.0, 0.0), (d * math.cos(a1), d * math.sin(a1), 0.0), (d * math.cos(a2), d * math.sin(a2), 0.0)]
    x = np.concatenate([sphere_x(p, centre=c) for c in centres])
    rng = np.random.default_rng(seed)
    nc2 = (p + 1) * (p + 2)

    def dens(nf):
        out = np.zeros(3 * nf * nc2)
        for blk in range(3 * nf):
            for n in range(p + 1):
                for m in range(n + 1):
                    k = blk * nc2 + 2 * tri(n, m)
                    out[k] = rng.standard_normal() / (n + 1) ** 2
                    if m:
                        out[k + 1] = rng.standard_normal() / (n + 1) ** 2
        return out
    f, u, sg = dens(3), dens(3), dens(1)
    pa = np.array([p, p, p], np.int32)
    return W.Suspension("near3", pa, 2 * pa, 2 * pa, 0, x, f, sg, u, np.array(centres), np.ones(3))


def test_near_correction_deterministic_with_two_pairs_per_target(E):
    """Targets closer than delta to two other drops get both corrections
    added in a fixed order: eager serial, overlap mode and graph replays give
    the same bits, in both far-field precisions, call after call."""
    import torch
    p, qc, delta = 8, 80, 0.35
    s = three_spheres(p, 0.02)
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    ctx.set_near(delta, 3 * math.pi / (qc + 1), 6, qc)
    T = ctx.ntargets
    x0 = torch.empty(3, T, dtype=torch.float64, device=dev)
    n0 = torch.empty_like(x0)
    ctx.target_geometry(x0, n0)
    x0 = x0.cpu().numpy()
    npt = (p + 1) * (2 * p + 2)
    near_count = np.zeros(T, int)
    for j in range(3):
        dist = np.linalg.norm(x0 - s.centres[j][:, None], axis=0) - 1.0
        own = np.arange(T) // npt == j
        near_count += (~own) & (dist < delta)
    say("pairs", ctx.near_pairs(), "targets near two drops", int((near_count >= 2).sum()))
    assert (near_count >= 2).sum() >= 2 and abs(ctx.near_pairs() - near_count.sum()) <= 2
    f, u, sg = (torch.from_numpy(a).to(dev) for a in (s.fcoef, s.ucoef, s.sigcoef))
    for prec in (E.FAR_FP64, E.FAR_FP32C):
        ref = torch.empty(9, T, dtype=torch.float64, device=dev)
        ctx.layer_potentials(f, u, sg, E.ALL_KINDS, prec, ref)
        ctx.sync()
        for ov in (False, True):
            ctx.set_overlap(ov)
            for graph in (False, True):
                ctx.set_graph(graph)
                for _ in range(3):
                    out = torch.full_like(ref, 7.0)
                    ctx.layer_potentials(f, u, sg, E.ALL_KINDS, prec, out)
                    ctx.sync()
                    assert torch.equal(out, ref), (prec, ov, graph)
            ctx.set_graph(False)
        ctx.set_overlap(False)
    ctx.close()
