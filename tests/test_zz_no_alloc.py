"""GPU: the allocation-free E_n solve (ehd_solve_En_noalloc, called through
the C ABI) against the allocating ehd_solve_En on the same inputs, on two
calls in a row of which the second has the smaller problem (the shared
device workspace then holds the first call's values); and its refusals of
sizes beyond that workspace, which must leave the output untouched."""
import numpy as np
import pytest

from paper_1811_10270_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


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


def set_drops(E, ctx, s):
    import torch
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(torch.device("cuda", 0)))


def zeros(E, ctx):
    import torch
    return torch.zeros(ctx.num_coefs(), dtype=torch.float64, device=torch.device("cuda", 0))


PARAMS = dict(R=0.5, Eu=1.0, Eq=0.3)


def test_noalloc_solve_matches_the_allocating_solve(E):
    big = W.two_drops(12, seed=11, gap=0.3)
    small = W.single_drop(8, seed=2)
    ref = {}
    for name, s in (("big", big), ("small", small)):
        say(f"[gpu] ehd_solve_En on {name}: ndrops={s.ndrops} p={s.p.tolist()}")
        ctx = E.Context(0)
        set_drops(E, ctx, s)
        en = zeros(E, ctx)
        it, rr = ctx.solve_En(PARAMS["R"], PARAMS["Eu"], PARAMS["Eq"], en, restart=20, tol=1e-12)
        ref[name] = (en.cpu().numpy(), it, rr)
        ctx.close()
    ctx = E.Context(0)
    for name, s in (("big", big), ("small", small)):       # two calls in a row, the second smaller
        say(f"[gpu] ehd_solve_En_noalloc on {name}")
        set_drops(E, ctx, s)
        en = zeros(E, ctx)
        it, rr = ctx.solve_En_noalloc(PARAMS["R"], PARAMS["Eu"], PARAMS["Eq"], en, restart=20, tol=1e-12)
        got = en.cpu().numpy()
        want, it0, rr0 = ref[name]
        err = np.abs(got - want).max() / np.abs(want).max()
        say(name, "iterations", it, it0, "relres", rr, rr0, "rel diff", err)
        assert it == it0 and rr <= 1e-12 and err <= TOL, (name, it, it0, rr, err)
    ctx.close()


def test_noalloc_solve_refusals(E):
    s = W.two_drops(6, seed=3, gap=0.5)
    ctx = E.Context(0)
    set_drops(E, ctx, s)
    en = zeros(E, ctx)
    en.fill_(7.0)
    with pytest.raises(E.EhdError) as ei:
        ctx.solve_En_noalloc(1.5, 1.0, 0.0, en, restart=65)
    assert ei.value.code == E.EHD_E_SHAPE
    ctx.set_graph(True)
    with pytest.raises(E.EhdError) as ei:
        ctx.solve_En_noalloc(1.5, 1.0, 0.0, en)
    assert ei.value.code == E.EHD_E_STATE
    ctx.set_graph(False)
    assert float(en.min()) == 7.0 and float(en.max()) == 7.0     # nothing was written
    # 256 drops of p = 32: (30 + 4) n + 7 T exceeds the 8 Mi doubles
    big = W.large_suspension(seed=5)
    set_drops(E, ctx, big)
    en = zeros(E, ctx)
    en.fill_(7.0)
    with pytest.raises(E.EhdError) as ei:
        ctx.solve_En_noalloc(1.5, 1.0, 0.0, en, restart=30)
    assert ei.value.code == E.EHD_E_SHAPE
    assert float(en.min()) == 7.0 and float(en.max()) == 7.0
    ctx.close()
