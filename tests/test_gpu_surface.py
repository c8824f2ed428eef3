"""GPU: mean curvature and surface gradients at the target nodes (ehd_surface)
against the oracle's surface quantities (a different route to the second
derivatives: the recurrence differentiated twice, not the Legendre
equation)."""
import math

import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("grid_mode", [0, 1])
def test_surface_quantities_match_oracle(E, grid_mode):
    import torch
    s = W.subset(W.batched_suspension(seed=3, grid_mode=grid_mode), [0, 1, 2, 3])
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    ctx.set_drops(s.p, s.q_self, s.q_far, s.grid_mode, torch.from_numpy(s.xcoef).to(dev))
    T = ctx.ntargets
    ng = 2
    g = np.concatenate([np.concatenate([s.fcoef[3 * int(o):3 * int(o) + 2 * (int(p) + 1) * (int(p) + 2)]])
                        for o, p in zip(W.drop_offsets(s.p)[:-1], s.p)])
    H = torch.zeros(T, dtype=torch.float64, device=dev)
    grad = torch.zeros(ng, 3, T, dtype=torch.float64, device=dev)
    lap = torch.zeros(ng, T, dtype=torch.float64, device=dev)
    ctx.surface(H, torch.from_numpy(g).to(dev), grad, ng=ng, lap=lap)
    ctx.sync()
    H, grad, lap = H.cpu().numpy(), grad.cpu().numpy(), lap.cpu().numpy()
    ctx.close()
    offs = W.drop_offsets(s.p)
    t0 = 0
    errH, errG, errL = 0.0, 0.0, 0.0
    for d, p in enumerate(int(x) for x in s.p):
        nl = 2 * p + 2 if grid_mode == 0 else 2 * p
        t, _ = oracle.gauss_legendre(p + 1)
        gd = g[2 * int(offs[d]):2 * int(offs[d]) + 2 * (p + 1) * (p + 2)]
        xd = s.xcoef[3 * int(offs[d]):3 * int(offs[d]) + 3 * (p + 1) * (p + 2)]
        for j in range(0, p + 1, 3):
            for k in range(0, nl, 5):
                _, _, Hr, gr, lr = oracle.surface_point(p, xd, math.acos(t[j]), 2 * math.pi * k / nl, gcoef=gd,
                                                        ng=ng, lap=True)
                tt = t0 + j * nl + k
                errH = max(errH, abs(H[tt] - Hr) / abs(Hr))
                errG = max(errG, np.abs(grad[:, :, tt] - gr).max() / max(1e-3, np.abs(gr).max()))
                errL = max(errL, np.abs(lap[:, tt] - lr).max() / max(1e-3, np.abs(lr).max()))
        t0 += (p + 1) * nl
    print("surface: max rel err H", errH, "grad", errG, "Laplace-Beltrami", errL, flush=True)
    assert errH < 1e-11 and errG < 1e-10 and errL < 1e-10
