"""GPU: the learned initial guess for the implicit surfactant-diffusion solve
(a perceptron trained by the library's own kernels on solves the library
generates) against the preconditioned solve without it, on drops deformed
by a field along z that carry a surfactant field of the same symmetry, at
the degree of the learned-guess workload (p = 32).  The training budget is
cut for test time: 4,000 generated solves and 40 epochs instead of the
workload's 10,000 and 60 (bench.py --learned runs the full budget)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P, NTRAIN, NTEST = 32, 4000, 32


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_10270_amd import ehdbim, learned_guess as L
    ehdbim.load()
    tr = L.solve_all(L.draw(NTRAIN, P, seed=1, kind="ehd"))
    te = L.solve_all(L.draw(NTEST, P, seed=2, kind="ehd"))
    return L, L.train(tr, epochs=40), te


def test_training_converges(trained):
    _, m, _ = trained
    assert np.all(np.isfinite(m.history))
    assert m.history[-1] < 0.1 * m.history[0]
    assert np.all((m.gain >= 0.0) & (m.gain <= 1.0))


def test_learned_guess_cuts_iterations(trained):
    """Iterations to a 1e-10 true residual: the learned start needs fewer
    than the plain preconditioned solve and no more than a start at
    M^{-1} b, and its true residual is below that of M^{-1} b."""
    L, m, te = trained
    r = L.compare(te, L.predict(m, te), tol=1e-10)
    assert r["guess_used"].all()
    assert r["iters_learned"].mean() < r["iters_plain"].mean()
    assert r["iters_learned"].mean() <= r["iters_precond"].mean()
    assert np.median(r["guess_relres"]) < 0.5 * np.median(r["precond_relres"])


def test_garbage_guess_falls_back(trained):
    """A guess whose true residual exceeds |b| is dropped for the zero
    guess, and the preconditioned solve still reaches 1e-10."""
    L, _, te = trained
    rng = np.random.default_rng(5)
    bad = 1e3 * rng.standard_normal(te.b.shape)
    r = L.compare(te.__class__(te.p, te.x[:4], te.b[:4], te.kappa[:4], te.gamma[:4]), bad[:4], tol=1e-10)
    assert not r["guess_used"].any()
    assert np.array_equal(r["iters_learned"], r["iters_plain"])


def test_learned_solution_matches_reference(trained):
    """The solve that starts from the learned guess ends at the reference
    solution (generated to 1e-13) within the 1e-10 tolerance."""
    import torch
    L, m, te = trained
    g = L.predict(m, te)
    dev = torch.device("cuda", 0)
    for i in range(4):
        ctx = L._context(te.p, te.x[i:i + 1], dev)
        x = torch.from_numpy(g[i].copy()).to(dev)
        its, rr = ctx.solve_surfactant(te.kappa[i], torch.from_numpy(te.b[i]).to(dev), x, tol=1e-10)
        ctx.close()
        assert rr <= 1e-10
        err = np.linalg.norm(x.cpu().numpy() - te.gamma[i]) / np.linalg.norm(te.gamma[i])
        assert err < 1e-9


def test_library_guess_and_features_match_numpy(trained):
    """ehd_surfactant_guess and ehd_learned_features against the same
    formulas in numpy: M^{-1} b + kappa |b| gain (y std + mean) with
    M = diag(1 + kappa n(n+1)), and [x without degree 0, b / |b|,
    log10 kappa] standardised."""
    import torch
    L, _, te = trained
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(9)
    k = 5
    nc = (P + 1) * (P + 2)
    ctx = L._context(P, te.x[:k], dev)
    b = torch.from_numpy(te.b[:k].ravel()).to(dev)
    y = rng.standard_normal((k, nc)).astype(np.float32)
    ym, ysd, gain = rng.standard_normal(nc), rng.uniform(0.5, 2.0, nc), rng.uniform(0.0, 1.0, nc)
    g = torch.empty(k * nc, dtype=torch.float64, device=dev)
    ctx.surfactant_guess(te.kappa[:k], b, g, torch.from_numpy(y).to(dev), torch.from_numpy(ym).to(dev),
                         torch.from_numpy(ysd).to(dev), torch.from_numpy(gain).to(dev))
    g0 = torch.empty_like(g)
    ctx.surfactant_guess(te.kappa[:k], b, g0)
    deg = np.concatenate([[n, n] for n in range(P + 1) for _ in range(n + 1)])
    for i in range(k):
        pre = te.b[i] / (1.0 + te.kappa[i] * deg * (deg + 1.0))
        want = pre + te.kappa[i] * np.linalg.norm(te.b[i]) * gain * (y[i].astype(np.float64) * ysd + ym)
        np.testing.assert_allclose(g.cpu().numpy()[i * nc:(i + 1) * nc], want, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(g0.cpu().numpy()[i * nc:(i + 1) * nc], pre, rtol=1e-14, atol=0)
    nf = 4 * nc + 1
    mean, sd = rng.standard_normal(nf) * 1e-3, rng.uniform(0.5, 2.0, nf)
    f = torch.empty(k, nf, dtype=torch.float32, device=dev)
    ctx.learned_features(te.kappa[:k], b, torch.from_numpy(mean).to(dev), torch.from_numpy(sd).to(dev), f)
    xd = torch.empty(3 * nc * k, dtype=torch.float64, device=dev)
    ctx.drop_coefs(xd)
    ctx.close()
    xd = xd.cpu().numpy().reshape(k, 3 * nc)
    for i in range(k):
        x = xd[i].copy()
        x[[0, 1, nc, nc + 1, 2 * nc, 2 * nc + 1]] = 0.0
        raw = np.concatenate([x, te.b[i] / np.linalg.norm(te.b[i]), [math.log10(te.kappa[i])]])
        np.testing.assert_allclose(f.cpu().numpy()[i], ((raw - mean) / sd).astype(np.float32), rtol=2e-7,
                                   atol=2e-7)
