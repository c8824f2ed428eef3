"""GPU: the learned initial guess for the implicit surfactant-diffusion solve
(a perceptron trained by the library's own kernels on solves the library
generates) against the preconditioned solve without it, on drops deformed
by a field along z that carry a surfactant field of the same symmetry."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P, NTRAIN, NTEST = 12, 3000, 32


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
