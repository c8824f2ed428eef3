"""Pins of the numpy perceptron used to check the GPU kernels: its gradients
against central finite differences of its own loss (FP64), and its Adam step
against closed forms of the method (constant gradients, the first step,
invariance under gradient scaling) that do not reuse its formula."""
import numpy as np

from oracle import mlp as M


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    spec, n = M.layers(7, 9, 3, 5)
    p = rng.standard_normal(n) * 0.5
    x = rng.standard_normal((4, 7))
    t = rng.standard_normal((4, 5))
    hs = M.forward(p, spec, x)
    _, dy = M.mse_and_grad(hs[-1], t)
    g = M.backward(p, spec, hs, dy)
    h = 1e-6
    for k in rng.choice(n, 40, replace=False):
        e = np.zeros(n)
        e[k] = h
        lp = M.mse_and_grad(M.forward(p + e, spec, x)[-1], t)[0]
        lm = M.mse_and_grad(M.forward(p - e, spec, x)[-1], t)[0]
        assert abs((lp - lm) / (2 * h) - g[k]) < 1e-7 * max(1.0, abs(g[k]))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step, so each Adam step moves every parameter by
    lr g / (|g| + eps).  A missing or wrong bias correction (e.g. b1^(t-1)),
    eps under the square root, or swapped b1/b2 breaks this; the tiny
    gradients make the eps placement visible."""
    lr, eps = 0.05, 1e-8
    g = np.array([3.0, -0.2, 1e-7, -4e-9, 0.0])
    p = np.array([1.0, -2.0, 0.5, 0.25, 7.0])
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    p0 = p.copy()
    for t in range(1, 8):
        p, m1, m2 = M.adam(p, g, m1, m2, t, lr, eps=eps)
        want = p0 - t * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(p, want, rtol=0, atol=1e-14)


def test_adam_first_step_and_scale_invariance():
    """The first step is lr g/(|g| + eps) for any b1, b2 (the bias
    corrections cancel the (1 - b) factors exactly), and for gradients far
    above eps the whole trajectory is unchanged when every gradient is
    scaled by the same c > 0."""
    rng = np.random.default_rng(2)
    lr = 0.01
    for b1, b2 in [(0.9, 0.999), (0.5, 0.9), (0.0, 0.99)]:
        g = rng.standard_normal(6)
        p, _, _ = M.adam(np.zeros(6), g, np.zeros(6), np.zeros(6), 1, lr, b1, b2)
        np.testing.assert_allclose(p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=0)
    gs = rng.standard_normal((5, 4)) + 2.0
    traj = []
    for c in (1.0, 37.0):
        p = np.zeros(4)
        m1 = np.zeros(4)
        m2 = np.zeros(4)
        for t in range(1, 6):
            p, m1, m2 = M.adam(p, c * gs[t - 1], m1, m2, t, lr, eps=0.0)
        traj.append(p)
    np.testing.assert_allclose(traj[0], traj[1], rtol=1e-13, atol=0)
