"""Pins of the numpy perceptron used to check the GPU kernels: its gradients
against central finite differences of its own loss (FP64)."""
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
