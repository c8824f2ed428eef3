"""Plain FP64 numpy perceptron with the library's parameter layout (for each
layer l: W_l[in][out] row-major, then b_l[out]; ReLU hidden layers, linear
output), its mean-squared-error loss, gradients by the chain rule, and one
Adam step.  TEST INFRASTRUCTURE ONLY (gradient checks of the GPU kernels)."""
from __future__ import annotations

import numpy as np


def layers(nin: int, nhid: int, nlay: int, nout: int):
    dims = [nin] + [nhid] * nlay + [nout]
    out, off = [], 0
    for l in range(nlay + 1):
        a, b = dims[l], dims[l + 1]
        out.append((off, a, b, off + a * b))
        off += a * b + b
    return out, off


def unpack(params, spec):
    return [(params[o:o + a * b].reshape(a, b).astype(np.float64), params[bo:bo + b].astype(np.float64))
            for (o, a, b, bo) in spec]


def forward(params, spec, x):
    hs = [np.asarray(x, np.float64)]
    wb = unpack(params, spec)
    for l, (W, b) in enumerate(wb):
        z = hs[-1] @ W + b
        hs.append(np.maximum(z, 0.0) if l < len(wb) - 1 else z)
    return hs


def mse_and_grad(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, spec, hs, dy):
    """Gradient vector (library layout) for the output gradient dy."""
    wb = unpack(params, spec)
    g = np.zeros(len(params))
    dz = np.asarray(dy, np.float64)
    for l in range(len(wb) - 1, -1, -1):
        o, a, b, bo = spec[l]
        g[o:o + a * b] = (hs[l].T @ dz).ravel()
        g[bo:bo + b] = dz.sum(axis=0)
        if l == 0:
            break
        dh = dz @ wb[l][0].T
        dz = np.where(hs[l] > 0.0, dh, 0.0)
    return g


def adam(params, grad, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    p = params - lr * (m1 / (1 - b1**t)) / (np.sqrt(m2 / (1 - b2**t)) + eps)
    return p, m1, m2
