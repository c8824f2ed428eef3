"""GPU: the perceptron kernels (forward, loss, backward, Adam) against the
FP64 numpy oracle with the same parameters, at sizes that leave ragged
64x64 tiles."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_10270_amd import ehdbim
    ehdbim.load()
    return ehdbim


@pytest.mark.parametrize("dims", [(37, 50, 3, 21, 13), (130, 96, 2, 70, 67)])
def test_forward_backward_adam_match_oracle(E, dims):
    import torch
    nin, nhid, nlay, nout, batch = dims
    dev = torch.device("cuda", 0)
    net = E.MLP(nin, nhid, nlay, nout, seed=7)
    spec, n = M.layers(nin, nhid, nlay, nout)
    assert n == net.nparams
    rng = np.random.default_rng(3)
    p = net.params().astype(np.float64)
    p[[bo + j for (_, _, b, bo) in spec for j in range(b)]] = 0.1 * rng.standard_normal(sum(b for (_, _, b, _) in spec))
    net.set_params(p.astype(np.float32))
    p = net.params().astype(np.float64)
    x = rng.standard_normal((batch, nin)).astype(np.float32)
    t = rng.standard_normal((batch, nout)).astype(np.float32)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    y = torch.zeros(batch, nout, dtype=torch.float32, device=dev)
    dy = torch.zeros_like(y)
    net.forward(xd, y)
    loss = net.mse(y, td, dy)
    net.backward(dy)
    g = net.grads().astype(np.float64)
    hs = M.forward(p, spec, x.astype(np.float64))
    ref_loss, ref_dy = M.mse_and_grad(hs[-1], t.astype(np.float64))
    ref_g = M.backward(p, spec, hs, ref_dy)
    ey = np.abs(y.cpu().numpy() - hs[-1]).max() / np.abs(hs[-1]).max()
    eg = np.abs(g - ref_g).max() / np.abs(ref_g).max()
    print("mlp dims", dims, "y err", ey, "loss", loss, ref_loss, "grad err", eg, flush=True)
    assert ey < 1e-5 and abs(loss - ref_loss) < 1e-5 * ref_loss and eg < 1e-4
    net.adam(1e-3)
    p2 = net.params().astype(np.float64)
    ref_p2, _, _ = M.adam(p, g, np.zeros(n), np.zeros(n), 1, 1e-3)
    assert np.abs(p2 - ref_p2).max() < 1e-6
    net.close()


def test_training_reduces_the_loss(E):
    """Fit a random linear map: the loss falls by two orders of magnitude."""
    import torch
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((32, 16)) / 6
    X = rng.standard_normal((512, 32)).astype(np.float32)
    Y = (X @ A).astype(np.float32)
    xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    net = E.MLP(32, 64, 2, 16, seed=11)
    out = torch.zeros(512, 16, dtype=torch.float32, device=dev)
    dy = torch.zeros_like(out)
    first = None
    for it in range(400):
        net.forward(xd, out)
        loss = net.mse(out, yd, dy, want_loss=(it % 50 == 0 or it == 399))
        if first is None:
            first = loss
        net.backward(dy)
        net.adam(3e-3)
    print("training loss", first, "->", loss, flush=True)
    assert loss < 1e-2 * first
    net.close()
