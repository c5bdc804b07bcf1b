"""Parity of the surrogate network's HIP kernels (through the C interface)
with the FP64 oracle: forward, loss and gradients in both precisions, Adam
training steps, and that training fits a known function."""
import numpy as np
import pytest

from oracle import mlp as omlp
from workloads import mlp_layer_sizes, mlp_init, minibatch_indices

pytestmark = pytest.mark.gpu

SIZES = mlp_layer_sizes(5, 128, 4, 2)


def _net(params, prec, max_batch=256, sizes=(5, 128, 4, 2)):
    from paper_1611_05712_amd.mlp import MLP
    return MLP(params, *sizes, prec=prec, max_batch=max_batch)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 1.5, (n, 5)).astype(np.float32)
    t = np.stack([np.sin(x[:, 0]) * x[:, 1], x[:, 2] ** 2 - x[:, 3] * x[:, 4]], axis=1).astype(np.float32)
    return x, t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 5e-4)])
def test_forward_matches_oracle(prec, tol):
    p = mlp_init(SIZES, seed=7)
    x, _ = _data(300, 1)                     # two launches: 256 + a ragged 44
    net = _net(p, prec)
    y = net.forward(x).cpu().numpy()
    want, _ = omlp.forward(p.astype(np.float64), SIZES, x.astype(np.float64), bf16=(prec == 1))
    assert _rel(y, want) < tol
    net.close()


@pytest.mark.parametrize("prec,tol", [(0, 2e-5), (1, 3e-3)])
@pytest.mark.parametrize("n", [256, 37])
def test_loss_and_gradient_match_oracle(prec, tol, n):
    p = mlp_init(SIZES, seed=8)
    x, t = _data(n, 2)
    net = _net(p, prec)
    loss, g = net.loss_grad(x, t)
    g = g.cpu().numpy()
    want_loss, want_g = omlp.loss_grad(p.astype(np.float64), SIZES, x.astype(np.float64), t.astype(np.float64),
                                       bf16=(prec == 1))
    assert loss == pytest.approx(want_loss, rel=tol)
    o = 0
    for (i, nn) in SIZES:
        for k in (nn * i, nn):                  # W_l, then b_l
            assert _rel(g[o:o + k], want_g[o:o + k]) < tol, (i, nn, k)
            o += k
    net.close()


def test_adam_steps_match_oracle():
    p = mlp_init(SIZES, seed=9)
    x, t = _data(512, 3)
    idx = minibatch_indices(512, 128, 25, seed=5)
    net = _net(p, 0, max_batch=128)
    losses = net.train(x, t, idx, 128, lr=1e-3).cpu().numpy()
    got = net.params()
    want, want_losses = omlp.train(p, SIZES, x.astype(np.float64), t.astype(np.float64), idx, 128,
                                   omlp.Adam(p.size, lr=1e-3))
    np.testing.assert_allclose(losses, want_losses, rtol=1e-4)
    # the update, not the parameters, carries the signal: compare p_25 - p_0
    assert _rel(got - p, want - p) < 1e-3
    assert net.steps() == 25
    net.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_training_fits_a_known_function(prec):
    p = mlp_init(SIZES, seed=10)
    x, t = _data(2048, 4)
    xv, tv = _data(512, 5)
    idx = minibatch_indices(2048, 256, 3000, seed=6)
    net = _net(p, prec)
    losses = net.train(x, t, idx, 256, lr=1e-3).cpu().numpy()
    assert np.isfinite(losses).all()
    yv = net.forward(xv).cpu().numpy()
    mse = float(((yv - tv) ** 2).mean())
    base = float(((tv - tv.mean(axis=0)) ** 2).mean())
    assert mse < 0.01 * base, (mse, base)
    net.close()


def test_bad_minibatch_index_is_reported():
    from paper_1611_05712_amd import PicError
    p = mlp_init(SIZES, seed=11)
    x, t = _data(64, 6)
    net = _net(p, 0, max_batch=32)
    idx = np.arange(32, dtype=np.int32)
    idx[5] = 64                                  # one past the data set
    with pytest.raises(PicError) as e:
        net.train(x, t, idx, 32)
    assert e.value.code == -1
    net.close()
