"""Pins of the fp64 network oracle (CPU only).

  * central finite differences on the loss (h = 1e-6) against the analytic
    gradient;
  * closed forms: zero weights give uniform probabilities, loss ln 12 and a
    last-layer bias gradient of mean(1/12 - onehot); Adam's first step is
    -lr * g / (|g| + eps) for every coordinate;
  * torch CPU autograd in float64 on the same network (a library routine
    that computes the same derivative independently);
  * the histogram feature on hand-counted size lists.
"""
import numpy as np
import pytest
import torch

from oracle import mlp
from workloads.mlp_init import he_uniform


def _data(seed, B=16):
    g = np.random.default_rng(seed)
    x = np.log2(1 + g.integers(0, 300, size=(B, 32))).astype(np.float64)
    y = g.integers(0, 12, size=B)
    return x, y


def test_param_count():
    assert mlp.N_PARAMS == 7052 and he_uniform().shape == (7052,)


def test_finite_differences():
    theta = he_uniform(0).astype(np.float64)
    x, y = _data(1)
    g = mlp.grad(theta, x, y)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(7052, 300, replace=False),
                          [0, 2047, 2048, 2111, 2112, 6207, 6208, 6975, 6976, 7051]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, x, y) - mlp.loss(tm, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 2e-9, (i, fd, g[i])


def test_zero_weights_closed_form():
    theta = np.zeros(7052)
    x, y = _data(3, B=10)
    assert mlp.loss(theta, x, y) == pytest.approx(np.log(12.0), abs=1e-15)
    g = mlp.unpack(mlp.grad(theta, x, y))
    onehot = np.eye(12)[y]
    assert np.allclose(g["b3"], (1 / 12 - onehot).mean(axis=0), atol=1e-15)
    # with zero hidden activations nothing else receives gradient
    for k in ["W1", "b1", "W2", "b2", "W3"]:
        assert not g[k].any()


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0, -7.0])
    opt = mlp.Adam(5)
    theta = opt.step(np.ones(5), g)
    assert np.allclose(theta, 1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # second step against the textbook recursion written out
    g2 = np.array([1.0, 1.0, -1.0, 2.0, 0.0])
    m = 0.9 * (0.1 * g) + 0.1 * g2
    v = 0.999 * (0.001 * g * g) + 0.001 * g2 * g2
    want = theta - 1e-3 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(opt.step(theta, g2), want, rtol=0, atol=1e-15)


def test_against_torch_autograd():
    theta = he_uniform(4).astype(np.float64)
    x, y = _data(5, B=32)
    p = {k: torch.tensor(v, requires_grad=True) for k, v in mlp.unpack(theta.copy()).items()}
    xt = torch.tensor(x)
    h1 = torch.relu(xt @ p["W1"].T + p["b1"])
    h2 = torch.relu(h1 @ p["W2"].T + p["b2"])
    z = h2 @ p["W3"].T + p["b3"]
    L = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    L.backward()
    tg = np.concatenate([p[k].grad.numpy().ravel() for k, _ in mlp.SHAPES])
    assert mlp.loss(theta, x, y) == pytest.approx(L.item(), rel=1e-14)
    assert np.allclose(mlp.grad(theta, x, y), tg, rtol=1e-12, atol=1e-15)
    zo, _ = mlp.forward(theta, x)
    assert np.allclose(zo, z.detach().numpy(), rtol=1e-13, atol=1e-13)


def test_features_hand_counted():
    sizes = [0, 1, 2, 3, 4, 7, 8, 255, 256, 2**31, 2**40, 2**63]
    f = mlp.features(np.array(sizes, dtype=np.uint64))
    counts = np.zeros(32)
    counts[0] = 2       # 0 and 1
    counts[1] = 2       # 2, 3
    counts[2] = 2       # 4, 7
    counts[3] = 1       # 8
    counts[7] = 1       # 255
    counts[8] = 1       # 256
    counts[31] = 3      # 2^31, 2^40, 2^63 fold into the last bin
    assert np.array_equal(f, np.log2(1 + counts))


def test_predict_ties_lowest():
    theta = np.zeros(7052)
    assert mlp.predict(theta, np.ones(32))[0] == 0
    p = mlp.unpack(theta)
    p["b3"][:] = 0
    p["b3"][[4, 9]] = 1.0
    assert mlp.predict(mlp.pack(p), np.ones(32))[0] == 4
