"""Pins of the FP64 iteration-count network: backward pass against central
finite differences, Adam against its closed form on a quadratic."""
import numpy as np

import oracle.mlp as M
import workloads as W


def test_gradient_matches_central_differences():
    p = W.mlp_init(seed=5)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(40, M.NF)) * 3 + 5
    p[0:M.NF] = x.mean(0)
    p[M.NF:2 * M.NF] = 1 / x.std(0)
    t = rng.normal(size=40) + 4
    loss, g = M.loss_and_grad(p, x, t)
    h = 1e-5
    idx = np.concatenate([rng.choice(np.arange(M.OFF_W1, M.NPARAM), 60, replace=False), [M.OFF_B3, M.OFF_B1]])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (M.loss_and_grad(p + e, x, t)[0] - M.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert np.all(g[:M.OFF_W1] == 0)
    assert abs(loss - np.mean((M.forward(p, x) - t) ** 2)) < 1e-12


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected moments are g and g^2,
    so Adam moves each weight by exactly -lr g / (|g| + eps)."""
    p = W.mlp_init(seed=2)
    g = np.zeros_like(p)
    g[M.OFF_W1:] = np.linspace(-1, 1, M.NPARAM - M.OFF_W1) + 0.01
    q, m, v = M.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, 1, 1e-3)
    gg = g[M.OFF_W1:]
    np.testing.assert_allclose(q[M.OFF_W1:] - p[M.OFF_W1:], -1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-9)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(512, M.NF))
    t = np.sin(3 * x[:, 0]) + x[:, 1] ** 2
    p = W.mlp_init(seed=9)
    p[0:M.NF] = x.mean(0)
    p[M.NF:2 * M.NF] = 1 / x.std(0)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = M.loss_and_grad(p, x, t)[0]
    for step in range(1, 301):
        b = rng.choice(512, 64, replace=False)
        _, g = M.loss_and_grad(p, x[b], t[b])
        p, m, v = M.adam_step(p, m, v, g, step, 3e-3)
    assert M.loss_and_grad(p, x, t)[0] < 0.1 * l0
