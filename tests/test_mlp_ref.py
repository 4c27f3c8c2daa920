"""Pins of the FP64 network reference: the analytic gradient against central
finite differences of the loss, and closed-form cases."""
import numpy as np

from oracle import mlp_ref


def _setup(seed=0, n=40):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp_ref.NPARAM)
    x = rng.normal(0, 1, (n, 16))
    t = rng.normal(0, 1, (n, 16))
    return p, x, t


def test_gradient_matches_finite_differences():
    p, x, t = _setup()
    loss, g = mlp_ref.loss_and_grad(p, x, t)
    rng = np.random.default_rng(1)
    idx = rng.choice(mlp_ref.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp_ref.OFF["b1"], mlp_ref.OFF["b2"] + 3, mlp_ref.OFF["b3"] + 5]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp_ref.loss_and_grad(pp, x, t)[0] - mlp_ref.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_closed_forms():
    # zero weights: the output is the last bias, the loss its mean squared error
    p = np.zeros(mlp_ref.NPARAM)
    p[mlp_ref.OFF["b3"]:] = np.arange(16) * 0.1
    x = np.ones((3, 16))
    t = np.zeros((3, 16))
    y, _ = mlp_ref.forward(p, x)
    assert np.allclose(y, np.arange(16) * 0.1)
    loss, g = mlp_ref.loss_and_grad(p, x, t)
    assert np.isclose(loss, np.mean((np.arange(16) * 0.1) ** 2))
    assert np.allclose(g[mlp_ref.OFF["b3"]:], 2 * np.arange(16) * 0.1 / 16)


def test_bf16_rounding():
    # 1 + 2^-8 is exactly halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert mlp_ref.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp_ref.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert mlp_ref.bf16(np.array([3.0]))[0] == 3.0
