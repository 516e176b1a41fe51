"""Pins of the selector-network oracle: finite differences for the backward
pass, a hand-set network for the forward pass, the pinball loss on known
residuals, and the closed form of Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def _net(seed):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.NPARAM) * 0.3
    X = rng.standard_normal((9, mlp.NIN)) * 2.0 + 1.0
    t = rng.integers(2, 13, 9).astype(np.float64)
    mu = rng.standard_normal(mlp.NIN) * 0.5
    sd = rng.uniform(0.5, 2.0, mlp.NIN)
    return p, X, t, mu, sd


def test_param_count():
    assert mlp.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5313
    p = np.arange(mlp.NPARAM, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)
    P = mlp.unpack(p)
    assert P["W1"][1, 0] == 16 and P["b1"][0] == 1024 and P["b3"][0] == 5312


def test_pinball_values():
    assert mlp.pinball(np.array([1.0]), np.array([3.0]), 0.9) == pytest.approx(1.8)
    assert mlp.pinball(np.array([3.0]), np.array([1.0]), 0.9) == pytest.approx(0.2)
    assert mlp.pinball(np.array([1.0, 3.0]), np.array([3.0, 1.0]), 0.9) == pytest.approx(1.0)


def test_forward_hand_set():
    P = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    P["W1"][:16, :16] = np.eye(16)
    P["W2"][:16, :16] = np.eye(16)
    P["W3"][:16] = 1.0
    P["b3"][0] = 0.5
    P["b2"][20] = 3.0       # a hidden unit that is on but not read
    P["W3"][20] = 0.0
    x = np.linspace(-2, 2, 16)[None, :]
    y, c = mlp.forward(mlp.pack(P), x, np.zeros(16), np.ones(16))
    assert y[0] == pytest.approx(np.sum(np.maximum(x, 0)) + 0.5, rel=1e-15)
    # normalisation: x = mu + sd * z gives the same output as z with (0, 1)
    mu, sd = np.full(16, 0.25), np.full(16, 2.0)
    y2, _ = mlp.forward(mlp.pack(P), mu + sd * x, mu, sd)
    assert y2[0] == pytest.approx(y[0], rel=1e-15)


def test_backward_finite_differences():
    p, X, t, mu, sd = _net(1)
    tau = 0.9
    loss, g = mlp.loss_grad(p, X, t, tau, mu, sd)
    # keep away from the kinks: every pre-activation and residual clear of 0
    _, c = mlp.forward(p, X, mu, sd)
    assert np.min(np.abs(c["Z1"])) > 1e-4 and np.min(np.abs(c["Z2"])) > 1e-4
    h = 1e-6
    rng = np.random.default_rng(0)
    idx = np.concatenate([np.arange(0, 1088, 17), 1088 + rng.choice(4096 + 64, 150, replace=False),
                          np.arange(5248, 5313)])
    fd = np.empty(idx.size)
    for j, i in enumerate(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[j] = (mlp.loss_grad(pp, X, t, tau, mu, sd)[0] - mlp.loss_grad(pm, X, t, tau, mu, sd)[0]) / (2 * h)
    err = np.abs(fd - g[idx])
    assert np.max(err) <= 1e-6 * max(1.0, np.max(np.abs(g[idx])))
    # a plausible mistake (dropping the ReLU mask in layer 2) is caught by the same check
    assert np.count_nonzero(g) > 0.3 * mlp.NPARAM


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    g[7] = 0.0
    lr, eps = 1e-3, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert p1[7] == p[7]
    # second step with the same gradient moves by the same amount again
    p2, _, _ = mlp.adam_step(p1, g, m, v, 2, lr, eps=eps)
    assert np.allclose(p2 - p1, p1 - p, rtol=1e-9, atol=1e-18)


def test_predict_slices():
    y = np.array([-3.0, 2.0, 2.01, 2.49, 6.5, 6.7, 11.2, 11.999, 40.0])
    assert list(mlp.predict_slices(y)) == [2, 2, 2, 2, 7, 7, 11, 12, 12]
