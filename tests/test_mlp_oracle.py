"""Pins of the CPU float64 work-predictor reference (no GPU)."""
import numpy as np

from oracle import mlp


def _data(seed, n=64):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, mlp.N_PARAMS)
    X = rng.uniform(-1, 1, (n, mlp.F))
    t = rng.normal(0, 1, n)
    return p, X, t


def test_layout_size():
    assert mlp.N_PARAMS == 32 * 10 + 32 + 32 * 32 + 32 + 32 + 1
    p, _, _ = _data(0)
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(p)), p)


def test_backward_matches_finite_differences():
    p, X, t = _data(1, n=96)
    # keep samples away from the ReLU kinks, where differences are not derivatives
    _, (_, z1, _, z2, _) = mlp.forward(p, X)
    keep = (np.abs(z1).min(axis=1) > 1e-3) & (np.abs(z2).min(axis=1) > 1e-3)
    X, t = X[keep], t[keep]
    assert X.shape[0] >= 32
    _, g = mlp.loss_grad(p, X, t)
    idx = list(range(mlp.N_PARAMS))
    fd = mlp.finite_diff(p, X, t, idx)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_closed_form_zero_hidden():
    """With all weights zero the output is b3 for every sample; the loss and
    the b3 gradient are then mean-square and mean residual (ReLU at 0 passes
    no gradient to the hidden layers)."""
    p = np.zeros(mlp.N_PARAMS)
    p[-1] = 0.75
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (10, mlp.F))
    t = rng.normal(0, 1, 10)
    y, _ = mlp.forward(p, X)
    np.testing.assert_allclose(y, 0.75)
    L, g = mlp.loss_grad(p, X, t)
    assert abs(L - 0.5 * np.mean((0.75 - t) ** 2)) < 1e-12
    assert abs(g[-1] - np.mean(0.75 - t)) < 1e-12
    assert np.all(g[:-1] == 0)


def test_linear_regime_closed_form():
    """Positive weights and inputs keep every ReLU open, so the network is the
    linear map y = W3.(W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(3)
    w = {"W1": rng.uniform(0.1, 1, (32, 10)), "b1": rng.uniform(0.1, 1, 32), "W2": rng.uniform(0.1, 1, (32, 32)),
         "b2": rng.uniform(0.1, 1, 32), "W3": rng.uniform(-1, 1, 32), "b3": np.array([0.3])}
    X = rng.uniform(0.1, 1, (5, 10))
    y, _ = mlp.forward(mlp.pack(w), X)
    lin = ((X @ w["W1"].T + w["b1"]) @ w["W2"].T + w["b2"]) @ w["W3"] + 0.3
    np.testing.assert_allclose(y, lin, rtol=1e-12)
