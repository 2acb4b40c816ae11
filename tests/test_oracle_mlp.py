"""Pins of the screener network's FP64 reference: gradients against central
differences, the asymmetric loss, and one Adam step by hand."""
import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    p = mlp.init(6, hidden=8, seed=1)
    x = rng.standard_normal((17, 6))
    t = rng.standard_normal(17)
    for alpha in (1.0, 4.0):
        _, g = mlp.backward(p, x, t, alpha)
        h = 1e-6
        for k in mlp.NAMES:
            it = np.nditer(p[k], flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                p2 = {q: v.copy() for q, v in p.items()}
                p2[k][idx] += h
                lp = mlp.loss(p2, x, t, alpha)
                p2[k][idx] -= 2 * h
                lm = mlp.loss(p2, x, t, alpha)
                num = (lp - lm) / (2 * h)
                assert abs(num - g[k][idx]) <= 1e-6 * max(1.0, abs(num)), (k, idx)


def test_asymmetric_loss_weights_underprediction():
    p = mlp.init(2, hidden=4, seed=0)
    x = np.zeros((1, 2))
    y, _ = mlp.forward(p, x)
    over = mlp.loss(p, x, y - 0.5, 4.0)
    under = mlp.loss(p, x, y + 0.5, 4.0)
    assert abs(over - 0.25) < 1e-12 and abs(under - 1.0) < 1e-12


def test_adam_single_step_by_hand():
    p = {k: np.array([1.0]) for k in mlp.NAMES}
    g = {k: np.array([0.5]) for k in mlp.NAMES}
    m = {k: np.zeros(1) for k in mlp.NAMES}
    v = {k: np.zeros(1) for k in mlp.NAMES}
    p, m, v = mlp.adam(p, g, m, v, 1, 0.01)
    # first step: m_hat = g, v_hat = g^2 -> p -= lr * sign(g) (up to eps)
    for k in mlp.NAMES:
        assert abs(p[k][0] - (1.0 - 0.01 * 0.5 / (0.5 + 1e-8))) < 1e-15
