"""Pins of the oracle's perceptron training step (test infrastructure):
central finite differences of the loss for every gradient, closed forms of
the loss and of the first SGD and Adam steps."""
import numpy as np
import pytest

import oracle


def _problem(seed=11, M=37, K2=12, hidden=9):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.normal(0, 1, (M, K2))
    y = rng.normal(0, 2, (M, 2))
    p = dict(W1=rng.normal(0, 0.5, (hidden, K2)), b1=rng.normal(0, 0.5, hidden),
             W2=rng.normal(0, 0.5, (2, hidden)), b2=rng.normal(0, 0.5, 2))
    return x, y, p


def test_gradients_match_central_differences():
    x, y, p = _problem()
    L, g = oracle.mlp_loss_grads(x, y, p["W1"], p["b1"], p["W2"], p["b2"])
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(12))
    for k in ("W1", "b1", "W2", "b2"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, min(12, flat.size), replace=False):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].reshape(-1)[idx] += h
            Lp, _ = oracle.mlp_loss_grads(x, y, q["W1"], q["b1"], q["W2"], q["b2"])
            q[k].reshape(-1)[idx] -= 2 * h
            Lm, _ = oracle.mlp_loss_grads(x, y, q["W1"], q["b1"], q["W2"], q["b2"])
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_loss_closed_form_with_silent_layer1():
    x, y, p = _problem()
    p["W1"][:] = 0.0
    p["b1"][:] = -1.0  # every hidden unit off: the prediction is b2
    L, g = oracle.mlp_loss_grads(x, y, p["W1"], p["b1"], p["W2"], p["b2"])
    assert L == pytest.approx(((p["b2"] - y) ** 2).sum(1).mean(), rel=1e-14)
    assert np.all(g["W1"] == 0) and np.all(g["b1"] == 0) and np.all(g["W2"] == 0)
    assert np.allclose(g["b2"], 2 * (p["b2"] - y).mean(0), rtol=1e-14)


def test_first_sgd_and_adam_steps():
    x, y, p = _problem()
    L, g, new, _ = oracle.mlp_train_step(x, y, p, "sgd", lr=0.05)
    for k in p:
        assert np.allclose(new[k], p[k] - 0.05 * g[k], rtol=0, atol=1e-15)
    # Adam at step 1: the bias-corrected moments are g and g^2, so the step
    # is lr g / (|g| + eps)
    L2, g2, new2, st = oracle.mlp_train_step(x, y, p, "adam", lr=0.01, t=1)
    for k in p:
        assert np.allclose(new2[k], p[k] - 0.01 * g2[k] / (np.abs(g2[k]) + 1e-8), rtol=1e-12,
                           atol=1e-15)
        assert np.allclose(st["m"][k], 0.1 * g2[k]) and np.allclose(st["v"][k], 0.001 * g2[k] ** 2)


def test_a_planted_error_is_caught():
    """A dropped ReLU mask in the backward pass (a plausible mistake) breaks
    the finite-difference agreement: the check above has teeth."""
    x, y, p = _problem()
    z = x @ p["W1"].T + p["b1"]
    h = np.maximum(z, 0)
    dp = 2 * (h @ p["W2"].T + p["b2"] - y) / x.shape[0]
    wrong = (dp @ p["W2"]).T @ x  # no ReLU mask
    _, g = oracle.mlp_loss_grads(x, y, p["W1"], p["b1"], p["W2"], p["b2"])
    assert np.abs(wrong - g["W1"]).max() > 1e-3
