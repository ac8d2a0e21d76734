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


def test_adam_bias_correction_constant_gradient():
    """Adam at t >= 2: with the same gradient g at every step the moment
    estimates are geometric series, (1 - b^t) g and (1 - b^t) g^2, so the
    bias-corrected moments equal g and g^2 exactly at every t and every step
    moves by lr g / (|g| + eps).  A wrong correction power (b^(t-1), or none)
    or a swapped beta moves the step at t = 2 by a factor of about 2."""
    x, y, p = _problem(seed=21)
    lr = 0.01
    st = None
    for t in (1, 2, 3, 7):
        L, g, new, st_next = oracle.mlp_train_step(x, y, p, "adam", lr=lr, state=st, t=t)
        for k in p:
            assert np.allclose(new[k], p[k] - lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-10,
                               atol=1e-14), (t, k)
        # same parameters (hence the same gradient) at the next step; the
        # moments carry over
        st = st_next
        if t == 3:  # skip to t = 7: run steps 4..6 on the same gradient first
            for tt in (4, 5, 6):
                _, _, _, st = oracle.mlp_train_step(x, y, p, "adam", lr=lr, state=st, t=tt)


def test_adam_two_steps_hand_derived():
    """Two Adam steps where only b2 learns (layer 1 silent: W1 = 0, b1 < 0),
    targets zero: the gradient of b2 is 2 b2.  From b2 = (1, -1/2), lr = 1/10:
    step 1 moves each component by lr sign(g) (to 1e-9), giving
    b2 = (0.9, -0.4) and g = (1.8, -0.8); then m = 0.9 (0.1 g1) + 0.1 g2 =
    (0.36, -0.17), v = 0.999 (0.001 g1^2) + 0.001 g2^2 = (0.007236, 0.001639),
    bias corrections 1 - 0.9^2 = 0.19 and 1 - 0.999^2 = 0.001999."""
    x, _, p = _problem(seed=22, K2=4, hidden=3)
    p["W1"][:] = 0.0
    p["b1"][:] = -1.0
    p["b2"] = np.array([1.0, -0.5])
    y = np.zeros((x.shape[0], 2))
    _, g1, p1, st = oracle.mlp_train_step(x, y, p, "adam", lr=0.1, t=1)
    np.testing.assert_allclose(g1["b2"], [2.0, -1.0], rtol=1e-15)
    np.testing.assert_allclose(p1["b2"], [0.9, -0.4], rtol=0, atol=1e-9)
    _, g2, p2, _ = oracle.mlp_train_step(x, y, p1, "adam", lr=0.1, state=st, t=2)
    np.testing.assert_allclose(g2["b2"], [1.8, -0.8], rtol=0, atol=1e-8)
    mhat = np.array([0.36, -0.17]) / 0.19
    vhat = np.array([0.007236, 0.001639]) / 0.001999
    expect = np.array([0.9, -0.4]) - 0.1 * mhat / np.sqrt(vhat)
    np.testing.assert_allclose(p2["b2"], expect, rtol=0, atol=1e-8)
    for k in ("W1", "b1", "W2"):
        assert np.array_equal(p2[k], p[k])
