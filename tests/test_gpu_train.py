"""GPU checks of the perceptron trainer through the C-ABI.

  * one gradient-descent step against the FP64 oracle's step on the same
    inputs (relL2 of the new weights' change <= 1e-4, loss <= 1e-5: fp32
    sums over a few thousand rows);
  * Adam steps against the oracle (the step is lr g / (|g| + eps) at first,
    which flips where a gradient is near zero; relL2 of the change <= 2e-3);
  * determinism (two trainers from the same start give identical weights);
  * learning: on encodings of synthetic edges (GPU encoder) with their true
    normal flows (four slices of 32 edges), Adam lowers the loss, and on a
    held-out slice the trained perceptron's flows point the right way
    (median cosine to the true normal flow > 0.8) with a squared error well
    below a constant predictor's (< 0.7 of it).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_19417_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def vk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19417_amd import veckm
    return veckm


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _batch(seed, m, d, hidden):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, (m, 2 * d)).astype(np.float32)
    y = rng.normal(0, 1.5, (m, 2)).astype(np.float32)
    W1, b1, W2, b2 = synth.init_mlp(d, hidden)
    return x, y, dict(W1=W1, b1=b1, W2=W2, b2=b2)


@pytest.mark.parametrize("m,d,hidden", [(3000, 64, 128), (777, 32, 64), (5000, 128, 256)])
def test_sgd_step_matches_oracle(vk, m, d, hidden):
    x, y, p = _batch(5001 + m, m, d, hidden)
    _say("case: trainer sgd step m=%d d=%d hidden=%d" % (m, d, hidden))
    tr = vk.Trainer(d, hidden, m, p["W1"], p["b1"], p["W2"], p["b2"])
    loss = torch.zeros(1, device="cuda")
    tr.step(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), "sgd", 0.05, loss)
    W1, b1, W2, b2 = tr.weights()
    L, g, new, _ = oracle.mlp_train_step(x, y, p, "sgd", lr=0.05)
    assert abs(float(loss.cpu()[0]) - L) <= 1e-5 * L
    for k, got in zip(("W1", "b1", "W2", "b2"), (W1, b1, W2, b2)):
        e = rel_l2(got.astype(np.float64) - p[k], new[k] - p[k])
        _say("  %s change relL2 %.2e" % (k, e))
        assert e <= 1e-4, k
    tr.close()


def test_adam_steps_match_oracle_and_are_deterministic(vk):
    m, d, hidden = 4000, 64, 128
    x, y, p = _batch(5101, m, d, hidden)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    trs = [vk.Trainer(d, hidden, m, p["W1"], p["b1"], p["W2"], p["b2"]) for _ in range(2)]
    ref, state = dict(p), None
    for t in range(1, 4):
        for tr in trs:
            tr.step(xt, yt, "adam", 1e-3)
        _, _, ref, state = oracle.mlp_train_step(x, y, ref, "adam", lr=1e-3, state=state, t=t)
    w_a, w_b = trs[0].weights(), trs[1].weights()
    for a, b in zip(w_a, w_b):
        assert np.array_equal(a, b)
    for k, got in zip(("W1", "b1", "W2", "b2"), w_a):
        e = rel_l2(got.astype(np.float64) - p[k], ref[k] - p[k])
        _say("adam 3 steps %s change relL2 %.2e" % (k, e))
        assert e <= 2e-3, k
    for tr in trs:
        tr.close()


def test_training_on_synthetic_edges_learns_normal_flow(vk):
    d, hidden, rx, rt = 64, 128, 3, 2
    A = synth.draw_frequencies(d, rx, rx, rt)

    def encoded(seed):
        ev, t0, T, f = synth.make_slice(synth.SliceSpec(346, 260, 25, 50_000, 32, seed=seed),
                                        with_flow=True)
        c = vk.Context(346, 260, rx, rx, rt, A, T, len(ev))
        emb = c.encode(torch.from_numpy(ev).cuda(), t0, T)
        torch.cuda.synchronize()
        assert c.status() == vk.VECKM_OK
        keep = ~np.isnan(f[:, 0])
        idx = torch.from_numpy(np.nonzero(keep)[0]).cuda()
        return c, ev, t0, T, emb[idx].contiguous(), f[keep].astype(np.float32), keep

    xs, ys = [], []
    for k in range(4):
        c, _, _, _, x, y, _ = encoded(5201 + k)
        xs.append(x)
        ys.append(y)
        c.close()
    x_tr, y_tr = torch.cat(xs).contiguous(), np.concatenate(ys)
    W1, b1, W2, b2 = synth.init_mlp(d, hidden)
    tr = vk.Trainer(d, hidden, len(y_tr), W1, b1, W2, b2)
    yt = torch.from_numpy(y_tr).cuda()
    loss = torch.zeros(1, device="cuda")
    losses = []
    for it in range(400):
        tr.step(x_tr, yt, "adam", 3e-3, loss)
        if it % 100 == 0 or it == 399:
            losses.append(float(loss.cpu()[0]))
    _say("training loss", ["%.3f" % v for v in losses])
    assert losses[-1] < 0.6 * losses[0]
    # held-out slice through the inference path with the trained weights
    c_te, ev, t0, T, _, y_te, keep = encoded(5301)
    c_te.set_mlp(*tr.weights())
    flow = c_te.flow(torch.from_numpy(ev).cuda(), t0, T).cpu().numpy()[keep]
    mse = float(((flow - y_te) ** 2).sum(1).mean())
    base = float(((y_te - y_tr.mean(0)) ** 2).sum(1).mean())
    cos = np.sum(flow * y_te, 1) / (np.linalg.norm(flow, axis=1) * np.linalg.norm(y_te, axis=1) + 1e-9)
    _say("held-out mse %.3f (constant predictor %.3f), median cosine %.3f"
         % (mse, base, float(np.median(cos))))
    assert mse < 0.7 * base and float(np.median(cos)) > 0.8
    tr.close()
    c_te.close()
