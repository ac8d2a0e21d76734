"""GPU checks of the launch graphs (veckm_graph_create / veckm_graph_launch).

A graph captured for a batch layout replays the batch call bit for bit: each
replay reads the event buffer as it is at launch time, so the buffer is
refilled between replays (alternating two event sets of the same layout),
with eager batch calls and other device work of the program in between, and
every replay is compared with the eager batch call on the same events.  The
first event set is also checked against the FP64 oracle on sampled events.
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


D, RX, RT, HIDDEN = 64, 3, 2, 128


def _layout():
    """Eight uneven slices on two sensors (one empty), and a second event set
    of the same layout (x mirrored within each slice)."""
    rng = np.random.Generator(np.random.PCG64(7301))
    specs, a, b = [], [], []
    for k, n in enumerate([20_000, 3_000, 0, 45_000, 700, 12_000, 64, 30_000]):
        W, H = (346, 260) if k % 2 == 0 else (640, 480)
        T, t0 = 25, 5_000 * k - 9_000
        ev = synth.random_events(rng, n, W, H, T, t_base=t0)
        specs.append((W, H, t0, T, n))
        a.append(ev)
        m = ev.copy()
        m[:, 0] = W - 1 - m[:, 0]
        b.append(m)
    return specs, np.concatenate(a).astype(np.int32), np.concatenate(b).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_graph_replays_match_eager_batch(vk, precision):
    specs, ev_a, ev_b = _layout()
    A = synth.draw_frequencies(D, RX, RX, RT)
    mlp = synth.init_mlp(D, HIDDEN)
    n = len(ev_a)
    _say("case: graph %s, %d slices, %d events" % (precision, len(specs), n))
    c = vk.Context(640, 480, RX, RX, RT, A, 25, n, precision, max_slices=8)
    c.set_mlp(*mlp)
    events = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    flow = torch.empty((n, 2), device="cuda")
    emb = torch.empty((n, 2 * D), device="cuda")
    g_flow = c.graph(specs, events, flow, flow=True)
    g_emb = c.graph(specs, events, emb, flow=False)
    sets = [torch.from_numpy(ev_a).cuda(), torch.from_numpy(ev_b).cuda()]
    eager = [c.flow_batch(specs, e).cpu().numpy() for e in sets]
    eager_emb = c.encode_batch(specs, sets[0]).cpu().numpy()
    torch.cuda.synchronize()
    assert c.status() == vk.VECKM_OK
    for r in range(5):
        k = r % 2
        events.copy_(sets[k])
        g_flow.launch()
        got = flow.cpu().numpy()
        assert np.array_equal(got, eager[k]), ("replay", r)
        if k == 0:
            g_emb.launch()
            assert np.array_equal(emb.cpu().numpy(), eager_emb), ("emb replay", r)
        # the program's own device work between replays
        x = torch.randn(4096, 256, device="cuda")
        (x @ x.T).sum().item()
        eager_again = c.flow_batch(specs, sets[1 - k]).cpu().numpy()
        assert np.array_equal(eager_again, eager[1 - k])
    assert c.status() == vk.VECKM_OK
    # set A against the oracle on sampled events of every non-empty slice
    off, got, ref = 0, [], []
    events.copy_(sets[0])
    g_flow.launch()
    flows = flow.cpu().numpy()
    for k, (W, H, t0, T, m) in enumerate(specs):
        if m:
            q = synth.sample_queries(m, 12, 7400 + k)
            e = ev_a[off:off + m]
            emb_o, _ = oracle.encode(e, A, RX, RX, RT, queries=q)
            ref.append(oracle.mlp(emb_o, *mlp))
            got.append(flows[off + q])
        off += m
    err = float(np.linalg.norm(np.concatenate(got) - np.concatenate(ref)) /
                np.linalg.norm(np.concatenate(ref)))
    _say("graph %s flow relL2 vs oracle %.2e" % (precision, err))
    assert err <= (1e-3 if precision == "fp32" else 2e-2)
    g_flow.close()
    g_emb.close()
    c.close()


def test_graph_create_errors(vk):
    specs, ev_a, _ = _layout()
    A = synth.draw_frequencies(D, RX, RX, RT)
    n = len(ev_a)
    c = vk.Context(640, 480, RX, RX, RT, A, 25, n, "fp32", max_slices=8)
    events = torch.from_numpy(ev_a).cuda()
    flow = torch.empty((n, 2), device="cuda")
    with pytest.raises(vk.VeckmError) as e:  # no perceptron yet
        c.graph(specs, events, flow, flow=True)
    assert e.value.code == vk.VECKM_E_STATE
    c.set_mlp(*synth.init_mlp(D, HIDDEN))
    bad = [(641, 480, 0, 25, n)]  # wider than the context
    with pytest.raises(vk.VeckmError) as e:
        c.graph(bad, events, flow, flow=True)
    assert e.value.code == vk.VECKM_E_RANGE
    c.close()
