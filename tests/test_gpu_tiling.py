"""GPU checks of the encoder tilings and the tuner (veckm_tiling_*, veckm_tune).

Every tiling a context offers must give bit-identical encodings (the per-row
arithmetic does not depend on how voxels are grouped into bricks or rows
into waves), for batches and single slices.  Flows are bit-identical among
the tilings whose encoder hands rows to the perceptron kernel, and among the
one-wave-per-SIMD tilings, whose encoder runs the perceptron itself (D = 64
and 128): the two groups sum layer 1 in different orders, so they agree to
fp32 rounding (relL2 <= 1e-5), and both match the FP64 oracle.  The tuner
must pick one of the tilings and leave results unchanged.
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


D, RX, RT, HIDDEN = 128, 5, 3, 256


def _batch():
    """Six slices: two sensors, uneven sizes (one dense, one tiny, one empty),
    events on the grid faces."""
    rng = np.random.Generator(np.random.PCG64(8101))
    specs, parts = [], []
    for k, (n, T) in enumerate([(30_000, 50), (200_000, 50), (0, 7), (900, 13), (60_000, 50),
                                (5_000, 3)]):
        W, H = (346, 260) if k % 2 == 0 else (640, 480)
        t0 = 1_000 * k - 2_500
        ev = synth.random_events(rng, n, W, H, T, t_base=t0)
        if n >= 4:
            ev[0, :3] = [0, 0, t0]
            ev[1, :3] = [W - 1, H - 1, t0 + T - 1]
        specs.append((W, H, t0, T, n))
        parts.append(ev)
    return specs, np.concatenate(parts).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp16", "fp32"])
def test_every_tiling_gives_identical_results(vk, precision):
    specs, ev = _batch()
    A = synth.draw_frequencies(D, RX, RX, RT)
    mlp = synth.init_mlp(D, HIDDEN)
    c = vk.Context(640, 480, RX, RX, RT, A, 50, len(ev), precision, max_slices=8)
    c.set_mlp(*mlp)
    tl = c.tilings()
    _say("case: tilings %s %s" % (precision, tl))
    assert len(tl) >= 1 and c.tiling() == 0
    if precision == "fp16":
        assert len(tl) >= 2, "a larger brick fits beside two fp16 slabs at D = 128, r = 5/3"
    evt = torch.from_numpy(ev).cuda()
    one = torch.from_numpy(ev[specs[0][4]:specs[0][4] + specs[1][4]]).cuda()  # slice 1 alone
    ref = None
    flows = {}  # the first flows of each group: False = perceptron kernel, True = fused

    def fused(t):  # the pipelined wave layouts run the perceptron inside the encoder
        return t[4] >= 2

    for i in range(len(tl)):
        _say("case: tiling %d %s" % (i, tl[i]))
        c.select_tiling(i)
        emb = c.encode_batch(specs, evt).cpu().numpy()
        flow = c.flow_batch(specs, evt).cpu().numpy()
        single = c.encode(one, specs[1][2], specs[1][3]).cpu().numpy()
        torch.cuda.synchronize()
        assert c.status() == vk.VECKM_OK
        if ref is None:
            ref = (emb, single)
        else:
            assert np.array_equal(emb, ref[0]), ("encodings", tl[i])
            assert np.array_equal(single, ref[1]), ("single slice", tl[i])
        g = fused(tl[i])
        if g in flows:
            assert np.array_equal(flow, flows[g]), ("flows", tl[i])
        else:
            flows[g] = flow
    if len(flows) == 2:
        a, b = flows[False].astype(np.float64), flows[True].astype(np.float64)
        d = float(np.linalg.norm(a - b) / np.linalg.norm(a))
        _say("fused vs perceptron-kernel flows relL2 %.2e" % d)
        assert d <= 1e-5
    chosen = c.tune(specs, evt, reps=2)
    _say("tuner picked %d %s" % (chosen, tl[chosen]))
    assert 0 <= chosen < len(tl) and c.tiling() == chosen
    assert np.array_equal(c.flow_batch(specs, evt).cpu().numpy(), flows[fused(tl[chosen])])
    # flows of each group against the oracle on sampled events of slice 1
    e1 = ev[specs[0][4]:specs[0][4] + specs[1][4]]
    q1 = synth.sample_queries(len(e1), 200, 8103)
    emb_o1, _ = oracle.encode(e1, A, RX, RX, RT, queries=q1)
    flow_o = oracle.mlp(emb_o1, *mlp)
    for g, f in flows.items():
        got = f[specs[0][4]:specs[0][4] + specs[1][4]][q1].astype(np.float64)
        err = float(np.linalg.norm(got - flow_o) / np.linalg.norm(flow_o))
        _say("flows (%s) relL2 vs oracle %.2e" % ("fused" if g else "perceptron kernel", err))
        assert err <= (1e-3 if precision == "fp32" else 3e-2)
    # the last tiling against the oracle on sampled events of slice 1
    c.select_tiling(len(tl) - 1)
    e1 = ev[specs[0][4]:specs[0][4] + specs[1][4]]
    q = synth.sample_queries(len(e1), 200, 8102)
    got = c.encode(one, specs[1][2], specs[1][3]).cpu().numpy()[q]
    emb_o, _ = oracle.encode(e1, A, RX, RX, RT, queries=q)
    err = float(np.linalg.norm(got - emb_o) / np.linalg.norm(emb_o))
    _say("tiling %s emb relL2 vs oracle %.2e" % (tl[-1], err))
    assert err <= (1e-4 if precision == "fp32" else 2e-3)
    with pytest.raises(vk.VeckmError):
        c.select_tiling(len(tl))
    c.close()
