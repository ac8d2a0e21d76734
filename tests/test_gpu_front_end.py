"""GPU checks of the sparse front end of bounded-window slice calls.

The scatter flags the brick x rows that hold events; ranking builds pair-grid
entries and row numbers only in flagged rows, and after each call the
flagged rows' counts, pair entries and flags go back to zero (the pair grid
is no longer rewritten densely per call).  Anything a call leaves behind, or
any entry it fails to write, shows up in a later call on the same context.
So each test runs a sequence of calls on one context: every tiling, all
events and query subsets, encodings, counts and flows, sensors of different
sizes, a batch, and a call with invalid events.  Each result must be
bit-identical to the same call on a fresh context, whose grids start zeroed.
The first call of each sequence is also checked against the FP64 oracle.
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


def _slices():
    """Three slices of different sensors, lengths and densities (moving edges
    plus uniform noise), with events on the grid faces."""
    out = []
    for k, (W, H, T, n) in enumerate([(346, 260, 20, 40_000), (64, 48, 9, 3_000),
                                      (200, 130, 14, 25_000)]):
        ev, t0, T = synth.make_slice(synth.SliceSpec(W, H, T, n, 6, seed=8800 + k))
        ev = ev.copy()
        ev[0, :3] = [0, 0, t0]
        ev[1, :3] = [W - 1, H - 1, t0 + T - 1]
        ev[2, :3] = [W - 1, 0, t0 + T - 1]
        out.append((W, H, ev, t0, T))
    return out


CONFIGS = [(64, 3, 2, 128), (128, 5, 3, 256)]


def _ctx(vk, cfg, precision, tiling):
    d, r, rt, hidden = cfg
    A = synth.draw_frequencies(d, r, r, rt)
    c = vk.Context(346, 260, r, r, rt, A, 20, 70_000, precision, max_slices=3)
    c.set_mlp(*synth.init_mlp(d, hidden))
    c.select_tiling(tiling)
    return c, A


def _calls(slices):
    """The call sequence: (kind, slice index or None for the batch, queries)."""
    q1 = synth.sample_queries(len(slices[1][2]), 700, 31)
    q1 = np.concatenate([q1, q1[:50]]).astype(np.int32)  # duplicates too
    q0 = synth.sample_queries(len(slices[0][2]), 5_000, 32)
    return [("flow", 0, None), ("flow", 1, q1), ("encode", 2, None), ("count", 0, None),
            ("flow", 2, None), ("batch", None, None), ("encode", 0, q0), ("bad", 1, None),
            ("flow", 1, None), ("flow", 0, None)]


def _run(vk, c, slices, kind, k, q):
    if kind == "batch":
        specs = [(W, H, t0, T, len(ev)) for (W, H, ev, t0, T) in slices]
        ev = torch.from_numpy(np.concatenate([s[2] for s in slices])).cuda()
        out = c.flow_batch(specs, ev)
    else:
        W, H, ev, t0, T = slices[k]
        if kind == "bad":  # a tenth of the events outside the slice: reported, not counted
            ev = ev.copy()
            ev[::10, 2] = t0 + T + 3
        evt = torch.from_numpy(ev).cuda()
        qt = None if q is None else torch.from_numpy(q).cuda()
        fn = {"flow": c.flow, "bad": c.flow, "encode": c.encode, "count": c.count}[kind]
        out = fn(evt, t0, T, queries=qt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), c.status()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("cfg", CONFIGS, ids=["d64", "d128"])
def test_call_sequences_match_fresh_contexts(vk, cfg, precision):
    slices = _slices()
    probe, _ = _ctx(vk, cfg, precision, 0)
    tilings = probe.tilings()
    probe.close()
    for ti, tl in enumerate(tilings):
        c, A = _ctx(vk, cfg, precision, ti)
        for step, (kind, k, q) in enumerate(_calls(slices)):
            _say("case: front end %s d=%d tiling %s step %d %s slice %s" %
                 (precision, cfg[0], tl, step, kind, k))
            got, st = _run(vk, c, slices, kind, k, q)
            fresh, _ = _ctx(vk, cfg, precision, ti)
            want, st2 = _run(vk, fresh, slices, kind, k, q)
            fresh.close()
            assert st == st2 == (vk.VECKM_E_RANGE if kind == "bad" else vk.VECKM_OK), (st, st2)
            # bitwise (invalid events' outputs are NaN)
            assert got.shape == want.shape and got.tobytes() == want.tobytes(), (tl, step, kind)
            if step == 0:
                W, H, ev, t0, T = slices[0]
                qs = synth.sample_queries(len(ev), 300, 33)
                emb, _ = oracle.encode(ev, A, cfg[1], cfg[1], cfg[2], queries=qs)
                ref = oracle.mlp(emb, *synth.init_mlp(cfg[0], cfg[3]))
                err = np.linalg.norm(got[qs] - ref) / np.linalg.norm(ref)
                assert err <= (1e-3 if precision == "fp32" else 3e-2), err
        c.close()


def test_counts_exact_after_sequences(vk):
    """The neighbour counts of every event (Eqn. 17) equal the oracle's
    exactly after calls that flagged other rows, other sensors and invalid
    events on the same context."""
    slices = _slices()
    c, A = _ctx(vk, CONFIGS[1], "fp32", 0)
    for kind, k, q in _calls(slices)[:8]:
        _run(vk, c, slices, kind, k, q)
    for k in range(3):
        W, H, ev, t0, T = slices[k]
        _say("case: exact counts after sequence, slice %d (%dx%dx%d)" % (k, W, H, T))
        got, st = _run(vk, c, slices, "count", k, None)
        assert st == vk.VECKM_OK
        qs = synth.sample_queries(len(ev), 2_000, 40 + k)
        _, cnt = oracle.encode(ev, A, 5, 5, 3, queries=qs)
        assert np.array_equal(got[qs].astype(np.int64), np.asarray(cnt, np.int64))
    c.close()
