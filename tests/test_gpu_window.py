"""GPU checks of the sliding-window (streaming) encoder through the C-ABI.

A recording is pushed a few bins at a time into a window of Tw bins (the ring
wraps several times, and one push skips bins).  After each push, query events
of the window are encoded and compared (a) bit for bit with veckm_encode /
veckm_flow of a slice holding exactly the window's events (t0 = end - Tw,
nbins = Tw), and (b) with the FP64 oracle over those events (relL2 <= 1e-4 for
encodings, the FP32 form's bar).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2504_19417_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W, H, TW, RX, RT, D = 346, 260, 12, 4, 2, 64


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


@pytest.fixture(scope="module")
def recording():
    ev, t0, T = synth.make_slice(synth.SliceSpec(W, H, 40, 200_000, 12, seed=4001))
    A = synth.draw_frequencies(D, RX, RX, RT)
    mlp = synth.init_mlp(D, 128)
    return ev, t0, T, A, mlp


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_window_matches_slice_encode_and_oracle(vk, recording, precision):
    ev, t0, T, A, mlp = recording
    win = vk.Window(W, H, RX, RX, RT, A, TW, len(ev), precision)
    win.set_mlp(*mlp)
    ref = vk.Context(W, H, RX, RX, RT, A, TW, len(ev), precision)
    ref.set_mlp(*mlp)
    rng = np.random.Generator(np.random.PCG64(4002))
    # bins pushed: 3 at a time, then a skipped stretch, then the rest
    pushes = [(b, 3) for b in range(0, 30, 3)] + [(33, 3), (36, 4)]
    checked = 0
    for b0, nb in pushes:
        sel = (ev[:, 2] >= t0 + b0) & (ev[:, 2] < t0 + b0 + nb)
        win.push(_cuda(ev[sel]), t0 + b0, nb)
        end = t0 + b0 + nb
        wsel = (ev[:, 2] >= end - TW) & (ev[:, 2] < end)
        if b0 >= 33:  # the skipped bins 30-32 hold nothing in the window
            wsel &= (ev[:, 2] < t0 + 30) | (ev[:, 2] >= t0 + 33)
        wev = np.ascontiguousarray(ev[wsel])
        q = rng.choice(len(wev), size=min(3000, len(wev)), replace=False).astype(np.int32)
        emb_w = win.encode_window(_cuda(wev[q])).cpu().numpy()
        flow_w = win.flow_window(_cuda(wev[q])).cpu().numpy()
        torch.cuda.synchronize()
        assert win.status() == vk.VECKM_OK
        emb_s = ref.encode(_cuda(wev), end - TW, TW, _cuda(q)).cpu().numpy()
        flow_s = ref.flow(_cuda(wev), end - TW, TW, _cuda(q)).cpu().numpy()
        assert ref.status() == vk.VECKM_OK
        assert np.array_equal(emb_w, emb_s), (b0, nb)
        assert np.array_equal(flow_w, flow_s), (b0, nb)
        if b0 in (0, 12, 27, 36):  # the oracle on a few windows (first, wrapped, after the gap)
            emb_o, _ = oracle.encode(wev, A, RX, RX, RT, queries=q[:800])
            e = rel_l2(emb_w[:800], emb_o)
            _say("window %s bins [%d, %d) emb relL2 %.3e" % (precision, end - TW - t0, end - t0, e))
            assert e <= (1e-4 if precision == "fp32" else 2e-3)
            checked += 1
    assert checked == 4
    win.close()
    ref.close()


def test_window_argument_errors_and_empty_neighbourhood(vk, recording):
    ev, t0, T, A, mlp = recording
    win = vk.Window(W, H, RX, RX, RT, A, TW, len(ev))
    with pytest.raises(vk.VeckmError) as e:  # nothing pushed yet
        win.encode_window(_cuda(ev[:10]))
    assert e.value.code == vk.VECKM_E_STATE
    sel = (ev[:, 2] >= t0) & (ev[:, 2] < t0 + 4)
    win.push(_cuda(ev[sel]), t0, 4)
    with pytest.raises(vk.VeckmError) as e:  # back in time
        win.push(_cuda(ev[sel][:10]), t0 + 2, 1)
    assert e.value.code == vk.VECKM_E_INVAL
    with pytest.raises(vk.VeckmError) as e:  # more bins than the window holds
        win.push(_cuda(ev[:0]), t0 + 4, TW + 1)
    assert e.value.code == vk.VECKM_E_RANGE
    with pytest.raises(vk.VeckmError) as e:  # single-slice calls are not for windows
        win.encode(_cuda(ev[sel]), t0, 4)
    assert e.value.code == vk.VECKM_E_INVAL
    # a query far from every event: zero encoding, no error
    lone = np.array([[W - 1, H - 1, t0 + 3, 1]], np.int32)
    occupied = (np.abs(ev[sel][:, 0] - (W - 1)) <= RX) & (np.abs(ev[sel][:, 1] - (H - 1)) <= RX)
    if not occupied.any():
        out = win.encode_window(_cuda(lone)).cpu().numpy()
        assert win.status() == vk.VECKM_OK and np.all(out == 0)
    # a query outside the window is reported
    win.encode_window(_cuda(np.array([[5, 5, t0 + 4, 1]], np.int32)))
    assert win.status() == vk.VECKM_E_RANGE
    # an event outside the pushed bins is reported
    win.push(_cuda(np.array([[5, 5, t0 + 9, 1]], np.int32)), t0 + 4, 2)
    assert win.status() == vk.VECKM_E_RANGE
    win.close()
