"""GPU parity of the batch entry points (veckm_encode_batch / veckm_flow_batch).

A batch result must be bit-identical, slice by slice, to encoding that slice
alone on a context of its own sensor size (slices are independent, and the
per-row arithmetic does not depend on which other rows share a launch), and
within the FP32-form tolerance of the FP64 oracle (relative L2 <= 1e-4 for
encodings, 1e-3 for flows).
"""
import ctypes
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


D, R, HIDDEN = 48, (4, 2, 3), 64


def _mixed_slices():
    """Slices of different sensors, lengths and sizes: ragged, empty, smaller
    than one brick, all events in one voxel, events on every grid face."""
    rng = np.random.Generator(np.random.PCG64(4242))
    specs = [(37, 29, 9, 1000, -5), (16, 12, 3, 0, 0), (64, 40, 12, 4097, 1 << 30),
             (5, 3, 1, 7, 123), (1, 1, 1, 3, 0), (64, 40, 2, 2500, -(1 << 20))]
    out = []
    for W, H, T, n, t0 in specs:
        ev = synth.random_events(rng, n, W, H, T, t_base=t0)
        if n >= 8:
            ev[0, :3] = [0, 0, t0]
            ev[1, :3] = [W - 1, H - 1, t0 + T - 1]
            ev[2, :3] = [0, H - 1, t0]
            ev[3, :3] = [W - 1, 0, t0 + T // 2]
        out.append(((W, H, t0, T, n), ev))
    return out


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_batch_equals_single_and_oracle(vk, precision):
    _say("case: mixed batch %s" % precision)
    sl = _mixed_slices()
    A = synth.draw_frequencies(D, *R)
    mlp = synth.init_mlp(D, HIDDEN)
    specs = [s for s, _ in sl]
    ev = np.concatenate([e for _, e in sl]).astype(np.int32)
    c = vk.Context(64, 40, *R, A, 12, len(ev), precision, max_slices=8)
    c.set_mlp(*mlp)
    evt = _gpu(ev)
    emb = c.encode_batch(specs, evt)
    flow = c.flow_batch(specs, evt)
    torch.cuda.synchronize()
    assert c.status() == vk.VECKM_OK
    emb, flow = emb.cpu().numpy(), flow.cpu().numpy()
    off = 0
    for (W, H, t0, T, n), e in sl:
        s = vk.Context(W, H, *R, A, T, max(n, 1), precision)
        s.set_mlp(*mlp)
        if n:
            one = s.encode(_gpu(e), t0, T).cpu().numpy()
            onef = s.flow(_gpu(e), t0, T).cpu().numpy()
            assert s.status() == vk.VECKM_OK
            assert np.array_equal(emb[off:off + n], one), (W, H, T, n)
            assert np.array_equal(flow[off:off + n], onef), (W, H, T, n)
            ref, _ = oracle.encode(e, A, *R)
            err = rel_l2(one, ref)
            ferr = rel_l2(onef, oracle.mlp(ref, *mlp))
            _say("slice %dx%dx%d n=%d emb relL2 %.2e flow relL2 %.2e" % (W, H, T, n, err, ferr))
            if precision == "fp32":
                assert err <= 1e-4 and ferr <= 1e-3
            else:
                assert err <= 2e-3 and ferr <= 3e-2
        s.close()
        off += n
    c.close()


def test_batch_slot_reuse(vk):
    """More batch calls in flight than the context's slice-table slots; every
    call keeps its own slice table."""
    _say("case: batch slot reuse")
    sl = _mixed_slices()
    A = synth.draw_frequencies(D, *R)
    c = vk.Context(64, 40, *R, A, 12, 10_000, max_slices=8)
    outs, refs = [], []
    for k in range(20):
        pick = [sl[(k + j) % len(sl)] for j in range(1 + k % 4)]
        specs = [s for s, _ in pick]
        ev = np.concatenate([e for _, e in pick]).astype(np.int32)
        outs.append(c.encode_batch(specs, _gpu(ev)))
        refs.append((specs, ev))
    torch.cuda.synchronize()
    assert c.status() == vk.VECKM_OK
    for (specs, ev), out in zip(refs, outs):
        again = c.encode_batch(specs, _gpu(ev))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), again.cpu().numpy())
    c.close()


def test_batch_argument_errors(vk):
    _say("case: batch argument errors")
    A = synth.draw_frequencies(32, 2, 2, 1)
    c = vk.Context(16, 16, 2, 2, 1, A, 4, 100, max_slices=3)
    ev = _gpu(np.array([[1, 1, 0, 1], [2, 2, 1, -1], [3, 3, 2, 1]], np.int32))
    out = torch.empty((3, 64), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call(specs, offsets=None, count=None):
        arr = vk.make_slices(specs)
        if offsets is not None:
            for k, o in enumerate(offsets):
                arr[k].offset = o
        return vk.veckm_encode_batch(c.handle, arr, len(specs) if count is None else count,
                                     ev.data_ptr(), out.data_ptr(), stream)

    assert call([(16, 16, 0, 4, 3)]) == vk.VECKM_OK
    assert call([(16, 16, 0, 4, 1), (16, 16, 0, 4, 2)], offsets=[0, 2]) == vk.VECKM_E_INVAL
    assert call([(16, 16, 0, 4, 1)] * 4) == vk.VECKM_E_INVAL          # > max_slices
    assert call([(16, 16, 0, 4, 3)], count=0) == vk.VECKM_E_INVAL
    assert call([(17, 16, 0, 4, 3)]) == vk.VECKM_E_RANGE               # wider than the sensor
    assert call([(16, 16, 0, 5, 3)]) == vk.VECKM_E_RANGE               # nbins > max_bins
    assert call([(16, 16, 0, 4, 101)]) == vk.VECKM_E_RANGE             # > max_events
    assert call([(16, 16, 0, 4, -1)]) == vk.VECKM_E_INVAL
    with pytest.raises(vk.VeckmError) as e:
        c.flow_batch([(16, 16, 0, 4, 3)], ev)
    assert e.value.code == vk.VECKM_E_STATE
    torch.cuda.synchronize()
    assert c.status() == vk.VECKM_OK
    # device-side check against each slice's own sensor and time window
    c.encode_batch([(16, 16, 0, 4, 1), (3, 3, 1, 2, 2)], ev)  # (3, 3) is outside 3x3
    assert c.status() == vk.VECKM_E_RANGE
    c.encode_batch([(16, 16, 0, 4, 1), (4, 4, 1, 2, 2)], ev)  # t = 2 is inside [1, 3)
    assert c.status() == vk.VECKM_OK
    c.close()


@pytest.fixture(scope="module")
def batch64():
    w = synth.workloads()["batch64"]
    parts = [synth.make_slice(s) for s in w.slices]
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    return w, parts, A, mlp


@pytest.mark.parametrize("precision", ["fp16", "fp32"])
def test_batch64_full_run_sampled_parity(vk, batch64, precision):
    """The 64-slice batch (5.7M events, 346x260 and 640x480 sensors, D=128,
    r=5/3) in the launch configuration the benchmark times; 64 sampled events
    per slice against the oracle."""
    w, parts, A, mlp = batch64
    _say("case: batch64 %s full run" % precision)
    specs = [(s.width, s.height, t0, T, len(ev)) for s, (ev, t0, T) in zip(w.slices, parts)]
    ev = np.concatenate([p[0] for p in parts]).astype(np.int32)
    c = vk.Context(640, 480, w.rx, w.ry, w.rt, A, 50, len(ev), precision, max_slices=64)
    c.set_mlp(*mlp)
    evt = _gpu(ev)
    emb = c.encode_batch(specs, evt)
    flow = c.flow_batch(specs, evt)
    torch.cuda.synchronize()
    assert c.status() == vk.VECKM_OK
    emb, flow = emb.cpu().numpy(), flow.cpu().numpy()
    off, errs, ferrs = 0, [], []
    got_e, ref_e, got_f, ref_f = [], [], [], []
    for k, (e, t0, T) in enumerate(parts):
        q = synth.sample_queries(len(e), 64, 500 + k)
        ref, _ = oracle.encode(e, A, w.rx, w.ry, w.rt, queries=q)
        got_e.append(emb[off + q])
        ref_e.append(ref)
        got_f.append(flow[off + q])
        ref_f.append(oracle.mlp(ref, *mlp))
        off += len(e)
    err = rel_l2(np.concatenate(got_e), np.concatenate(ref_e))
    ferr = rel_l2(np.concatenate(got_f), np.concatenate(ref_f))
    _say("batch64 %s sampled emb relL2 %.3e flow relL2 %.3e" % (precision, err, ferr))
    if precision == "fp32":
        assert err <= 1e-4 and ferr <= 1e-3
    else:
        assert err <= 2e-3 and ferr <= 3e-2
    assert np.hypot(emb[:, :w.d], emb[:, w.d:]).max() <= 1.0 + 1e-3
    c.close()
