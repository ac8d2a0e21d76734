"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances (relative L2 over the whole output array, oracle as reference):
  FP32 form: encodings <= 1e-4, flows <= 1e-3.
  FP16 form (fp16 offset phases, bf16 perceptron): encodings <= 2e-3,
  flows <= 3e-2; the measured error is printed.
Integer results (the all-ones count pin, isolated events) must be exact.
"""
import sys

import numpy as np
import pytest

import oracle
import parity
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


def _ctx(vk, W, H, r, A, max_bins, max_events, precision="fp32", mlp=None):
    c = vk.Context(W, H, r[0], r[1], r[2], A, max_bins, max_events, precision)
    if mlp is not None:
        c.set_mlp(*mlp)
    return c


def _run_encode(c, ev, t0, nbins, queries=None):
    evt = torch.from_numpy(np.ascontiguousarray(ev)).cuda()
    qt = None if queries is None else torch.from_numpy(np.asarray(queries, np.int32)).cuda()
    out = c.encode(evt, t0, nbins, qt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), c.status()


def _run_flow(c, ev, t0, nbins, queries=None):
    evt = torch.from_numpy(np.ascontiguousarray(ev)).cuda()
    qt = None if queries is None else torch.from_numpy(np.asarray(queries, np.int32)).cuda()
    out = c.flow(evt, t0, nbins, qt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), c.status()


@pytest.fixture(scope="module")
def tiny():
    w = synth.workloads()["tiny"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    emb, cnt = oracle.encode(ev, A, w.rx, w.ry, w.rt)
    flow = oracle.mlp(emb, *mlp)
    return dict(w=w, ev=ev, t0=t0, T=T, A=A, mlp=mlp, emb=emb, cnt=cnt, flow=flow)


def test_tiny_fp32_all_queries(vk, tiny):
    w = tiny["w"]
    _say("case: tiny fp32 encode+flow, n=%d" % len(tiny["ev"]))
    c = _ctx(vk, 346, 260, (w.rx, w.ry, w.rt), tiny["A"], w.slices[0].nbins, len(tiny["ev"]),
             mlp=tiny["mlp"])
    emb, st = _run_encode(c, tiny["ev"], tiny["t0"], tiny["T"])
    assert st == vk.VECKM_OK
    parity.check(emb, tiny["emb"], "fp32", "emb", kp=parity.padded_slots(w.rx, w.ry, w.rt),
                 say=_say)
    flow, st = _run_flow(c, tiny["ev"], tiny["t0"], tiny["T"])
    assert st == vk.VECKM_OK
    parity.check(flow, tiny["flow"], "fp32", "flow", say=_say)
    # P1: the windowed count of every event, bit for bit
    cnt = c.count(torch.from_numpy(tiny["ev"]).cuda(), tiny["t0"], tiny["T"]).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    np.testing.assert_array_equal(cnt, tiny["cnt"])
    q = synth.sample_queries(len(tiny["ev"]), 777, 5).astype(np.int32)
    cq = c.count(torch.from_numpy(tiny["ev"]).cuda(), tiny["t0"], tiny["T"],
                 torch.from_numpy(q).cuda()).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    np.testing.assert_array_equal(cq, tiny["cnt"][q])
    c.close()


def test_tiny_fp16_precision_form(vk, tiny):
    w = tiny["w"]
    _say("case: tiny fp16/bf16 encode+flow")
    c = _ctx(vk, 346, 260, (w.rx, w.ry, w.rt), tiny["A"], w.slices[0].nbins, len(tiny["ev"]),
             precision="fp16", mlp=tiny["mlp"])
    emb, st = _run_encode(c, tiny["ev"], tiny["t0"], tiny["T"])
    assert st == vk.VECKM_OK
    e = rel_l2(emb, tiny["emb"])
    flow, st = _run_flow(c, tiny["ev"], tiny["t0"], tiny["T"])
    f = rel_l2(flow, tiny["flow"])
    _say("tiny fp16 emb relL2 %.3e flow relL2 %.3e" % (e, f))
    assert st == vk.VECKM_OK
    assert e <= 2e-3 and f <= 3e-2
    c.close()


def test_query_subset_with_duplicates(vk, tiny):
    w = tiny["w"]
    _say("case: tiny query subset")
    rng = np.random.Generator(np.random.PCG64(8))
    q = rng.integers(0, len(tiny["ev"]), 3001).astype(np.int32)
    q[:10] = q[0]
    c = _ctx(vk, 346, 260, (w.rx, w.ry, w.rt), tiny["A"], w.slices[0].nbins, len(tiny["ev"]),
             mlp=tiny["mlp"])
    emb, st = _run_encode(c, tiny["ev"], tiny["t0"], tiny["T"], q)
    assert st == vk.VECKM_OK
    assert rel_l2(emb, tiny["emb"][q]) <= 1e-4
    flow, st = _run_flow(c, tiny["ev"], tiny["t0"], tiny["T"], q)
    assert st == vk.VECKM_OK
    assert rel_l2(flow, tiny["flow"][q]) <= 1e-3
    c.close()


def test_count_pin_and_isolated_events_exact(vk):
    """A = 0: every encoding is exactly 1 + 0i (exact neighbour count of an
    all-ones feature).  An isolated event encodes to exactly 1 + 0i for any A."""
    _say("case: count pin / isolated events")
    rng = np.random.Generator(np.random.PCG64(31))
    ev = synth.random_events(rng, 50_000, 120, 90, 20, t_base=-777)
    c = _ctx(vk, 120, 90, (5, 5, 3), np.zeros((128, 3)), 20, len(ev))
    emb, st = _run_encode(c, ev, -777, 20)
    assert st == vk.VECKM_OK
    assert np.all(emb[:, :128] == 1.0) and np.all(emb[:, 128:] == 0.0)
    c.close()
    A = synth.draw_frequencies(64, 3, 3, 2)
    iso = np.array([[0, 0, 0, 1], [50, 50, 5, -1], [119, 89, 19, 1], [60, 0, 19, 1]], np.int32)
    c = _ctx(vk, 120, 90, (3, 3, 2), A, 20, 16)
    emb, st = _run_encode(c, iso, 0, 20)
    assert st == vk.VECKM_OK
    assert np.all(emb[:, :64] == 1.0) and np.all(emb[:, 64:] == 0.0)
    c.close()


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 4097])
def test_ragged_sizes_and_grid_edges(vk, n):
    """Ragged event counts, events on every face of the grid (window clipped
    at the faces), duplicates in one voxel."""
    _say("case: ragged n=%d" % n)
    rng = np.random.Generator(np.random.PCG64(100 + n))
    W, H, T = 37, 29, 9
    ev = synth.random_events(rng, n, W, H, T, t_base=1 << 30)
    if n >= 8:
        ev[0, :3] = [0, 0, 1 << 30]
        ev[1, :3] = [W - 1, H - 1, (1 << 30) + T - 1]
        ev[2, :3] = [0, H - 1, 1 << 30]
        ev[3, :3] = ev[4, :3] = ev[5, :3] = [W - 1, 0, (1 << 30) + 4]
    A = synth.draw_frequencies(48, 4, 2, 3)
    mlp = synth.init_mlp(48, 64)
    ref, cnt = oracle.encode(ev, A, 4, 2, 3)
    c = _ctx(vk, W, H, (4, 2, 3), A, T, max(n, 16), mlp=mlp)
    emb, st = _run_encode(c, ev, 1 << 30, T)
    assert st == vk.VECKM_OK
    parity.check(emb, ref, "fp32", "emb", kp=parity.padded_slots(4, 2, 3), say=_say)
    got = c.count(torch.from_numpy(ev).cuda(), 1 << 30, T).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    np.testing.assert_array_equal(got, cnt)
    flow, st = _run_flow(c, ev, 1 << 30, T)
    assert st == vk.VECKM_OK
    assert rel_l2(flow, oracle.mlp(ref, *mlp)) <= 1e-3
    c.close()


def test_empty_slice(vk):
    _say("case: empty")
    A = synth.draw_frequencies(32, 2, 2, 1)
    c = _ctx(vk, 16, 16, (2, 2, 1), A, 4, 8)
    ev = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    out = c.encode(ev, 0, 4)
    torch.cuda.synchronize()
    assert out.shape == (0, 64) and c.status() == vk.VECKM_OK
    c.close()


def test_input_errors_are_reported(vk):
    _say("case: input errors")
    A = synth.draw_frequencies(32, 2, 2, 1)
    c = _ctx(vk, 16, 16, (2, 2, 1), A, 4, 4096)
    good = np.array([[1, 1, 10, 1], [2, 2, 11, -1]], np.int32)
    _, st = _run_encode(c, good, 10, 4)
    assert st == vk.VECKM_OK
    for bad in ([[16, 1, 10, 1]], [[1, -1, 10, 1]], [[1, 1, 14, 1]], [[1, 1, 9, 1]], [[1, 1, 10, 0]]):
        _, st = _run_encode(c, np.vstack([good, np.array(bad, np.int32)]), 10, 4)
        assert st == vk.VECKM_E_RANGE, bad
    _, st = _run_encode(c, good, 10, 4, queries=[0, 2])
    assert st == vk.VECKM_E_RANGE
    crowd = np.tile(np.array([[3, 3, 10, 1]], np.int32), (vk.VECKM_MAX_VOXEL_EVENTS + 1, 1))
    _, st = _run_encode(c, crowd, 10, 4)
    assert st == vk.VECKM_E_OVERFLOW
    crowd = crowd[:vk.VECKM_MAX_VOXEL_EVENTS]
    emb, st = _run_encode(c, crowd, 10, 4)
    assert st == vk.VECKM_OK
    assert np.all(emb[:, :32] == 1.0) and np.all(emb[:, 32:] == 0.0)
    # host-side argument errors
    evt = torch.from_numpy(good).cuda()
    with pytest.raises(vk.VeckmError) as e:
        c.encode(evt, 10, 5)  # nbins > max_bins
    assert e.value.code == vk.VECKM_E_RANGE
    with pytest.raises(vk.VeckmError) as e:
        c.flow(evt, 10, 4)  # no perceptron set
    assert e.value.code == vk.VECKM_E_STATE
    c.close()


def _full_size_sample(ev, t0, n_random, seed, brick=(32, 16, 8), n_faces=4096):
    """Sampled queries of a full-size slice: n_random seeded events plus up to
    n_faces events whose voxel lies on a face of the encoder's default brick
    (where the count box's halo and the brick edges meet)."""
    q = synth.sample_queries(len(ev), n_random, seed)
    t = ev[:, 2] - t0
    face = ((ev[:, 0] % brick[0] == 0) | (ev[:, 0] % brick[0] == brick[0] - 1) |
            (ev[:, 1] % brick[1] == 0) | (ev[:, 1] % brick[1] == brick[1] - 1) |
            (t % brick[2] == 0) | (t % brick[2] == brick[2] - 1))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    fq = np.flatnonzero(face)
    fq = rng.choice(fq, min(n_faces, len(fq)), replace=False)
    return np.unique(np.concatenate([q, fq])).astype(np.int64)


@pytest.fixture(scope="module")
def slice1m():
    w = synth.workloads()["slice1m"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    q = _full_size_sample(ev, t0, 16384, 77)
    emb, cnt = oracle.encode(ev, A, w.rx, w.ry, w.rt, queries=q)
    return dict(w=w, ev=ev, t0=t0, T=T, A=A, mlp=mlp, q=q, emb=emb,
                flow=oracle.mlp(emb, *mlp), cnt_all=oracle.box_count(ev, w.rx, w.ry, w.rt))


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_slice1m_full_run_sampled_parity(vk, slice1m, precision):
    """The 1M-event, 346x260x50, D=128, r=5/3 workload in the launch
    configuration the benchmark times (all events queried): about 20k
    sampled rows (16384 random, the rest on brick faces) against the oracle
    with whole-sample, per-row and per-element bounds, and the windowed count
    of every one of the 1M events bit for bit against the exact box count."""
    s = slice1m
    w = s["w"]
    _say("case: slice1m %s full run" % precision)
    c = _ctx(vk, 346, 260, (w.rx, w.ry, w.rt), s["A"], s["T"], len(s["ev"]), precision,
             mlp=s["mlp"])
    emb, st = _run_encode(c, s["ev"], s["t0"], s["T"])
    assert st == vk.VECKM_OK
    flow, st = _run_flow(c, s["ev"], s["t0"], s["T"])
    assert st == vk.VECKM_OK
    parity.check(emb[s["q"]], s["emb"], precision, "emb", say=_say)
    parity.check(flow[s["q"]], s["flow"], precision, "flow", say=_say)
    # the sampled events as a query subset (about 15 per brick: most go to
    # the encoder as single rows with their own count boxes): bit-identical
    # to the same rows of the full run
    _say("case: slice1m %s query subset of %d" % (precision, len(s["q"])))
    emb_q, st = _run_encode(c, s["ev"], s["t0"], s["T"], queries=s["q"])
    assert st == vk.VECKM_OK and np.array_equal(emb_q, emb[s["q"]])
    flow_q, st = _run_flow(c, s["ev"], s["t0"], s["T"], queries=s["q"])
    assert st == vk.VECKM_OK and np.array_equal(flow_q, flow[s["q"]])
    # P1: the exact windowed count of every event
    evt = torch.from_numpy(s["ev"]).cuda()
    cnt = c.count(evt, s["t0"], s["T"]).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    np.testing.assert_array_equal(cnt, s["cnt_all"])
    # modulus bound and determinism at full size
    assert np.hypot(emb[:, :128], emb[:, 128:]).max() <= 1.0 + 1e-5
    emb2, _ = _run_encode(c, s["ev"], s["t0"], s["T"])
    assert np.array_equal(emb, emb2)
    # translation by 2^30 in time (and t0) is bit-identical
    ev2 = s["ev"].copy()
    ev2[:, 2] += 1 << 30
    emb3, st = _run_encode(c, ev2, s["t0"] + (1 << 30), s["T"])
    assert st == vk.VECKM_OK and np.array_equal(emb, emb3)
    c.close()


@pytest.fixture(scope="module")
def precision5m():
    w = synth.workloads()["precision5m"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    q = _full_size_sample(ev, t0, 16384, 78)
    emb, cnt = oracle.encode(ev, A, w.rx, w.ry, w.rt, queries=q)
    return dict(w=w, ev=ev, t0=t0, T=T, A=A, mlp=mlp, q=q, emb=emb,
                flow=oracle.mlp(emb, *mlp), cnt_all=oracle.box_count(ev, w.rx, w.ry, w.rt))


def test_precision5m_full_run_sampled_parity(vk, precision5m):
    """The precision workload (1280x720, 5M events with textured-blob noise,
    100 bins, D=128, r=5/3) at full size in the benchmark's launch
    configuration, both forms: about 20k sampled rows against the oracle
    (whole-sample, per-row and per-element bounds), every event's windowed
    count bit for bit, and the FP16/BF16 form's flows against the FP32
    form's over the whole slice."""
    s = precision5m
    w = s["w"]
    evt = torch.from_numpy(s["ev"]).cuda()
    qt = torch.from_numpy(s["q"]).cuda()
    flows = {}
    for precision in ("fp32", "fp16"):
        _say("case: precision5m %s full run" % precision)
        c = _ctx(vk, 1280, 720, (w.rx, w.ry, w.rt), s["A"], s["T"], len(s["ev"]), precision,
                 mlp=s["mlp"])
        emb = c.encode(evt, s["t0"], s["T"])
        emb_q = emb[qt].cpu().numpy()
        del emb
        flow = c.flow(evt, s["t0"], s["T"]).cpu().numpy()
        torch.cuda.synchronize()
        assert c.status() == vk.VECKM_OK
        if precision == "fp32":
            cnt = c.count(evt, s["t0"], s["T"]).cpu().numpy()
            assert c.status() == vk.VECKM_OK
            np.testing.assert_array_equal(cnt, s["cnt_all"])
        c.close()
        parity.check(emb_q, s["emb"], precision, "emb", say=_say)
        parity.check(flow[s["q"]], s["flow"], precision, "flow", say=_say)
        assert np.isfinite(flow).all()
        flows[precision] = flow
    d = rel_l2(flows["fp16"], flows["fp32"].astype(np.float64))
    _say("precision5m fp16 vs fp32 flow relL2 %.3e" % d)
    assert d <= 3e-2
