"""GPU tests of the serving layer (veckm_server_* / veckm_stream_* /
veckm_submit / veckm_poll).

The central property: a slice's flows are the same whether it runs alone or
continuously batched with slices of other streams arriving concurrently
(bit-identical, since slices are independent and each row's arithmetic does
not depend on its batch), and they match the FP64 oracle within the BF16
form's tolerance (relative L2 <= 3e-2 on flows).
"""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_2504_19417_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

D, R, HIDDEN = 64, (3, 3, 2), 128


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


def _streams(seed=77, count=6, per=3):
    """Slices of `count` streams (346x260 or 640x480), `per` each, of 300 to
    20,000 events over 4 to 16 one-ms bins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(count):
        W, H = (346, 260) if s % 2 == 0 else (640, 480)
        slices = []
        for k in range(per):
            n = int(rng.integers(300, 20_000))
            T = int(rng.integers(4, 17))
            spec = synth.SliceSpec(W, H, T, n, 4, seed=5000 + 10 * s + k,
                                   t_base=1_000_000 + 100 * k)
            ev, t0, nb = synth.make_slice(spec)
            slices.append((ev, t0, nb))
        out.append(((W, H), slices))
    return out


def _server(vk, A, mlp, max_events=120_000, streams=8, depth=4, max_voxels=0):
    s = vk.Server(640, 480, *R, A, 16, max_events, "fp16", hbm_budget_bytes=32 << 30,
                  max_streams=streams, depth=depth, max_voxels=max_voxels)
    s.set_mlp(*mlp)
    return s


def test_alone_equals_in_mix_and_oracle(vk):
    _say("case: server alone vs mix")
    A = synth.draw_frequencies(D, *R)
    mlp = synth.init_mlp(D, HIDDEN)
    data = _streams()
    srv = _server(vk, A, mlp)
    sids = [srv.open_stream(W, H, 16, 20_000) for (W, H), _ in data]
    # alone: one slice at a time
    alone = []
    for sid, (_, slices) in zip(sids, data):
        res = []
        for ev, t0, T in slices:
            rc, f = srv.poll(srv.submit(sid, ev, t0, T))
            assert rc == vk.VECKM_OK
            res.append(f)
        alone.append(res)
    srv.stats(reset=True)
    # in the mix: every stream submits all its slices at once, from its own thread
    tickets = [[None] * len(sl) for _, sl in data]
    barrier = threading.Barrier(len(data))

    def feed(i):
        barrier.wait()
        for k, (ev, t0, T) in enumerate(data[i][1]):
            tickets[i][k] = srv.submit(sids[i], ev, t0, T)

    th = [threading.Thread(target=feed, args=(i,)) for i in range(len(data))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(len(data)):
        for k in range(len(data[i][1])):
            rc, f = srv.poll(tickets[i][k])
            assert rc == vk.VECKM_OK
            assert np.array_equal(f, alone[i][k]), (i, k)
    st = srv.stats()
    _say("mix: %d slices in %d batches, p50 %.3f ms p99 %.3f ms"
         % (st["slices"], st["batches"], st["p50_ms"], st["p99_ms"]))
    assert st["slices"] == sum(len(sl) for _, sl in data)
    assert st["batches"] < st["slices"]  # slices shared batches
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    # resident grids: every slice of a stream reused its stream's grid; each
    # result equals a fresh slice on a context of its own sensor
    fresh = {}
    for (W, H), _ in data:
        if (W, H) not in fresh:
            c = vk.Context(W, H, *R, A, 16, 20_000, "fp16")
            c.set_mlp(*mlp)
            fresh[(W, H)] = c
    for i, ((W, H), slices) in enumerate(data):
        for k, (ev, t0, T) in enumerate(slices):
            f = fresh[(W, H)].flow(torch.from_numpy(ev).cuda(), t0, T).cpu().numpy()
            assert np.array_equal(f, alone[i][k]), (i, k)
    for c in fresh.values():
        c.close()
    # oracle on a sample of each stream's first slice
    for i, (_, slices) in enumerate(data):
        ev = slices[0][0]
        q = synth.sample_queries(len(ev), 256, 40 + i)
        ref = oracle.mlp(oracle.encode(ev, A, *R, queries=q)[0], *mlp)
        err = rel_l2(alone[i][0][q], ref)
        assert err <= 3e-2, err
    for sid in sids:
        srv.close_stream(sid)
    srv.close()


def test_admission_by_capacity_and_close(vk):
    _say("case: server admission")
    A = synth.draw_frequencies(D, *R)
    mlp = synth.init_mlp(D, HIDDEN)
    # room for exactly three 20k-event streams
    srv = _server(vk, A, mlp, max_events=60_000, streams=8)
    sids = [srv.open_stream(346, 260, 16, 20_000) for _ in range(3)]
    with pytest.raises(vk.VeckmError) as e:
        srv.open_stream(346, 260, 16, 20_000)
    assert e.value.code == vk.VECKM_E_BUDGET
    with pytest.raises(vk.VeckmError) as e:
        srv.open_stream(641, 480, 16, 100)  # wider than the server's sensor
    assert e.value.code == vk.VECKM_E_RANGE
    srv.close_stream(sids[1])
    sids[1] = srv.open_stream(346, 260, 16, 20_000)
    # a slice beyond the stream's limits
    ev = synth.random_events(np.random.Generator(np.random.PCG64(3)), 10, 346, 260, 4)
    with pytest.raises(vk.VeckmError) as e:
        srv.submit(sids[0], ev, 0, 17)
    assert e.value.code == vk.VECKM_E_RANGE
    for sid in sids:
        srv.close_stream(sid)
    srv.close()


def test_resident_grid_arena_admission(vk):
    """Each open stream holds its grids in the server's arena: with room for
    two 346x260x16 streams a third is refused (as is a larger sensor), a
    close gives its region back, and slices of streams opened in a reused
    region give the same flows as before."""
    _say("case: server grid arena")
    A = synth.draw_frequencies(D, *R)
    mlp = synth.init_mlp(D, HIDDEN)
    srv = _server(vk, A, mlp, max_events=60_000, streams=8, max_voxels=2 * 346 * 260 * 16)
    a = srv.open_stream(346, 260, 16, 10_000)
    b = srv.open_stream(346, 260, 16, 10_000)
    for W, H in ((346, 260), (640, 480)):
        with pytest.raises(vk.VeckmError) as e:
            srv.open_stream(W, H, 16, 1000)
        assert e.value.code == vk.VECKM_E_BUDGET
    rng = np.random.Generator(np.random.PCG64(12))
    ev = synth.random_events(rng, 8000, 346, 260, 12, t_base=300)
    rc, ref = srv.poll(srv.submit(a, ev, 300, 12))
    assert rc == vk.VECKM_OK
    srv.close_stream(a)
    c = srv.open_stream(346, 260, 8, 10_000)  # a smaller stream in the freed region
    for sid in (b, c):
        rc, f = srv.poll(srv.submit(sid, ev[ev[:, 2] < 308], 300, 8))
        assert rc == vk.VECKM_OK
        rc, f = srv.poll(srv.submit(b, ev, 300, 12))
        assert rc == vk.VECKM_OK and np.array_equal(f, ref)
    srv.close_stream(b)
    srv.close_stream(c)
    srv.close()


def test_depth_poll_and_errors(vk):
    _say("case: server depth / poll / device errors")
    A = synth.draw_frequencies(D, *R)
    mlp = synth.init_mlp(D, HIDDEN)
    srv = _server(vk, A, mlp, depth=2)
    sid = srv.open_stream(346, 260, 8, 5000)
    other = srv.open_stream(640, 480, 8, 5000)
    rng = np.random.Generator(np.random.PCG64(11))
    good = synth.random_events(rng, 4000, 346, 260, 8, t_base=50)
    bad = good.copy()
    bad[17, 0] = 346  # outside the sensor
    ref_rc, ref = srv.poll(srv.submit(sid, good, 50, 8))
    assert ref_rc == vk.VECKM_OK
    # depth: two slices not yet polled fill the stream
    t1 = srv.submit(sid, good, 50, 8)
    t2 = srv.submit(sid, bad, 50, 8)
    with pytest.raises(vk.VeckmError) as e:
        srv.submit(sid, good, 50, 8)
    assert e.value.code == vk.VECKM_E_AGAIN
    t3 = srv.submit(other, good, 50, 8)
    assert srv.poll(987654321)[0] == vk.VECKM_E_INVAL
    rc1, f1 = srv.poll(t1)
    rc2, f2 = srv.poll(t2)
    rc3, f3 = srv.poll(t3)
    assert (rc1, rc2, rc3) == (vk.VECKM_OK, vk.VECKM_E_RANGE, vk.VECKM_OK)
    assert f2 is None
    assert np.array_equal(f1, ref) and np.array_equal(f3, ref)
    # overflow of one voxel is reported for that slice only
    crowd = np.tile(np.array([[5, 5, 51, 1]], np.int32), (vk.VECKM_MAX_VOXEL_EVENTS + 1, 1))
    t4 = srv.submit(sid, crowd, 50, 8)
    t5 = srv.submit(other, good, 50, 8)
    assert srv.poll(t4)[0] == vk.VECKM_E_OVERFLOW
    rc5, f5 = srv.poll(t5)
    assert rc5 == vk.VECKM_OK and np.array_equal(f5, ref)
    # a poll that does not wait
    t6 = srv.submit(sid, good, 50, 8)
    rc, _ = srv.poll(t6, timeout_us=0)
    assert rc in (vk.VECKM_OK, vk.VECKM_E_AGAIN)
    if rc == vk.VECKM_E_AGAIN:
        assert srv.poll(t6)[0] == vk.VECKM_OK
    srv.close_stream(sid)
    srv.close_stream(other)
    srv.close()
