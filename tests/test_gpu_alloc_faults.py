"""Out-of-memory unwinding, forced from the host (VECKM_FAULT_ALLOC=n makes
the n-th device or pinned allocation of the library fail).

For each object the library builds (context with its perceptron weights,
paper-form context, sliding window, server with a stream and its first
batch, trainer), every allocation point in turn is made to fail: the call must
return VECKM_E_NOMEM, leave nothing behind (device memory back to where it
was), and the device must still give correct results afterwards.  No kernel
misbehaves here: the failures happen before launches.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2504_19417_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SLACK = 16 << 20  # device bytes a failed build may leave in the runtime's own pools


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def vk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19417_amd import veckm
    return veckm


@pytest.fixture()
def fault_env():
    yield
    os.environ.pop("VECKM_FAULT_ALLOC", None)


def _free(at_least=None):
    """Free device memory; with at_least, waits up to a second for it to
    reach that level (the runtime may hand freed memory back a little
    later)."""
    import time
    torch.cuda.synchronize()
    free = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        if at_least is None or free >= at_least:
            break
        time.sleep(0.05)
        free = torch.cuda.mem_get_info()[0]
    return free


def _params(vk, rt=2, precision="fp32"):
    A = synth.draw_frequencies(64, 3, 3, max(rt, 1))
    return vk.make_params(width=346, height=260, rx=3, ry=3, rt=rt, A=A, max_bins=50,
                          max_events=1_000_000, precision=precision)


def _sweep(vk, build, max_points=200):
    """Runs build() with allocation n failing for n = 1, 2, ... until it
    succeeds; returns the number of allocation points that failed cleanly.
    One unfaulted build first, so that the HIP runtime's own lazy set-up
    (module load, copy staging) is not counted as a leak."""
    os.environ["VECKM_FAULT_ALLOC"] = "0"
    rc, cleanup = build()
    assert rc == vk.VECKM_OK, rc
    cleanup()
    base = _free()
    n = 0
    while True:
        n += 1
        assert n <= max_points, "build never succeeded"
        os.environ["VECKM_FAULT_ALLOC"] = str(n)
        rc, cleanup = build()
        os.environ["VECKM_FAULT_ALLOC"] = "0"
        if rc == vk.VECKM_OK:
            cleanup()
            break
        assert rc == vk.VECKM_E_NOMEM, (n, rc)
        free = _free(base - SLACK)
        assert free >= base - SLACK, "allocation point %d leaked %d bytes" % (n, base - free)
    free = _free(base - SLACK)
    assert free >= base - SLACK, "the successful build leaked %d bytes" % (base - free)
    return n - 1


def test_context_and_perceptron(vk, fault_env):
    W1, b1, W2, b2 = [np.ascontiguousarray(a, np.float32) for a in synth.init_mlp(64, 128)]

    def build():
        p = _params(vk)
        h = ctypes.c_void_p()
        rc = vk._lib.veckm_create(ctypes.byref(p), ctypes.byref(h))
        if rc:
            assert not h.value
            return rc, None
        rc = vk._lib.veckm_set_mlp(h, 128, W1.ctypes.data, b1.ctypes.data, W2.ctypes.data,
                                   b2.ctypes.data)
        if rc:
            vk.veckm_destroy(h)
            return rc, None
        return rc, lambda: vk.veckm_destroy(h)

    points = _sweep(vk, build)
    _say("context + perceptron: %d allocation points" % points)
    assert points >= 15


def test_paper_form_context(vk, fault_env):
    def build():
        p = _params(vk, rt=-1)
        h = ctypes.c_void_p()
        rc = vk._lib.veckm_create(ctypes.byref(p), ctypes.byref(h))
        return rc, (lambda: vk.veckm_destroy(h))

    assert _sweep(vk, build) >= 15


def test_window(vk, fault_env):
    def build():
        p = _params(vk)
        h = ctypes.c_void_p()
        rc = vk._lib.veckm_window_create(ctypes.byref(p), ctypes.byref(h))
        return rc, (lambda: vk.veckm_destroy(h))

    assert _sweep(vk, build) >= 10


def test_trainer(vk, fault_env):
    W1, b1, W2, b2 = [np.ascontiguousarray(a, np.float32) for a in synth.init_mlp(64, 128)]

    def build():
        h = ctypes.c_void_p()
        rc = vk._lib.veckm_trainer_create(64, 128, 200_000, W1.ctypes.data, b1.ctypes.data,
                                          W2.ctypes.data, b2.ctypes.data, ctypes.byref(h))
        return rc, (lambda: vk._lib.veckm_trainer_destroy(h))

    assert _sweep(vk, build) >= 8


def test_server_stream_and_first_batch(vk, fault_env):
    W1, b1, W2, b2 = synth.init_mlp(64, 128)
    spec = synth.SliceSpec(346, 260, 8, 5000, 4, seed=4711)
    ev, t0, T = synth.make_slice(spec)

    def build():
        p = _params(vk, precision="fp16")
        p.max_events = 50_000
        h = ctypes.c_void_p()
        rc = vk._lib.veckm_server_create(ctypes.byref(p), 1 << 34, 4, 2, ctypes.byref(h))
        if rc:
            return rc, None
        done = lambda: vk.veckm_server_destroy(h)  # noqa: E731
        rc = vk.veckm_server_set_mlp(h, 128, W1, b1, W2, b2)
        if rc:
            done()
            return rc, None
        sid = ctypes.c_int32(-1)
        rc = vk._lib.veckm_stream_open(h, 346, 260, 50, 50_000, ctypes.byref(sid))
        if rc:
            done()
            return rc, None
        # the first batch takes pinned memory for its error word: a failure
        # there reaches the slice through its poll
        tk = ctypes.c_uint64()
        rc = vk._lib.veckm_submit(h, sid.value, ev.ctypes.data, len(ev), t0, T, ctypes.byref(tk))
        if rc:
            done()
            return rc, None
        out = np.zeros((len(ev), 2), np.float32)
        rc = vk._lib.veckm_poll(h, tk.value, out.ctypes.data, 10_000_000)
        done()
        return rc, (lambda: None)

    assert _sweep(vk, build) >= 6


def test_device_still_correct_after_faults(vk, fault_env):
    os.environ["VECKM_FAULT_ALLOC"] = "3"
    h = ctypes.c_void_p()
    p = _params(vk)
    assert vk._lib.veckm_create(ctypes.byref(p), ctypes.byref(h)) == vk.VECKM_E_NOMEM
    os.environ.pop("VECKM_FAULT_ALLOC")
    spec = synth.SliceSpec(96, 64, 12, 6000, 6, seed=4242)
    ev, t0, T = synth.make_slice(spec)
    A = synth.draw_frequencies(64, 3, 3, 2)
    mlp = synth.init_mlp(64, 128)
    ctx = vk.Context(96, 64, 3, 3, 2, A, T, len(ev), "fp32")
    ctx.set_mlp(*mlp)
    flow = ctx.flow(torch.from_numpy(ev).cuda(), t0, T)
    torch.cuda.synchronize()
    assert ctx.status() == vk.VECKM_OK
    ctx.close()
    emb, _ = oracle.encode(ev, A, 3, 3, 2)
    ref = oracle.mlp(emb, *mlp)
    f = flow.cpu().numpy()
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) <= 1e-3
