"""The allocation-free flow entry point against veckm_flow, through the C-ABI.

veckm_flow_noalloc runs the same kernels as veckm_flow with every per-call
workspace in the library's static device array, so its flows must equal
veckm_flow's bit for bit (and therefore meet the oracle tolerance veckm_flow
meets).  Two calls in a row, the second on a smaller slice, check that the
array's leftovers from a larger call do not leak into a smaller one."""
import ctypes
import sys

import numpy as np
import pytest

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


def _noalloc(vk, ctx, evt, t0, nbins):
    out = torch.full((evt.shape[0], 2), float("nan"), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = vk.veckm_flow_noalloc(ctx.handle, evt.data_ptr(), evt.shape[0], t0, nbins,
                               out.data_ptr(), s)
    assert rc == vk.VECKM_OK, vk.veckm_strerror(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_noalloc_matches_flow_two_calls(vk, precision):
    w = synth.workloads()["tiny"]
    spec = w.slices[0]
    ev, t0, T = synth.make_slice(spec)
    small = synth.SliceSpec(spec.width, spec.height, 10, 5000, 8, seed=4321)
    ev2, t02, T2 = synth.make_slice(small)
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    ctx = vk.Context(spec.width, spec.height, w.rx, w.ry, w.rt, A, T, len(ev), precision)
    ctx.set_mlp(*mlp)
    for e, t, nb in ((ev, t0, T), (ev2, t02, T2)):
        _say("case: noalloc %s n=%d nbins=%d" % (precision, len(e), nb))
        evt = torch.from_numpy(e).cuda()
        got = _noalloc(vk, ctx, evt, t, nb)
        assert ctx.status() == vk.VECKM_OK
        ref = ctx.flow(evt, t, nb).cpu().numpy()
        assert ctx.status() == vk.VECKM_OK
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)
    # a slice whose workspaces exceed the array is refused, nothing launched
    big = vk.Context(1280, 720, w.rx, w.ry, w.rt, A, 100, 64, precision)
    big.set_mlp(*mlp)
    evt = torch.from_numpy(ev[:64].copy()).cuda()
    out = torch.zeros((64, 2), dtype=torch.float32, device="cuda")
    rc = vk.veckm_flow_noalloc(big.handle, evt.data_ptr(), 64, t0, 100, out.data_ptr(),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == vk.VECKM_E_BUDGET
    big.close()
    ctx.close()
