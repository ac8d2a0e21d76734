"""GPU parity over the corners of the parameter space the library accepts.

Every shape here is accepted by veckm_params_check and runs a code path the
main workloads do not: the smallest and largest D (one frequency tile per
wave; four waves across frequencies), the degenerate window (the centre
only), the largest radii, asymmetric radii, and every perceptron form the
FP32 and FP16 paths choose by shape (register-resident fp16 hi/lo and bf16
kernels, the fp32 matrix-core kernel for W1 too large for registers, the
generic fp32 and bf16 kernels).  Every row is compared with the FP64 oracle
(encodings, flows) and the windowed count is compared bit for bit.
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


# name: (W, H, nbins, n, edges, D, rx, ry, rt, hidden, precision)
#   perceptron kernel chosen (FP32 form: fp16 hi/lo rows when W1 fits in
#   registers, else fp32 rows; FP16 form: bf16 rows)
SHAPES = {
    "d16_r12_6_fp32": (64, 48, 16, 3000, 6, 16, 12, 12, 6, 64, "fp32"),     # fp32 generic, K2 = 32
    "d16_r12_6_fp16": (64, 48, 16, 3000, 6, 16, 12, 12, 6, 64, "fp16"),     # bf16 generic
    "d48_r0_fp32": (40, 30, 8, 2500, 4, 48, 0, 0, 0, 128, "fp32"),          # centre only; K2 = 96
    "d64_r12_6_fp32": (80, 60, 20, 6000, 8, 64, 12, 12, 6, 128, "fp32"),    # hi/lo, K2 = 128
    "d64_r12_6_fp16": (80, 60, 20, 6000, 8, 64, 12, 12, 6, 128, "fp16"),    # bf16 resident
    "d64_h448_fp32": (60, 50, 10, 4000, 6, 64, 3, 3, 2, 448, "fp32"),       # fp32 MFMA, K2 = 128
    "d64_h512_fp32": (60, 50, 10, 4000, 6, 64, 3, 3, 2, 512, "fp32"),       # fp32 MFMA, 8 tiles
    "d128_h320_fp32": (70, 50, 12, 5000, 6, 128, 5, 5, 3, 320, "fp32"),     # fp32 MFMA, K2 = 256
    "d128_h512_fp16": (70, 50, 12, 5000, 6, 128, 5, 5, 3, 512, "fp16"),     # bf16 generic, K2 = 256
    "d128_r12_6_fp32": (70, 50, 16, 5000, 6, 128, 12, 12, 6, 256, "fp32"),  # two frequency waves
    "d256_fp32": (60, 40, 12, 3000, 6, 256, 5, 5, 3, 256, "fp32"),          # 4 frequency waves; K2 = 512
    "d256_fp16": (60, 40, 12, 3000, 6, 256, 5, 5, 3, 512, "fp16"),          # bf16 generic, K2 = 512
    "d256_r8_4_fp32": (60, 40, 12, 3000, 6, 256, 8, 8, 4, 64, "fp32"),      # largest D=256 window
    "d32_asym_fp32": (50, 40, 12, 4000, 6, 32, 7, 2, 4, 192, "fp32"),       # hi/lo, K2 = 64
    "d32_asym_fp16": (50, 40, 12, 4000, 6, 32, 2, 7, 1, 192, "fp16"),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_shape_every_row(vk, name):
    W, H, T, n, edges, d, rx, ry, rt, hidden, prec = SHAPES[name]
    _say("case: shape %s" % name)
    spec = synth.SliceSpec(W, H, T, n, edges, seed=900 + sum(map(ord, name)))
    ev, t0, nb = synth.make_slice(spec)
    A = synth.draw_frequencies(d, rx, ry, rt)
    mlp = synth.init_mlp(d, hidden)
    ref, cnt = oracle.encode(ev, A, rx, ry, rt)
    rflow = oracle.mlp(ref, *mlp)
    c = vk.Context(W, H, rx, ry, rt, A, nb, len(ev), prec)
    c.set_mlp(*mlp)
    evt = torch.from_numpy(ev).cuda()
    emb = c.encode(evt, t0, nb).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    flow = c.flow(evt, t0, nb).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    got_cnt = c.count(evt, t0, nb).cpu().numpy()
    assert c.status() == vk.VECKM_OK
    c.close()
    np.testing.assert_array_equal(got_cnt, cnt)
    kp = parity.padded_slots(rx, ry, rt)
    parity.check(emb, ref, prec, "emb", kp=kp, say=_say)
    parity.check(flow, rflow, prec, "flow", say=_say)
    if rx == ry == rt == 0:  # the centre only: every event sees its own voxel
        assert np.all(emb[:, :d] == 1.0) and np.all(emb[:, d:] == 0.0)


def test_rejected_shapes_fail_cleanly(vk):
    """Shapes whose encoder box does not fit in LDS beside two table slabs
    are refused at creation, before any launch."""
    A = np.zeros((256, 3))
    for r in ((12, 12, 6), (10, 10, 6)):
        p = vk.make_params(346, 260, *r, A, 50, 1000, "fp32")
        assert vk.veckm_params_check(p) == vk.VECKM_E_INVAL
        with pytest.raises(vk.VeckmError) as e:
            vk.Context(346, 260, *r, A, 50, 1000, "fp32")
        assert e.value.code == vk.VECKM_E_INVAL
