"""Host-side checks of the C-ABI library: it loads, exports every function
the header declares, validates parameters, and builds the offset-phase table
(FP64 on the host, rounded for the matrix cores) correctly.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2504_19417_amd import synth, veckm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "veckm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int64_t|int|void)\s+(veckm_\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_api():
    names = _declared_functions()
    for required in ["veckm_create", "veckm_destroy", "veckm_encode", "veckm_flow",
                     "veckm_set_mlp", "veckm_status", "veckm_strerror", "veckm_encode_batch",
                     "veckm_flow_batch", "veckm_server_create", "veckm_server_destroy",
                     "veckm_server_set_mlp", "veckm_stream_open", "veckm_stream_close",
                     "veckm_submit", "veckm_poll", "veckm_server_stats", "veckm_window_create",
                     "veckm_window_push", "veckm_window_encode", "veckm_window_flow",
                     "veckm_trainer_create", "veckm_trainer_step", "veckm_trainer_get",
                     "veckm_trainer_destroy", "veckm_graph_create", "veckm_graph_launch",
                     "veckm_graph_destroy", "veckm_tiling_count", "veckm_tiling_selected",
                     "veckm_tiling_info", "veckm_tiling_select", "veckm_tune"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(veckm.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _params(**kw):
    A = synth.draw_frequencies(kw.pop("d", 64), 3, 3, 2)
    args = dict(width=346, height=260, rx=3, ry=3, rt=2, A=A, max_bins=25, max_events=20000)
    args.update(kw)
    return veckm.make_params(**args)


def test_params_check():
    assert veckm.veckm_params_check(_params()) == veckm.VECKM_OK
    for d in (16, 32, 48, 64, 128, 256):
        assert veckm.veckm_params_check(_params(d=d)) == veckm.VECKM_OK
    # rt = -1 is the paper's unbounded window (up to 1024 bins per slice)
    assert veckm.veckm_params_check(_params(rt=-1)) == veckm.VECKM_OK
    assert veckm.veckm_params_check(_params(rt=-1, max_bins=1024)) == veckm.VECKM_OK
    bad = [dict(width=0), dict(height=-1), dict(rx=-1), dict(ry=13), dict(rt=7), dict(rt=-2),
           dict(rt=-1, max_bins=1025), dict(max_bins=0), dict(max_events=0),
           dict(max_events=1 << 40), dict(precision=5)]
    for b in bad:
        assert veckm.veckm_params_check(_params(**b)) == veckm.VECKM_E_INVAL, b
    for d in (8, 40, 96, 512):
        assert veckm.veckm_params_check(_params(d=d)) == veckm.VECKM_E_INVAL, d
    p = _params()
    p.A = ctypes.POINTER(ctypes.c_double)()
    assert veckm.veckm_params_check(p) == veckm.VECKM_E_INVAL
    A = synth.draw_frequencies(64, 3, 3, 2)
    A[5, 1] = np.nan
    assert veckm.veckm_params_check(_params(A=A)) == veckm.VECKM_E_INVAL


def test_strerror_covers_codes():
    for c in range(0, -10, -1):
        assert veckm.veckm_strerror(c) != "unknown error"
    assert veckm.veckm_strerror(-99) == "unknown error"


@pytest.mark.parametrize("r", [(0, 0, 0), (3, 3, 2), (5, 5, 3), (2, 4, 1), (12, 12, 6)])
def test_half_window_offsets(r):
    rx, ry, rt = r
    p = _params(rx=rx, ry=ry, rt=rt)
    off, _ = veckm.veckm_offset_table(p, with_phases=False)
    full = (2 * rx + 1) * (2 * ry + 1) * (2 * rt + 1)
    assert off.shape == ((full + 1) // 2, 3)
    assert tuple(off[0]) == (0, 0, 0)
    pos = [tuple(o) for o in off[1:]]
    assert len(set(pos)) == len(pos)
    # every entry is lexicographically positive in (dt, dy, dx) and inside the window
    for dx, dy, dt in pos:
        assert (dt, dy, dx) > (0, 0, 0)
        assert abs(dx) <= rx and abs(dy) <= ry and abs(dt) <= rt
    # centre + half + mirrored half = the whole window, exactly once
    allo = {(0, 0, 0)} | set(pos) | {(-a, -b, -c) for a, b, c in pos}
    assert len(allo) == full


def _f16(bits):
    return bits.view(np.float16).astype(np.float64)


@pytest.mark.parametrize("d,r", [(64, (3, 3, 2)), (128, (5, 5, 3))])
def test_phase_table_fp64_build(d, r):
    """hi = fp16(cos theta) exactly (numpy's round-to-nearest-even), hi + lo
    carries theta to ~2^-22, the centre is cos = 1/2, sin = 0."""
    rx, ry, rt = r
    A = synth.draw_frequencies(d, rx, ry, rt)
    p = _params(rx=rx, ry=ry, rt=rt, A=A, d=d)
    off, bits = veckm.veckm_offset_table(p)
    th = off[1:].astype(np.float64) @ A.T                      # [K-1, D]
    c, s = np.cos(th), np.sin(th)
    assert np.array_equal(bits[1:, :, 0], c.astype(np.float16).view(np.uint16))
    assert np.array_equal(bits[1:, :, 2], s.astype(np.float16).view(np.uint16))
    lo_c = (c - _f16(bits[1:, :, 0])).astype(np.float16)
    assert np.array_equal(bits[1:, :, 1], lo_c.view(np.uint16))
    err_c = np.abs(_f16(bits[1:, :, 0]) + _f16(bits[1:, :, 1]) - c)
    err_s = np.abs(_f16(bits[1:, :, 2]) + _f16(bits[1:, :, 3]) - s)
    assert err_c.max() < 2 ** -22 and err_s.max() < 2 ** -22
    assert np.all(_f16(bits[0, :, 0]) == 0.5) and np.all(_f16(bits[0, :, 1]) == 0.0)
    assert np.all(_f16(bits[0, :, 2]) == 0.0) and np.all(_f16(bits[0, :, 3]) == 0.0)


def test_workspace_bytes():
    p = _params()
    b0 = veckm.veckm_workspace_bytes(p, 0)
    b1 = veckm.veckm_workspace_bytes(p, 128)
    assert b0 > 346 * 260 * 25 * 9 and b1 > b0
    big = veckm.veckm_workspace_bytes(_params(max_events=1_000_000), 0)
    assert big > b0
    assert veckm.veckm_workspace_bytes(_params(d=8), 0) == veckm.VECKM_E_INVAL
    # the paper form holds two D-wide complex fp32 pixel grids (G, S)
    bp = veckm.veckm_workspace_bytes(_params(rt=-1), 0)
    assert bp > 2 * 2 * 64 * 346 * 260 * 4


def test_paper_form_has_no_offset_table_and_no_server():
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_offset_table(_params(rt=-1), with_phases=False)
    assert e.value.code == veckm.VECKM_E_INVAL
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_server_create(_params(rt=-1), 1 << 40, 4, 2)
    assert e.value.code == veckm.VECKM_E_INVAL


def test_create_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the GPU tests")
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_create(_params())
    assert e.value.code == veckm.VECKM_E_NODEVICE


def test_create_rejects_bad_params_before_device():
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_create(_params(rx=99))
    assert e.value.code == veckm.VECKM_E_INVAL


def test_server_create_checks_before_device():
    """Argument and HBM-budget checks happen on the host, before any device
    call; without a device the server reports VECKM_E_NODEVICE."""
    p = _params()
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_server_create(p, 1 << 20, 4, 2)  # 1 MiB cannot hold the workspaces
    assert e.value.code == veckm.VECKM_E_BUDGET
    for streams, depth, budget in ((0, 2, 1 << 40), (4, 0, 1 << 40), (4, 17, 1 << 40), (4, 2, 0)):
        with pytest.raises(veckm.VeckmError) as e:
            veckm.veckm_server_create(p, budget, streams, depth)
        assert e.value.code == veckm.VECKM_E_INVAL
    import torch
    if torch.cuda.is_available():
        return
    with pytest.raises(veckm.VeckmError) as e:
        veckm.veckm_server_create(p, 1 << 40, 4, 2)
    assert e.value.code == veckm.VECKM_E_NODEVICE


def test_window_checks_before_device():
    for bad in (dict(rt=-1), dict(max_slices=2)):
        with pytest.raises(veckm.VeckmError) as e:
            veckm.veckm_window_create(_params(**bad))
        assert e.value.code == veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_window_push(None, None, 0, 0, 1, None) == veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_window_encode(None, None, 0, None, None) == veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_window_flow(None, None, 0, None, None) == veckm.VECKM_E_INVAL


def test_trainer_argument_checks():
    z = np.zeros(1, np.float32).ctypes.data
    h = ctypes.c_void_p()
    for d, hidden, rows in ((0, 64, 10), (64, 32, 10), (64, 96, 10), (64, 576, 10), (64, 64, 0)):
        assert veckm._lib.veckm_trainer_create(d, hidden, rows, z, z, z, z, ctypes.byref(h)) == \
            veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_trainer_step(None, None, None, 1, 0, 0.1, None, None) == \
        veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_trainer_get(None, None, None, None, None) == veckm.VECKM_E_INVAL
    veckm._lib.veckm_trainer_destroy(None)


def test_server_null_handles():
    assert veckm._lib.veckm_stream_close(None, 0) == veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_poll(None, 1, None, 0) == veckm.VECKM_E_INVAL
    assert veckm._lib.veckm_server_set_mlp(None, 64, None, None, None, None) == veckm.VECKM_E_INVAL
    veckm._lib.veckm_server_destroy(None)
