"""Python binding of the veckm C-ABI (``include/veckm.h``).

Argument marshalling only: every function below forwards to the function of
the same name in ``_lib/libveckm.so``, and every step of the computation runs
in that library's HIP kernels.  Importing this module fails loudly when the
library has not been built (``python -m paper_2504_19417_amd.build``).

``Context`` is a convenience holder for a ``veckm_ctx*`` that takes torch
CUDA tensors, passes their device pointers and the current HIP stream, and
allocates outputs with torch.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VECKM_LIB names another build of the same library (the host-sanitizer
# build of the checks); by default the in-tree build.
LIB_PATH = os.environ.get("VECKM_LIB") or os.path.join(_HERE, "_lib", "libveckm.so")

VECKM_OK = 0
VECKM_E_INVAL = -1
VECKM_E_RANGE = -2
VECKM_E_NOMEM = -3
VECKM_E_BUDGET = -4
VECKM_E_AGAIN = -5
VECKM_E_HIP = -6
VECKM_E_NODEVICE = -7
VECKM_E_OVERFLOW = -8
VECKM_E_STATE = -9
VECKM_MAX_VOXEL_EVENTS = 1024
VECKM_NOALLOC_SCRATCH_BYTES = 64 << 20
VECKM_FP32 = 0
VECKM_FP16 = 1
VECKM_STAGE_PREPARE = 0
VECKM_STAGE_ENCODE = 1
VECKM_STAGE_MLP = 2
VECKM_STAGE_EXPAND = 3
VECKM_NUM_STAGES = 4
STAGE_NAMES = ("prepare", "encode", "mlp", "expand")

PRECISIONS = {"fp32": VECKM_FP32, "fp16": VECKM_FP16}


class veckm_params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("rx", ctypes.c_int32), ("ry", ctypes.c_int32), ("rt", ctypes.c_int32),
        ("d", ctypes.c_int32), ("max_bins", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("max_events", ctypes.c_int64),
        ("A", ctypes.POINTER(ctypes.c_double)),
        ("max_slices", ctypes.c_int32),
        ("max_voxels", ctypes.c_int64),
    ]


class veckm_slice(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("t0", ctypes.c_int32), ("nbins", ctypes.c_int32),
        ("offset", ctypes.c_int64), ("n", ctypes.c_int64),
    ]


class veckm_serving_stats(ctypes.Structure):
    _fields_ = [
        ("slices", ctypes.c_int64), ("flows", ctypes.c_int64), ("batches", ctypes.c_int64),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
        ("busy_s", ctypes.c_double),
    ]


class VeckmError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, veckm_strerror(code), code))


if not os.path.exists(LIB_PATH):
    raise ImportError("libveckm.so is not built (%s); run "
                      "`python -m paper_2504_19417_amd.build`" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_sig = {
    "veckm_params_check": (ctypes.c_int, [ctypes.POINTER(veckm_params)]),
    "veckm_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(veckm_params), ctypes.c_int32]),
    "veckm_offset_table": (ctypes.c_int, [ctypes.POINTER(veckm_params), ctypes.POINTER(ctypes.c_int32),
                                          _P, _P]),
    "veckm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "veckm_create": (ctypes.c_int, [ctypes.POINTER(veckm_params), ctypes.POINTER(_P)]),
    "veckm_destroy": (None, [_P]),
    "veckm_set_mlp": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "veckm_encode": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P,
                                    ctypes.c_int64, _P, _P]),
    "veckm_flow": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P,
                                  ctypes.c_int64, _P, _P]),
    "veckm_count": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P,
                                   ctypes.c_int64, _P, _P]),
    "veckm_flow_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, _P, _P]),
    "veckm_encode_batch": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P]),
    "veckm_flow_batch": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P]),
    "veckm_status": (ctypes.c_int, [_P, _P]),
    "veckm_graph_create": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                          ctypes.POINTER(_P)]),
    "veckm_graph_launch": (ctypes.c_int, [_P, _P]),
    "veckm_graph_destroy": (None, [_P]),
    "veckm_tiling_count": (ctypes.c_int, [_P]),
    "veckm_tiling_selected": (ctypes.c_int, [_P]),
    "veckm_tiling_info": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "veckm_tiling_select": (ctypes.c_int, [_P, ctypes.c_int32]),
    "veckm_tune": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P,
                                  ctypes.POINTER(ctypes.c_int32)]),
    "veckm_window_create": (ctypes.c_int, [ctypes.POINTER(veckm_params), ctypes.POINTER(_P)]),
    "veckm_window_push": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         _P]),
    "veckm_window_encode": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "veckm_window_flow": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
    "veckm_trainer_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P,
                                            _P, _P, ctypes.POINTER(_P)]),
    "veckm_trainer_destroy": (None, [_P]),
    "veckm_trainer_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_float, _P, _P]),
    "veckm_trainer_get": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "veckm_server_create": (ctypes.c_int, [ctypes.POINTER(veckm_params), ctypes.c_int64,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "veckm_server_destroy": (None, [_P]),
    "veckm_server_set_mlp": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "veckm_stream_open": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "veckm_stream_close": (ctypes.c_int, [_P, ctypes.c_int32]),
    "veckm_submit": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "veckm_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.c_int32]),
    "veckm_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(veckm_serving_stats), ctypes.c_int32]),
    "veckm_server_stats_sensor": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.POINTER(veckm_serving_stats)]),
    "veckm_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "veckm_profile_read": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "veckm_last_rows": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def make_params(width, height, rx, ry, rt, A, max_bins, max_events, precision="fp32",
                max_slices=0, max_voxels=0):
    """Build a veckm_params; the returned object keeps A alive."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    p = veckm_params()
    p.width, p.height, p.rx, p.ry, p.rt = int(width), int(height), int(rx), int(ry), int(rt)
    p.d = int(A.shape[0])
    p.max_bins = int(max_bins)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.max_events = int(max_events)
    p.A = A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.max_slices = int(max_slices)
    p.max_voxels = int(max_voxels)
    p._A_keepalive = A
    return p


def make_slices(specs):
    """A veckm_slice array from (width, height, t0, nbins, n) tuples, events
    back to back in the given order."""
    arr = (veckm_slice * len(specs))()
    off = 0
    for k, (w, h, t0, nbins, n) in enumerate(specs):
        arr[k].width, arr[k].height, arr[k].t0, arr[k].nbins = int(w), int(h), int(t0), int(nbins)
        arr[k].offset, arr[k].n = off, int(n)
        off += int(n)
    return arr


def veckm_params_check(params):
    return _lib.veckm_params_check(ctypes.byref(params))


def veckm_workspace_bytes(params, hidden=0):
    return _lib.veckm_workspace_bytes(ctypes.byref(params), int(hidden))


def veckm_offset_table(params, with_phases=True):
    """(offsets int32[K,3], phase_bits uint16[K,D,4] or None)."""
    k = ctypes.c_int32(0)
    rc = _lib.veckm_offset_table(ctypes.byref(params), ctypes.byref(k), None, None)
    if rc:
        raise VeckmError(rc, "veckm_offset_table")
    off = np.zeros((k.value, 3), dtype=np.int32)
    bits = np.zeros((k.value, params.d, 4), dtype=np.uint16) if with_phases else None
    rc = _lib.veckm_offset_table(ctypes.byref(params), ctypes.byref(k), off.ctypes.data,
                                 None if bits is None else bits.ctypes.data)
    if rc:
        raise VeckmError(rc, "veckm_offset_table")
    return off, bits


def veckm_strerror(code):
    return _lib.veckm_strerror(int(code)).decode()


def veckm_create(params):
    h = _P()
    rc = _lib.veckm_create(ctypes.byref(params), ctypes.byref(h))
    if rc:
        raise VeckmError(rc, "veckm_create")
    return h


def veckm_destroy(ctx):
    _lib.veckm_destroy(ctx)


def veckm_set_mlp(ctx, hidden, W1, b1, W2, b2):
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in (W1, b1, W2, b2)]
    rc = _lib.veckm_set_mlp(ctx, int(hidden), *[a.ctypes.data for a in arrs])
    if rc:
        raise VeckmError(rc, "veckm_set_mlp")


def veckm_encode(ctx, events_ptr, n, t0, nbins, queries_ptr, m, emb_ptr, stream):
    return _lib.veckm_encode(ctx, events_ptr, int(n), int(t0), int(nbins), queries_ptr, int(m),
                             emb_ptr, stream)


def veckm_flow(ctx, events_ptr, n, t0, nbins, queries_ptr, m, flow_ptr, stream):
    return _lib.veckm_flow(ctx, events_ptr, int(n), int(t0), int(nbins), queries_ptr, int(m),
                           flow_ptr, stream)


def veckm_count(ctx, events_ptr, n, t0, nbins, queries_ptr, m, counts_ptr, stream):
    return _lib.veckm_count(ctx, events_ptr, int(n), int(t0), int(nbins), queries_ptr, int(m),
                            counts_ptr, stream)


def veckm_flow_noalloc(ctx, events_ptr, n, t0, nbins, flow_ptr, stream):
    return _lib.veckm_flow_noalloc(ctx, events_ptr, int(n), int(t0), int(nbins), flow_ptr, stream)


def veckm_encode_batch(ctx, slices, count, events_ptr, emb_ptr, stream):
    return _lib.veckm_encode_batch(ctx, ctypes.cast(slices, _P), int(count), events_ptr, emb_ptr,
                                   stream)


def veckm_flow_batch(ctx, slices, count, events_ptr, flow_ptr, stream):
    return _lib.veckm_flow_batch(ctx, ctypes.cast(slices, _P), int(count), events_ptr, flow_ptr,
                                 stream)


def veckm_status(ctx, stream):
    return _lib.veckm_status(ctx, stream)


def veckm_window_create(params):
    h = _P()
    rc = _lib.veckm_window_create(ctypes.byref(params), ctypes.byref(h))
    if rc:
        raise VeckmError(rc, "veckm_window_create")
    return h


def veckm_window_push(ctx, events_ptr, n, t0, nbins, stream):
    return _lib.veckm_window_push(ctx, events_ptr, int(n), int(t0), int(nbins), stream)


def veckm_window_encode(ctx, queries_ptr, m, emb_ptr, stream):
    return _lib.veckm_window_encode(ctx, queries_ptr, int(m), emb_ptr, stream)


def veckm_window_flow(ctx, queries_ptr, m, flow_ptr, stream):
    return _lib.veckm_window_flow(ctx, queries_ptr, int(m), flow_ptr, stream)


def veckm_profile_enable(ctx, enable):
    rc = _lib.veckm_profile_enable(ctx, int(enable))
    if rc:
        raise VeckmError(rc, "veckm_profile_enable")


def veckm_profile_read(ctx):
    """{stage name: (milliseconds, launches)} since the last read."""
    ms = np.zeros(VECKM_NUM_STAGES, dtype=np.float64)
    cnt = np.zeros(VECKM_NUM_STAGES, dtype=np.int64)
    rc = _lib.veckm_profile_read(ctx, ms.ctypes.data, cnt.ctypes.data, VECKM_NUM_STAGES)
    if rc:
        raise VeckmError(rc, "veckm_profile_read")
    return {STAGE_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(VECKM_NUM_STAGES)}


def veckm_last_rows(ctx, stream):
    r = ctypes.c_int64(0)
    rc = _lib.veckm_last_rows(ctx, stream, ctypes.byref(r))
    if rc:
        raise VeckmError(rc, "veckm_last_rows")
    return r.value


class Context:
    """A veckm context driven with torch CUDA tensors."""

    def __init__(self, width, height, rx, ry, rt, A, max_bins, max_events, precision="fp32",
                 max_slices=0, max_voxels=0):
        self.params = make_params(width, height, rx, ry, rt, A, max_bins, max_events, precision,
                                  max_slices, max_voxels)
        self.d = self.params.d
        self.handle = veckm_create(self.params)
        self.hidden = 0

    def close(self):
        if self.handle:
            veckm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mlp(self, W1, b1, W2, b2):
        hidden = np.asarray(W1).shape[0]
        veckm_set_mlp(self.handle, hidden, W1, b1, W2, b2)
        self.hidden = hidden

    @staticmethod
    def _stream(stream):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        return ctypes.c_void_p(s.cuda_stream)

    def _check_inputs(self, events, queries):
        import torch
        if not (events.is_cuda and events.dtype == torch.int32 and events.dim() == 2
                and events.shape[1] == 4 and events.is_contiguous()):
            raise ValueError("events must be a contiguous int32 CUDA tensor [n, 4]")
        if queries is not None and not (queries.is_cuda and queries.dtype == torch.int32
                                        and queries.dim() == 1 and queries.is_contiguous()):
            raise ValueError("queries must be a contiguous int32 CUDA tensor [m]")

    def encode(self, events, t0, nbins, queries=None, out=None, stream=None):
        import torch
        self._check_inputs(events, queries)
        n = events.shape[0]
        m = n if queries is None else queries.shape[0]
        if out is None:
            out = torch.empty((m, 2 * self.d), dtype=torch.float32, device=events.device)
        rc = veckm_encode(self.handle, events.data_ptr(), n, t0, nbins,
                          None if queries is None else queries.data_ptr(), m,
                          out.data_ptr(), self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_encode")
        return out

    def flow(self, events, t0, nbins, queries=None, out=None, stream=None):
        import torch
        self._check_inputs(events, queries)
        n = events.shape[0]
        m = n if queries is None else queries.shape[0]
        if out is None:
            out = torch.empty((m, 2), dtype=torch.float32, device=events.device)
        rc = veckm_flow(self.handle, events.data_ptr(), n, t0, nbins,
                        None if queries is None else queries.data_ptr(), m,
                        out.data_ptr(), self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_flow")
        return out

    def count(self, events, t0, nbins, queries=None, out=None, stream=None):
        """Windowed neighbour count (int32) of each queried event."""
        import torch
        self._check_inputs(events, queries)
        n = events.shape[0]
        m = n if queries is None else queries.shape[0]
        if out is None:
            out = torch.empty((m,), dtype=torch.int32, device=events.device)
        rc = veckm_count(self.handle, events.data_ptr(), n, t0, nbins,
                         None if queries is None else queries.data_ptr(), m,
                         out.data_ptr(), self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_count")
        return out

    def _batch(self, fn, name, width, slices, events, out, stream):
        import torch
        self._check_inputs(events, None)
        arr = make_slices(slices)
        n = sum(int(s[4]) for s in slices)
        if n != events.shape[0]:
            raise ValueError("slice sizes add up to %d events, got %d" % (n, events.shape[0]))
        if out is None:
            out = torch.empty((n, width), dtype=torch.float32, device=events.device)
        rc = fn(self.handle, arr, len(slices), events.data_ptr(), out.data_ptr(),
                self._stream(stream))
        if rc:
            raise VeckmError(rc, name)
        return out

    def encode_batch(self, slices, events, out=None, stream=None):
        """slices: (width, height, t0, nbins, n) per slice, events back to back."""
        return self._batch(veckm_encode_batch, "veckm_encode_batch", 2 * self.d, slices, events,
                           out, stream)

    def flow_batch(self, slices, events, out=None, stream=None):
        return self._batch(veckm_flow_batch, "veckm_flow_batch", 2, slices, events, out, stream)

    def status(self, stream=None):
        return veckm_status(self.handle, self._stream(stream))

    def tilings(self):
        """[(bx, by, bt, slabs, layout)] of the encoder tilings this context offers."""
        n = _lib.veckm_tiling_count(self.handle)
        out = []
        for i in range(n):
            info = (ctypes.c_int32 * 5)()
            rc = _lib.veckm_tiling_info(self.handle, i, ctypes.cast(info, _P))
            if rc:
                raise VeckmError(rc, "veckm_tiling_info")
            out.append(tuple(int(v) for v in info))
        return out

    def tiling(self):
        return _lib.veckm_tiling_selected(self.handle)

    def select_tiling(self, index):
        rc = _lib.veckm_tiling_select(self.handle, int(index))
        if rc:
            raise VeckmError(rc, "veckm_tiling_select")

    def tune(self, slices, events, reps=3, stream=None):
        """Times every tiling on this batch and keeps the fastest; returns its index."""
        self._check_inputs(events, None)
        arr = make_slices(slices)
        chosen = ctypes.c_int32(-1)
        rc = _lib.veckm_tune(self.handle, ctypes.cast(arr, _P), len(slices), events.data_ptr(),
                             int(reps), self._stream(stream), ctypes.byref(chosen))
        if rc:
            raise VeckmError(rc, "veckm_tune")
        return chosen.value

    def graph(self, slices, events, out, flow=True):
        """A launch graph of flow_batch (flow=True) or encode_batch over
        exactly these slices, event tensor and output tensor."""
        self._check_inputs(events, None)
        n = sum(int(s[4]) for s in slices)
        width = 2 if flow else 2 * self.d
        import torch
        if n != events.shape[0] or tuple(out.shape) != (n, width) or not out.is_contiguous() \
                or not out.is_cuda or out.dtype != torch.float32:
            raise ValueError("events / out (contiguous float32 CUDA) do not match the slices")
        arr = make_slices(slices)
        h = _P()
        rc = _lib.veckm_graph_create(self.handle, ctypes.cast(arr, _P), len(slices),
                                     events.data_ptr(), out.data_ptr(), 1 if flow else 0,
                                     ctypes.byref(h))
        if rc:
            raise VeckmError(rc, "veckm_graph_create")
        return Graph(h, self, events, out)

    def profile(self, enable=True):
        veckm_profile_enable(self.handle, enable)

    def profile_read(self):
        return veckm_profile_read(self.handle)

    def last_rows(self, stream=None):
        return veckm_last_rows(self.handle, self._stream(stream))


# ---------------------------------------------------------------- serving


def veckm_server_create(params, hbm_budget_bytes, max_streams, depth):
    h = _P()
    rc = _lib.veckm_server_create(ctypes.byref(params), int(hbm_budget_bytes), int(max_streams),
                                  int(depth), ctypes.byref(h))
    if rc:
        raise VeckmError(rc, "veckm_server_create")
    return h


def veckm_server_destroy(server):
    _lib.veckm_server_destroy(server)


def veckm_server_set_mlp(server, hidden, W1, b1, W2, b2):
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in (W1, b1, W2, b2)]
    return _lib.veckm_server_set_mlp(server, int(hidden), *[a.ctypes.data for a in arrs])


def veckm_stream_open(server, width, height, max_bins, max_events):
    """(code, sid)."""
    sid = ctypes.c_int32(-1)
    rc = _lib.veckm_stream_open(server, int(width), int(height), int(max_bins), int(max_events),
                                ctypes.byref(sid))
    return rc, sid.value


def veckm_stream_close(server, sid):
    return _lib.veckm_stream_close(server, int(sid))


def veckm_submit(server, sid, events, t0, nbins):
    """events: host int32 [n, 4] (C-contiguous).  (code, ticket)."""
    ev = np.ascontiguousarray(events, dtype=np.int32)
    if ev.ndim != 2 or ev.shape[1] != 4:
        raise ValueError("events must be int32 [n, 4]")
    t = ctypes.c_uint64(0)
    rc = _lib.veckm_submit(server, int(sid), ev.ctypes.data if len(ev) else None, len(ev),
                           int(t0), int(nbins), ctypes.byref(t))
    return rc, t.value


def veckm_poll(server, ticket, flows, timeout_us):
    """flows: host float32 [n, 2] array to fill, or None."""
    ptr = None
    if flows is not None:
        if not (flows.dtype == np.float32 and flows.flags["C_CONTIGUOUS"]):
            raise ValueError("flows must be a C-contiguous float32 array")
        ptr = flows.ctypes.data
    return _lib.veckm_poll(server, ctypes.c_uint64(ticket), ptr, int(timeout_us))


def veckm_server_stats(server, reset=False):
    st = veckm_serving_stats()
    rc = _lib.veckm_server_stats(server, ctypes.byref(st), int(bool(reset)))
    if rc:
        raise VeckmError(rc, "veckm_server_stats")
    return {f: getattr(st, f) for f, _ in veckm_serving_stats._fields_}


def veckm_server_stats_sensor(server, width, height):
    st = veckm_serving_stats()
    rc = _lib.veckm_server_stats_sensor(server, int(width), int(height), ctypes.byref(st))
    if rc:
        raise VeckmError(rc, "veckm_server_stats_sensor")
    return {f: getattr(st, f) for f, _ in veckm_serving_stats._fields_}


class Graph:
    """A captured batch launch (holds its context, event and output tensors)."""

    def __init__(self, handle, ctx, events, out):
        self.handle, self.ctx, self.events, self.out = handle, ctx, events, out

    def launch(self, stream=None):
        rc = _lib.veckm_graph_launch(self.handle, self.ctx._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_graph_launch")
        return self.out

    def close(self):
        if self.handle:
            _lib.veckm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Window(Context):
    """A sliding-window (streaming) encoder: push the events of new time bins,
    encode query events against the resident window."""

    def __init__(self, width, height, rx, ry, rt, A, window_bins, max_events, precision="fp32"):
        self.params = make_params(width, height, rx, ry, rt, A, window_bins, max_events, precision)
        self.d = self.params.d
        self.handle = veckm_window_create(self.params)
        self.hidden = 0

    def push(self, events, t0, nbins, stream=None):
        self._check_inputs(events, None)
        rc = veckm_window_push(self.handle, events.data_ptr(), events.shape[0], t0, nbins,
                               self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_window_push")

    def encode_window(self, queries, out=None, stream=None):
        import torch
        self._check_inputs(queries, None)
        m = queries.shape[0]
        if out is None:
            out = torch.empty((m, 2 * self.d), dtype=torch.float32, device=queries.device)
        rc = veckm_window_encode(self.handle, queries.data_ptr(), m, out.data_ptr(),
                                 self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_window_encode")
        return out

    def flow_window(self, queries, out=None, stream=None):
        import torch
        self._check_inputs(queries, None)
        m = queries.shape[0]
        if out is None:
            out = torch.empty((m, 2), dtype=torch.float32, device=queries.device)
        rc = veckm_window_flow(self.handle, queries.data_ptr(), m, out.data_ptr(),
                               self._stream(stream))
        if rc:
            raise VeckmError(rc, "veckm_window_flow")
        return out


class Trainer:
    """Trains the perceptron on device encodings with target flows (torch
    CUDA tensors); weights come and go as numpy float32 arrays."""

    def __init__(self, d, hidden, max_rows, W1, b1, W2, b2):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in (W1, b1, W2, b2)]
        if arrs[0].shape != (hidden, 2 * d) or arrs[1].shape != (hidden,) or \
                arrs[2].shape != (2, hidden) or arrs[3].shape != (2,):
            raise ValueError("perceptron shapes do not match")
        h = _P()
        rc = _lib.veckm_trainer_create(int(d), int(hidden), int(max_rows),
                                       *[a.ctypes.data for a in arrs], ctypes.byref(h))
        if rc:
            raise VeckmError(rc, "veckm_trainer_create")
        self.handle, self.d, self.hidden = h, d, hidden

    def close(self):
        if self.handle:
            _lib.veckm_trainer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, emb, target, optimizer="adam", lr=1e-3, loss=None, stream=None):
        import torch
        for t, w in ((emb, 2 * self.d), (target, 2)):
            if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[1] == w
                    and t.is_contiguous()):
                raise ValueError("emb [m, 2d] and target [m, 2] must be contiguous float32 CUDA")
        s = torch.cuda.current_stream() if stream is None else stream
        rc = _lib.veckm_trainer_step(self.handle, emb.data_ptr(), target.data_ptr(),
                                     int(emb.shape[0]), 0 if optimizer == "sgd" else 1,
                                     float(lr), None if loss is None else loss.data_ptr(),
                                     ctypes.c_void_p(s.cuda_stream))
        if rc:
            raise VeckmError(rc, "veckm_trainer_step")

    def weights(self):
        W1 = np.zeros((self.hidden, 2 * self.d), np.float32)
        b1 = np.zeros(self.hidden, np.float32)
        W2 = np.zeros((2, self.hidden), np.float32)
        b2 = np.zeros(2, np.float32)
        rc = _lib.veckm_trainer_get(self.handle, W1.ctypes.data, b1.ctypes.data, W2.ctypes.data,
                                    b2.ctypes.data)
        if rc:
            raise VeckmError(rc, "veckm_trainer_get")
        return W1, b1, W2, b2


class Server:
    """A veckm server driven with numpy host arrays."""

    def __init__(self, width, height, rx, ry, rt, A, max_bins, max_events, precision="fp16",
                 hbm_budget_bytes=64 << 30, max_streams=32, depth=4, max_voxels=0):
        self.params = make_params(width, height, rx, ry, rt, A, max_bins, max_events, precision,
                                  max_streams, max_voxels)
        self.handle = veckm_server_create(self.params, hbm_budget_bytes, max_streams, depth)
        self.sizes = {}

    def close(self):
        if self.handle:
            veckm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mlp(self, W1, b1, W2, b2):
        rc = veckm_server_set_mlp(self.handle, np.asarray(W1).shape[0], W1, b1, W2, b2)
        if rc:
            raise VeckmError(rc, "veckm_server_set_mlp")

    def open_stream(self, width, height, max_bins, max_events):
        rc, sid = veckm_stream_open(self.handle, width, height, max_bins, max_events)
        if rc:
            raise VeckmError(rc, "veckm_stream_open")
        return sid

    def close_stream(self, sid):
        rc = veckm_stream_close(self.handle, sid)
        if rc:
            raise VeckmError(rc, "veckm_stream_close")

    def submit(self, sid, events, t0, nbins):
        rc, ticket = veckm_submit(self.handle, sid, events, t0, nbins)
        if rc:
            raise VeckmError(rc, "veckm_submit")
        self.sizes[ticket] = len(events)
        return ticket

    def poll(self, ticket, timeout_us=-1):
        """(code, flows or None): code VECKM_E_AGAIN while the slice runs."""
        n = self.sizes.get(ticket)
        if n is None:
            return VECKM_E_INVAL, None
        out = np.empty((n, 2), dtype=np.float32)
        rc = veckm_poll(self.handle, ticket, out, timeout_us)
        if rc == VECKM_E_AGAIN:
            return rc, None
        del self.sizes[ticket]
        return rc, (out if rc == VECKM_OK else None)

    def stats(self, reset=False):
        return veckm_server_stats(self.handle, reset)

    def stats_sensor(self, width, height):
        return veckm_server_stats_sensor(self.handle, width, height)
