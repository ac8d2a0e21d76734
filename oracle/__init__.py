"""CPU oracle for the normal-flow estimator (FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

Contents
  * ``encode`` / ``mlp`` -- ctypes front end of ``veckm_oracle.c``: the plain
    quadratic adjacency-row encoding (Eqn. 10 over the neighbourhood of
    Eqn. 1, normalised by the count of Eqn. 17) and the two-layer perceptron
    (Eqns. 5-6), in FP64.
  * ``alg1_paper_form`` -- the staged 2-D form of Sec. 2.2.2 (Eqns.
    14-17): a per-pixel grid of summed temporal phases and event counts,
    pooled over the spatial window with the spatial offset phases, then
    turned back by the conjugate temporal phase of the query and divided by
    the count.  No temporal bound, as in Eqn. 1.
  * ``pooling_form_3d`` -- the same pooling idea generalised to a temporal
    radius: a 3-D (x, y, t) count grid pooled with (dx, dy, dt) offset
    phases.
  * ``box_count`` -- the windowed neighbour count of Eqn. 17 alone, exact
    in integers, from a summed-volume table of the event histogram (cheap
    enough for every event of the largest slices).

These two numpy routines are independent routes to the same numbers and
are used to pin the C oracle (they share no code with it).

  * ``mlp_train_step`` -- one training step of the perceptron on a batch of
    encodings with target normal flows (the paper delegates its loss to its
    predecessor, so the loss here is our own: the mean over rows of the
    squared error of the 2-vector), with the gradients of layer 2 and layer 1
    written out by the chain rule, then plain gradient descent or Adam.
    FP64, numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "veckm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def compile_source(src: str, out: str, sanitize: bool = False) -> str:
    """gcc -O2 without FMA contraction, OpenMP, as a shared library.  With
    `sanitize`, instrumented by AddressSanitizer and UndefinedBehaviorSanitizer
    (the library then needs gcc's libasan preloaded into the process)."""
    tmp = out + ".tmp%d" % os.getpid()
    extra = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"] if sanitize else []
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC"] + extra +
                          ["-shared", src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


def load_library(path: str):
    """Open a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    lib.oracle_encode.restype = ctypes.c_int
    lib.oracle_encode.argtypes = [
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.oracle_mlp.restype = ctypes.c_int
    lib.oracle_mlp.argtypes = [
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int32]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load_library(_LIB)
    return _lib


def encode(events, A, rx, ry, rt, queries=None, search="bucket", threads=0, lib=None):
    """FP64 encodings of the queried events.

    events: int[n,4] (x, y, t, p); A: float64[D,3] (columns x, y, t);
    queries: None (all events) or int[m] event indices.
    Returns (emb float64[m, 2D] planar [Re | Im], cnt int64[m])."""
    lib = lib or _load()
    ev = np.ascontiguousarray(np.asarray(events, dtype=np.int32))
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n = ev.shape[0]
    D = A.shape[0]
    if queries is None:
        q = None
        m = n
    else:
        q = np.ascontiguousarray(np.asarray(queries, dtype=np.int64))
        m = q.shape[0]
        if m and (q.min() < 0 or q.max() >= n):
            raise IndexError("query index out of range")
    emb = np.zeros((m, 2 * D), dtype=np.float64)
    cnt = np.zeros(m, dtype=np.int64)
    rc = lib.oracle_encode(ev.ctypes.data, n, None if q is None else q.ctypes.data, m,
                           A.ctypes.data, D, int(rx), int(ry), int(rt),
                           1 if search == "bucket" else 0, emb.ctypes.data, cnt.ctypes.data,
                           int(threads))
    if rc != 0:
        raise RuntimeError("oracle_encode failed (%d)" % rc)
    return emb, cnt


def mlp(x, W1, b1, W2, b2, threads=0, lib=None):
    """FP64 two-layer perceptron: W2 relu(W1 x + b1) + b2, per row of x."""
    lib = lib or _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    W1 = np.ascontiguousarray(np.asarray(W1, dtype=np.float64))
    b1 = np.ascontiguousarray(np.asarray(b1, dtype=np.float64))
    W2 = np.ascontiguousarray(np.asarray(W2, dtype=np.float64))
    b2 = np.ascontiguousarray(np.asarray(b2, dtype=np.float64))
    m, din = x.shape
    hidden = W1.shape[0]
    if W1.shape != (hidden, din) or W2.shape != (2, hidden) or b1.shape != (hidden,) \
            or b2.shape != (2,):
        raise ValueError("perceptron shapes do not match")
    out = np.zeros((m, 2), dtype=np.float64)
    rc = lib.oracle_mlp(x.ctypes.data, m, din, hidden, W1.ctypes.data, b1.ctypes.data,
                        W2.ctypes.data, b2.ctypes.data, out.ctypes.data, int(threads))
    if rc != 0:
        raise RuntimeError("oracle_mlp failed (%d)" % rc)
    return out


def flow(events, A, rx, ry, rt, W1, b1, W2, b2, queries=None, search="bucket", threads=0):
    emb, cnt = encode(events, A, rx, ry, rt, queries, search, threads)
    return mlp(emb, W1, b1, W2, b2, threads), emb, cnt


def alg1_paper_form(events, A, rx, ry, queries=None):
    """The staged 2-D form of Sec. 2.2.2 (no temporal bound), FP64.

    Eqns. 14-15: a per-pixel grid holding, for each pixel p, the sum of the
    temporal phases exp(i A_t t_k) of its events (PixelEmbed) and their
    number (PixelCount).  Eqns. 16-17: for a query at pixel q, the window sum
    over spatial offsets o of PixelEmbed(q + o) times the spatial offset
    phase exp(i (A_x o_x + A_y o_y)), and the window count.  The query's own
    temporal phase is then removed (conjugate factor) and the sum divided by
    the count.  Time is measured from the earliest event: a constant shift
    that cancels between the two temporal phases.  Evaluated offset by
    offset over all queries at once (grid padded by the radii)."""
    ev = np.asarray(events, dtype=np.int64)
    A = np.asarray(A, dtype=np.float64)
    D = A.shape[0]
    qs = np.arange(len(ev)) if queries is None else np.asarray(queries, dtype=np.int64)
    # pixel coordinates inside a grid padded by the window radii
    px = ev[:, 0] - ev[:, 0].min() + rx
    py = ev[:, 1] - ev[:, 1].min() + ry
    tt = (ev[:, 2] - ev[:, 2].min()).astype(np.float64)
    GW, GH = int(px.max()) + rx + 1, int(py.max()) + ry + 1
    flat = py * GW + px
    tphase = np.exp(1j * tt[:, None] * A[None, :, 2])                 # [n, D]
    pix_embed = np.zeros((GH * GW, D), dtype=np.complex128)
    np.add.at(pix_embed, flat, tphase)                               # Eqn. 14
    pix_count = np.bincount(flat, minlength=GH * GW)                 # Eqn. 15
    dxs = np.arange(-rx, rx + 1)
    dys = np.arange(-ry, ry + 1)
    # spatial offset phases, [2ry+1, 2rx+1, D]
    ophase = np.exp(1j * (dys[:, None, None] * A[None, None, :, 1] +
                          dxs[None, :, None] * A[None, None, :, 0]))
    qflat = flat[qs]
    acc = np.zeros((len(qs), D), dtype=np.complex128)
    cnt = np.zeros(len(qs), dtype=np.int64)
    for iy, dy in enumerate(dys):                                    # Eqns. 16-17
        for ix, dx in enumerate(dxs):
            nb = qflat + dy * GW + dx
            acc += pix_embed[nb] * ophase[iy, ix][None, :]
            cnt += pix_count[nb]
    emb = acc * np.conj(tphase[qs]) / cnt[:, None]
    return np.concatenate([emb.real, emb.imag], axis=1), cnt


def box_count(events, rx, ry, rt, queries=None):
    """Windowed neighbour count of Eqn. 17 for every queried event, exact.

    N(q) = number of events k with |x_k - x_q| <= rx, |y_k - y_q| <= ry and
    |t_k - t_q| <= rt (rt < 0: no temporal bound, Eqn. 1 as written), the
    query included.  Computed as a box sum of the integer event histogram
    over (t, y, x) voxels, read off a summed-volume table (inclusion-exclusion
    over the 8 corners of the clipped box).  int64[m]."""
    ev = np.asarray(events, dtype=np.int64)
    if len(ev) == 0:
        return np.zeros(0, dtype=np.int64)
    x, y, t = ev[:, 0] - ev[:, 0].min(), ev[:, 1] - ev[:, 1].min(), ev[:, 2] - ev[:, 2].min()
    W, H, T = int(x.max()) + 1, int(y.max()) + 1, int(t.max()) + 1
    if rt < 0:
        rt = T
    hist = np.zeros((T, H, W), dtype=np.int64)
    np.add.at(hist, (t, y, x), 1)
    sv = np.zeros((T + 1, H + 1, W + 1), dtype=np.int64)   # sv[a, b, c] = hist[:a, :b, :c].sum()
    sv[1:, 1:, 1:] = hist.cumsum(0).cumsum(1).cumsum(2)
    qs = np.arange(len(ev)) if queries is None else np.asarray(queries, dtype=np.int64)
    t0, t1 = np.maximum(t[qs] - rt, 0), np.minimum(t[qs] + rt + 1, T)
    y0, y1 = np.maximum(y[qs] - ry, 0), np.minimum(y[qs] + ry + 1, H)
    x0, x1 = np.maximum(x[qs] - rx, 0), np.minimum(x[qs] + rx + 1, W)
    return (sv[t1, y1, x1] - sv[t0, y1, x1] - sv[t1, y0, x1] - sv[t1, y1, x0]
            + sv[t0, y0, x1] + sv[t0, y1, x0] + sv[t1, y0, x0] - sv[t0, y0, x0])


def pooling_form_3d(events, A, rx, ry, rt, queries=None):
    """Pooling over a 3-D (x, y, t) count grid with a temporal radius, FP64.

    Every event sharing a voxel has the same phase relative to the query,
    so the window sum is a sum over voxels of count * offset phase."""
    ev = np.asarray(events, dtype=np.int64)
    A = np.asarray(A, dtype=np.float64)
    x, y, t = ev[:, 0], ev[:, 1], ev[:, 2]
    gx, gy, gt = x - x.min() + rx, y - y.min() + ry, t - t.min() + rt
    grid = np.zeros((gx.max() + rx + 1, gy.max() + ry + 1, gt.max() + rt + 1), dtype=np.int64)
    np.add.at(grid, (gx, gy, gt), 1)
    offs = [(dx, dy, dt) for dx in range(-rx, rx + 1) for dy in range(-ry, ry + 1)
            for dt in range(-rt, rt + 1)]
    table = {o: np.exp(1j * (A[:, 0] * o[0] + A[:, 1] * o[1] + A[:, 2] * o[2])) for o in offs}
    D = A.shape[0]
    qs = np.arange(len(ev)) if queries is None else np.asarray(queries)
    out = np.zeros((len(qs), 2 * D))
    cnt = np.zeros(len(qs), dtype=np.int64)
    for i, q in enumerate(qs):
        e = np.zeros(D, dtype=np.complex128)
        c = 0
        for o in offs:
            k = grid[gx[q] + o[0], gy[q] + o[1], gt[q] + o[2]]
            if k:
                c += k
                e += k * table[o]
        e /= c
        out[i, :D], out[i, D:] = e.real, e.imag
        cnt[i] = c
    return out, cnt


def mlp_loss_grads(x, y, W1, b1, W2, b2):
    """Loss and gradients of L = (1/M) sum_r ||W2 relu(W1 x_r + b1) + b2 - y_r||^2.

    x: [M, K2], y: [M, 2].  The ReLU derivative at 0 is taken as 0.
    Returns (L, dict(W1=..., b1=..., W2=..., b2=...)), all FP64."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    W1 = np.asarray(W1, np.float64); b1 = np.asarray(b1, np.float64)
    W2 = np.asarray(W2, np.float64); b2 = np.asarray(b2, np.float64)
    M = x.shape[0]
    z = x @ W1.T + b1                 # pre-activations [M, hidden]
    h = np.maximum(z, 0.0)
    p = h @ W2.T + b2                 # predictions [M, 2]
    r = p - y
    L = float((r * r).sum() / M)
    dp = 2.0 * r / M                  # dL/dp
    gW2 = dp.T @ h
    gb2 = dp.sum(0)
    dz = (dp @ W2) * (z > 0)          # back through W2 and the ReLU
    gW1 = dz.T @ x
    gb1 = dz.sum(0)
    return L, dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2)


def mlp_train_step(x, y, params, opt="sgd", lr=1e-3, state=None, t=1, betas=(0.9, 0.999),
                   eps=1e-8):
    """One step on (x, y): returns (loss, grads, new params, new state).

    params: dict W1, b1, W2, b2.  opt "sgd": p - lr g.  opt "adam": the
    moment estimates m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2 (state
    holds them, zero before step 1), bias-corrected by 1 - b^t, and
    p - lr m_hat / (sqrt(v_hat) + eps)."""
    L, g = mlp_loss_grads(x, y, params["W1"], params["b1"], params["W2"], params["b2"])
    new, st = {}, {}
    for k in ("W1", "b1", "W2", "b2"):
        p = np.asarray(params[k], np.float64)
        if opt == "sgd":
            new[k] = p - lr * g[k]
        else:
            m0 = np.zeros_like(p) if state is None else state["m"][k]
            v0 = np.zeros_like(p) if state is None else state["v"][k]
            m1 = betas[0] * m0 + (1.0 - betas[0]) * g[k]
            v1 = betas[1] * v0 + (1.0 - betas[1]) * g[k] * g[k]
            mh = m1 / (1.0 - betas[0] ** t)
            vh = v1 / (1.0 - betas[1] ** t)
            new[k] = p - lr * mh / (np.sqrt(vh) + eps)
            st.setdefault("m", {})[k] = m1
            st.setdefault("v", {})[k] = v1
    return L, g, new, (st if opt == "adam" else None)
