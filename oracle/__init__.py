"""CPU oracle for the normal-flow estimator (FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path never imports it.

Contents
  * ``encode`` / ``mlp`` -- ctypes front end of ``veckm_oracle.c``: the plain
    quadratic adjacency-row encoding (Eqn. 10 over the neighbourhood of
    Eqn. 1, normalised by the count of Eqn. 17) and the two-layer perceptron
    (Eqns. 5-6), in FP64.
  * ``alg1_paper_form`` -- Algorithm 1 as the paper states it: a 2-D
    PixelEmbed/PixelCount grid filled with temporal phases (Eqns. 14-15),
    pooled over the spatial window with the precomputed spatial offset
    phases (Eqn. 16, count of Eqn. 17), then multiplied by the conjugate
    temporal phase of the query and divided by the count.  No temporal
    bound, as in Eqn. 1.
  * ``pooling_form_3d`` -- the same pooling idea generalised to a temporal
    radius: a 3-D (x, y, t) count grid pooled with (dx, dy, dt) offset
    phases.

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


def compile_source(src: str, out: str) -> str:
    """gcc -O2 without FMA contraction, OpenMP, as a shared library."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", src, "-o", tmp, "-lm"])
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
    """Algorithm 1 in numpy (no temporal bound), FP64.

    Per pixel: PixelEmbed[x, y, :] = sum of exp(i * A_t * t_k) over its
    events, PixelCount[x, y] = number of events (Eqns. 14-15).  Per query:
    pool PixelEmbed over the window with the precomputed spatial offset
    phases exp(i (A_x dx + A_y dy)), pool the counts (Eqns. 16-17), then
    multiply by exp(-i A_t t_q) and divide by the count.  Time is measured
    from the earliest event, a constant shift that cancels between the
    scattered and the conjugate temporal phase."""
    ev = np.asarray(events, dtype=np.int64)
    A = np.asarray(A, dtype=np.float64)
    x, y, t = ev[:, 0], ev[:, 1], ev[:, 2] - ev[:, 2].min()
    x0, y0 = x.min() - rx, y.min() - ry
    gx, gy = x - x0, y - y0
    Wg, Hg = gx.max() + rx + 1, gy.max() + ry + 1
    D = A.shape[0]
    embed = np.zeros((Wg, Hg, D), dtype=np.complex128)
    count = np.zeros((Wg, Hg), dtype=np.int64)
    temporal = np.exp(1j * np.outer(t.astype(np.float64), A[:, 2]))      # [n, D]
    for k in range(len(ev)):                                              # scatter
        embed[gx[k], gy[k]] += temporal[k]
        count[gx[k], gy[k]] += 1
    offs = [(dx, dy) for dx in range(-rx, rx + 1) for dy in range(-ry, ry + 1)]
    table = {o: np.exp(1j * (A[:, 0] * o[0] + A[:, 1] * o[1])) for o in offs}  # precomputed
    qs = np.arange(len(ev)) if queries is None else np.asarray(queries)
    out = np.zeros((len(qs), 2 * D))
    cnt = np.zeros(len(qs), dtype=np.int64)
    for i, q in enumerate(qs):
        e = np.zeros(D, dtype=np.complex128)
        c = 0
        for (dx, dy) in offs:
            c += count[gx[q] + dx, gy[q] + dy]
            e += embed[gx[q] + dx, gy[q] + dy] * table[(dx, dy)]
        e = e * np.exp(-1j * t[q] * A[:, 2]) / c
        out[i, :D], out[i, D:] = e.real, e.imag
        cnt[i] = c
    return out, cnt


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
