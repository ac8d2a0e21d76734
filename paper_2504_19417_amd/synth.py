"""Seeded synthetic inputs for the normal-flow estimator.

This module is the only code shared by the HIP path's tests/benchmarks and
the CPU oracle.  It draws inputs and nothing else: event slices, the random
Fourier frequency matrix ``A``, the two-layer perceptron weights and query
subsets.  None of the estimator's arithmetic (phases, window sums,
normalisation, the perceptron) lives here.

Event model (stands in for the EVIMO2 recordings the paper trains and
evaluates on, which are not available): straight edges of random
orientation translating at 0.5-3 px/ms across the sensor, each edge firing
events along its current position with 0.5 px jitter along its normal, plus
10 % uniform noise (or, for the 1280x720 precision workload, noise drawn
from textured Gaussian blobs).  Timestamps are integer 1 ms bins offset by a
large base time so that every consumer has to rebase them.  Events are sorted
by time with seeded tie-breaking, as a camera would emit them.

Frequencies follow Algorithm 1 (frequency draw): three D-vectors drawn from
N(0, 25) with seeds 0, 1, 2 for the t, x, y axes, divided by the radius of
their axis so that ``A`` acts directly on integer (dx, dy, dt) offsets.  When
the temporal radius is negative (no temporal bound, the paper's neighbourhood
of Eqn. (1)) the temporal scale is half the slice length, as in the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SIGMA2 = 25.0          # variance of the frequency draw (Algorithm 1)
FREQ_SEEDS = (0, 1, 2)  # seeds of the T, X, Y draws (Algorithm 1)
MLP_SEED = 7


@dataclass
class SliceSpec:
    """Shape of one synthetic event slice."""
    width: int
    height: int
    nbins: int                 # number of 1 ms bins in the slice
    n: int                     # events in the slice
    edges: int                 # moving edges
    noise_frac: float = 0.10
    blob_noise: bool = False   # textured-blob noise instead of uniform noise
    t_base: int = 1_000_000    # absolute time of bin 0
    seed: int = 0


@dataclass
class Workload:
    """One named workload: slices plus encoder/perceptron sizes."""
    name: str
    slices: list
    d: int                     # complex RFF dimension D
    rx: int
    ry: int
    rt: int
    hidden: int                # perceptron hidden width
    precision: str = "fp32"    # "fp32" or "fp16" (fp16 phase table + bf16 MLP)
    notes: str = ""
    extra: dict = field(default_factory=dict)


def _lognormal_sizes(rng, count, median, sigma, lo, hi):
    n = np.exp(rng.normal(math.log(median), sigma, size=count))
    return np.clip(np.round(n), lo, hi).astype(np.int64)


def workloads() -> dict:
    """The workloads: tiny CPU case, 1M-event FP32 slice, 5M-event precision
    slice, 64-slice batch (the 32-stream serving mix is `serving_streams`),
    and the paper's own form at its training recipes (640x480, D=64, no
    temporal bound, delta-t = half the slice): radius 8 over 32 ms and radius
    10 over 24 ms, each 0.5M events (the size of the paper's worked timing
    example)."""
    w = {}
    w["tiny"] = Workload(
        "tiny", [SliceSpec(346, 260, 25, 20_000, 8, seed=1001)],
        d=64, rx=3, ry=3, rt=2, hidden=128,
        notes="346x260, 20k events, 8 edges, 25 bins, D=64, r=3/2, MLP 128-128-2")
    w["slice1m"] = Workload(
        "slice1m", [SliceSpec(346, 260, 50, 1_000_000, 32, seed=1002)],
        d=128, rx=5, ry=5, rt=3, hidden=256,
        notes="346x260, 1M events, 32 edges, 50 bins, D=128, r=5/3, MLP 256-256-2 FP32")
    w["precision5m"] = Workload(
        "precision5m", [SliceSpec(1280, 720, 100, 5_000_000, 64, blob_noise=True, seed=1003)],
        d=128, rx=5, ry=5, rt=3, hidden=256, precision="fp16",
        notes="1280x720, 5M events, 64 edges + blob noise, 100 bins, D=128, r=5/3, "
              "fp16 phase table + bf16 MLP")
    rng = np.random.Generator(np.random.PCG64(1004))
    sizes = _lognormal_sizes(rng, 64, 70_711, 0.652, 10_000, 500_000)
    coins = rng.integers(0, 2, size=64)
    slices = []
    for i in range(64):
        W, H = (346, 260) if coins[i] == 0 else (640, 480)
        slices.append(SliceSpec(W, H, 50, int(sizes[i]), 32, seed=2000 + i,
                                t_base=1_000_000 + 50 * i))
    w["batch64"] = Workload("batch64", slices, d=128, rx=5, ry=5, rt=3, hidden=256,
                            precision="fp16",
                            notes="64 slices, lognormal 10k-500k events, 346x260 / 640x480")
    # the launch-bound end of the batched form: 64 slices of 10k events each
    # (the lower clip of the lognormal mix), same sensors
    slices = [SliceSpec(*((346, 260) if coins[i] == 0 else (640, 480)), 50, 10_000, 32,
                        seed=3000 + i, t_base=2_000_000 + 50 * i) for i in range(64)]
    w["batch64x10k"] = Workload("batch64x10k", slices, d=128, rx=5, ry=5, rt=3, hidden=256,
                                precision="fp16",
                                notes="64 slices of 10k events, 346x260 / 640x480")
    w["paper_k8"] = Workload(
        "paper_k8", [SliceSpec(640, 480, 32, 500_000, 32, seed=1006)],
        d=64, rx=8, ry=8, rt=-1, hidden=128,
        notes="640x480, 0.5M events, 32 edges, 32 bins (32 ms, delta-t 16 ms), D=64, "
              "delta-x = delta-y = 8, no temporal bound, MLP 128-128-2 FP32")
    w["paper_k10"] = Workload(
        "paper_k10", [SliceSpec(640, 480, 24, 500_000, 32, seed=1007)],
        d=64, rx=10, ry=10, rt=-1, hidden=128,
        notes="640x480, 0.5M events, 32 edges, 24 bins (24 ms, delta-t 12 ms), D=64, "
              "delta-x = delta-y = 10, no temporal bound, MLP 128-128-2 FP32")
    return w


@dataclass
class StreamSpec:
    """One event stream of the serving workload: a sensor, a Poisson event
    rate and a slice window (the stream closes a slice every `window_ms`)."""
    width: int
    height: int
    rate_mev_s: float
    window_ms: int
    seed: int


def serving_streams(count: int = 32, seed: int = 1005):
    """The serving workload: `count` streams, sensors 346x260 or 1280x720 by
    coin, rates U[0.5, 10] Mev/s, slice windows U{1..20} ms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        W, H = (346, 260) if rng.integers(0, 2) == 0 else (1280, 720)
        out.append(StreamSpec(W, H, float(rng.uniform(0.5, 10.0)), int(rng.integers(1, 21)),
                              seed=3000 + i))
    return out


def stream_slices(spec: StreamSpec, count: int):
    """`count` consecutive slices of a stream: Poisson(rate x window) events
    each over `window_ms` one-ms bins, from the moving-edge generator."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    out = []
    for k in range(count):
        n = max(1, int(rng.poisson(spec.rate_mev_s * 1e3 * spec.window_ms)))
        sl = SliceSpec(spec.width, spec.height, spec.window_ms, n, 16,
                       t_base=1_000_000 + k * spec.window_ms, seed=spec.seed * 100 + k)
        out.append(make_slice(sl))
    return out


def _edge_events(rng, W, H, T, count, E):
    """Events of E moving edges, ``count`` in total, and the true normal flow
    of each (sign * speed * normal, px per bin; NaN for the noise that tops
    up an edge that rarely crosses the sensor)."""
    theta = rng.uniform(0.0, math.pi, E)
    nu = np.stack([np.cos(theta), np.sin(theta)], 1)
    nu_perp = np.stack([-np.sin(theta), np.cos(theta)], 1)
    sign = rng.choice([-1.0, 1.0], E)
    speed = rng.uniform(0.5, 3.0, E)
    length = rng.uniform(0.3, 0.8, E) * math.hypot(W, H)
    centre = rng.uniform([0.0, 0.0], [W, H], (E, 2))
    pol = rng.choice([-1, 1], E)
    share = np.full(E, count // E, dtype=np.int64)
    share[: count - share.sum()] += 1
    xs, ys, ts, ps, fs = [], [], [], [], []
    for e in range(E):
        need = int(share[e])
        got = 0
        for _ in range(1000):
            if got >= need:
                break
            batch = max(256, 2 * (need - got))
            tau = rng.uniform(0.0, T, batch)
            ell = rng.uniform(-length[e] / 2, length[e] / 2, batch)
            eps = rng.normal(0.0, 0.5, batch)
            off = sign[e] * speed[e] * (tau - T / 2.0)
            px = centre[e, 0] + off * nu[e, 0] + ell * nu_perp[e, 0] + eps * nu[e, 0]
            py = centre[e, 1] + off * nu[e, 1] + ell * nu_perp[e, 1] + eps * nu[e, 1]
            x = np.floor(px).astype(np.int64)
            y = np.floor(py).astype(np.int64)
            t = np.minimum(np.floor(tau).astype(np.int64), T - 1)
            ok = (x >= 0) & (x < W) & (y >= 0) & (y < H)
            x, y, t = x[ok][: need - got], y[ok][: need - got], t[ok][: need - got]
            xs.append(x); ys.append(y); ts.append(t)
            ps.append(np.full(len(x), pol[e], dtype=np.int64))
            fs.append(np.tile(sign[e] * speed[e] * nu[e], (len(x), 1)))
            got += len(x)
        if got < need:  # an edge that almost never crosses the sensor: top up with noise
            k = need - got
            xs.append(rng.integers(0, W, k)); ys.append(rng.integers(0, H, k))
            ts.append(rng.integers(0, T, k)); ps.append(rng.choice([-1, 1], k))
            fs.append(np.full((k, 2), np.nan))
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(ts), np.concatenate(ps),
            np.concatenate(fs))


def _blob_noise(rng, W, H, T, count, blobs=32):
    """Textured blobs: Gaussian blobs whose samples are thinned by a random
    plane-wave texture (1 + cos(k . pos)) / 2."""
    centre = rng.uniform([0.0, 0.0], [W, H], (blobs, 2))
    sig = rng.uniform(4.0, 24.0, blobs)
    kmag = rng.uniform(0.2, 1.0, blobs)
    kang = rng.uniform(0.0, 2 * math.pi, blobs)
    kvec = np.stack([kmag * np.cos(kang), kmag * np.sin(kang)], 1)
    xs, ys = [], []
    got = 0
    while got < count:
        batch = 2 * (count - got) + 256
        b = rng.integers(0, blobs, batch)
        pos = centre[b] + rng.normal(0.0, 1.0, (batch, 2)) * sig[b, None]
        keep = rng.uniform(0.0, 1.0, batch) < 0.5 * (1.0 + np.cos((kvec[b] * pos).sum(1)))
        x = np.floor(pos[:, 0]).astype(np.int64)
        y = np.floor(pos[:, 1]).astype(np.int64)
        keep &= (x >= 0) & (x < W) & (y >= 0) & (y < H)
        x, y = x[keep][: count - got], y[keep][: count - got]
        xs.append(x); ys.append(y)
        got += len(x)
    x = np.concatenate(xs); y = np.concatenate(ys)
    t = rng.integers(0, T, count)
    p = rng.choice([-1, 1], count)
    return x, y, t, p


def make_slice(spec: SliceSpec, with_flow: bool = False):
    """Return (events int32[n,4] as (x, y, t, p), t0, nbins), and with
    ``with_flow`` also the true normal flow float64[n, 2] of every event (px
    per bin; NaN for noise events).

    t is absolute (``t_base`` + bin); every event satisfies
    t0 <= t < t0 + nbins and 0 <= x < width, 0 <= y < height.  The flow is
    computed alongside and draws no random numbers, so the events do not
    depend on ``with_flow``."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    W, H, T = spec.width, spec.height, spec.nbins
    n_noise = int(round(spec.noise_frac * spec.n))
    n_edge = spec.n - n_noise
    ex, ey, et, ep, ef = _edge_events(rng, W, H, T, n_edge, spec.edges)
    if spec.blob_noise:
        nx, ny, nt, np_ = _blob_noise(rng, W, H, T, n_noise)
    else:
        nx = rng.integers(0, W, n_noise); ny = rng.integers(0, H, n_noise)
        nt = rng.integers(0, T, n_noise); np_ = rng.choice([-1, 1], n_noise)
    x = np.concatenate([ex, nx]); y = np.concatenate([ey, ny])
    t = np.concatenate([et, nt]); p = np.concatenate([ep, np_])
    f = np.concatenate([ef, np.full((len(nx), 2), np.nan)])
    perm = rng.permutation(len(x))          # seeded tie-break ...
    x, y, t, p, f = x[perm], y[perm], t[perm], p[perm], f[perm]
    order = np.argsort(t, kind="stable")    # ... then camera (time) order
    ev = np.stack([x[order], y[order], t[order] + spec.t_base, p[order]], 1).astype(np.int32)
    if with_flow:
        return np.ascontiguousarray(ev), int(spec.t_base), int(T), np.ascontiguousarray(f[order])
    return np.ascontiguousarray(ev), int(spec.t_base), int(T)


def temporal_scale(rt: int, nbins: int) -> float:
    """delta-t of Algorithm 1 for a temporal radius ``rt`` (in bins)."""
    if rt < 0:
        return nbins / 2.0
    return float(max(rt, 1))


def draw_frequencies(d: int, rx: int, ry: int, rt: int, nbins: int = 0,
                     sigma2: float = SIGMA2, seeds=FREQ_SEEDS) -> np.ndarray:
    """Frequency matrix A (float64, d x 3, columns x, y, t).

    T, X, Y ~ N(0, sigma2) with seeds (0, 1, 2) as in Algorithm 1, divided by
    delta-x = rx, delta-y = ry and delta-t so that A multiplies integer
    offsets directly."""
    sd = math.sqrt(sigma2)
    zt = np.random.Generator(np.random.PCG64(seeds[0])).normal(0.0, 1.0, d)
    zx = np.random.Generator(np.random.PCG64(seeds[1])).normal(0.0, 1.0, d)
    zy = np.random.Generator(np.random.PCG64(seeds[2])).normal(0.0, 1.0, d)
    A = np.empty((d, 3), dtype=np.float64)
    A[:, 0] = sd * zx / max(rx, 1)
    A[:, 1] = sd * zy / max(ry, 1)
    A[:, 2] = sd * zt / temporal_scale(rt, nbins)
    return A


def init_mlp(d: int, hidden: int, seed: int = MLP_SEED):
    """Random-init two-layer perceptron (2D -> hidden -> 2), float32, torch
    Linear layout ([out][in]) and torch's default U(+-1/sqrt(fan_in))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fin1 = 2 * d
    b1w = 1.0 / math.sqrt(fin1)
    b2w = 1.0 / math.sqrt(hidden)
    W1 = rng.uniform(-b1w, b1w, (hidden, fin1)).astype(np.float32)
    b1 = rng.uniform(-b1w, b1w, hidden).astype(np.float32)
    W2 = rng.uniform(-b2w, b2w, (2, hidden)).astype(np.float32)
    b2 = rng.uniform(-b2w, b2w, 2).astype(np.float32)
    return W1, b1, W2, b2


def sample_queries(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct event indices out of n, sorted, int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = min(m, n)
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)


def random_events(rng, n, W, H, T, t_base=0):
    """Uniform random events (used for small edge-case inputs)."""
    ev = np.stack([rng.integers(0, W, n), rng.integers(0, H, n),
                   rng.integers(0, T, n) + t_base, rng.choice([-1, 1], n)], 1)
    return np.ascontiguousarray(ev.astype(np.int32))
