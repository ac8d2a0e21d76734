"""Benchmark: normal flows per second on a 1M-event slice, FP32 and FP16/BF16.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one veckm_flow call over the whole slice: validate and bin the
events, rank the query voxels, the encoder contraction, the perceptron and
the per-event output, with the events already resident in HBM.  Every event
is queried (one flow per event).  Workload: 346x260 sensor, 1,000,000
events of 32 moving edges plus 10 % noise over 50 one-bin time steps,
D = 128, window +-5 px, +-3 bins, perceptron 256 -> 256 -> 2.

Prints one JSON line.  `value` is the FP32 form's flows/s; the FP16/BF16
form, per-step latency percentiles, per-stage device times, the roofline of
the dominant kernel and the CPU oracle timed on a bounded sample are extra
keys.  The timed steps run the plain call; the latency percentiles (an event
pair around each call) and the stage times (the library's stage timers) come
from passes of the same number of steps after them.  Only one GPU is used.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp16_TFLOPs": 2500.0,
    "bf16_TFLOPs": 2500.0,
    "fp32_TFLOPs": 157.3,
}


def encoder_flops_per_row(K, d):
    """Algorithmic flops of one encoder row: the window sum written over the
    centre plus half window (conjugate symmetry), real count pair sums times
    cos for Re (K terms) and pair differences times sin for Im (K-1 terms),
    one multiply-add = 2 flops, for each of the d frequencies."""
    return 2 * (2 * K - 1) * d


def mlp_flops_per_row(d, hidden):
    """Layer 1 (2d -> hidden) and layer 2 (hidden -> 2) multiply-adds."""
    return 2 * (2 * d) * hidden + 2 * hidden * 2


def encode_stage_flops_per_row(K, d, hidden, stages):
    """Algorithmic flops per row of the encode stage: the encoder's, plus the
    perceptron's when the encoder ran it itself (no perceptron stage timed)."""
    fused = stages.get("mlp") is None
    return encoder_flops_per_row(K, d) + (mlp_flops_per_row(d, hidden) if fused else 0), fused


def paper_encode_bytes(W, H, T, d, rows, row_bytes):
    """Algorithmic HBM bytes of the paper form's encode stage (no temporal
    bound): the temporal phase pass reads the T x H x W count grid and writes
    the complex D-wide fp32 pixel grid G; the fused window pass reads G and
    writes S; the box sums read and write four int32 pixel grids; the row
    pass reads S (8D bytes) and writes one row per query voxel."""
    V2 = W * H
    grid = 2 * d * 4 * V2
    return 4 * T * V2 + grid + 2 * grid + 4 * 4 * V2 + rows * (2 * d * 4 + row_bytes)


def eqn18_split(n, m_small, ms_small, ms_all):
    """The runtime model of Eqn. 18, time = c n + C m, fitted through the
    all-events point (m = n) and a sparse point (m = m_small)."""
    C = (ms_all - ms_small) / (n - m_small)       # ms per flow
    c = (ms_small - C * m_small) / n              # ms per event
    return {"c_ns_per_event": round(c * 1e6, 4), "C_ns_per_flow": round(C * 1e6, 4),
            "points": [[m_small, round(ms_small, 4)], [n, round(ms_all, 4)]]}


def run_form(vk, torch, w, ev, t0, T, A, mlp, precision, steps, warmup, queries=None,
             tune=False):
    ctx = vk.Context(w.slices[0].width, w.slices[0].height, w.rx, w.ry, w.rt, A, T, len(ev),
                     precision)
    ctx.set_mlp(*mlp)
    evt = torch.from_numpy(ev).cuda()
    tiling = None
    qt = None if queries is None else torch.from_numpy(np.asarray(queries, np.int32)).cuda()
    m = len(ev) if queries is None else len(queries)
    out = torch.empty((m, 2), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.flow(evt, t0, T, qt, out=out)
    if tune:
        # the library's tuner picks the encoder tiling (set-up, not timed),
        # once the device has warmed up: the first few tens of calls run slow
        W, H = w.slices[0].width, w.slices[0].height
        tiling = list(ctx.tilings()[ctx.tune([(W, H, t0, T, len(ev))], evt, reps=5)])
        for _ in range(warmup):
            ctx.flow(evt, t0, T, qt, out=out)
    torch.cuda.synchronize()
    if ctx.status() != vk.VECKM_OK:
        raise RuntimeError("input error reported by the device")
    # the timed steps: the plain call, nothing recorded around it
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        ctx.flow(evt, t0, T, qt, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # after them, not part of the timed value: the latency of each call (an
    # event pair around it), then the stage split from the library's stage
    # timers (six event records per call, which add about 20 us to a step)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for i in range(steps):
        starts[i].record(stream)
        ctx.flow(evt, t0, T, qt, out=out)
        ends[i].record(stream)
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ctx.profile(True)
    ctx.profile_read()
    for i in range(steps):
        ctx.flow(evt, t0, T, qt, out=out)
    torch.cuda.synchronize()
    stages = ctx.profile_read()
    ctx.profile(False)
    rows = ctx.last_rows()
    flows = out.cpu().numpy()
    st = ctx.status()
    ctx.close()
    if st != vk.VECKM_OK:
        raise RuntimeError("input error reported by the device")
    return dict(elapsed=elapsed, lat=lat, stages=stages, rows=rows, flows=flows, tiling=tiling)


def host_cpu():
    """The host's processor model and logical CPU count (lscpu, else /proc)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except Exception:
            pass
    return {"model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _timed(fn):
    t = time.perf_counter()
    fn()
    return time.perf_counter() - t


def cpu_baseline(oracle, w, ev, A, mlp, target_s):
    """The FP64 oracle, as it stands, on the host's cores.

    Headline (value): a seeded sample of the same slice's queries, bucketed
    neighbour search, OpenMP over queries on every available thread, sized to
    about 0.6 target_s.  Further legs: the same search on one thread; the
    20k-event workload (346x260x25, D = 64, r = 3/2, perceptron 128-128-2) in
    full with the bucketed and with the literal quadratic search; and the
    literal quadratic scan on 1024 queries of this slice."""
    from paper_2504_19417_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()

    def rate(queries, nthreads, search="bucket", events=ev, A_=A, wl=w, mlp_=mlp):
        def go():
            e, _ = oracle.encode(events, A_, wl.rx, wl.ry, wl.rt, queries=queries,
                                 search=search, threads=nthreads)
            oracle.mlp(e, *mlp_, threads=nthreads)
        dt = _timed(go)
        m = len(events) if queries is None else len(queries)
        return m, dt

    def sized(nthreads, budget, seed):
        m0, t0 = rate(synth.sample_queries(len(ev), 512, seed), nthreads)
        m = int(min(len(ev), max(512, 512 * budget / max(t0, 1e-3))))
        return rate(synth.sample_queries(len(ev), m, seed + 1), nthreads)

    m, dt = sized(threads, 0.6 * target_s, 901)
    m1, dt1 = sized(1, 0.15 * target_s, 911)
    tw = synth.workloads()["tiny"]
    tev, _, _ = synth.make_slice(tw.slices[0])
    tA = synth.draw_frequencies(tw.d, tw.rx, tw.ry, tw.rt)
    tmlp = synth.init_mlp(tw.d, tw.hidden)
    tb = rate(None, threads, "bucket", tev, tA, tw, tmlp)
    tq = rate(None, threads, "scan", tev, tA, tw, tmlp)
    q1k = rate(synth.sample_queries(len(ev), 1024, 921), threads, "scan")
    return {"value": m / dt, "unit": "flows/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the slice's %d queries (seeded), FP64 quadratic adjacency-row "
                      "encoding with bucketed neighbour search + FP64 perceptron, %d threads, "
                      "%.1f s" % (m, len(ev), threads, dt),
            "host": host_cpu(),
            "legs": {
                "one_thread_bucketed": {"flows_per_s": m1 / dt1, "queries": m1,
                                        "seconds": round(dt1, 2), "threads": 1},
                "tiny_full_bucketed": {"flows_per_s": tb[0] / tb[1], "queries": tb[0],
                                       "seconds": round(tb[1], 3), "threads": threads},
                "tiny_full_quadratic": {"flows_per_s": tq[0] / tq[1], "queries": tq[0],
                                        "seconds": round(tq[1], 3), "threads": threads},
                "slice_quadratic_1024": {"flows_per_s": q1k[0] / q1k[1], "queries": q1k[0],
                                         "seconds": round(q1k[1], 2), "threads": threads,
                                         "extrapolated_full_slice_s":
                                             round(q1k[1] * len(ev) / q1k[0], 1)}}}


def sampled_error(oracle, w, ev, A, mlp, flows, seed=903, count=2048):
    """Flow error against the FP64 oracle on `count` seeded events: relative
    L2 over the sample, the largest absolute error, and the 99.9th percentile
    of the per-event relative error."""
    from paper_2504_19417_amd import synth
    q = synth.sample_queries(len(ev), count, seed)
    e, _ = oracle.encode(ev, A, w.rx, w.ry, w.rt, queries=q)
    ref = oracle.mlp(e, *mlp)
    got = flows[q].astype(np.float64)
    d = np.linalg.norm(got - ref, axis=1)
    return {"flow_relL2_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "flow_maxabs_sampled": float(np.abs(got - ref).max()),
            "flow_row_rel_p999": float(np.percentile(d / np.maximum(np.linalg.norm(ref, axis=1),
                                                                    1e-300), 99.9)),
            "sampled_events": int(count)}


def serving_run(vk, seconds, pool=3, scale=1.0):
    """The serving workload: 32 streams (346x260 or 1280x720, Poisson event
    rates 0.5-10 Mev/s times `scale`, slice windows 1-20 ms, D = 128,
    r = 5/3, BF16 perceptron 256-256-2) replayed in real time for `seconds`:
    each stream's thread submits a slice every window (cycling over `pool`
    pre-generated slices) and polls its previous one.  Latency is measured by
    the server from submit to completion, overall and per sensor class;
    flows/s is completed flows over the span from the first submit to the
    last completion."""
    import dataclasses
    import threading
    from paper_2504_19417_amd import synth
    w = synth.workloads()["slice1m"]
    specs = [dataclasses.replace(sp, rate_mev_s=sp.rate_mev_s * scale)
             for sp in synth.serving_streams()]
    slices = [synth.stream_slices(sp, pool) for sp in specs]
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    per = [max(len(e) for e, _, _ in sl) for sl in slices]
    srv = vk.Server(1280, 720, w.rx, w.ry, w.rt, A, 20, int(sum(per)), "fp16",
                    hbm_budget_bytes=96 << 30, max_streams=len(specs), depth=4)
    srv.set_mlp(*mlp)
    sids = [srv.open_stream(sp.width, sp.height, sp.window_ms, n) for sp, n in zip(specs, per)]
    # warm-up: one slice of every stream
    for sid, sl in zip(sids, slices):
        ev, t0, T = sl[0]
        rc, _ = srv.poll(srv.submit(sid, ev, t0, T))
        if rc != vk.VECKM_OK:
            raise RuntimeError("serving warm-up failed: %d" % rc)
    srv.stats(reset=True)
    errors = []
    start = time.perf_counter() + 0.05

    def feed(i):
        sp, sid, sl = specs[i], sids[i], slices[i]
        prev, k = None, 0
        rng = np.random.Generator(np.random.PCG64(77 + i))
        t_next = start + rng.uniform(0.0, sp.window_ms * 1e-3)  # random phase
        while t_next < start + seconds:
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ev, t0, T = sl[k % len(sl)]
            try:
                ticket = srv.submit(sid, ev, t0, T)
            except vk.VeckmError as e:
                errors.append(e.code)
                break
            if prev is not None:
                rc, _ = srv.poll(prev)
                if rc != vk.VECKM_OK:
                    errors.append(rc)
            prev, k = ticket, k + 1
            t_next += sp.window_ms * 1e-3
        if prev is not None:
            rc, _ = srv.poll(prev)
            if rc != vk.VECKM_OK:
                errors.append(rc)

    th = [threading.Thread(target=feed, args=(i,)) for i in range(len(specs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    classes = {}
    for W, H in sorted({(sp.width, sp.height) for sp in specs}):
        c = srv.stats_sensor(W, H)
        classes["%dx%d" % (W, H)] = {
            "streams": sum(1 for sp in specs if (sp.width, sp.height) == (W, H)),
            "slices": c["slices"], "p50_ms": round(c["p50_ms"], 3),
            "p99_ms": round(c["p99_ms"], 3), "max_ms": round(c["max_ms"], 3)}
    st = srv.stats()
    for sid in sids:
        srv.close_stream(sid)
    srv.close()
    if errors:
        raise RuntimeError("serving errors: %s" % sorted(set(errors)))
    # offered event rate of the replayed slices (Mev/s)
    offered = sum(np.mean([len(e) for e, _, _ in sl]) / (sp.window_ms * 1e-3)
                  for sp, sl in zip(specs, slices)) / 1e6
    return {"streams": len(specs), "rate_scale": scale,
            "offered_mev_s": round(float(offered), 1),
            "seconds": seconds, "slices": st["slices"], "batches": st["batches"],
            "flows_per_s": st["flows"] / st["busy_s"] if st["busy_s"] > 0 else None,
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "max_ms": round(st["max_ms"], 3), "per_sensor": classes}


def serving_sweep(vk, seconds, scales=(0.5, 1.0, 2.0)):
    """The serving replay at x0.5, x1 and x2 of the stream rates: where the
    served rate stops tracking the offered rate the server is saturated."""
    pts = [serving_run(vk, seconds, scale=f) for f in scales]
    return {"points": pts,
            "latency": "submit to completion (host copies and device work included)",
            "dtype": "fp16 phase table, bf16 perceptron, fp32 accumulation",
            "served_over_offered": [round(p["flows_per_s"] / (p["offered_mev_s"] * 1e6), 3)
                                    if p["flows_per_s"] else None for p in pts]}


KERNEL_SOURCES = {  # kernel name prefix (template form) -> source file it is built from
    "k_encode<4": "paper_2504_19417_amd/csrc/kernels_encode.hip",   # FP32 form encoder
    "k_encode<2": "paper_2504_19417_amd/csrc/kernels_encode.hip",   # FP16 form encoder
    "k_mlp_res<2": "paper_2504_19417_amd/csrc/kernels_mlp.hip",     # FP32 form perceptron
    "k_mlp_split<": "paper_2504_19417_amd/csrc/kernels_mlp.hip",    # FP32 form, paper form
    "k_mlp_res<0": "paper_2504_19417_amd/csrc/kernels_mlp.hip",     # FP16 form perceptron
    "k_pool2d<": "paper_2504_19417_amd/csrc/kernels_paper.hip",     # paper form window sum
    "k_tphase<": "paper_2504_19417_amd/csrc/kernels_paper.hip",     # paper form phase sums
}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written


def source_sha(rel):
    import hashlib
    return hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters (scaled by the copy calibration), if they were taken
    on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    try:
        rec = json.load(open(TRAFFIC_JSON))["kernels"][kernel]
        if source_sha(rec["source"]) != rec["source_sha"]:
            return None
        return rec["hbm_bytes_per_launch"]
    except Exception:
        return None


def copy_calibration(torch):
    """A plain device copy of known size (elementwise negation of a 1 GiB
    float32 buffer into another), for scaling the HBM byte counters."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def _read_counters(path):
    """{kernel name: [mean counter value over dispatches, dispatches]} from a
    rocprofv3 counter_collection.csv holding one counter."""
    import csv
    acc = {}
    for row in csv.DictReader(open(path)):
        name = row["Kernel_Name"]
        a = acc.setdefault(name, [0.0, 0])
        a[0] += float(row["Counter_Value"])
        a[1] += 1
    return {k: [v[0] / v[1], v[1]] for k, v in acc.items()}


def _find_csv(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, d))


PROFILE_WORKLOADS = {
    "precision5m": "precision form (1280x720x100, 5M events with textured-blob noise, D=128, "
                   "r=5/3, perceptron 256-256-2), FP16/BF16 and FP32 forms",
    "batch64": "64-slice batch (lognormal 10k-500k events, 346x260 / 640x480, 50 bins, D=128, "
               "r=5/3, perceptron 256-256-2), FP16/BF16 and FP32 forms, tuned tiling",
    "slice1m": "1M-event slice (346x260x50, D=128, r=5/3, perceptron 256-256-2), "
               "FP32 and FP16/BF16 forms",
    "paper_k8": "paper form, 640x480 recipe (0.5M events, 32 bins, D=64, delta 8, no temporal "
                "bound, perceptron 128-128-2), FP32 and FP16/BF16 forms, all events and 10k "
                "queries",
    "paper_k10": "paper form, 640x480 recipe (0.5M events, 24 bins, D=64, delta 10, no temporal "
                 "bound, perceptron 128-128-2), FP32 and FP16/BF16 forms, all events and 10k "
                 "queries",
}
PROFILE_NOTES = {
    "slice1m": "As the bench runs it (the 10k-query run and serving skipped): each form "
               "warms up 50 steps, runs the tuner's trials of every tiling, warms up 50 more "
               "steps on the tuner's pick, times 20, then runs 20 with an event pair around "
               "each call and 20 with the library's stage timers; the averages are over each "
               "kernel's last 60 dispatches (those three passes; the first few tens of calls "
               "after start run up to 12 % slower).  The encoders run the "
               "perceptron themselves (template arguments: operand terms, slab tiles, wave "
               "layout, ring depth, row format): `k_encode<4, 8, 4, 2, 5>` is the FP32 form "
               "(16 waves, fp16 hi/lo operands, 32x16x8 brick), `k_encode<2, 8, 4, 2, 4>` the "
               "FP16/BF16 form (16 waves, bf16 perceptron, 32x16x16 brick); the other encoder "
               "instances are tuner trials; the front-end and expansion kernels serve both.  "
               "`__amd_rocclr_*` are runtime copies and fills outside the steps.",
    "paper_k8": "Three runs of 2 warm-up + 5 timed steps: FP32 form over all events, FP16/BF16 "
                "form over all events, FP32 form over the 10k-query subset (7 calls each).  "
                "`k_paper_rows<false>` and `k_mlp_split` serve the FP32 runs (all events and 10k "
                "queries: hence the min/max spread), `k_paper_rows<true>` and `k_mlp_res` the "
                "FP16/BF16 run; `k_tphase`, `k_pool2d`, the box sums and the prepare kernels "
                "serve all three.",
}
PROFILE_NOTES["paper_k10"] = PROFILE_NOTES["paper_k8"]
PROFILE_NOTES["precision5m"] = (
    "Each form runs the tuner (every tiling: 1 untimed + 2 timed runs of the front end, encoder "
    "and perceptron), 2 warm-up and 5 timed steps.  Template arguments of `k_encode`: operand "
    "terms (2: FP16/BF16 form, 4: FP32 form's hi/lo), slab tiles, wave layout, ring depth, row "
    "format (1: bf16 rows, 3: hi/lo rows, both for `k_mlp_res`; 4 and 5: perceptron inside the "
    "encoder, bf16 and hi/lo operands).  The fused `<2, 8, 4, 2, 4>` (16 waves, 32x32x8 brick "
    "in this run) and `<4, 8, 3, 2, 5>` (8 waves, 32x16x8 brick) are the tuner's picks and run "
    "the timed "
    "steps (the same template names also cover tuner trials on other bricks); the rest are "
    "tuner trials.  The brick scan runs as three launches (23,400 bricks: three 8192-brick "
    "tiles).")
PROFILE_NOTES["batch64"] = (
    "Each form runs the tuner (every tiling: 1 untimed + 2 timed runs of the front end, "
    "encoder and perceptron), 1 warm-up and 3 timed steps.  Template arguments of "
    "`k_encode`: operand terms (2: FP16/BF16 form, 4: FP32 form's hi/lo), slab tiles, wave "
    "layout, ring depth, row format (0-3: rows written for `k_mlp_res`; 4, 5: perceptron "
    "inside the encoder).  The tuner's picks on this batch write rows in wave layout 0: "
    "`k_encode<2, 8, 0, 2, 1>` (FP16 form, 32x32x8 brick) and `k_encode<4, 8, 0, 2, 3>` "
    "(FP32 form, 32x16x8), with `k_mlp_res` after them; the other encoder instances are "
    "tuner trials.  `k_rank_lines` ranks the flagged rows of the batch's bricks (a wave per "
    "brick: the batch is sparse), `k_clear_events` returns the grids to zero after each "
    "call, and the brick scan runs as three launches (`k_scan_totals`, `k_scan_tiles`, "
    "`k_scan_place`).  The front-end kernels serve both forms and the tuner runs.")


KERNELS_JSON = os.path.join(ROOT, "profiles", "kernels.json")


def record_kernel_times(rows, workload):
    """Keeps the rocprofv3 average duration of the hot kernels of `workload`
    (with the hash of their source) in profiles/kernels.json."""
    rec = json.load(open(KERNELS_JSON)) if os.path.exists(KERNELS_JSON) else {}
    out = {}
    for r in rows:
        for short, src in KERNEL_SOURCES.items():
            if ("veckm::%s" % short) in r["Name"] and short not in out:
                out[short] = {"kernel": r["Name"], "calls": int(r["Calls"]),
                              "avg_us": round(float(r["AverageNs"]) / 1e3, 2),
                              "source": src, "source_sha": source_sha(src)}
    rec[workload] = out
    with open(KERNELS_JSON, "w") as f:
        json.dump(rec, f, indent=1)


def profiled_ms(workload, kernel):
    """The committed rocprofv3 average of `kernel` (ms) on `workload`, if it
    was taken on the current source; else None."""
    try:
        r = json.load(open(KERNELS_JSON))[workload][kernel]
        return r["avg_us"] / 1e3 if source_sha(r["source"]) == r["source_sha"] else None
    except Exception:
        return None


def summarize_kernels(stats_dir, command, workload="slice1m", last=0):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run.  With
    last > 0 the table also gives each kernel's average over its last
    `last` dispatches (the timed steps, after warm-up and tuner trials),
    and that average is the one recorded for the bench's cross-check."""
    import csv
    rows = list(csv.DictReader(open(_find_csv(stats_dir, "kernel_stats.csv"))))
    tail = {}
    if last > 0:
        trace = list(csv.DictReader(open(_find_csv(stats_dir, "kernel_trace.csv"))))
        trace.sort(key=lambda r: int(r["Start_Timestamp"]))
        per = {}
        for r in trace:
            per.setdefault(r["Kernel_Name"], []).append(
                int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        tail = {k: sum(v[-last:]) / len(v[-last:]) for k, v in per.items()}
        for r in rows:
            if r["Name"] in tail:
                r["AverageNs"] = str(tail[r["Name"]])
                r["Calls"] = str(min(int(r["Calls"]), last))
    record_kernel_times(rows, workload)
    out = ["# Kernel times: " + PROFILE_WORKLOADS[workload], "",
           "Commands (R = repository root, one MI355X, ROCm 7.2):", ""]
    out += ["    " + c for c in command.split(" ; ")]
    head = "average (us)" if not last else "average of the last %d (us)" % last
    out += ["", PROFILE_NOTES[workload], "",
            "| kernel | calls | %s | min (us) | max (us) | share of GPU time |" % head,
            "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f %% |" % (
            r["Name"].replace("|", "\\|"), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def traffic_markdown(rec, workload="slice1m"):
    out = ["# HBM traffic per launch: " + PROFILE_WORKLOADS[workload], "",
           "Commands (R = repository root, one MI355X, ROCm 7.2):", ""]
    out += ["    " + c for c in rec["command"].split(" ; ")]
    out += ["", "Calibration: the same counters on a plain device copy of known size "
            "(`torch.neg` of a 1 GiB float32 buffer into another: 1 GiB read, 1 GiB written) "
            "read FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB per dispatch, so fetched "
            "bytes are scaled by %.4f and written bytes by %.4f.  The counters see the L2's "
            "traffic to the memory fabric (Infinity Cache hits included)."
            % (rec["copy_bytes"] / 1024 / rec["fetch_scale"], rec["copy_bytes"] / 1024 / rec["write_scale"],
               rec["fetch_scale"], rec["write_scale"]), "",
            "| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | bytes, scaled |",
            "|---|---:|---:|---:|---:|"]
    for k, v in rec["all"].items():
        out.append("| `%s` | %d | %.1f | %.1f | %d |" % (k.replace("|", "\\|")[:110], v["dispatches"],
                                                      v["fetch_kib"], v["write_kib"], v["hbm_bytes"]))
    return "\n".join(out) + "\n"


def summarize_traffic(fetch_dir, write_dir, command):
    """Writes the traffic summary: per-launch FETCH_SIZE and WRITE_SIZE (KiB)
    of each kernel, scaled by what the same counters read for the 1 GiB
    calibration copy."""
    fetch = _read_counters(_find_csv(fetch_dir, "counter_collection.csv"))
    write = _read_counters(_find_csv(write_dir, "counter_collection.csv"))
    copy = [k for k in fetch if "neg" in k.lower()]
    if len(copy) != 1:
        raise RuntimeError("calibration copy kernel not found uniquely: %s" % copy)
    kib = COPY_BYTES / 1024.0
    f_scale = kib / fetch[copy[0]][0]
    w_scale = kib / write[copy[0]][0]
    out = {"command": command, "copy_kernel": copy[0], "copy_bytes": COPY_BYTES,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}, "all": {}}
    for name in sorted(fetch):
        if name not in write:
            continue
        fk, wk = fetch[name][0], write[name][0]
        out["all"][name] = {"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                            "dispatches": fetch[name][1],
                            "hbm_bytes": int(round((fk * f_scale + wk * w_scale) * 1024))}
        for short, src in KERNEL_SOURCES.items():
            if ("veckm::%s" % short) in name:
                out["kernels"].setdefault(short, {
                    "kernel": name, "source": src, "source_sha": source_sha(src),
                    "fetch_kib_per_launch": round(fk, 1), "write_kib_per_launch": round(wk, 1),
                    "hbm_bytes_per_launch": out["all"][name]["hbm_bytes"]})
    return out


COUNTER_NOTES = {
    "MfmaUtil": "matrix cores busy, % of kernel time (SQ_VALU_MFMA_BUSY_CYCLES over "
                "GRBM_GUI_ACTIVE x 1024 SIMDs)",
    "MfmaFlopsF16": "fp16 matrix-core flops per dispatch (SQ_INSTS_VALU_MFMA_MOPS_F16 x 512)",
    "MfmaFlopsBF16": "bf16 matrix-core flops per dispatch (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512)",
    "LdsUtil": "LDS busy with indexed reads and writes, % of kernel time (SQ_LDS_IDX_ACTIVE)",
    "LdsBankConflict": "LDS cycles lost to bank conflicts per conflict-free LDS cycle "
                       "(SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT))",
    "TCC_HIT_sum": "L2 hits per dispatch", "TCC_MISS_sum": "L2 misses per dispatch",
    "TCP_TCC_READ_REQ_sum": "vector L1 -> L2 read requests per dispatch",
    "TCP_TCC_READ_REQ_LATENCY_sum": "summed latency of those requests (cycles)",
}


def summarize_counters(dirs, command, workload="slice1m"):
    """Markdown summary of rocprofv3 --pmc runs (derived and raw counters),
    one row per kernel of the library, counters averaged over dispatches."""
    import csv
    acc = {}
    for d in dirs:
        for row in csv.DictReader(open(_find_csv(d, "counter_collection.csv"))):
            name = row["Kernel_Name"]
            if "veckm::" not in name:
                continue
            c = acc.setdefault(name, {})
            v = c.setdefault(row["Counter_Name"], [0.0, 0])
            v[0] += float(row["Counter_Value"])
            v[1] += 1
    cols = [k for k in COUNTER_NOTES if any(k in c for c in acc.values())]
    out = ["# Hardware counters: " + PROFILE_WORKLOADS[workload], "",
           "Commands (R = repository root, one MI355X, ROCm 7.2; each --pmc pass is a run "
           "of its own):", ""]
    out += ["    " + c for c in command.split(" ; ")]
    out += ["", "Counters (averages over the dispatches of each kernel):", ""]
    out += ["* `%s`: %s" % (k, COUNTER_NOTES[k]) for k in cols]
    derived = "TCC_HIT_sum" in cols and "TCC_MISS_sum" in cols
    lat = "TCP_TCC_READ_REQ_sum" in cols and "TCP_TCC_READ_REQ_LATENCY_sum" in cols
    if derived:
        out.append("* L2 hit %: TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)")
    if lat:
        out.append("* L1->L2 read latency: TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum")
    head = ["kernel"] + ["`%s`" % k for k in cols] + (["L2 hit %"] if derived else []) + \
        (["L1->L2 read latency (cycles)"] if lat else [])
    out += ["", "| " + " | ".join(head) + " |", "|---|" + "---:|" * (len(head) - 1)]
    for name in sorted(acc):
        c = {k: v[0] / v[1] for k, v in acc[name].items()}
        cells = []
        for k in cols:
            v = c.get(k)
            cells.append("" if v is None else ("%.4g" % v))
        if derived:
            h, m = c.get("TCC_HIT_sum"), c.get("TCC_MISS_sum")
            cells.append("" if h is None or m is None or h + m == 0 else "%.1f" % (100 * h / (h + m)))
        if lat:
            r, l = c.get("TCP_TCC_READ_REQ_sum"), c.get("TCP_TCC_READ_REQ_LATENCY_sum")
            cells.append("" if not r or l is None else "%.0f" % (l / r))
        out.append("| `%s` | %s |" % (name.replace("|", "\\|")[:100], " | ".join(cells)))
    return "\n".join(out) + "\n"


def paper_main(args, name):
    """The paper's own form (no temporal bound) at one of its training
    recipes: 640x480, D = 64, delta-x = delta-y = 8 over 32 ms or 10 over
    24 ms, 0.5M events (the size of the paper's worked timing example), every
    event queried; then the worked example's 10k-flow query set."""
    import torch
    import oracle
    from paper_2504_19417_amd import synth, veckm as vk

    w = synth.workloads()[name]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt, nbins=T)
    mlp = synth.init_mlp(w.d, w.hidden)
    n = len(ev)
    W, H = w.slices[0].width, w.slices[0].height
    res = {f: run_form(vk, torch, w, ev, t0, T, A, mlp, f, args.steps, args.warmup)
           for f in ("fp32", "fp16")}
    q10k = synth.sample_queries(n, 10_000, 79)
    sparse = run_form(vk, torch, w, ev, t0, T, A, mlp, "fp32", args.steps, args.warmup,
                      queries=q10k)

    def stages(r):
        return {k: (round(v[0] / v[1], 4) if v[1] else None) for k, v in r["stages"].items()}

    st32, st16 = stages(res["fp32"]), stages(res["fp16"])
    rows = res["fp32"]["rows"]
    enc_bytes = paper_encode_bytes(W, H, T, w.d, rows, 2 * w.d * 4)
    cand = {
        "encode": dict(ms=st32["encode"], bound="hbm", amount=enc_bytes / 1e9,
                       peak=PEAK["hbm_GBps"], unit="GB/s",
                       kernel="paper encode stage (k_tphase, k_pool2d, k_boxx, k_boxy, "
                              "k_paper_rows)"),
        "mlp": dict(ms=st32["mlp"], bound="mfma", amount=mlp_flops_per_row(w.d, w.hidden) * rows / 1e12,
                    peak=PEAK["fp16_TFLOPs"], unit="TFLOP/s", kernel="k_mlp_split<"),
    }
    dom = max(cand, key=lambda k: cand[k]["ms"])
    c = cand[dom]
    achieved = c["amount"] / (c["ms"] * 1e-3)
    roofline = {"bound": c["bound"], "achieved": round(achieved, 2), "peak": c["peak"],
                "unit": c["unit"], "frac": round(achieved / c["peak"], 4), "traffic": None,
                "kernel": c["kernel"], "avg_launch_ms": c["ms"], "rows_per_launch": rows}
    err32 = sampled_error(oracle, w, ev, A, mlp, res["fp32"]["flows"])
    err16 = sampled_error(oracle, w, ev, A, mlp, res["fp16"]["flows"])
    cpu = None if args.no_cpu_baseline else cpu_baseline(oracle, w, ev, A, mlp, args.cpu_seconds)
    ms_sparse = sparse["elapsed"] / args.steps * 1e3
    line = {
        "metric": "normal flows/sec, paper form (no temporal bound), 640x480 D=64 recipe",
        "value": n * args.steps / res["fp32"]["elapsed"],
        "unit": "flows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["fp32"]["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (fp32 encoder; fp16 hi/lo perceptron operands)",
        "data": "synthetic (seeded moving edges + 10% uniform noise)",
        "config": {"workload": name, "sensor": "%dx%d" % (W, H), "events": n, "bins": T,
                   "d": w.d, "radius_xy": w.rx, "radius_t": "none (whole slice)",
                   "delta_t_bins": T / 2, "hidden": w.hidden, "queries": "all events"},
        "stages_ms": st32,
        "err_vs_oracle": err32,
        "fp16_bf16": {"value": n * args.steps / res["fp16"]["elapsed"],
                      "ms_per_step": round(res["fp16"]["elapsed"] / args.steps * 1e3, 4),
                      "stages_ms": st16, "err_vs_oracle": err16,
                      "dtype": "fp32 encoder, bf16 perceptron"},
        "worked_example_10k_flows": {"ms_per_call": round(ms_sparse, 4),
                                     "stages_ms": stages(sparse),
                                     "paper_estimate_ms_rtx2080ti_r8": 7.04},
        "eqn18": eqn18_split(n, 10_000, ms_sparse, res["fp32"]["elapsed"] / args.steps * 1e3),
        "rows": rows,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration:
        copy_calibration(torch)


def window_main(args):
    """The sliding-window encoder on the 1M-event recording (346x260, 50 bins,
    D = 128, r = 5/3): the window holds 2 rt + 1 = 7 bins; each step pushes
    the next bin's events and computes the flows of the events rt bins back,
    whose neighbourhoods are then complete (a live stream's steady state)."""
    import torch
    import oracle
    from paper_2504_19417_amd import synth, veckm as vk

    w = synth.workloads()["slice1m"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    tw = 2 * w.rt + 1
    bins = [np.ascontiguousarray(ev[ev[:, 2] == t0 + b]) for b in range(T)]
    per = max(len(b) for b in bins)
    res = {}
    for form in ("fp32", "fp16"):
        win = vk.Window(346, 260, w.rx, w.ry, w.rt, A, tw, per, form)
        win.set_mlp(*mlp)
        dev = [torch.from_numpy(b).cuda() for b in bins]
        outs = [torch.empty((len(b), 2), device="cuda") for b in bins]
        stream = torch.cuda.current_stream()

        def step(b):
            win.push(dev[b], t0 + b, 1)
            if b >= w.rt:
                win.flow_window(dev[b - w.rt], out=outs[b - w.rt])

        for b in range(T):  # warm-up pass over the recording
            step(b)
        torch.cuda.synchronize()
        if win.status() != vk.VECKM_OK:
            raise RuntimeError("input error reported by the device")
        rounds = max(1, args.steps // T)
        t_start = time.perf_counter()
        flows = 0
        for r in range(rounds):
            win.close()
            win = vk.Window(346, 260, w.rx, w.ry, w.rt, A, tw, per, form)
            win.set_mlp(*mlp)
            torch.cuda.synchronize()
            t_r = time.perf_counter()
            for b in range(T):
                step(b)
            torch.cuda.synchronize()
            flows += sum(len(bins[b]) for b in range(T - w.rt))
            res.setdefault(form, []).append(time.perf_counter() - t_r)
        st = win.status()
        win.close()
        if st != vk.VECKM_OK:
            raise RuntimeError("input error reported by the device")
        res[form] = dict(seconds=sum(res[form]), flows=flows, steps=T * rounds,
                         flows_np=torch.cat(outs[:T - w.rt]).cpu().numpy())
    # the streamed flows equal the oracle's over the 7-bin windows (sampled)
    rng = np.random.Generator(np.random.PCG64(905))
    errs = []
    for b in rng.choice(np.arange(w.rt, T - w.rt), 3, replace=False):
        lo = max(0, b - w.rt)
        wev = np.ascontiguousarray(np.concatenate(bins[lo:b + w.rt + 1]))
        off = sum(len(x) for x in bins[lo:b])
        q = off + rng.choice(len(bins[b]), 300, replace=False)
        e, _ = oracle.encode(wev, A, w.rx, w.ry, w.rt, queries=q)
        ref = oracle.mlp(e, *mlp)
        base = sum(len(x) for x in bins[:b])
        f32 = res["fp32"]["flows_np"][base + (q - off)]
        errs.append(float(np.linalg.norm(f32 - ref) / np.linalg.norm(ref)))
    line = {
        "metric": "normal flows/sec, sliding-window streaming encoder (push one bin, flow the "
                  "bin rt back)",
        "value": res["fp32"]["flows"] / res["fp32"]["seconds"],
        "unit": "flows/s", "n_gpus": 1, "steps": res["fp32"]["steps"], "warmup": T,
        "ms_per_step": round(res["fp32"]["seconds"] / res["fp32"]["steps"] * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (fp32 sums; 22-bit operands)",
        "data": "synthetic (the 1M-event 346x260x50 recording, one 1 ms bin per step)",
        "config": {"workload": "window", "sensor": "346x260", "events": int(len(ev)),
                   "bins": T, "window_bins": tw, "d": w.d, "radius_xy": w.rx,
                   "radius_t": w.rt, "hidden": w.hidden,
                   "per_step": "push ~20k events of one bin, flows of the bin rt back"},
        "fp16_bf16": {"value": res["fp16"]["flows"] / res["fp16"]["seconds"],
                      "ms_per_step": round(res["fp16"]["seconds"] / res["fp16"]["steps"] * 1e3, 4)},
        "err_vs_oracle": {"flow_relL2_sampled_fp32": max(errs)},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def batch_main(args):
    """The batched form: 64 slices in one launch sequence per step, every
    event queried, D = 128, r = 5/3, 50 bins, 346x260 and 640x480 sensors.
    `batch64`: lognormal 10k-500k events per slice; `batch64x10k`: 10k events
    per slice (launch overhead dominates).  Each form (FP16/BF16, the
    configuration's precision, and FP32) is timed twice on the same inputs:
    replaying the launch graph captured for the batch (the timed value) and
    calling flow_batch eagerly; the two give bit-identical flows."""
    import torch
    import oracle
    from paper_2504_19417_amd import synth, veckm as vk

    wl = args.workload
    w = synth.workloads()[wl]
    parts = [synth.make_slice(s) for s in w.slices]
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    specs = [(s.width, s.height, t0, T, len(e)) for s, (e, t0, T) in zip(w.slices, parts)]
    ev = np.concatenate([p[0] for p in parts]).astype(np.int32)
    n = len(ev)
    evt = torch.from_numpy(ev).cuda()
    res = {}
    for form in ("fp16", "fp32"):
        c = vk.Context(640, 480, w.rx, w.ry, w.rt, A, 50, n, form, max_slices=64)
        c.set_mlp(*mlp)
        # the encoder tiling for this batch, picked by the library's tuner
        # (set-up, outside the timed region)
        tiling = c.tilings()[c.tune(specs, evt, reps=2)]
        out = torch.empty((n, 2), device="cuda")
        for _ in range(args.warmup):
            c.flow_batch(specs, evt, out=out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            c.flow_batch(specs, evt, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        # the stage split, from the library's stage timers (after the timed
        # steps: their event records add to each call)
        c.profile(True)
        c.profile_read()
        for _ in range(args.steps):
            c.flow_batch(specs, evt, out=out)
        torch.cuda.synchronize()
        st = {k: (round(v[0] / v[1], 4) if v[1] else None) for k, v in c.profile_read().items()}
        c.profile(False)
        status = c.status()
        rows = c.last_rows()
        flows = out.cpu().numpy()
        # the same batch through its captured launch graph
        gout = torch.empty((n, 2), device="cuda")
        g = c.graph(specs, evt, gout, flow=True)
        for _ in range(args.warmup):
            g.launch()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            g.launch()
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t) / args.steps
        gflows = gout.cpu().numpy()
        g.close()
        status = status or c.status()
        c.close()
        if status != vk.VECKM_OK:
            raise RuntimeError("input error reported by the device")
        if not np.array_equal(gflows, flows):
            raise RuntimeError("graph replay differs from the eager batch call")
        # 16 sampled events per slice against the oracle
        got, ref, off = [], [], 0
        for k, (e, t0, T) in enumerate(parts):
            q = synth.sample_queries(len(e), 16, 600 + k)
            emb, _ = oracle.encode(e, A, w.rx, w.ry, w.rt, queries=q)
            ref.append(oracle.mlp(emb, *mlp))
            got.append(flows[off + q])
            off += len(e)
        got, ref = np.concatenate(got).astype(np.float64), np.concatenate(ref)
        res[form] = dict(value=n / dtg, ms=dtg * 1e3, eager_value=n / dt, eager_ms=dt * 1e3,
                         stages=st, tiling=list(tiling), rows=rows,
                         err=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    # the encoder (the dominant kernel) against the fp16 matrix-core peak
    K = ((2 * w.rx + 1) * (2 * w.ry + 1) * (2 * w.rt + 1) + 1) // 2
    r16 = res["fp16"]
    fpr, fused = encode_stage_flops_per_row(K, w.d, w.hidden, r16["stages"])
    achieved = fpr * r16["rows"] / (r16["stages"]["encode"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["fp16_TFLOPs"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK["fp16_TFLOPs"], 4),
                "traffic": None, "kernel": "k_encode<2", "avg_launch_ms": r16["stages"]["encode"],
                "rows_per_launch": r16["rows"], "flops_per_row": fpr,
                "perceptron_in_encoder": fused}
    sizes = "lognormal 10k-500k events" if wl == "batch64" else "10k events each"

    def eager(r):
        return {"value": r["eager_value"], "ms_per_step": round(r["eager_ms"], 4)}

    line = {
        "metric": "normal flows/sec, 64-slice batch replayed as one captured launch graph "
                  "(BF16 perceptron)",
        "value": res["fp16"]["value"], "unit": "flows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(res["fp16"]["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp16 phase table, bf16 perceptron, fp32 accumulation",
        "data": "synthetic (seeded moving edges + 10% uniform noise, 64 slices)",
        "config": {"workload": wl, "slices": 64, "events": n, "slice_sizes": sizes,
                   "sensors": "346x260 / 640x480", "bins": 50, "d": w.d, "radius_xy": w.rx,
                   "radius_t": w.rt, "hidden": w.hidden, "queries": "all events",
                   "tiling_brick_slabs": res["fp16"]["tiling"]},
        "eager_flow_batch": eager(res["fp16"]),
        "stages_ms": res["fp16"]["stages"],
        "err_vs_oracle": {"flow_relL2_sampled": res["fp16"]["err"]},
        "fp32": {"value": res["fp32"]["value"], "ms_per_step": round(res["fp32"]["ms"], 4),
                 "eager_flow_batch": eager(res["fp32"]),
                 "stages_ms": res["fp32"]["stages"], "tiling_brick_slabs": res["fp32"]["tiling"],
                 "err_vs_oracle": {"flow_relL2_sampled": res["fp32"]["err"]}},
        "roofline": roofline, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def precision_main(args):
    """The precision form: one 1280x720 slice of 5M events (64 moving edges
    plus textured-blob noise), 100 bins, D = 128, r = 5/3, every event
    queried; the FP16/BF16 form timed and compared with the FP32 form (whole
    slice) and with the FP64 oracle (sampled events)."""
    import torch
    import oracle
    from paper_2504_19417_amd import synth, veckm as vk

    w = synth.workloads()["precision5m"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    n = len(ev)
    res = {f: run_form(vk, torch, w, ev, t0, T, A, mlp, f, args.steps, args.warmup, tune=True)
           for f in ("fp16", "fp32")}

    def stages(r):
        return {k: (round(v[0] / v[1], 4) if v[1] else None) for k, v in r["stages"].items()}

    st16, st32 = stages(res["fp16"]), stages(res["fp32"])
    err16 = sampled_error(oracle, w, ev, A, mlp, res["fp16"]["flows"])
    err32 = sampled_error(oracle, w, ev, A, mlp, res["fp32"]["flows"])
    f16 = res["fp16"]["flows"].astype(np.float64)
    f32 = res["fp32"]["flows"].astype(np.float64)
    vs32 = float(np.linalg.norm(f16 - f32) / np.linalg.norm(f32))
    K = ((2 * w.rx + 1) * (2 * w.ry + 1) * (2 * w.rt + 1) + 1) // 2
    rows = res["fp16"]["rows"]
    fpr, fused = encode_stage_flops_per_row(K, w.d, w.hidden, st16)
    achieved = fpr * rows / (st16["encode"] * 1e-3) / 1e12
    line = {
        "metric": "normal flows/sec, precision form (FP16 grid, BF16 perceptron) at 5M events",
        "value": n * args.steps / res["fp16"]["elapsed"], "unit": "flows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["fp16"]["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp16 phase table, bf16 perceptron, fp32 accumulation",
        "data": "synthetic (seeded moving edges + textured-blob noise)",
        "config": {"workload": "precision5m", "sensor": "1280x720", "events": n, "bins": T,
                   "d": w.d, "radius_xy": w.rx, "radius_t": w.rt, "hidden": w.hidden,
                   "queries": "all events", "tiling_brick_slabs": res["fp16"]["tiling"]},
        "stages_ms": st16, "rows": rows,
        "err_vs_oracle": err16,
        "flow_relL2_vs_fp32_form": vs32,
        "fp32": {"value": n * args.steps / res["fp32"]["elapsed"],
                 "ms_per_step": round(res["fp32"]["elapsed"] / args.steps * 1e3, 4),
                 "stages_ms": st32, "tiling_brick_slabs": res["fp32"]["tiling"],
                 "err_vs_oracle": err32},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2),
                     "peak": PEAK["fp16_TFLOPs"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK["fp16_TFLOPs"], 4), "traffic": None,
                     "kernel": "k_encode<2", "avg_launch_ms": st16["encode"],
                     "rows_per_launch": rows, "flops_per_row": fpr,
                     "perceptron_in_encoder": fused},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def train_main(args):
    """Training the perceptron on the 1M-event slice's edge events (about 0.9M
    rows of FP32 encodings, D = 128, hidden 256, their true normal flows):
    one Adam step over all rows per step."""
    import torch
    from paper_2504_19417_amd import synth, veckm as vk

    w = synth.workloads()["slice1m"]
    ev, t0, T, f = synth.make_slice(w.slices[0], with_flow=True)
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    ctx = vk.Context(346, 260, w.rx, w.ry, w.rt, A, T, len(ev))
    emb = ctx.encode(torch.from_numpy(ev).cuda(), t0, T)
    torch.cuda.synchronize()
    keep = np.nonzero(~np.isnan(f[:, 0]))[0]
    x = emb[torch.from_numpy(keep).cuda()].contiguous()
    del emb
    y = torch.from_numpy(f[keep].astype(np.float32)).cuda()
    ctx.close()
    m = len(keep)
    tr = vk.Trainer(w.d, w.hidden, m, *synth.init_mlp(w.d, w.hidden))
    loss = torch.zeros(1, device="cuda")
    for _ in range(args.warmup):
        tr.step(x, y, "adam", 1e-3, loss)
    torch.cuda.synchronize()
    l0 = float(loss.cpu()[0])
    t = time.perf_counter()
    for _ in range(args.steps):
        tr.step(x, y, "adam", 1e-3, loss)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    l1 = float(loss.cpu()[0])
    tr.close()
    k2, hid = 2 * w.d, w.hidden
    flops = m * (2 * k2 * hid * 2 + 8 * hid + 16)  # layer 1 forward, dW1, layer 2 and its way back
    line = {
        "metric": "perceptron training rows/sec (one Adam step over the slice's edge events)",
        "value": m / dt, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (encodings of the 1M-event slice's edge events, true normal flows)",
        "config": {"workload": "train", "rows": m, "d": w.d, "hidden": hid,
                   "optimizer": "adam", "lr": 1e-3},
        "loss": {"after_warmup": l0, "after_steps": l1},
        "roofline": {"bound": "alu", "achieved": round(flops / dt / 1e12, 2),
                     "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(flops / dt / 1e12 / 78.6, 4), "traffic": None,
                     "kernel": "training step (fp32 FMA GEMMs on the vector ALU, without "
                               "packed-fp32 instructions: 256 CUs x 4 SIMDs x 16 lanes x 2 flops "
                               "x 2.4 GHz = 78.6 TFLOP/s)"},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="slice1m",
                    choices=["slice1m", "paper_k8", "paper_k10", "window", "train", "batch64",
                             "batch64x10k", "precision5m"],
                    help="slice1m: the bounded-window 1M-event slice (the headline line); "
                         "paper_k8 / paper_k10: the paper's own form at its recipes")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the 10k-query run (profiling runs: one call size per kernel)")
    ap.add_argument("--no-tune", action="store_true",
                    help="slice1m: keep each form's default encoder tiling instead of the "
                         "tuner's pick (profiling runs: no tuner trials among the kernels)")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="real-time replay of the 32-stream serving workload (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 1 GiB on the device (counter calibration)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) "
                         "into profiles/traffic_<workload>.md (and, for slice1m, "
                         "profiles/traffic.json) and exit (no GPU needed)")
    ap.add_argument("--summarize-kernels", metavar="STATS_DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats run into "
                         "profiles/kernels_<workload>.md and exit (no GPU needed)")
    ap.add_argument("--last", type=int, default=0,
                    help="with --summarize-kernels: average each kernel over its last N "
                         "dispatches (the timed steps)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_DIR",
                    help="summarise rocprofv3 --pmc runs (MFMA, LDS and L2 counters) into "
                         "profiles/counters_<workload>.md and exit (no GPU needed)")
    ap.add_argument("--command", default="", help="commands recorded with the summaries "
                                                  "(separated by ' ; ')")
    args = ap.parse_args()
    if args.summarize_traffic or args.summarize_kernels or args.summarize_counters:
        wl = args.workload
        if args.summarize_counters:
            with open(os.path.join(ROOT, "profiles", "counters_%s.md" % wl), "w") as f:
                f.write(summarize_counters(args.summarize_counters, args.command, wl))
        if args.summarize_traffic:
            rec = summarize_traffic(*args.summarize_traffic, args.command)
            if wl == "slice1m":  # the headline line's roofline reads this record
                with open(TRAFFIC_JSON, "w") as f:
                    json.dump(rec, f, indent=1)
            with open(os.path.join(ROOT, "profiles", "traffic_%s.md" % wl), "w") as f:
                f.write(traffic_markdown(rec, wl))
            print(json.dumps(rec["kernels"], indent=1))
        if args.summarize_kernels:
            text = summarize_kernels(args.summarize_kernels, args.command, wl, args.last)
            with open(os.path.join(ROOT, "profiles", "kernels_%s.md" % wl), "w") as f:
                f.write(text)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent slices shard across GPUs with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "window":
        window_main(args)
        return
    if args.workload == "train":
        train_main(args)
        return
    if args.workload in ("batch64", "batch64x10k"):
        batch_main(args)
        return
    if args.workload == "precision5m":
        precision_main(args)
        return
    if args.workload != "slice1m":
        paper_main(args, args.workload)
        return

    import torch
    import oracle
    from paper_2504_19417_amd import synth, veckm as vk

    w = synth.workloads()["slice1m"]
    ev, t0, T = synth.make_slice(w.slices[0])
    A = synth.draw_frequencies(w.d, w.rx, w.ry, w.rt)
    mlp = synth.init_mlp(w.d, w.hidden)
    K = ((2 * w.rx + 1) * (2 * w.ry + 1) * (2 * w.rt + 1) + 1) // 2
    n = len(ev)

    res = {}
    for form in ("fp32", "fp16"):
        # the encoder tiling picked by the library's tuner (set-up, not timed)
        res[form] = run_form(vk, torch, w, ev, t0, T, A, mlp, form, args.steps, args.warmup,
                             tune=not args.no_tune)
    # sparse query set (Eqn. 18's C m term shrinks, the c n term stays)
    sparse = None
    if not args.no_sparse:
        q10k = synth.sample_queries(n, 10_000, 79)
        sparse = run_form(vk, torch, w, ev, t0, T, A, mlp, "fp32", args.steps, args.warmup,
                          queries=q10k)
        ms_sparse = sparse["elapsed"] / args.steps * 1e3

    def summary(r):
        ms = r["elapsed"] / args.steps * 1e3
        st = {k: (v[0] / v[1] if v[1] else None) for k, v in r["stages"].items()}
        return ms, st

    ms32, st32 = summary(res["fp32"])
    ms16, st16 = summary(res["fp16"])
    rows = res["fp32"]["rows"]

    # dominant kernel of the FP32 form, from the live per-stage event times
    # (the encoder, which also runs the perceptron when no perceptron stage
    # was timed)
    fpr, fused = encode_stage_flops_per_row(K, w.d, w.hidden, st32)
    cand = {
        "encode": dict(ms=st32["encode"], flops=fpr * rows,
                       peak=PEAK["fp16_TFLOPs"], kernel="k_encode<4"),
    }
    if not fused:
        # FP32-form perceptron: fp16 hi/lo operand pairs on the fp16 matrix cores
        cand["mlp"] = dict(ms=st32["mlp"], flops=mlp_flops_per_row(w.d, w.hidden) * rows,
                           peak=PEAK["fp16_TFLOPs"], kernel="k_mlp_res<2")
    dom = max(cand, key=lambda k: cand[k]["ms"])
    c = cand[dom]
    achieved = c["flops"] / (c["ms"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": c["peak"],
                "unit": "TFLOP/s", "frac": round(achieved / c["peak"], 4),
                "traffic": load_traffic(c["kernel"]), "kernel": c["kernel"],
                "avg_launch_ms": round(c["ms"], 4), "rows_per_launch": rows,
                "flops_per_row": c["flops"] // rows, "perceptron_in_encoder": fused,
                "clock": "HIP events around the kernel's launch on its stream"}
    # the same figure from the committed rocprofv3 kernel trace of this source
    pms = profiled_ms("slice1m", c["kernel"])
    if pms:
        roofline["rocprof_avg_ms"] = round(pms, 4)
        roofline["rocprof_frac"] = round(c["flops"] / (pms * 1e-3) / 1e12 / c["peak"], 4)

    err32 = sampled_error(oracle, w, ev, A, mlp, res["fp32"]["flows"])
    err16 = sampled_error(oracle, w, ev, A, mlp, res["fp16"]["flows"])
    serving = serving_sweep(vk, args.serving_seconds) if args.serving_seconds > 0 else None
    cpu = None if args.no_cpu_baseline else cpu_baseline(oracle, w, ev, A, mlp, args.cpu_seconds)

    def lat(r):
        return {"p50": round(float(np.percentile(r["lat"], 50)), 4),
                "p99": round(float(np.percentile(r["lat"], 99)), 4)}

    line = {
        "metric": "normal flows/sec at 1M-event slices (FP32 vs BF16); p99 slice latency",
        "value": n * args.steps / res["fp32"]["elapsed"],
        "unit": "flows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (fp32 sums; 22-bit operands: exact counts, fp16 hi/lo phase table, "
                 "fp16 hi/lo perceptron operands)",
        "data": "synthetic (seeded moving edges + 10% uniform noise)",
        "config": {"workload": "slice1m", "sensor": "346x260", "events": n, "bins": T,
                   "d": w.d, "radius_xy": w.rx, "radius_t": w.rt, "hidden": w.hidden,
                   "queries": "all events", "tiling_brick_slabs": res["fp32"]["tiling"]},
        "latency_ms": lat(res["fp32"]),
        "err_vs_oracle": err32,
        "stages_ms": {k: (round(v, 4) if v is not None else None) for k, v in st32.items()},
        "fp16_bf16": {
            "value": n * args.steps / res["fp16"]["elapsed"],
            "ms_per_step": round(ms16, 4),
            "latency_ms": lat(res["fp16"]),
            "stages_ms": {k: (round(v, 4) if v is not None else None) for k, v in st16.items()},
            "err_vs_oracle": err16,
            "dtype": "fp16 phase table, bf16 perceptron, fp32 accumulation",
            "tiling_brick_slabs": res["fp16"]["tiling"],
        },
        "sparse_10k_queries": None if sparse is None else {
            "ms_per_call": round(ms_sparse, 4),
            "stages_ms": {k: (round(v[0] / v[1], 4) if v[1] else None)
                          for k, v in sparse["stages"].items()},
            "eqn18": eqn18_split(n, 10_000, ms_sparse, ms32)},
        "rows": rows,
        "roofline": roofline,
        "serving": serving,
        "cpu_baseline": cpu,
        "paper_context_flows_per_s": {"rtx3070": 4e6, "rtx_a5000": 6e6},
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration:
        copy_calibration(torch)


if __name__ == "__main__":
    main()
