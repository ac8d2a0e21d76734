"""The seeded input generator: determinism, shapes and ranges."""
import numpy as np
import pytest

from paper_2504_19417_amd import synth


def test_workload_table():
    w = synth.workloads()
    assert set(w) >= {"tiny", "slice1m", "precision5m", "batch64"}
    assert w["tiny"].d == 64 and (w["tiny"].rx, w["tiny"].ry, w["tiny"].rt) == (3, 3, 2)
    assert w["slice1m"].slices[0].n == 1_000_000 and w["slice1m"].d == 128
    b = w["batch64"].slices
    assert len(b) == 64
    sizes = np.array([s.n for s in b])
    assert sizes.min() >= 10_000 and sizes.max() <= 500_000
    assert {(s.width, s.height) for s in b} == {(346, 260), (640, 480)}
    for name, r, T in (("paper_k8", 8, 32), ("paper_k10", 10, 24)):
        p = w[name]
        assert (p.rx, p.ry, p.rt, p.d) == (r, r, -1, 64)
        s = p.slices[0]
        assert (s.width, s.height, s.nbins, s.n) == (640, 480, T, 500_000)


def test_slice_is_deterministic_and_in_range():
    spec = synth.workloads()["tiny"].slices[0]
    ev1, t0, T = synth.make_slice(spec)
    ev2, _, _ = synth.make_slice(spec)
    assert np.array_equal(ev1, ev2)
    assert ev1.dtype == np.int32 and ev1.shape == (spec.n, 4)
    assert ev1[:, 0].min() >= 0 and ev1[:, 0].max() < spec.width
    assert ev1[:, 1].min() >= 0 and ev1[:, 1].max() < spec.height
    assert ev1[:, 2].min() >= t0 and ev1[:, 2].max() < t0 + T
    assert set(np.unique(ev1[:, 3])) <= {-1, 1}
    assert np.all(np.diff(ev1[:, 2]) >= 0)  # camera (time) order


def test_blob_noise_slice_small():
    spec = synth.SliceSpec(200, 120, 20, 20_000, 6, blob_noise=True, seed=9)
    ev, t0, T = synth.make_slice(spec)
    assert ev.shape == (20_000, 4)
    assert ev[:, 0].max() < 200 and ev[:, 1].max() < 120


def test_frequencies_follow_algorithm1_draw():
    A = synth.draw_frequencies(4096, 5, 5, 3)
    # seeds 0,1,2 for T, X, Y; variance 25 before division by the radius
    z_t = np.random.Generator(np.random.PCG64(0)).normal(size=4096)
    assert np.allclose(A[:, 2], 5 * z_t / 3)
    assert abs(np.var(A[:, 0] * 5) - 25) < 2.5
    # no temporal bound: delta-t is half the slice length
    A2 = synth.draw_frequencies(16, 5, 5, -1, nbins=50)
    assert np.allclose(A2[:, 2], 5 * z_t[:16] / 25)


def test_mlp_init_layout():
    W1, b1, W2, b2 = synth.init_mlp(64, 128)
    assert W1.shape == (128, 128) and b1.shape == (128,)
    assert W2.shape == (2, 128) and b2.shape == (2,)
    assert W1.dtype == np.float32
    assert np.abs(W1).max() <= 1 / np.sqrt(128)


def test_sample_queries():
    q = synth.sample_queries(1000, 100, 1)
    assert len(np.unique(q)) == 100 and q.min() >= 0 and q.max() < 1000
    assert np.array_equal(q, synth.sample_queries(1000, 100, 1))
