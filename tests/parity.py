"""Error measures and tolerances shared by the GPU parity tests.

Tolerances of the whole-array comparison (relative L2 against the FP64
oracle) are the stated targets: FP32 form <= 1e-4 on encodings and <= 1e-3
on flows; the FP16/BF16 form is reported, and held to 2e-3 / 3e-2.

Per-element bounds on encodings, derived from the arithmetic (the count
operands are exact integers and every product is exact in fp32, so only the
table and the fp32 sums round):
  * table: each offset phase is an fp16 hi + lo pair within 2^-22 of the
    FP64 value (FP32 form) or one fp16 within 2^-11 (FP16 form); summed over
    the window and divided by the count this moves an element by at most
    that much.
  * sums: an element of S is a sum of n products (n = the padded half-window
    slots KP, twice that in the FP32 form: hi and lo terms) whose absolute
    values add up to at most twice the count N (the pair sums add up to N
    plus the centre's count), so fp32 summation in any order is off by at
    most n 2^-24 2N, i.e. 2 n 2^-24 after the division by N.
  So enc_maxabs = table + 2 n 2^-24: 1.15e-4 (FP32 form) and 5.4e-4 (FP16
  form) at r = 5/3 (KP = 480).  These are worst cases; measured errors are
  orders of magnitude below.
Per-row bounds: every sampled row's error norm, relative to the RMS row norm
of the sample, must meet the whole-array tolerance (so a defect confined to
a few rows cannot hide in an aggregate); the 99.9th percentile of the
per-row relative error is reported.
"""
import numpy as np

EMB_REL = {"fp32": 1e-4, "fp16": 2e-3}
FLOW_REL = {"fp32": 1e-3, "fp16": 3e-2}


def enc_maxabs(precision, kp=480):
    table = 2.0 ** -22 if precision == "fp32" else 2.0 ** -11
    terms = 2 * kp if precision == "fp32" else kp
    return table + 2 * terms * 2.0 ** -24


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def row_errors(got, ref):
    """(per-row error norm / RMS row norm, per-row relative error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    e = np.linalg.norm(got - ref, axis=1)
    n = np.linalg.norm(ref, axis=1)
    rms = max(float(np.sqrt(np.mean(n * n))), 1e-300)
    return e / rms, e / np.maximum(n, 1e-300)


def check(got, ref, precision, what, kp=480, say=None):
    """Whole-array, per-row and (encodings) per-element checks; returns a
    summary dict of the measured errors."""
    tol = EMB_REL[precision] if what == "emb" else FLOW_REL[precision]
    agg = rel_l2(got, ref)
    per_rms, per_rel = row_errors(got, ref)
    maxabs = float(np.abs(np.asarray(got, np.float64) - ref).max()) if len(ref) else 0.0
    out = dict(relL2=agg, row_max=float(per_rms.max()) if len(ref) else 0.0,
               row_rel_p999=float(np.percentile(per_rel, 99.9)) if len(ref) else 0.0,
               maxabs=maxabs)
    if say:
        say("%s %s: relL2 %.3e  worst row %.3e  row p99.9 %.3e  maxabs %.3e" % (
            what, precision, agg, out["row_max"], out["row_rel_p999"], maxabs))
    assert agg <= tol, (what, precision, agg)
    assert out["row_max"] <= tol, (what, precision, out["row_max"])
    if what == "emb":
        assert maxabs <= enc_maxabs(precision, kp), (what, precision, maxabs)
    return out


def padded_slots(rx, ry, rt):
    """Slots of the encoder's half window: the centre row (dx = 0..rx) and
    every other window row of the positive half (2 rx + 1 offsets), each
    padded to a multiple of 4, the total to a multiple of 32."""
    row = lambda k: (k + 3) // 4 * 4
    n = row(rx + 1) + (ry + rt * (2 * ry + 1)) * row(2 * rx + 1)
    return (n + 31) // 32 * 32
