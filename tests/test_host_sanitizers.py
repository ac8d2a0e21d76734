"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two instrumented builds, each driven in a child process with its sanitizer
runtime preloaded (leak checking off: the Python interpreter itself is not
instrumented):

* the C-ABI library with its host C++ instrumented (parameter validation,
  the half-window slot layout, the FP64 phase table and its matrix-core
  fragments, tiling and workspace sizing, and the create calls of every
  object up to the device check, which fails cleanly without a GPU);
* the C oracle (quadratic scan and pixel buckets, with and without the
  temporal bound, and the perceptron), whose results must also be bitwise
  equal to the regular build's.

Any sanitizer report aborts the child and fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

HOST_SCRIPT = r"""
import ctypes
import numpy as np
from paper_2504_19417_amd import synth, veckm as vk
assert vk.LIB_PATH.endswith("libveckm_hostsan.so"), vk.LIB_PATH

def params(d=64, rx=3, ry=3, rt=2, **kw):
    A = synth.draw_frequencies(d, max(rx, 1), max(ry, 1), max(rt, 1))
    args = dict(width=346, height=260, rx=rx, ry=ry, rt=rt, A=A, max_bins=25, max_events=20000)
    args.update(kw)
    return vk.make_params(**args)

checked = 0
for d in (16, 32, 48, 64, 128, 256):
    for r in ((0, 0, 0), (3, 3, 2), (5, 5, 3), (2, 4, 1), (12, 12, 6), (8, 8, -1), (10, 10, -1)):
        for prec in ("fp32", "fp16"):
            p = params(d, *r, precision=prec, max_bins=32 if r[2] < 0 else 25)
            rc = vk.veckm_params_check(p)
            assert rc in (vk.VECKM_OK, vk.VECKM_E_INVAL), rc
            if rc == vk.VECKM_OK:
                assert vk.veckm_workspace_bytes(p, 256) > 0
                assert vk.veckm_workspace_bytes(p, 0) > 0
                if r[2] >= 0:
                    vk.veckm_offset_table(p, with_phases=True)
                    vk.veckm_offset_table(p, with_phases=False)
            checked += 1
for bad in (dict(width=0), dict(height=-1), dict(rx=-1), dict(ry=13), dict(rt=7), dict(rt=-2),
            dict(rt=-1, max_bins=1025), dict(max_bins=0), dict(max_events=0),
            dict(max_events=1 << 40), dict(precision=5)):
    assert vk.veckm_params_check(params(**bad)) == vk.VECKM_E_INVAL, bad
for c in range(1, -12, -1):
    vk.veckm_strerror(c)
# object creation reaches the device check and unwinds (no GPU here)
p = params()
h = ctypes.c_void_p()
assert vk._lib.veckm_create(ctypes.byref(p), ctypes.byref(h)) == vk.VECKM_E_NODEVICE
assert vk._lib.veckm_window_create(ctypes.byref(p), ctypes.byref(h)) == vk.VECKM_E_NODEVICE
assert vk._lib.veckm_server_create(ctypes.byref(p), 1 << 34, 4, 2, ctypes.byref(h)) < 0
W1 = np.zeros((128, 128), np.float32); b1 = np.zeros(128, np.float32)
W2 = np.zeros((2, 128), np.float32); b2 = np.zeros(2, np.float32)
assert vk._lib.veckm_trainer_create(64, 128, 1000, W1.ctypes.data, b1.ctypes.data, W2.ctypes.data,
                                    b2.ctypes.data, ctypes.byref(h)) == vk.VECKM_E_NODEVICE
vk._lib.veckm_destroy(None)
vk._lib.veckm_server_destroy(None)
vk._lib.veckm_trainer_destroy(None)
print("host checks:", checked)
"""

ORACLE_SCRIPT = r"""
import sys
import numpy as np
import oracle
from paper_2504_19417_amd import synth
san = oracle.load_library(sys.argv[1])
reg = oracle.load_library(oracle.build())
spec = synth.SliceSpec(64, 48, 10, 3000, 4, seed=77)
ev, t0, T = synth.make_slice(spec)
A = synth.draw_frequencies(32, 3, 3, 2)
q = np.array([0, 5, 5, 2999, 1234], np.int64)
for rt in (2, -1):
    for search in ("scan", "bucket"):
        for queries in (None, q):
            e1, c1 = oracle.encode(ev, A, 3, 3, rt, queries, search, lib=san)
            e2, c2 = oracle.encode(ev, A, 3, 3, rt, queries, search, lib=reg)
            assert np.array_equal(e1, e2) and np.array_equal(c1, c2)
W1, b1, W2, b2 = synth.init_mlp(32, 64)
x = np.random.default_rng(3).standard_normal((500, 64))
assert np.array_equal(oracle.mlp(x, W1, b1, W2, b2, lib=san), oracle.mlp(x, W1, b1, W2, b2, lib=reg))
e1, c1 = oracle.encode(ev[:1], A, 3, 3, 2, lib=san)
assert c1[0] == 1
print("oracle checks passed")
"""

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(args, env_extra):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c"] + args, cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=900)
    report = r.stdout[-2000:] + "\n" + r.stderr[-8000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
    return r.stdout


def test_host_library_under_asan_and_ubsan():
    from paper_2504_19417_amd import hostsan
    lib = hostsan.build_host_sanitized()
    out = _run([HOST_SCRIPT], {"VECKM_LIB": lib, "LD_PRELOAD": hostsan.asan_runtime(),
                               "HIP_VISIBLE_DEVICES": ""})
    assert "host checks:" in out


def test_oracle_under_asan_and_ubsan():
    import oracle
    out_dir = os.path.join(ROOT, "_build", "oracle_san")
    os.makedirs(out_dir, exist_ok=True)
    path = oracle.compile_source(os.path.join(ROOT, "oracle", "veckm_oracle.c"),
                                 os.path.join(out_dir, "liboracle_san.so"), sanitize=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE,
                             text=True).stdout.strip()
    out = _run([ORACLE_SCRIPT, path], {"LD_PRELOAD": libasan})
    assert "oracle checks passed" in out
