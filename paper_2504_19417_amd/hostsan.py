"""Host-sanitizer build of the library (CPU checks only).

    python -m paper_2504_19417_amd.hostsan

Compiles the library's host C++ (API, validation, tables, server, trainer)
with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only,
links it with the kernels of the regular build, and writes
``_build/veckm_hostsan/libveckm_hostsan.so``.  Nothing on the product path
loads it; the checks load it through ``VECKM_LIB`` with the compiler's ASan
runtime preloaded.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

from .build import ARCH, CFLAGS, CSRC, HIPCC, OBJ_DIR, ROOT, build

SAN_DIR = os.path.join(ROOT, "_build", "veckm_hostsan")
SAN_LIB = os.path.join(SAN_DIR, "libveckm_hostsan.so")
# AddressSanitizer + UndefinedBehaviorSanitizer on the host side only (the
# device code of the same sources is built as usual)
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build_host_sanitized() -> str:
    """The library with its host C++ (API, validation, tables, server,
    trainer) instrumented by AddressSanitizer and UBSan, linked with the
    kernels of the regular build (built first if missing).  Loading it needs
    the compiler's ASan runtime preloaded; see `asan_runtime()`."""
    objs = []
    if not all(os.path.exists(os.path.join(OBJ_DIR, os.path.basename(f) + ".o"))
               for f in glob.glob(os.path.join(CSRC, "*.hip"))):
        build(verbose=False)
    os.makedirs(SAN_DIR, exist_ok=True)

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + CFLAGS + SAN_FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stdout))
        return obj

    srcs = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    objs += sorted(os.path.join(OBJ_DIR, os.path.basename(f) + ".o")
                   for f in glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def asan_runtime() -> str:
    """The compiler's shared ASan runtime matching `build_host_sanitized`."""
    res = subprocess.run([HIPCC, "-print-resource-dir"], stdout=subprocess.PIPE,
                         stderr=subprocess.DEVNULL, text=True).stdout.strip()
    return os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")


if __name__ == "__main__":
    print(build_host_sanitized())
