"""Build libte.so (HIP kernels for gfx950 + host runtime) in-tree with hipcc.

`python -m paper_1401_4068_amd.build --sanitize address|thread` builds a copy of the
library whose host code is instrumented with AddressSanitizer or ThreadSanitizer
(device code is compiled as usual), as _build/<kind>/libte_<kind>.so, for CPU runs of
the host-logic tests with the sanitizer runtime preloaded (commands in the design notes).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libte.so")
OBJ = os.path.join(ROOT, "_build")

ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]
# host-only instrumentation: each sanitizer flag applies to the host compilation alone
SANITIZE = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"],
    "thread": ["-Xarch_host", "-fsanitize=thread", "-g"],
}


def _compile(src: str, objdir: str, extra: list) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = ["hipcc", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS + extra + ["-c", src, "-o", obj]

    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + src)
    return obj


def build(verbose: bool = False, sanitize: str = "") -> str:
    extra = SANITIZE[sanitize] if sanitize else []
    objdir = os.path.join(OBJ, sanitize) if sanitize else OBJ
    out = os.path.join(objdir, "libte_%s.so" % sanitize) if sanitize else OUT
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, extra), srcs))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread", "-lrocprofiler-sdk-roctx"]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=" + sanitize, "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--sanitize", choices=sorted(SANITIZE), default="")
    build(verbose=True, sanitize=ap.parse_args().sanitize)
