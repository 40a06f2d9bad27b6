"""Build recipe of libifdlbm.so: hipcc for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libifdlbm.so")
SOURCES = ["api.hip", "kernels_common.hip", "step_staged.hip", "step_fused.hip", "gradient.hip", "adjoint.hip", "regime.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-I", INCLUDE, "-I", CSRC,
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-parameter",
]
# Flags of single sources.  The step kernels are scheduled for instruction-level parallelism (LLVM's
# iterative-ilp strategy) instead of occupancy first: they keep their occupancy either way (two waves per SIMD
# with FP32 arithmetic, one with FP64), and that schedule measured faster in every storage mode (FP64 +6 %,
# FP16DEV +3.4 %, FP32SRF +1.6 %, FP32 +0.8 % over the default).
FILE_FLAGS = {"step_fused.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}


def source_files():
    """Every file the library is built from: the sources, the headers beside them and the C-ABI header."""
    heads = sorted(f for f in os.listdir(CSRC) if f.endswith(".h"))
    return [os.path.join(CSRC, f) for f in SOURCES + heads] + [os.path.join(INCLUDE, "ifdlbm.h")]


def source_digest() -> str:
    """SHA-256 of the library's sources (names and contents) and of the per-source flags, compiled into the library as
    ifdlbm_build_digest() so that the binding can refuse a library built from other sources."""
    import hashlib
    h = hashlib.sha256()
    h.update(repr(sorted(FILE_FLAGS.items())).encode() + b"\0")
    for path in source_files():
        with open(path, "rb") as f:
            data = f.read()
        h.update(os.path.basename(path).encode() + b"\0" + str(len(data)).encode() + b"\0" + data)
    return h.hexdigest()


def _compile(src: str, obj: str, extra) -> None:
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % src)


def build(extra=(), jobs: int = 4, out: str = LIB, objdir: str = "") -> str:
    """Compile every source with the flags above plus `extra` (e.g. -D tuning
    knobs of step_fused.hip) and link `out`."""
    objdir = objdir or os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    extra = list(extra) + ['-DIFD_SOURCE_DIGEST="%s"' % source_digest()]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], extra), zip(SOURCES, objs)))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("link of libifdlbm.so failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
