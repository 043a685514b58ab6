"""Build libsv.so (HIP, gfx950) in-tree with hipcc.

Each translation unit under csrc/ is compiled to an object with
``--offload-arch=gfx950`` and linked into ``paper_1608_00263_amd/libsv.so``.
Packed-FP32 instructions are disabled for the device code
(``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsv.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["api.cpp", "plan.cpp", "emulate.cpp", "sweeps.hip", "reduce.hip", "adjoint.hip", "batch.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # keep the per-case register-tile code separate: merging the switch
            # cases makes the amplitude registers addressable (scratch spills)
            "-mllvm", "-simplifycfg-sink-common=false",
            # leave regions under wave-uniform branches unstructured: the op
            # dispatch of the tile programs branches on scalar values only,
            # and structuring it merges the amplitude registers through
            # flow blocks (register copies at every op)
            "-mllvm", "-structurizecfg-skip-uniform-regions=true",
            "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
            "-D__HIP_PLATFORM_AMD__"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + lang + _flags() + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    # keep warnings other than the host pass's note about the device feature
    msg = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if msg.strip():
        sys.stderr.write(msg + "\n")
    return obj


def build(jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
