"""Compiles the gfx950 HIP library ``librt_mi355x.so`` in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librt_mi355x.so")
SOURCES = ["rt_api.hip", "rt_build.hip", "rt_trace.hip", "rt_batch.hip", "rt_rays.hip", "rt_probe.hip",
           "rt_receive.hip", "rt_diffract.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off: plain scalar float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-function",
]
# the builder's decisions must not depend on fused multiply-add contraction
PER_FILE = {"rt_build.hip": ["-ffp-contract=off"]}


def build(verbose: bool = False, extra=None) -> str:
    extra = list(extra or [])
    with tempfile.TemporaryDirectory(prefix="rtbuild") as tmp:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [HIPCC, *FLAGS, *PER_FILE.get(src, []), *extra, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            objs.append(obj)
        out_tmp = os.path.join(tmp, "librt_mi355x.so")
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB) if os.path.dirname(out_tmp) == os.path.dirname(LIB) else \
            _copy(out_tmp, LIB)
    return LIB


def _copy(src, dst):
    tmp = dst + ".tmp%d" % os.getpid()
    with open(src, "rb") as f, open(tmp, "wb") as g:
        g.write(f.read())
    os.chmod(tmp, 0o755)
    os.replace(tmp, dst)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
