"""Build libzfpx.so (HIP, gfx950) in-tree with hipcc.

Always recompiles.  ``python -m paper_2609_24294_amd.build`` or
``__graft_entry__.build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libzfpx.so")
SOURCES = ["kernels.hip", "api.cpp", "server.cpp", "plan_tables.cpp"]

# packed FP32 instructions are disabled on purpose; plain float code only
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False, jobs: int = 3) -> str:
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with tempfile.TemporaryDirectory(prefix="zfpx_build_") as tmp:
        procs = []
        objs = []
        for s in srcs:
            obj = os.path.join(tmp, s + ".o")
            objs.append(obj)
            cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        failed = False
        for cmd, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                failed = True
                sys.stderr.write(out)
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            raise RuntimeError("hipcc failed")
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB_PATH + ".tmp"]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def build_program(src: str, out: str, verbose: bool = False) -> str:
    """Compile a standalone HIP program (a measurement probe) with the
    library's flags."""
    cmd = [hipcc(), *[f for f in HIPCC_FLAGS if f != "-fPIC"], src, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    print(LIB_PATH)
