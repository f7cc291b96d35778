"""Build libpdlp.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdlp.so")
SOURCES = ["pdlp.hip"]
HEADERS = ["pdlp_internal.h", "pdlp_kernels.h", "gnn_kernels.h", "gnn_host.h", "fix_kernels.h", "fix_host.h", "prop_kernels.h", "prop_host.h", "snap_kernels.h"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no product is fused into a sum unless the code asks for fma() itself: every update rounds
    # its product and its sum separately, as the method's formulas are written
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-parameter", "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(out: str = LIB, verbose: bool = False) -> str:
    srcs = sources()
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    noise = ("packed-fp32-ops",)
    msgs = [ln for ln in r.stdout.splitlines() if not any(k in ln for k in noise)]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building libpdlp.so")
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, out)
    return out


def stale(out: str = LIB) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "pdlp.h"))
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


if __name__ == "__main__":
    print(build(verbose=True))
