"""Build the HIP library (libps.so) in-tree for gfx950 with hipcc.

    python -m paper_2605_04550_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libps.so")
SOURCES = (["ps_kernels.hip", "ps_mask.hip", "ps_api.cpp", "ps_bisect.hip", "ps_eval_batch.hip", "ps_noalloc.hip", "ps_dense.hip"] + ["ps_eval_kl%d.hip" % k for k in range(5)]
           + ["ps_bis_h%d.hip" % h for h in range(1, 9)])
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++20", "-fPIC",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every source to an object and link libps.so (always rebuilds)."""
    objs = []
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(outdir, src + ".o")
        cmd = [_hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        elif verbose and out:
            sys.stdout.write(out.decode(errors="replace"))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
