"""Build libplan.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libplan.so")
SOURCES = ["rollout.hip", "rollout_onelane_1wave.hip", "rollout_multilane.hip", "est.hip",
           "select.hip", "plan_api.hip", "serve.hip", "adjoint.hip", "terrain_prep.hip",
           "order.hip"]

# Per-source flags (none at present). Every unit uses the default instruction
# scheduler: the max-ILP scheduler, once 3-4 % faster for the kernels of one
# wave per SIMD, measured slower on the current step (one-lane stress plan
# 196.7 against 193.4 us; one-lane sampled paper-shape plans at 49 152 and
# 65 536 candidates 0.89-0.90 against 0.83-0.85 ms; two lanes at 32 768
# candidates 71.0 against 69.5 us) and equal at four lanes.
SOURCE_FLAGS = {}

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 ops stay off: the scalar float code is compiled to plain VALU
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit contraction: every fused multiply-add is written as fmaf, so
    # all kernel variants evaluate identical arithmetic
    "-ffp-contract=off",
    "-Wall",
]


def build(verbose: bool = False, extra=None) -> str:
    """Compile every HIP source and link the shared library; returns its path."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = ["hipcc", *HIPCC_FLAGS, *SOURCE_FLAGS.get(src, []), *(extra or []), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
