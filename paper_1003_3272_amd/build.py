"""Compile the gfx950 HIP library libnmf.so in place (hipcc, no torch)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnmf.so")
SOURCES = ["nmf_kernels.hip", "nmf_objective.hip", "nmf_update.hip", "nmf_kl.hip", "nmf_qn.hip",
           "nmf_runtime.hip", "nmf_mlp.hip", "nmf_batch.hip", "nmf_pet.hip", "nmf_ceiling.hip"]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for device code; hipcc's host pass
# warns that it does not know the feature, which is harmless.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 into libnmf.so; returns its path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", *FLAGS,
           "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
