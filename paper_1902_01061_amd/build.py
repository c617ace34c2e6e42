"""Compile the HIP kernels and the C-ABI layer into libsgreg.so (gfx950)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libsgreg.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["descriptors.hip", "force.hip", "pose.hip", "residual.hip", "adjoint.hip", "mixed.hip", "knn_grid.hip",
           "sort.hip", "change.hip", "radius.hip", "vdesc.hip", "vforce.hip", "psum.hip", "capi.cpp"]
# Translation units whose results are integers decided by floating point
# (neighbour ranks by the float32 key (dx*dx + dy*dy) + dz*dz, change flags)
# are compiled without fused multiply-add, so that every operation is
# rounded on its own exactly as the key is defined; the others may fuse.
NO_FUSION = {"descriptors.hip", "knn_grid.hip", "change.hip", "radius.hip"}
# The vector-descriptor force and the mixed-precision force keep their
# matrix-instruction accumulators in ordinary VGPRs: in accumulation
# registers the compiler rotates them through register moves at every step
# (one move per pair weight in the vector form; 12 per 64 pairs a lane in
# the mixed form, which runs 5 % faster without them).
EXTRA = {"vforce.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"], "mixed.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
# Packed FP32 instructions are disabled for every HIP translation unit.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-munsafe-fp-atomics", "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    contract = "-ffp-contract=off" if src in NO_FUSION else "-ffp-contract=fast"
    cmd = ["hipcc", *FLAGS, contract, *EXTRA.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
    sys.exit(0)
