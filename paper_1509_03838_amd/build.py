"""Builds libne.so for gfx950 with hipcc (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libne.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["api.hip", "stream_kernels.hip", "conv_valu.hip", "chain.hip", "fused.hip", "plan.hip",
           "gemm.hip", "word32.hip", "bandwidth.hip",
           "failstop.hip"]

# fused_conv.hip is compiled once per (kernel class, slot count), and
# fused_stream.hip and fused_single.hip (the single-launch kernel) once per
# kernel class: entangled
# groups of 3..8 streams, plain groups of 1..8, checksum groups of 2..8 data
# streams (3..9 slots).
CONV_VARIANTS = ([(0, n) for n in range(3, 9)] + [(1, n) for n in range(1, 9)] +
                 [(2, n) for n in range(3, 10)])

# Packed-FP32 instructions are disabled for all device code. Matrix-core
# results stay in ordinary VGPRs (no accumulation-register copies in the
# convolution loops).
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form=1",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    units = [(src, src.replace(".hip", ".o"), []) for src in SOURCES]
    units += [("fused_conv.hip", f"fused_conv_{k}_{n}.o", [f"-DNE_KCLASS={k}", f"-DNE_SLOTS={n}"])
              for k, n in CONV_VARIANTS]
    units += [("fused_stream.hip", f"fused_stream_{k}.o", [f"-DNE_KCLASS={k}"]) for k in range(3)]
    units += [("gemm_kernels.hip", f"gemm_kernels_{k}.o", [f"-DNE_KCLASS={k}"]) for k in range(3)]
    # the single-launch units compile longest: started first
    units = [("fused_single.hip", f"fused_single_{k}.o", [f"-DNE_KCLASS={k}", "-DNE_SINGLE_LAUNCH"])
             for k in range(3)] + units
    objs = []
    pending = list(units)
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            src, o, defs = pending.pop(0)
            obj = os.path.join(CSRC, "_build", o)
            os.makedirs(os.path.dirname(obj), exist_ok=True)
            cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((o, subprocess.Popen(cmd)))
            objs.append(obj)
        o, p = running.pop(0)
        if p.wait() != 0:
            for _, q in running:
                q.wait()
            raise RuntimeError(f"hipcc failed on {o}")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
