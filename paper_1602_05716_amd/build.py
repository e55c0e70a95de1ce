"""Builds the gfx950 shared library libmc.so in-tree with hipcc.

Flags: contraction off (the double path must round every product and sum as
written; the float path asks for its fused multiply-adds explicitly) and
packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmc.so")
PEAK_EXE = os.path.join(HERE, "valu_peak")
SOURCES = ["mc_lib.hip", "mc_train.hip"]
HEADERS = ["mc_device.hpp", "mc_sweep_kernel.hpp", "mc_aux_kernels.hpp", "mc_reduce_kernel.hpp", "mc_internal.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libmc.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the VALU / v_rsq_f32 issue-rate probe used for the roofline denominator
    tmpx = PEAK_EXE + ".tmp%d" % os.getpid()
    cmdx = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
        "-o", tmpx, os.path.join(CSRC, "valu_peak.hip")]
    if verbose:
        print(" ".join(cmdx), flush=True)
    subprocess.check_call(cmdx)
    os.replace(tmpx, PEAK_EXE)
    return LIB


def asm(out_path: str) -> str:
    """Writes the gfx950 assembly of the device code (for inspection), all
    sources concatenated into out_path."""
    parts = []
    for src in SOURCES:
        part = out_path + "." + src + ".s"
        cmd = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
            "--cuda-device-only", "-S", "-I", os.path.join(HERE, "..", "include"), "-o", part,
            os.path.join(CSRC, src)]
        subprocess.check_call(cmd)
        parts.append(part)
    with open(out_path, "w") as out:
        for part in parts:
            with open(part) as f:
                out.write(f.read())
            os.remove(part)
    return out_path


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "asm":
        print(asm(sys.argv[2] if len(sys.argv) > 2 else "/tmp/mc_gfx950.s"))
    else:
        print(build(verbose=True))
