"""Builds libscalp.so (HIP, gfx950) in-tree with hipcc.

Floating-point flags are part of the contract of the library: the distance of
the assignment is evaluated operation by operation in IEEE FP32, so no
contraction into FMA (-ffp-contract=off), no fast-math, denormals preserved,
and packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libscalp.so")
SOURCES = ["scalp_kernels.hip", "scalp_soft.hip", "scalp_metrics.hip", "scalp_maps.hip",
           "scalp_abi.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every HIP source of the library into `out` (always recompiles)."""
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(extra or []), f"-I{INCLUDE}", f"-I{CSRC}", *sources(),
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


PROBE_SRC = os.path.join(CSRC, "peaks_probe.hip")
PROBE_BIN = os.path.join(HERE, "peaks_probe")


def build_probe(verbose: bool = False) -> str:
    """Compile the peak-rate microbenchmark (always recompiles)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    tmp = PROBE_BIN + ".tmp"
    cmd = [hipcc(), *flags, PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PROBE_BIN)
    return PROBE_BIN


def disassemble(out_dir: str) -> list[str]:
    """Writes the gfx950 assembly of every source into out_dir (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    paths = []
    for src in sources():
        dst = os.path.join(out_dir, os.path.basename(src) + ".s")
        cmd = [hipcc(), *[f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")],
               f"-I{INCLUDE}", f"-I{CSRC}", "--cuda-device-only", "-S", src, "-o", dst]
        subprocess.run(cmd, check=True)
        paths.append(dst)
    return paths


if __name__ == "__main__":
    build(verbose=True)
    build_probe(verbose=True)
    print(LIB)
    sys.exit(0)
