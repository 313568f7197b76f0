"""Build the HIP libraries in-tree for gfx950 with hipcc: librt3d.so (the
tracer, the two-stream column and the denoiser) and librt3d_probe.so (the
memory-system measurement the benchmark uses; not part of the tracer)."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = [os.path.join(PKG, "csrc", n) for n in ("rt3d.hip", "denoise.hip", "two_stream.hip")]
LIB = os.path.join(PKG, "librt3d.so")
PROBE_SOURCES = [os.path.join(PKG, "csrc", "probe.hip")]
PROBE_LIB = os.path.join(PKG, "librt3d_probe.so")
ARCH = os.environ.get("RT3D_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def flags() -> list:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=fast", "-munsafe-fp-atomics",
        # no packed FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wall", "-Wno-unused-function",
    ]


def _compile(sources, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [hipcc()] + flags() + sources + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build_library(verbose: bool = False) -> str:
    """Compile librt3d.so and librt3d_probe.so (always recompiles)."""
    _compile(SOURCES, LIB, verbose)
    _compile(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
