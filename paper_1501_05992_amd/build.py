"""Build libcorrx.so (HIP, gfx950) in place with hipcc, and the instruction
issue-rate probes (libceiling.so) the benchmark measures ceilings with.

    python -m paper_1501_05992_amd.build

The library is a plain shared object with a C ABI (include/corrx.h); it links
the HIP runtime by soname, so inside a process that already loaded PyTorch it
binds to the runtime PyTorch loaded.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcorrx.so")
SOURCES = ["api.hip", "batch.hip", "xengine_mfma.hip", "xengine_plain.hip", "dump.hip", "fpfb.hip"]
CEILING_LIB = os.path.join(HERE, "libceiling.so")
CEILING_SOURCES = ["ceiling.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-fp32 instructions are disabled for every device compile.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, save_temps_dir: str | None = None) -> str:
    _build_one(LIB, SOURCES, verbose, save_temps_dir)
    _build_one(CEILING_LIB, CEILING_SOURCES, verbose, None)
    return LIB


def _build_one(lib: str, sources: list[str], verbose: bool, save_temps_dir: str | None) -> None:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = lib + ".tmp"
    # --no-undefined: a missing definition fails the build instead of the load.
    cmd = [HIPCC, *DEVICE_FLAGS, "-shared", "-Wl,--no-undefined", "-I", os.path.join(ROOT, "include"), "-o", tmp,
           *srcs]
    if save_temps_dir:
        os.makedirs(save_temps_dir, exist_ok=True)
        cmd.insert(1, f"-save-temps={save_temps_dir}")
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, lib)


if __name__ == "__main__":
    print(build(verbose=True))
