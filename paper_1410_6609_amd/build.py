"""Compile the HIP library libccmg.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ccmg.hip")
LIB = os.path.join(HERE, "libccmg.so")
# a second build with other tile macros, for the test that the iterates do not
# depend on the tiling: 4-wave FP64 blocks (64x16 loaded tiles, as few as 6
# owned rows beside the 5-row halos) and 8-wave FP32 blocks (64x32)
TILES_LIB = os.path.join(HERE, "libccmg_tiles.so")
TILES_DEFINES = ("CCMG_WAVES=4", "CCMG_WAVES_F32=8", "CCMG_CHUNK_CAPACITY_SCALE=3", "CCMG_PAD_MIN_PLANES=8")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off: plain scalar FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# host code only (the device code is built as usual): AddressSanitizer and
# UndefinedBehaviorSanitizer, UB aborting
HOST_SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                       "-shared-libsan"]


def _command(out: str, defines=(), sanitize_host: bool = False):
    return [hipcc(), *HIPCC_FLAGS, *[f"-D{d}" for d in defines], *(HOST_SANITIZE_FLAGS if sanitize_host else []),
            "-o", out + ".tmp", SRC]


def build(verbose: bool = False, out: str = LIB, defines=(), sanitize_host: bool = False) -> str:
    """Compile libccmg.so; `defines` are extra -D tuning macros (tile shape)."""
    cmd = _command(out, defines, sanitize_host)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(out + ".tmp", out)
    return out


def build_all(verbose: bool = False) -> None:
    """libccmg.so and the other-tiling build beside it, compiled side by side."""
    jobs = [(LIB, ()), (TILES_LIB, TILES_DEFINES)]
    procs = []
    for out, defines in jobs:
        cmd = _command(out, defines)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, cwd=HERE))
    codes = [p.wait() for p in procs]
    for (out, _), code in zip(jobs, codes):
        if code != 0:
            raise subprocess.CalledProcessError(code, out)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
    print(LIB, TILES_LIB)
