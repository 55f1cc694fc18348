"""Build libctu.so (HIP, gfx950) in-tree with hipcc.

The three translation units (host API, FP32 and FP64 kernel
instantiations) compile in parallel, then link into
``paper_1110_0740_amd/libctu.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libctu.so")
BUILD = os.path.join(HERE, "_build")
UNITS = ["ctu_lib.hip", "ctu_inst_f32.hip", "ctu_inst_f64.hip", "ctu_inst_mt_f32.hip", "ctu_inst_mt_f64.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# FP32 translation unit: divide and square root as the hardware's
# approximate reciprocal / root (a few ulp) instead of the correctly rounded
# expansions, and FP32 subnormals flushed to zero, which lets both map to
# single instructions without range scaling (the state variables stay many
# orders of magnitude above 1e-38); FP64 keeps the correctly rounded forms
# and subnormals.
_F32 = ["-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero"]
UNIT_FLAGS = {"ctu_inst_f32.hip": _F32, "ctu_inst_mt_f32.hip": _F32}


def _compile(unit: str, extra: list[str], build_dir: str = BUILD) -> str:
    src = os.path.join(CSRC, unit)
    obj = os.path.join(build_dir, unit.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *UNIT_FLAGS.get(unit, []), *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stderr[-8000:]}")
    return obj


def build(extra: list[str] | None = None, verbose: bool = False, out: str = OUT) -> str:
    """Compile every HIP source and link the library (default: the in-tree
    libctu.so); always rebuilds."""
    extra = list(extra or [])
    build_dir = BUILD if out == OUT else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(lambda u: _compile(u, extra, build_dir), UNITS))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(extra=sys.argv[1:], verbose=True)
