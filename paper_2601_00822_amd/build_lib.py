"""Build liblsfft.so for gfx950 with hipcc (in-tree, no JIT).

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled, and linked with the host orchestration into one shared library
next to this file.  Sources compile in parallel; the link runs last.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblsfft.so")

# Translation units built from k_pass.hip: (object name, defines).  Outer
# pass launchers first (the slowest to compile), then the x and y passes; the
# schedule variants other than 0 (FP32 3D, lengths from 32 on) each get a
# unit of their own.
PASS_UNITS = (
    [(f"k_pass_g_{p}_{d}d_{'l' if lng else 's'}", {"LSFFT_PASS": 2, "LSFFT_F64": int(p == "f64"), "LSFFT_DIM": d,
                                                    "LSFFT_LONG": int(lng)})
     for lng in (True, False) for p in ("f32", "f64") for d in (3, 2)]
    + [(f"k_pass_g_f32_3d_l_v{v}", {"LSFFT_PASS": 2, "LSFFT_F64": 0, "LSFFT_DIM": 3, "LSFFT_LONG": 1,
                                    "LSFFT_VARIANT": v}) for v in (1, 2)]
    + [(f"k_pass_x_{p}_{d}d", {"LSFFT_PASS": 0, "LSFFT_F64": int(p == "f64"), "LSFFT_DIM": d})
       for p in ("f32", "f64") for d in (3, 2)]
    + [(f"k_pass_x_f32_3d_v{v}", {"LSFFT_PASS": 0, "LSFFT_F64": 0, "LSFFT_DIM": 3, "LSFFT_VARIANT": v})
       for v in (1, 2)]
    + [(f"k_pass_y_{p}", {"LSFFT_PASS": 1, "LSFFT_F64": int(p == "f64")}) for p in ("f32", "f64")]
    + [(f"k_pass_y_f32_v{v}", {"LSFFT_PASS": 1, "LSFFT_F64": 0, "LSFFT_VARIANT": v}) for v in (1, 2)]
)


def sources():
    """Every translation unit: (source in csrc/, object name, defines)."""
    units = [("k_pass.hip", name, defs) for name, defs in PASS_UNITS]
    others = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f != "k_pass.hip")
    units += [(f, os.path.splitext(f)[0], {}) for f in others]
    units += [("lsfft.cpp", "lsfft", {}), ("fno.cpp", "fno", {})]
    return units

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", INCLUDE,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build liblsfft")


def _compile(unit) -> str:
    src, name, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *COMMON, *[f"-D{k}={v}" for k, v in defs.items()], "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
