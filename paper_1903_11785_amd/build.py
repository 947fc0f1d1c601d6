"""Build the gfx950 HIP library ``libfvv.so`` in-tree with hipcc.

Every call recompiles.  Device code is compiled without fp contraction (all
fused multiply-adds are explicit) and without fast-math, which the bit-exact
occupancy test relies on; packed-fp32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfvv.so")
SOURCES = ["carve.hip", "ccl.hip", "surface.hip", "isovalue.hip", "mesh.hip", "visibility.hip",
           "soft.hip", "measure.hip", "api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-value", "-Wno-unused-command-line-argument", f"-I{INCLUDE}"]


def _compile(src: str, obj_dir: str, defines) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 8, defines=(), out: str = LIB) -> str:
    """Compile every source and link `out` (the library by default).  `defines`
    are preprocessor macros of a measurement build (e.g. FVV_LABEL_PHASES),
    which goes to another path."""
    obj_dir = BUILD if not defines else os.path.join(BUILD, "_".join(defines))
    os.makedirs(obj_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir, defines), SOURCES))
    tmp = out + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
