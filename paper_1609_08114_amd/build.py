"""Build libblp.so (HIP kernels + C-ABI runtime) for gfx950 with hipcc.

Objects go to ``_build/`` next to this file; the shared library is written
in-tree as ``libblp.so`` so that it travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libblp.so")
# the same library with in-kernel phase cycle counters (-DBLP_PHASE_TIMERS),
# for the per-phase breakdown of a solve; never the default
LIB_TIMERS = os.path.join(HERE, "libblp_timers.so")
BUILD_TIMERS = os.path.join(HERE, "_build_timers")
SOURCES = ["simplex_reg.hip", "simplex_lane.hip", "simplex_gm.hip", "aux_kernels.hip", "blp_runtime.cpp"]
HEADERS = ["blp_kernels.hpp", "simplex_common.hpp", "simplex_blk.hpp", "simplex_lane.hpp", "simplex_cols.hpp", "variants.hpp",
           "aux_kernels.hpp"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # only explicit fma() calls fuse: the pivot arithmetic must match its
    # specification operation by operation
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every atomic here is issued by one lane; the wave-aggregating rewrite
    # would wait for its result at once and defeat the work-list prefetch
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wno-unused-command-line-argument",
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False, jobs: int = 4, out: str = LIB, build_dir: str = BUILD, extra=()) -> str:
    """Compile and link.  `extra` adds compiler flags (e.g. -DBLP_PHASE_TIMERS
    for the instrumented build, written to another `out`)."""
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, extra), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


def build_timers(verbose: bool = False) -> str:
    """The phase-timer build (same sources, -DBLP_PHASE_TIMERS)."""
    return build(verbose=verbose, out=LIB_TIMERS, build_dir=BUILD_TIMERS, extra=("-DBLP_PHASE_TIMERS",))


if __name__ == "__main__":
    build(verbose=True)
    build_timers(verbose=True)
    sys.exit(0)
