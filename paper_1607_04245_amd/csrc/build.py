"""Build libfemq.so, the HIP library behind include/fem.h, for gfx950.

Every translation unit is compiled with hipcc in parallel and linked into
one shared library next to the Python binding. Packed FP32 instructions are
disabled. FMA contraction is off: the kernels write every fused multiply-add
explicitly, so an element's operation sequence is fixed by the source and is
the same in every kernel that evaluates it (batched and single-mesh results
are bitwise equal).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
PKG = HERE.parent
ROOT = PKG.parent
BUILD = PKG / "_build"
LIB = PKG / "libfemq.so"
SOURCES = ["fem_abi.hip", "geometry.hip", "residual_lane.hip", "residual_transpose.hip", "residual_mesh.hip",
           "residual_gather.hip", "backward_lane.hip", "batch.hip", "tune.hip", "assembly.hip",
           "residual_p2.hip", "residual_p3.hip", "residual_p3_mfma.hip", "residual_p3_comp.hip", "jacobian.hip", "mesh_plan.hip",
           "residual_dedup.hip", "stream_rows.hip"]

ARCH = "gfx950"
FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I", str(ROOT / "include"), "-I", str(HERE)]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    p = pathlib.Path(rocm) / "bin" / "hipcc"
    return str(p) if p.exists() else "hipcc"


def _compile(src: str, verbose: bool) -> pathlib.Path:
    obj = BUILD / (pathlib.Path(src).stem + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", str(HERE / src), "-o", str(obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def _stale(src: str) -> bool:
    """Whether src's object is missing or older than src or any header."""
    obj = BUILD / (pathlib.Path(src).stem + ".o")
    if not obj.exists():
        return True
    deps = [HERE / src, *HERE.glob("*.hpp"), *(ROOT / "include").glob("*.h")]
    return obj.stat().st_mtime < max(d.stat().st_mtime for d in deps)


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> pathlib.Path:
    """Compile every source (or, with incremental, the stale ones) and link."""
    BUILD.mkdir(exist_ok=True)
    todo = [s for s in SOURCES if not incremental or _stale(s)]
    jobs = jobs or min(max(len(todo), 1), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [BUILD / (pathlib.Path(s).stem + ".o") for s in SOURCES]
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
