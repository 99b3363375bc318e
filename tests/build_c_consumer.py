"""Build tests/c_abi_consumer (the plain C user of include/fem.h) with gcc,
linking libfemq.so, the oracle library and the HIP runtime. Test
infrastructure: run by the repository's build step after both libraries."""
from __future__ import annotations

import os
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parent
SRC = HERE / "c_abi_consumer.c"
OUT = HERE / "c_abi_consumer"


def build() -> pathlib.Path:
    rocm = pathlib.Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", f"-I{rocm / 'include'}",
           f"-I{ROOT / 'include'}", str(SRC), "-o", str(OUT),
           f"-L{ROOT / 'paper_1607_04245_amd'}", "-lfemq", f"-L{ROOT / 'oracle'}", "-loracle",
           f"-L{rocm / 'lib'}", "-lamdhip64", "-lm",
           f"-Wl,-rpath,$ORIGIN/../paper_1607_04245_amd:$ORIGIN/../oracle:{rocm / 'lib'}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C consumer failed:\n{r.stderr}")
    return OUT


if __name__ == "__main__":
    print(build())
