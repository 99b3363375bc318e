"""Build the FP64 reference integrator (test infrastructure) with gcc.

Plain C, -O2, FMA contraction off so every product and sum rounds as written.
"""
import pathlib
import subprocess

HERE = pathlib.Path(__file__).resolve().parent
SRC = HERE / "fem_oracle.c"
LIB = HERE / "liboracle.so"


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(out: pathlib.Path, verbose: bool = False) -> pathlib.Path:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer
    (any finding aborts). Loading it needs the sanitizer runtimes preloaded."""
    cmd = ["gcc", "-std=c11", "-O1", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           *SANITIZE, "-o", str(out), str(SRC), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> pathlib.Path:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", str(LIB) + ".tmp", str(SRC), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    pathlib.Path(str(LIB) + ".tmp").replace(LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
