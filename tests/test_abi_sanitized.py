"""The ABI's host-side argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer. The translation units with host logic beyond
launching (entry points and validation, batch and no-allocation launches,
the tuning cache parser, mesh and assembly plans) are rebuilt with the
sanitizers on their host code only, linked with the regular objects of the
other units, and tests/test_abi_cpu.py runs against that library in a child
process with the sanitizer runtime preloaded; any finding aborts the run.
CPU only (no device is touched)."""
import concurrent.futures as cf
import os
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

from paper_1607_04245_amd.csrc import build as lb  # noqa: E402

HOST_UNITS = ["fem_abi", "batch", "tune", "mesh_plan", "assembly"]
# each sanitizer flag applies to the host compilation only
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split() + \
    "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer".split()


def _asan_runtime():
    clang = pathlib.Path(os.environ.get("ROCM_PATH", "/opt/rocm")) / "llvm" / "bin" / "clang"
    if not clang.exists():
        return None
    r = subprocess.run([str(clang), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = pathlib.Path(r.stdout.strip())
    return p if r.returncode == 0 and p.is_absolute() and p.exists() else None


def _build_host_sanitized(work: pathlib.Path) -> pathlib.Path:
    flags = [f for f in lb.FLAGS if f != "-Wall"]

    def compile_unit(stem):
        obj = work / f"{stem}.o"
        cmd = [lb._hipcc(), *flags, *HOST_SANITIZE, "-c", str(lb.HERE / f"{stem}.hip"), "-o", str(obj)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(len(HOST_UNITS)) as ex:
        list(ex.map(compile_unit, HOST_UNITS))
    objs = []
    for src in lb.SOURCES:
        stem = pathlib.Path(src).stem
        objs.append(work / f"{stem}.o" if stem in HOST_UNITS else lb.BUILD / f"{stem}.o")
    out = work / "libfemq_host_sanitized.so"
    cmd = [lb._hipcc(), "-shared", "-fPIC", f"--offload-arch={lb.ARCH}", *HOST_SANITIZE[:4], "-shared-libasan",
           "-o", str(out), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def test_abi_validation_under_asan_ubsan(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("clang AddressSanitizer runtime not installed")
    missing = [s for s in lb.SOURCES if not (lb.BUILD / (pathlib.Path(s).stem + ".o")).exists()]
    if missing:
        pytest.skip(f"regular objects not built ({missing[0]} missing): run __graft_entry__.build() first")
    lib = _build_host_sanitized(tmp_path)
    env = dict(os.environ)
    env.update(FEMQ_LIB=str(lib), LD_PRELOAD=str(asan),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the child really maps the sanitized library
    probe = ("from paper_1607_04245_amd import _native as N; N.lib(); "
             "print(any(l.rstrip().endswith('libfemq_host_sanitized.so') for l in open('/proc/self/maps')))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), (r.stdout + r.stderr)[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi_cpu.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    assert " passed" in tail, tail
