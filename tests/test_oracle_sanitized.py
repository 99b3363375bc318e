"""The oracle's pins, run once more against a build of fem_oracle.c with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc; any finding aborts the
run), in a child process with the sanitizer runtimes preloaded. CPU only."""
import os
import pathlib
import subprocess
import sys

import pytest

from oracle import build as ob

ROOT = pathlib.Path(__file__).resolve().parents[1]
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_spaces.py", "tests/test_oracle_assembly.py",
        "tests/test_oracle_p2.py", "tests/test_oracle_p3.py", "tests/test_oracle_jacobian.py", "tests/test_golden.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = ob.build_sanitized(tmp_path / "liboracle_san.so")
    env = dict(os.environ)
    env.update(FEMQ_ORACLE_LIB=str(lib), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:allocator_may_return_null=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    assert " passed" in tail, tail
