"""The C ABI from a plain C program (tests/c_abi_consumer.c): HIP runtime
allocations, libfemq calls, checks against the oracle library. Built by the
repository's build step; run here as a child process."""
import pathlib
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = pathlib.Path(__file__).resolve().parent / "c_abi_consumer"


def test_c_consumer_program():
    if not BIN.exists():
        pytest.fail("tests/c_abi_consumer is not built (run __graft_entry__.build())")
    r = subprocess.run([str(BIN)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "ok" in r.stdout
