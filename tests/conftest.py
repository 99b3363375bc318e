import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _oracle_ready():
    lib = ROOT / "oracle" / "liboracle.so"
    src = ROOT / "oracle" / "fem_oracle.c"
    if not lib.exists() or lib.stat().st_mtime < src.stat().st_mtime:
        from oracle import build as ob
        ob.build()


_oracle_ready()


@pytest.fixture(scope="session")
def gpu_available():
    import torch
    return torch.cuda.is_available()
