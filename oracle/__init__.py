"""FP64 CPU reference for P1 element integration -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path never does.
Functions marked "parity unpinned" have no independent pin; at present every
function here is pinned by tests/test_oracle_*.py.
"""
from .oracle import (  # noqa: F401
    rule, geometry, integrate, integrate_abs, residual, backward, load, n_qpts, assemble, restrict, n_basis,
    jacobian, jacobian_abs,
)
