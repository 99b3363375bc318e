"""P1 finite-element residual integration on MI355X (gfx950).

The compute path is the HIP library ``libfemq.so`` behind the C ABI declared
in include/fem.h; this package is its thin Python binding. Importing the
package does not load the library: the first call does, and it raises if the
library has not been built.
"""
from .meshgen import LAPLACE, ELASTICITY, MASS, RULE_TRI3, RULE_TET4, RULE_CENTROID  # noqa: F401

__all__ = ["LAPLACE", "ELASTICITY", "MASS", "RULE_TRI3", "RULE_TET4", "RULE_CENTROID"]
