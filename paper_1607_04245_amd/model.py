"""Performance model: the paper's flop/traffic model and compulsory HBM bytes.

The paper (Section 3, subsection "Memory Traffic and Computation") counts,
per cell,
  flops = ((2 + (2 + 2d) d) N_bt + 2 d N_comp) N_q + (2 + 2d) d N_q N_bt
  bytes = 4 ((d^2 + 1) + N_bt + (d + 1) N_q)          (single precision)
and reports GF/s as elements/s times that flop count; for d = 2, N_b = 3,
N_comp = 1, N_q = 1 the balance is 41/22 flop/byte. "Model GF/s" in this
project is that convention, at the actual N_q of each rule.

The roofline instead counts compulsory bytes of the library's calls: every
input word is read once and every output word written once.
"""
from __future__ import annotations

from fractions import Fraction

# MI355X published peaks used as roofline denominators.
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6


def paper_flops_per_cell(d: int, n_b: int, n_comp: int, n_q: int) -> int:
    n_bt = n_b * n_comp
    return ((2 + (2 + 2 * d) * d) * n_bt + 2 * d * n_comp) * n_q + (2 + 2 * d) * d * n_q * n_bt


def paper_bytes_per_cell(d: int, n_b: int, n_comp: int, n_q: int, word: int = 4) -> int:
    n_bt = n_b * n_comp
    return word * ((d * d + 1) + n_bt + (d + 1) * n_q)


def paper_beta(d: int, n_b: int, n_comp: int, n_q: int) -> Fraction:
    """Algorithmic balance in flop/byte (exact fraction)."""
    return Fraction(paper_flops_per_cell(d, n_b, n_comp, n_q), paper_bytes_per_cell(d, n_b, n_comp, n_q))


def n_comp(dim: int, physics: int) -> int:
    return dim if physics == 1 else 1


def n_coef(physics: int) -> int:
    return 2 if physics == 1 else 1


def n_qpts(dim: int, rule: int) -> int:
    return 1 if rule == 2 else dim + 1


def model_flops(dim: int, physics: int, rule: int) -> int:
    """Paper-model flops per element for a (dim, physics, rule) of this library."""
    return paper_flops_per_cell(dim, dim + 1, n_comp(dim, physics), n_qpts(dim, rule))


def forward_words(dim: int, physics: int, rule: int) -> int:
    """Words moved by one element of fem_integrate_residual: invJ, detJ,
    closure u, coefficients in; element vector out."""
    nbt = (dim + 1) * n_comp(dim, physics)
    return (dim * dim + 1) + 2 * nbt + n_coef(physics) * n_qpts(dim, rule)


def forward_bytes(dim: int, physics: int, rule: int, word: int) -> int:
    return word * forward_words(dim, physics, rule)


def backward_bytes(dim: int, physics: int, rule: int, word: int, want_du=True, want_dcoef=True) -> int:
    """Compulsory bytes per element of fem_integrate_residual_backward."""
    nbt = (dim + 1) * n_comp(dim, physics)
    ncq = n_coef(physics) * n_qpts(dim, rule)
    words = (dim * dim + 1) + nbt   # geometry and w in
    if want_du:
        words += ncq + nbt           # coefficients in, du out
    if want_dcoef:
        words += nbt + ncq           # u in, dcoef out
    return word * words


def geometry_bytes(dim: int, n_elem: int, n_vert: int, word: int) -> float:
    """Compulsory bytes per element of fem_geometry: connectivity, each vertex
    read once (amortised), invJ and detJ written."""
    return 4 * (dim + 1) + 8.0 * dim * n_vert / max(n_elem, 1) + word * (dim * dim + 1)


def residual_mesh_bytes(dim: int, physics: int, rule: int, n_elem: int, n_vert: int, word: int,
                        store_geometry: bool = False) -> float:
    """Compulsory bytes per element of fem_integrate_residual_mesh:
    connectivity, each vertex once (amortised), closure and coefficients in,
    element vector out (and the geometry, if stored)."""
    nbt = (dim + 1) * n_comp(dim, physics)
    words = 2 * nbt + n_coef(physics) * n_qpts(dim, rule) + ((dim * dim + 1) if store_geometry else 0)
    return 4 * (dim + 1) + 8.0 * dim * n_vert / max(n_elem, 1) + word * words
