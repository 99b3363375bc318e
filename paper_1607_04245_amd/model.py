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

import math
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
    return {2: 1, 3: 6, 4: 11}.get(rule, dim + 1)


def n_basis(dim: int, order: int = 1) -> int:
    return math.comb(dim + order, order)


def n_coef_words(dim: int, rule: int, coef_space: int = 0) -> int:
    """Words per coefficient and element: values at the N_q points (0), the
    d+1 vertex values of a P1 field (1), or one cell value (2)."""
    return {0: n_qpts(dim, rule), 1: dim + 1, 2: 1}[coef_space]


def model_flops(dim: int, physics: int, rule: int) -> int:
    """Paper-model flops per element for a (dim, physics, rule) of this library."""
    return paper_flops_per_cell(dim, dim + 1, n_comp(dim, physics), n_qpts(dim, rule))


def forward_words(dim: int, physics: int, rule: int, coef_space: int = 0) -> int:
    """Words moved by one element of fem_integrate_residual: invJ, detJ,
    closure u, coefficients in; element vector out."""
    nbt = (dim + 1) * n_comp(dim, physics)
    return (dim * dim + 1) + 2 * nbt + n_coef(physics) * n_coef_words(dim, rule, coef_space)


def forward_bytes(dim: int, physics: int, rule: int, word: int, coef_space: int = 0) -> int:
    return word * forward_words(dim, physics, rule, coef_space)


def backward_bytes(dim: int, physics: int, rule: int, word: int, want_du=True, want_dcoef=True,
                   coef_space: int = 0) -> int:
    """Compulsory bytes per element of fem_integrate_residual_backward."""
    nbt = (dim + 1) * n_comp(dim, physics)
    ncq = n_coef(physics) * n_coef_words(dim, rule, coef_space)
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
                        store_geometry: bool = False, coef_space: int = 0) -> float:
    """Compulsory bytes per element of fem_integrate_residual_mesh:
    connectivity, each vertex once (amortised), closure and coefficients in,
    element vector out (and the geometry, if stored)."""
    nbt = (dim + 1) * n_comp(dim, physics)
    words = 2 * nbt + n_coef(physics) * n_coef_words(dim, rule, coef_space) + \
        ((dim * dim + 1) if store_geometry else 0)
    return 4 * (dim + 1) + 8.0 * dim * n_vert / max(n_elem, 1) + word * words


def residual_gather_bytes(dim: int, physics: int, rule: int, n_elem: int, n_vert: int, word: int,
                          coef_space: int = 0, store_geometry: bool = False) -> float:
    """Compulsory bytes per element of fem_integrate_residual_gather:
    connectivity; each vertex's coordinates, u (and P1 coefficient) once,
    amortised; point or cell coefficients per element; element vector out."""
    nbt = (dim + 1) * n_comp(dim, physics)
    per_vertex = 8.0 * dim + word * n_comp(dim, physics) + (word * n_coef(physics) if coef_space == 1 else 0)
    per_elem = word * (nbt + (0 if coef_space == 1 else n_coef(physics) * n_coef_words(dim, rule, coef_space)) +
                       ((dim * dim + 1) if store_geometry else 0))
    return 4 * (dim + 1) + per_vertex * n_vert / max(n_elem, 1) + per_elem


def planned_bytes(dim: int, physics: int, rule: int, n_elem: int, n_vert: int, tile_vertices: int, word: int,
                  gather: bool = False, coef_space: int = 0) -> float:
    """Compulsory bytes per element of the planned residuals: the packed
    local indices (4 bytes) and the tiles' vertex lists in place of the
    connectivity, otherwise as fem_integrate_residual_mesh (gather=False) or
    fem_integrate_residual_gather (gather=True)."""
    base = (residual_gather_bytes if gather else residual_mesh_bytes)(dim, physics, rule, n_elem, n_vert, word,
                                                                        coef_space=coef_space)
    return base - 4 * (dim + 1) + 4 + 4.0 * tile_vertices / max(n_elem, 1)


def assemble_bytes(dim: int, n_comp_: int, n_elem: int, n_vert: int, word: int) -> float:
    """Compulsory bytes per element of fem_assemble: the slot index and the
    element vectors in, row offsets in and the vertex field out (amortised)."""
    nb = dim + 1
    return 4.0 * nb + word * nb * n_comp_ + (4.0 + word * n_comp_) * n_vert / max(n_elem, 1)


def p2_model_flops(dim: int, physics: int, rule: int) -> int:
    """The paper's per-cell flop formula with the P2 basis (N_b = (d+1)(d+2)/2)."""
    return paper_flops_per_cell(dim, n_basis(dim, 2), n_comp(dim, physics), n_qpts(dim, rule))


def jacobian_bytes(dim: int, physics: int, rule: int, word: int, coef_space: int = 0, order: int = 1) -> int:
    """Compulsory bytes per element of fem_integrate_jacobian: the geometry
    (det J only for the mass form, which has no gradients), the coefficient
    words, and the N_bt^2 matrix entries written."""
    nbt = n_basis(dim, order) * n_comp(dim, physics)
    geo = 1 if physics == 2 else dim * dim + 1
    return word * (geo + n_coef(physics) * n_coef_words(dim, rule, coef_space) + nbt * nbt)


def p2_forward_bytes(dim: int, physics: int, rule: int, word: int, coef_space: int = 0) -> int:
    """Compulsory bytes per element of fem_integrate_residual_p2."""
    nbt = n_basis(dim, 2) * n_comp(dim, physics)
    return word * ((dim * dim + 1) + 2 * nbt + n_coef(physics) * n_coef_words(dim, rule, coef_space))


def p3_model_flops(dim: int, physics: int, rule: int) -> int:
    """The paper's per-cell flop formula with the P3 basis (N_b = (d+1)(d+2)(d+3)/6)."""
    return paper_flops_per_cell(dim, n_basis(dim, 3), n_comp(dim, physics), n_qpts(dim, rule))


def p3_forward_bytes(dim: int, physics: int, rule: int, word: int, coef_space: int = 0) -> int:
    """Compulsory bytes per element of fem_integrate_residual_p3."""
    nbt = n_basis(dim, 3) * n_comp(dim, physics)
    return word * ((dim * dim + 1) + 2 * nbt + n_coef(physics) * n_coef_words(dim, rule, coef_space))


def p3_backward_bytes(dim: int, physics: int, rule: int, word: int, coef_space: int = 0) -> int:
    """Compulsory bytes per element of fem_integrate_residual_p3_backward with
    both outputs: geometry, w, u and coefficients in, du and dcoef out."""
    nbt = n_basis(dim, 3) * n_comp(dim, physics)
    ncq = n_coef(physics) * n_coef_words(dim, rule, coef_space)
    return word * ((dim * dim + 1) + 3 * nbt + 2 * ncq)
