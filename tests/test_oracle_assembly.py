"""Pins of the oracle's assembly (Section 2: the global residual is the sum of
the element vectors mapped back through the element restriction) and of its
adjoint, the restriction (closure) of a vertex field.

The pins do not reuse the oracle's own loops: dense global matrices built
from closed-form element matrices, the patch test, force and torque balance,
mass-matrix row sums, and the duality of assembly and restriction.
"""
import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg

from test_oracle_pins import bary_gradients, voigt_B, voigt_D

LAP, EL, MASS = mg.LAPLACE, mg.ELASTICITY, mg.MASS
RULES = {2: mg.RULE_TRI3, 3: mg.RULE_TET4}


def grid(dim, n, seed):
    rng = np.random.default_rng(seed)
    return (mg.tri_grid if dim == 2 else mg.tet_grid)(n, None, rng)


def residual(dim, phys, coords, conn, uv, coef):
    R, nd = oracle.residual(dim, phys, RULES[dim], coords, conn, mg.closure(conn, uv), coef)
    assert nd == 0
    return R


@pytest.mark.parametrize("dim", [2, 3])
def test_laplace_assembled_equals_dense_stiffness(dim):
    """F = K u with K assembled densely from |T| kappa g_i . g_j (closed-form
    barycentric gradients), one element at a time, by matrix indexing."""
    coords, conn = grid(dim, 4 if dim == 2 else 2, 3)
    nv, ne = coords.shape[0], conn.shape[0]
    rng = np.random.default_rng(4)
    kap = rng.uniform(0.5, 2, ne)
    K = np.zeros((nv, nv))
    for e in range(ne):
        g, V = bary_gradients(coords[conn[e]])
        K[np.ix_(conn[e], conn[e])] += kap[e] * V * g @ g.T
    uv = rng.uniform(-1, 1, (nv, 1))
    coef = np.repeat(kap[None, None, :], dim + 1, axis=1)
    F = oracle.assemble(dim, 1, nv, conn, residual(dim, LAP, coords, conn, uv, coef))
    assert np.allclose(F[:, 0], K @ uv[:, 0], rtol=1e-12, atol=1e-13)
    assert np.allclose(K, K.T)


@pytest.mark.parametrize("dim", [2, 3])
def test_elasticity_assembled_equals_dense_stiffness(dim):
    coords, conn = grid(dim, 3 if dim == 2 else 2, 5)
    nv, ne = coords.shape[0], conn.shape[0]
    rng = np.random.default_rng(6)
    lam, mu = rng.uniform(1, 10, ne), rng.uniform(0.5, 5, ne)
    K = np.zeros((nv * dim, nv * dim))
    for e in range(ne):
        g, V = bary_gradients(coords[conn[e]])
        B = voigt_B(g)                       # columns b*dim + c
        Ke = V * B.T @ voigt_D(dim, lam[e], mu[e]) @ B
        dofs = (conn[e][:, None] * dim + np.arange(dim)).ravel()
        K[np.ix_(dofs, dofs)] += Ke
    uv = rng.uniform(-1e-2, 1e-2, (nv, dim))
    coef = np.stack([np.repeat(lam[None, :], dim + 1, 0), np.repeat(mu[None, :], dim + 1, 0)])
    F = oracle.assemble(dim, dim, nv, conn, residual(dim, EL, coords, conn, uv, coef))
    assert np.allclose(F.ravel(), K @ uv.ravel(), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("dim,phys", [(2, LAP), (3, LAP), (2, EL), (3, EL)])
def test_patch_test_assembled(dim, phys):
    """Constant coefficients and a linear field: zero at interior vertices."""
    n = 6 if dim == 2 else 3
    coords, conn = grid(dim, n, 7)
    ne = conn.shape[0]
    nc = dim if phys == EL else 1
    coef = np.stack([np.full((dim + 1, ne), 3.0), np.full((dim + 1, ne), 1.5)]) if phys == EL \
        else np.full((1, dim + 1, ne), 1.7)
    rng = np.random.default_rng(8)
    uv = coords @ rng.normal(size=(nc, dim)).T + rng.normal(size=nc)
    F = oracle.assemble(dim, nc, coords.shape[0], conn, residual(dim, phys, coords, conn, uv, coef))
    idx = np.stack(np.unravel_index(np.arange(coords.shape[0]), (n + 1,) * dim), axis=1)
    interior = np.all((idx > 0) & (idx < n), axis=1)
    assert interior.any()
    assert np.abs(F[interior]).max() < 1e-12
    assert np.abs(F[~interior]).max() > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_force_and_torque_balance(dim):
    """Any u, any coefficients: the assembled elastic forces sum to zero and
    so does their moment (rigid modes are in the kernel of every element)."""
    coords, conn = grid(dim, 5 if dim == 2 else 3, 9)
    ne, nv = conn.shape[0], coords.shape[0]
    rng = np.random.default_rng(10)
    coef = np.stack([rng.uniform(1, 10, (dim + 1, ne)), rng.uniform(0.5, 5, (dim + 1, ne))])
    uv = rng.uniform(-1, 1, (nv, dim))
    F = oracle.assemble(dim, dim, nv, conn, residual(dim, EL, coords, conn, uv, coef))
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale * nv
    if dim == 2:
        torque = np.sum(coords[:, 0] * F[:, 1] - coords[:, 1] * F[:, 0])
    else:
        torque = np.cross(coords, F).sum(axis=0)
    assert np.abs(torque).max() < 1e-12 * scale * nv
    # the Laplacian with a random coefficient: rows sum to zero
    Fl = oracle.assemble(dim, 1, nv, conn, residual(dim, LAP, coords, conn, uv[:, :1],
                                                    rng.uniform(0.5, 2, (1, dim + 1, ne))))
    assert abs(Fl.sum()) < 1e-12 * np.abs(Fl).max() * nv


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_row_sums(dim):
    """u = 1, unit coefficient: F_v = integral of phi_v = sum over the
    elements at v of |T| / (d + 1)."""
    coords, conn = grid(dim, 5 if dim == 2 else 3, 11)
    ne, nv = conn.shape[0], coords.shape[0]
    F = oracle.assemble(dim, 1, nv, conn, residual(dim, MASS, coords, conn, np.ones((nv, 1)),
                                                   np.ones((1, dim + 1, ne))))
    expect = np.zeros(nv)
    for e in range(ne):
        _, V = bary_gradients(coords[conn[e]])
        expect[conn[e]] += V / (dim + 1)
    assert np.allclose(F[:, 0], expect, rtol=1e-12, atol=1e-16)
    assert np.isclose(F.sum(), 1.0, rtol=1e-12)   # the unit square / cube


@pytest.mark.parametrize("dim,nc", [(2, 1), (2, 2), (3, 1), (3, 3)])
def test_assembly_restriction_duality(dim, nc):
    coords, conn = grid(dim, 4, 12)
    ne, nv = conn.shape[0], coords.shape[0]
    rng = np.random.default_rng(13)
    R = rng.normal(size=((dim + 1) * nc, ne))
    W = rng.normal(size=(nv, nc))
    lhs = np.sum(oracle.assemble(dim, nc, nv, conn, R) * W)
    rhs = np.sum(R * oracle.restrict(dim, nc, conn, W))
    assert np.isclose(lhs, rhs, rtol=1e-12)
    assert np.array_equal(oracle.restrict(dim, nc, conn, W), mg.closure(conn, W))


def test_summation_order_is_element_order():
    """Element vectors are added in increasing element order from zero: a
    vertex shared by values that cancel only in that order shows it."""
    conn = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 1]], dtype=np.int32)
    R = np.zeros((3, 3))
    R[0] = [1.0, -1.0, 1e-17]    # vertex 0 gets 1, then -1, then 1e-17
    assert oracle.assemble(2, 1, 4, conn, R)[0, 0] == 1e-17   # reversed order would give 0
    R[0] = [1e-17, 1.0, -1.0]
    assert oracle.assemble(2, 1, 4, conn, R)[0, 0] == 0.0     # reversed order would give 1e-17


def test_bad_index_and_arguments_rejected():
    conn = np.array([[0, 1, 4]], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.assemble(2, 1, 4, conn, np.zeros((3, 1)))
    with pytest.raises(ValueError):
        oracle.restrict(2, 1, conn, np.zeros((4, 1)))
    with pytest.raises(ValueError):
        oracle.assemble(2, 4, 5, conn, np.zeros((12, 1)))
