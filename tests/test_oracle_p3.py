"""Pins of the oracle's third-order (P3) elements.

The element order is a parameter of the quadrature discretization of
Eq. (2) (Section 3 tabulates any basis at the points); the paper evaluates
P1 (Section 6). These pins fix the P3 extension against results that do not
come from the oracle's pointwise evaluation: the P3 basis written here as
exact rational polynomials (its Lagrange property at the cubic lattice is
checked first), exact monomial integration on the reference simplex, the
textbook integrals of the triangle's P3 functions (|T|/30 at vertices,
3|T|/40 at edge nodes, 9|T|/20 at the centre), rigid motions, symmetry,
cubic reproduction and central differences of the adjoint. The degree-4
rules integrate every P3 stiffness entry (degree 4) exactly.

P3 node order: vertices 0..d; per edge (i, j), i < j, lexicographic, the
node at (2/3, 1/3) of (i, j) then the node at (1/3, 2/3); per face
(i, j, k), i < j < k, lexicographic, its centroid.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg

from test_oracle_p2 import _add, _der, _integral, _mul, _scale, geom, physical_gradient_integrals, vol
from test_oracle_pins import random_simplices

LAP, EL, MASS = mg.LAPLACE, mg.ELASTICITY, mg.MASS
HIGH = {2: mg.RULE_TRI6, 3: mg.RULE_TET11}
EDGES = {d: list(itertools.combinations(range(d + 1), 2)) for d in (2, 3)}
FACES = {d: list(itertools.combinations(range(d + 1), 3)) for d in (2, 3)}


def nb3(d):
    return (d + 1) * (d + 2) * (d + 3) // 6


def node_barycentrics(d):
    """Barycentric coordinates (exact) of the P3 nodes, in node order."""
    nodes = []
    for v in range(d + 1):
        nodes.append([Fr(1) if k == v else Fr(0) for k in range(d + 1)])
    for i, j in EDGES[d]:
        for a, b in ((i, j), (j, i)):
            nodes.append([Fr(2, 3) if k == a else (Fr(1, 3) if k == b else Fr(0)) for k in range(d + 1)])
    for f in FACES[d]:
        nodes.append([Fr(1, 3) if k in f else Fr(0) for k in range(d + 1)])
    return nodes


def _eval(p, xi):
    return sum(c * math.prod(x ** a for x, a in zip(xi, al)) for al, c in p.items())


def p3_basis_polys(d):
    """The P3 Lagrange basis as exact polynomials in xi_1..xi_d, built as the
    products of barycentric factors that vanish on the other nodes."""
    z = (0,) * d
    e = [tuple(1 if i == k else 0 for i in range(d)) for k in range(d)]
    one = {z: Fr(1)}
    lam = [_add(one, {ek: Fr(-1) for ek in e})] + [{ek: Fr(1)} for ek in e]

    def lin(l, a, b):          # a * l + b
        return _add(_scale(l, Fr(a)), {z: Fr(b)})
    phi = [_scale(_mul(_mul(l, lin(l, 3, -1)), lin(l, 3, -2)), Fr(1, 2)) for l in lam]
    for i, j in EDGES[d]:
        for a, b in ((i, j), (j, i)):
            phi.append(_scale(_mul(_mul(lam[a], lam[b]), lin(lam[a], 3, -1)), Fr(9, 2)))
    for i, j, k in FACES[d]:
        phi.append(_scale(_mul(_mul(lam[i], lam[j]), lam[k]), Fr(27)))
    return phi


def reference_gradient_integrals3(d):
    phi = p3_basis_polys(d)
    nb = len(phi)
    dphi = [[_der(p, k) for k in range(d)] for p in phi]
    I = np.zeros((d, d, nb, nb))
    for k in range(d):
        for l in range(d):
            for a in range(nb):
                for b in range(a, nb):
                    v = float(_integral(_mul(dphi[a][k], dphi[b][l])))
                    I[k, l, a, b] = v
                    I[l, k, b, a] = v
    return I


def p3_nodes(x):
    """Physical node coordinates of one simplex x[d+1, d]."""
    d = x.shape[1]
    lam = np.array([[float(c) for c in n] for n in node_barycentrics(d)])
    return lam @ x


def columns3(dim, phys, rule, ij, dj, coef, nc):
    n = dj.shape[0]
    nbt = nb3(dim) * nc
    K = np.zeros((nbt, nbt, n))
    for j in range(nbt):
        u = np.zeros((nbt, n))
        u[j] = 1.0
        K[:, j, :] = oracle.integrate(dim, phys, rule, ij, dj, u, coef, order=3)
    return K


# -------------------------------------------------------------------- pins ---

@pytest.mark.parametrize("dim", [2, 3])
def test_p3_test_basis_is_the_lagrange_basis(dim):
    """The polynomials above are 1 at their own node and 0 at the others, and
    sum to one: they are the P3 Lagrange basis in the stated node order."""
    phi = p3_basis_polys(dim)
    nodes = node_barycentrics(dim)
    assert len(phi) == len(nodes) == nb3(dim) == oracle.n_basis(dim, 3)
    for b, p in enumerate(phi):
        for c, lam in enumerate(nodes):
            assert _eval(p, lam[1:]) == (1 if b == c else 0), (b, c)
    total = {}
    for p in phi:
        total = _add(total, p)
    assert {k: v for k, v in total.items() if v != 0} == {(0,) * dim: Fr(1)}


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_laplace_stiffness_exact(dim):
    rng = np.random.default_rng(110 + dim)
    x = random_simplices(dim, 6, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    kap = rng.uniform(0.5, 2, n)
    rule = HIGH[dim]
    coef = np.repeat(kap[None, None, :], oracle.n_qpts(dim, rule), axis=1)
    K = columns3(dim, LAP, rule, ij, dj, coef, 1)
    I = reference_gradient_integrals3(dim)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        assert np.allclose(K[:, :, e], kap[e] * np.einsum("iiab->ab", A), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_elasticity_stiffness_exact(dim):
    rng = np.random.default_rng(120 + dim)
    x = random_simplices(dim, 3, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    lam, mu = rng.uniform(1, 10, n), rng.uniform(0.5, 5, n)
    nq = oracle.n_qpts(dim, HIGH[dim])
    coef = np.stack([np.repeat(lam[None, :], nq, 0), np.repeat(mu[None, :], nq, 0)])
    K = columns3(dim, EL, HIGH[dim], ij, dj, coef, dim)
    I = reference_gradient_integrals3(dim)
    nb = nb3(dim)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        ref = np.zeros((nb * dim, nb * dim))
        for c in range(dim):
            for cp in range(dim):
                ref[c::dim, cp::dim] = lam[e] * A[c, cp] + mu[e] * ((c == cp) * np.einsum("iiab->ab", A) + A[cp, c])
        assert np.allclose(K[:, :, e], ref, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("dim,phys", [(2, LAP), (3, LAP), (2, EL), (3, EL)])
def test_p3_element_matrices_exact(dim, phys):
    """The oracle's element-matrix routine (written from g0/g3, not from its
    residual routine) at order 3 against exact integration of the P3
    gradient products."""
    rng = np.random.default_rng(170 + dim + 5 * phys)
    x = random_simplices(dim, 3, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    nq = oracle.n_qpts(dim, HIGH[dim])
    nb = nb3(dim)
    I = reference_gradient_integrals3(dim)
    if phys == LAP:
        kap = rng.uniform(0.5, 2, n)
        coef = np.repeat(kap[None, None, :], nq, axis=1)
    else:
        lam, mu = rng.uniform(1, 10, n), rng.uniform(0.5, 5, n)
        coef = np.stack([np.repeat(lam[None, :], nq, 0), np.repeat(mu[None, :], nq, 0)])
    nbt = nb * (dim if phys == EL else 1)
    K = oracle.jacobian(dim, phys, HIGH[dim], ij, dj, coef, order=3).reshape(nbt, nbt, n)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        if phys == LAP:
            ref = kap[e] * np.einsum("iiab->ab", A)
        else:
            ref = np.zeros((nbt, nbt))
            for c in range(dim):
                for cp in range(dim):
                    ref[c::dim, cp::dim] = lam[e] * A[c, cp] + mu[e] * ((c == cp) * np.einsum("iiab->ab", A) + A[cp, c])
        assert np.allclose(K[:, :, e], ref, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_basis_integrals(dim):
    """Mass form with u = 1 and unit coefficient gives the integral of every
    basis function (degree 3, exact with the degree-4 rules): the exact
    rational integrals, and on triangles the textbook 1/30, 3/40, 9/20."""
    rng = np.random.default_rng(130 + dim)
    x = random_simplices(dim, 5, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    nq = oracle.n_qpts(dim, HIGH[dim])
    R = oracle.integrate(dim, MASS, HIGH[dim], ij, dj, np.ones((nb3(dim), n)), np.ones((1, nq, n)), order=3)
    exact = np.array([float(_integral(p)) for p in p3_basis_polys(dim)]) * math.factorial(dim)
    if dim == 2:
        assert np.allclose(exact, [1 / 30] * 3 + [3 / 40] * 6 + [9 / 20], rtol=0, atol=1e-15)
    for e in range(n):
        assert np.allclose(R[:, e], vol(x[e]) * exact, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_cubic_reproduction(dim):
    """u interpolating a cubic p is p itself, so with unit coefficient R_b is
    the exact integral of grad p . grad phi_b (computed in exact algebra on
    the reference element mapped affinely)."""
    rng = np.random.default_rng(140 + dim)
    x = random_simplices(dim, 3, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    nq = oracle.n_qpts(dim, HIGH[dim])
    phi = p3_basis_polys(dim)
    # a cubic in reference coordinates, with rational coefficients
    monos = [al for deg in range(4) for al in itertools.product(range(deg + 1), repeat=dim) if sum(al) == deg]
    p = {al: Fr(int(rng.integers(-9, 10)), int(rng.integers(1, 6))) for al in monos}
    nodes = node_barycentrics(dim)
    u_ref = np.array([float(_eval(p, lam[1:])) for lam in nodes])
    R = oracle.integrate(dim, LAP, HIGH[dim], ij, dj, np.repeat(u_ref[:, None], n, 1), np.ones((1, nq, n)), order=3)
    # reference-coordinate gradient integrals G[k][l][b] = int dp/dxi_k dphi_b/dxi_l
    G = np.array([[[float(_integral(_mul(_der(p, k), _der(phi[b], l)))) for b in range(len(phi))]
                   for l in range(dim)] for k in range(dim)])
    for e in range(n):
        J = np.stack([x[e, k + 1] - x[e, 0] for k in range(dim)], axis=1)
        Ji = np.linalg.inv(J)
        ref = abs(np.linalg.det(J)) * np.einsum("ki,li,klb->b", Ji, Ji, G)
        assert np.allclose(R[:, e], ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_p3_rigid_modes_symmetry_and_nulls(dim):
    rng = np.random.default_rng(150 + dim)
    x = random_simplices(dim, 6, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    nq = oracle.n_qpts(dim, HIGH[dim])
    nb = nb3(dim)
    coef = np.stack([rng.uniform(1, 10, (nq, n)), rng.uniform(0.5, 5, (nq, n))])
    X = np.stack([p3_nodes(x[e]) for e in range(n)])
    modes = [np.broadcast_to(np.eye(dim)[c], X.shape) for c in range(dim)]
    if dim == 2:
        modes.append(np.stack([-X[..., 1], X[..., 0]], axis=-1))
    else:
        for w in np.eye(3):
            modes.append(np.cross(w, X))
    for m in modes:
        u = np.ascontiguousarray(m.reshape(n, nb * dim).T)
        assert np.abs(oracle.integrate(dim, EL, HIGH[dim], ij, dj, u, coef, order=3)).max() < 1e-11
    ku = rng.uniform(0.5, 2, (1, nq, n))
    R = oracle.integrate(dim, LAP, HIGH[dim], ij, dj, np.full((nb, n), 0.7), ku, order=3)
    assert np.abs(R).max() < 1e-12
    for phys, nc, cf in [(LAP, 1, ku), (EL, dim, coef), (MASS, 1, ku)]:
        u = rng.normal(size=(nb * nc, n))
        w = rng.normal(size=(nb * nc, n))
        a = np.sum(w * oracle.integrate(dim, phys, HIGH[dim], ij, dj, u, cf, order=3), axis=0)
        b = np.sum(u * oracle.integrate(dim, phys, HIGH[dim], ij, dj, w, cf, order=3), axis=0)
        assert np.allclose(a, b, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("dim,phys,space", [(2, LAP, 0), (3, EL, 1), (3, MASS, 2)])
def test_p3_backward_central_differences(dim, phys, space):
    rng = np.random.default_rng(160 + dim + phys)
    x = random_simplices(dim, 3, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    rule = HIGH[dim]
    nc = dim if phys == EL else 1
    nb = nb3(dim)
    ncoef = 2 if phys == EL else 1
    nw = {0: oracle.n_qpts(dim, rule), 1: dim + 1, 2: 1}[space]
    u = rng.uniform(-1, 1, (nb * nc, n))
    coef = rng.uniform(0.5, 2, (ncoef, nw, n))
    w = rng.uniform(-1, 1, u.shape)
    du, dc = oracle.backward(dim, phys, rule, ij, dj, u, coef, w, space=space, order=3)

    def L(uu, cc):
        return np.sum(w * oracle.integrate(dim, phys, rule, ij, dj, uu, cc, space=space, order=3), axis=0)

    scale = max(np.abs(du).max(), np.abs(dc).max())
    h = 1e-3
    for j in range(0, nb * nc, 5):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        assert np.abs((L(up, coef) - L(um, coef)) / (2 * h) - du[j]).max() <= 1e-9 * scale
    for m in range(ncoef):
        for k in range(nw):
            cp, cm = coef.copy(), coef.copy()
            cp[m, k] += h
            cm[m, k] -= h
            assert np.abs((L(u, cp) - L(u, cm)) / (2 * h) - dc[m, k]).max() <= 1e-9 * scale


def test_p3_order_validation():
    x = random_simplices(2, 2, np.random.default_rng(1))
    ij, dj = geom(x)
    with pytest.raises(ValueError):
        oracle.integrate(2, LAP, mg.RULE_TRI6, ij, dj, np.zeros((15, 2)), np.ones((1, 6, 2)), order=4)
