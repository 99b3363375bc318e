"""Pins of the oracle's second-order (P2) elements and degree-4 rules.

The element order and the rule are parameters of the quadrature
discretization of Eq. (2); the paper evaluates P1 (Section 6), and these pins
fix the P2 extension against closed forms that do not come from the oracle:
exact monomial integration on the reference simplex (a small exact
polynomial algebra below, independent of the oracle's pointwise
evaluation), the textbook P2 mass matrices |T|/180 [...] and |T|/420 [...],
the P2 stiffness of the reference right triangle, the integrals of the P2
basis functions (0 and |T|/3 on triangles, -|T|/20 and |T|/5 on
tetrahedra) through a quadratic patch test, rigid motions, symmetry and
central differences of the adjoint.

P2 node order: vertices 0..d, then the edges (i, j), i < j, in lexicographic
order.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg

from test_oracle_pins import cayley_menger_volume, heron_area, mesh_from_simplices, random_simplices

LAP, EL, MASS = mg.LAPLACE, mg.ELASTICITY, mg.MASS
HIGH = {2: mg.RULE_TRI6, 3: mg.RULE_TET11}
LOW = {2: mg.RULE_TRI3, 3: mg.RULE_TET4}
EDGES = {d: list(itertools.combinations(range(d + 1), 2)) for d in (2, 3)}


# ------------------------------------------------- exact polynomial algebra ---
# polynomials in xi_1..xi_d as {exponent tuple: Fraction}

def _mono_int(alpha):
    return Fr(math.prod(math.factorial(a) for a in alpha), math.factorial(sum(alpha) + len(alpha)))


def _mul(p, q):
    r = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            r[k] = r.get(k, 0) + ca * cb
    return r


def _scale(p, s):
    return {k: s * v for k, v in p.items()}


def _add(p, q):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0) + v
    return r


def _der(p, k):
    r = {}
    for a, c in p.items():
        if a[k]:
            b = list(a)
            b[k] -= 1
            r[tuple(b)] = r.get(tuple(b), 0) + c * a[k]
    return r


def _integral(p):
    return sum(c * _mono_int(a) for a, c in p.items())


def p2_basis_polys(d):
    z = (0,) * d
    e = [tuple(1 if i == k else 0 for i in range(d)) for k in range(d)]
    lam = [_add({z: Fr(1)}, {ek: Fr(-1) for ek in e})] + [{ek: Fr(1)} for ek in e]
    phi = [_mul(l, _add(_scale(l, 2), {z: Fr(-1)})) for l in lam]
    phi += [_scale(_mul(lam[i], lam[j]), 4) for i, j in EDGES[d]]
    return phi


def reference_gradient_integrals(d):
    """I[k][l][a][b] = integral over the reference simplex of
    d phi_a / d xi_k * d phi_b / d xi_l (exact)."""
    phi = p2_basis_polys(d)
    nb = len(phi)
    return np.array([[[[float(_integral(_mul(_der(phi[a], k), _der(phi[b], l)))) for b in range(nb)]
                       for a in range(nb)] for l in range(d)] for k in range(d)])


def jacobian(x):
    d = x.shape[1]
    J = np.stack([x[k + 1] - x[0] for k in range(d)], axis=1)   # J[i][k]
    return J, np.linalg.inv(J), abs(np.linalg.det(J))


def physical_gradient_integrals(x, I):
    """A[i][j][a][b] = integral over the element of d phi_a/dx_i d phi_b/dx_j."""
    _, Ji, dJ = jacobian(x)          # Ji[k][i] = d xi_k / d x_i
    return dJ * np.einsum("ki,lj,klab->ijab", Ji, Ji, I)


# ------------------------------------------------------------------ helpers ---

def p2_nodes(x):
    """Node coordinates of one simplex x[d+1, d]: vertices then edge midpoints."""
    d = x.shape[1]
    return np.concatenate([x, np.array([(x[i] + x[j]) / 2 for i, j in EDGES[d]])])


def geom(x):
    coords, conn = mesh_from_simplices(x)
    ij, dj, nd = oracle.geometry(coords, conn)
    assert nd == 0
    return ij, dj


def vol(p):
    return heron_area(p) if p.shape[1] == 2 else cayley_menger_volume(p)


def textbook_mass(d):
    """P2 mass matrix / |T| (vertices, then lexicographic edges)."""
    nb = (d + 1) * (d + 2) // 2
    M = np.zeros((nb, nb))
    if d == 2:
        for a in range(3):
            for b in range(3):
                M[a, b] = 6 if a == b else -1
        for v in range(3):
            for k, (i, j) in enumerate(EDGES[2]):
                M[v, 3 + k] = M[3 + k, v] = 0 if v in (i, j) else -4
        for k in range(3):
            for m in range(3):
                M[3 + k, 3 + m] = 32 if k == m else 16
        return M / 180
    for a in range(4):
        for b in range(4):
            M[a, b] = 6 if a == b else 1
    for v in range(4):
        for k, (i, j) in enumerate(EDGES[3]):
            M[v, 4 + k] = M[4 + k, v] = -4 if v in (i, j) else -6
    for k, e in enumerate(EDGES[3]):
        for m, f in enumerate(EDGES[3]):
            M[4 + k, 4 + m] = 32 if k == m else (16 if set(e) & set(f) else 8)
    return M / 420


def columns(dim, phys, rule, ij, dj, coef, nc):
    """Element matrices K[:, :, e] with K[:, j] = R(u = unit_j) (linear forms)."""
    n = dj.shape[0]
    nbt = oracle.n_basis(dim, 2) * nc
    K = np.zeros((nbt, nbt, n))
    for j in range(nbt):
        u = np.zeros((nbt, n))
        u[j] = 1.0
        K[:, j, :] = oracle.integrate(dim, phys, rule, ij, dj, u, coef, order=2)
    return K


# -------------------------------------------------------------------- pins ---

@pytest.mark.parametrize("dim", [2, 3])
def test_degree4_rules(dim):
    xi, w = oracle.rule(dim, HIGH[dim])
    assert np.isclose(w.sum(), 1 / math.factorial(dim), rtol=0, atol=1e-16)
    for deg in range(6):
        err = 0.0
        for al in itertools.product(range(deg + 1), repeat=dim):
            if sum(al) != deg:
                continue
            err = max(err, abs(np.sum(w * np.prod(xi ** np.array(al), axis=1)) - float(_mono_int(al))))
        if deg <= 4:
            assert err < 1e-16, (deg, err)
        else:
            assert err > 1e-6, deg


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_mass_matrix_textbook(dim):
    rng = np.random.default_rng(dim)
    x = random_simplices(dim, 12, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    K = columns(dim, MASS, HIGH[dim], ij, dj, np.ones((1, oracle.n_qpts(dim, HIGH[dim]), n)), 1)
    for e in range(n):
        assert np.allclose(K[:, :, e], vol(x[e]) * textbook_mass(dim), rtol=1e-12, atol=1e-15)
    # a degree-2 rule does not integrate the P2 mass matrix exactly
    K2 = columns(dim, MASS, LOW[dim], ij, dj, np.ones((1, dim + 1, n)), 1)
    assert not np.allclose(K2[:, :, 0], vol(x[0]) * textbook_mass(dim), rtol=1e-6)


@pytest.mark.parametrize("rule", [mg.RULE_TRI3, mg.RULE_TRI6])
def test_p2_stiffness_reference_triangle(rule):
    """Reference right triangle, unit coefficient: the textbook matrix
    (1/6) [[6,1,1,-4,-4,0],[1,3,0,-4,0,0],[1,0,3,0,-4,0],[-4,-4,0,16,0,-8],
    [-4,0,-4,0,16,-8],[0,0,0,-8,-8,16]] (any degree >= 2 rule is exact)."""
    x = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    ij, dj = geom(x)
    K = columns(2, LAP, rule, ij, dj, np.ones((1, oracle.n_qpts(2, rule), 1)), 1)[:, :, 0]
    gold = np.array([[6, 1, 1, -4, -4, 0], [1, 3, 0, -4, 0, 0], [1, 0, 3, 0, -4, 0],
                     [-4, -4, 0, 16, 0, -8], [-4, 0, -4, 0, 16, -8], [0, 0, 0, -8, -8, 16]]) / 6
    assert np.allclose(K, gold, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("which", ["low", "high"])
def test_p2_laplace_stiffness_exact(dim, which):
    rule = (LOW if which == "low" else HIGH)[dim]
    rng = np.random.default_rng(10 + dim)
    x = random_simplices(dim, 10, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    kap = rng.uniform(0.5, 2, n)
    coef = np.repeat(kap[None, None, :], oracle.n_qpts(dim, rule), axis=1)
    K = columns(dim, LAP, rule, ij, dj, coef, 1)
    I = reference_gradient_integrals(dim)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        assert np.allclose(K[:, :, e], kap[e] * np.einsum("iiab->ab", A), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_elasticity_stiffness_exact(dim):
    """Constant Lame coefficients: K[(a,c),(b,c')] = lambda A_{c c'}[a,b]
    + mu (delta_{c c'} sum_i A_ii[a,b] + A_{c' c}[a,b]), A the exact
    physical gradient integrals."""
    rng = np.random.default_rng(20 + dim)
    x = random_simplices(dim, 6, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    lam, mu = rng.uniform(1, 10, n), rng.uniform(0.5, 5, n)
    nq = oracle.n_qpts(dim, HIGH[dim])
    coef = np.stack([np.repeat(lam[None, :], nq, 0), np.repeat(mu[None, :], nq, 0)])
    K = columns(dim, EL, HIGH[dim], ij, dj, coef, dim)
    I = reference_gradient_integrals(dim)
    nb = oracle.n_basis(dim, 2)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        ref = np.zeros((nb * dim, nb * dim))
        for c in range(dim):
            for cp in range(dim):
                blk = lam[e] * A[c, cp] + mu[e] * ((c == cp) * np.einsum("iiab->ab", A) + A[cp, c])
                ref[c::dim, cp::dim] = blk
        assert np.allclose(K[:, :, e], ref, rtol=1e-11, atol=1e-12)


def p2_mesh(dim, n, seed):
    """A jittered grid with P2 nodes: vertices then one node per edge."""
    coords, conn = (mg.tri_grid if dim == 2 else mg.tet_grid)(n, None, np.random.default_rng(seed))
    edge_id = {}
    extra = []
    conn2 = np.zeros((conn.shape[0], oracle.n_basis(dim, 2)), dtype=np.int64)
    conn2[:, :dim + 1] = conn
    for e in range(conn.shape[0]):
        for k, (i, j) in enumerate(EDGES[dim]):
            key = tuple(sorted((conn[e, i], conn[e, j])))
            if key not in edge_id:
                edge_id[key] = coords.shape[0] + len(extra)
                extra.append((coords[key[0]] + coords[key[1]]) / 2)
            conn2[e, dim + 1 + k] = edge_id[key]
    return coords, conn, np.concatenate([coords, np.array(extra)]), conn2


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_quadratic_patch_test(dim):
    """u = p(x) quadratic (reproduced by P2), constant kappa: at interior
    nodes the assembled residual is -kappa (Lap p) (integral of phi_node),
    with the integrals 0 and |T|/3 (triangle vertices, edges) and -|T|/20,
    |T|/5 (tetrahedron vertices, edges)."""
    n = 4 if dim == 2 else 2
    coords, conn, nodes, conn2 = p2_mesh(dim, n, 30 + dim)
    ne, nn = conn.shape[0], nodes.shape[0]
    rng = np.random.default_rng(40 + dim)
    Q = rng.normal(size=(dim, dim))
    Q = Q + Q.T
    g = rng.normal(size=dim)
    p = np.einsum("ni,ij,nj->n", nodes, Q, nodes) + nodes @ g + 0.3     # Lap p = 2 tr Q
    kappa = 1.7
    ij, dj, _ = oracle.geometry(coords, conn)
    u = p[conn2].T
    nq = oracle.n_qpts(dim, HIGH[dim])
    R = oracle.integrate(dim, LAP, HIGH[dim], ij, dj, u, np.full((1, nq, ne), kappa), order=2)
    F = np.zeros(nn)
    np.add.at(F, conn2.T.ravel(), R.ravel())
    expect = np.zeros(nn)
    w_v, w_e = (0.0, 1 / 3) if dim == 2 else (-1 / 20, 1 / 5)
    for e in range(ne):
        V = vol(coords[conn[e]])
        expect[conn2[e, :dim + 1]] += w_v * V
        expect[conn2[e, dim + 1:]] += w_e * V
    expect *= -kappa * 2 * np.trace(Q)
    # interior nodes: away from the boundary of the unit square / cube
    interior = np.all((nodes > 1e-9) & (nodes < 1 - 1e-9), axis=1)
    assert interior.sum() > 3
    assert np.allclose(F[interior], expect[interior], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_rigid_modes_symmetry_and_nulls(dim):
    rng = np.random.default_rng(50 + dim)
    x = random_simplices(dim, 8, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    nq = oracle.n_qpts(dim, HIGH[dim])
    nb = oracle.n_basis(dim, 2)
    coef = np.stack([rng.uniform(1, 10, (nq, n)), rng.uniform(0.5, 5, (nq, n))])
    X = np.stack([p2_nodes(x[e]) for e in range(n)])                # [n, nb, d]
    modes = [np.broadcast_to(np.eye(dim)[c], X.shape) for c in range(dim)]
    if dim == 2:
        modes.append(np.stack([-X[..., 1], X[..., 0]], axis=-1))
    else:
        for w in np.eye(3):
            modes.append(np.cross(w, X))
    for m in modes:
        u = np.ascontiguousarray(m.reshape(n, nb * dim).T)
        R = oracle.integrate(dim, EL, HIGH[dim], ij, dj, u, coef, order=2)
        assert np.abs(R).max() < 1e-12
    ku = rng.uniform(0.5, 2, (1, nq, n))
    R = oracle.integrate(dim, LAP, HIGH[dim], ij, dj, np.full((nb, n), 0.7), ku, order=2)
    assert np.abs(R).max() < 1e-13
    for phys, nc, cf in [(LAP, 1, ku), (EL, dim, coef), (MASS, 1, ku)]:
        u = rng.normal(size=(nb * nc, n))
        w = rng.normal(size=(nb * nc, n))
        a = np.sum(w * oracle.integrate(dim, phys, HIGH[dim], ij, dj, u, cf, order=2), axis=0)
        b = np.sum(u * oracle.integrate(dim, phys, HIGH[dim], ij, dj, w, cf, order=2), axis=0)
        assert np.allclose(a, b, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dim,phys", [(2, LAP), (3, LAP), (2, EL), (3, EL), (3, MASS)])
@pytest.mark.parametrize("space", [0, 1, 2])
def test_p2_backward_central_differences(dim, phys, space):
    rng = np.random.default_rng(60 + 7 * dim + phys + 3 * space)
    x = random_simplices(dim, 5, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    rule = HIGH[dim]
    nc = dim if phys == EL else 1
    nb = oracle.n_basis(dim, 2)
    ncoef = 2 if phys == EL else 1
    nw = {0: oracle.n_qpts(dim, rule), 1: dim + 1, 2: 1}[space]
    u = rng.uniform(-1, 1, (nb * nc, n))
    coef = rng.uniform(0.5, 2, (ncoef, nw, n))
    w = rng.uniform(-1, 1, u.shape)
    du, dc = oracle.backward(dim, phys, rule, ij, dj, u, coef, w, space=space, order=2)

    def L(uu, cc):
        return np.sum(w * oracle.integrate(dim, phys, rule, ij, dj, uu, cc, space=space, order=2), axis=0)

    scale = max(np.abs(du).max(), np.abs(dc).max())
    for j in range(0, nb * nc, 3):
        h = 1e-3
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        assert np.abs((L(up, coef) - L(um, coef)) / (2 * h) - du[j]).max() <= 1e-9 * scale
    for m in range(ncoef):
        for k in range(nw):
            h = 1e-3
            cp, cm = coef.copy(), coef.copy()
            cp[m, k] += h
            cm[m, k] -= h
            assert np.abs((L(u, cp) - L(u, cm)) / (2 * h) - dc[m, k]).max() <= 1e-9 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_linear_coefficient_same_in_every_space(dim):
    """A coefficient linear in x has exact P1 nodal values: with the P2 basis
    for u, the P1 space still gives the point-value result."""
    rng = np.random.default_rng(70 + dim)
    x = random_simplices(dim, 8, rng)
    ij, dj = geom(x)
    n = x.shape[0]
    rule = HIGH[dim]
    xi, _ = oracle.rule(dim, rule)
    lam = np.concatenate([1 - xi.sum(1, keepdims=True), xi], axis=1)
    xq = np.einsum("qb,nbi->nqi", lam, x)
    a = rng.normal(size=dim)
    cq = (xq @ a + 3.0).T[None]
    c1 = (x @ a + 3.0).T[None]
    u = rng.normal(size=(oracle.n_basis(dim, 2), n))
    Rq = oracle.integrate(dim, LAP, rule, ij, dj, u, cq, space=0, order=2)
    R1 = oracle.integrate(dim, LAP, rule, ij, dj, u, c1, space=1, order=2)
    assert np.allclose(R1, Rq, rtol=1e-12, atol=1e-13)


def test_order_and_rule_validation():
    x = random_simplices(2, 2, np.random.default_rng(1))
    ij, dj = geom(x)
    with pytest.raises(ValueError):
        oracle.integrate(2, LAP, mg.RULE_TRI6, ij, dj, np.zeros((6, 2)), np.ones((1, 6, 2)), order=4)
    with pytest.raises(ValueError):
        oracle.integrate(2, LAP, mg.RULE_TET11, ij, dj, np.zeros((6, 2)), np.ones((1, 11, 2)), order=2)
