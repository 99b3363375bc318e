"""Pins of the oracle's element matrices K_e = dR_e/du_e (the Jacobian of
the bracket of Eq. (2) with respect to the closure).

The oracle writes K from the pointwise derivatives of f0 and f1, not from
its residual routine. These pins tie it to results fixed elsewhere:
  - textbook closed forms: the P1 stiffness |T| kappa g g^T from the
    barycentric gradients of the geometry alone, the constant-strain
    elasticity element |T| B^T D B, the P1 mass matrices |T|/12 (1 + delta)
    and |T|/20 (1 + delta), the P2 mass matrices and the P2 stiffness of the
    reference right triangle;
  - exact polynomial integration of P2 gradient products on the reference
    simplex (no quadrature rule involved);
  - K_e u_e = R_e(u_e) for linear forms, against the residual routine, which
    is pinned on its own;
  - symmetry, the null spaces (constants for the Laplacian, rigid motions for
    elasticity), semi-definiteness and rank, coefficient-space equivalences,
    the absolute-value bound.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg

from test_oracle_pins import bary_gradients, element_arrays, random_simplices, voigt_B, voigt_D
from test_oracle_p2 import (EDGES, geom, p2_nodes, physical_gradient_integrals, reference_gradient_integrals,
                            textbook_mass, vol)
from test_oracle_p3 import p3_nodes

LAP, EL, MASS = mg.LAPLACE, mg.ELASTICITY, mg.MASS
RULES = {(2, 1): [mg.RULE_TRI3, mg.RULE_CENTROID], (3, 1): [mg.RULE_TET4, mg.RULE_CENTROID],
         (2, 2): [mg.RULE_TRI3, mg.RULE_TRI6], (3, 2): [mg.RULE_TET4, mg.RULE_TET11],
         (2, 3): [mg.RULE_TRI6], (3, 3): [mg.RULE_TET11]}
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]


def ncomp(dim, phys):
    return dim if phys == EL else 1


def as_matrices(K, nbt):
    """[N_bt*N_bt, n] -> [n, N_bt, N_bt] (row = test function)."""
    return np.moveaxis(K.reshape(nbt, nbt, -1), 2, 0)


def coefficients(dim, phys, rule, space, n, rng):
    nw = oracle.n_qpts(dim, rule) if space == mg.COEF_QUAD else (dim + 1 if space == mg.COEF_P1 else 1)
    if phys == EL:
        return np.stack([rng.uniform(1, 10, (nw, n)), rng.uniform(0.5, 5, (nw, n))])
    return rng.uniform(0.5, 2, (1, nw, n))


def constant_coef(dim, phys, rule, values):
    """Coefficient array (space QUAD) with one value per field at every point."""
    nq = oracle.n_qpts(dim, rule)
    vals = np.atleast_2d(values)                       # [N_coef, n]
    return np.repeat(vals[:, None, :], nq, axis=1)


# ------------------------------------------------------------ closed forms ---

@pytest.mark.parametrize("dim,rule", [(2, mg.RULE_TRI3), (3, mg.RULE_TET4), (2, mg.RULE_CENTROID),
                                      (3, mg.RULE_CENTROID)])
def test_p1_laplace_stiffness_from_barycentric_gradients(dim, rule):
    """P1, coefficient kappa_q at the points (equal weights): K = |T| mean(kappa) g g^T,
    g the barycentric gradients computed from face normals / edge vectors."""
    rng = np.random.default_rng(100 + dim + rule)
    x = random_simplices(dim, 20, rng)
    ij, dj, _, coef = element_arrays(dim, LAP, rule, x, rng)
    K = as_matrices(oracle.jacobian(dim, LAP, rule, ij, dj, coef), dim + 1)
    for e in range(x.shape[0]):
        g, v = bary_gradients(x[e])
        assert np.allclose(K[e], v * coef[0, :, e].mean() * g @ g.T, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dim,rule", [(2, mg.RULE_TRI3), (3, mg.RULE_TET4), (2, mg.RULE_CENTROID),
                                      (3, mg.RULE_CENTROID)])
def test_p1_elasticity_constant_strain_element(dim, rule):
    """K = |T| B^T D B with the mean Lame coefficients (textbook constant-strain element)."""
    rng = np.random.default_rng(110 + dim + rule)
    x = random_simplices(dim, 20, rng)
    ij, dj, _, coef = element_arrays(dim, EL, rule, x, rng)
    K = as_matrices(oracle.jacobian(dim, EL, rule, ij, dj, coef), (dim + 1) * dim)
    for e in range(x.shape[0]):
        g, v = bary_gradients(x[e])
        B = voigt_B(g)
        D = voigt_D(dim, coef[0, :, e].mean(), coef[1, :, e].mean())
        assert np.allclose(K[e], v * B.T @ D @ B, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dim,rule", [(2, mg.RULE_TRI3), (3, mg.RULE_TET4)])
def test_p1_mass_matrix_closed_form(dim, rule):
    """Degree-2 rules integrate P1 products exactly: |T|/12 (1 + delta) in 2D,
    |T|/20 (1 + delta) in 3D, times a constant kappa."""
    rng = np.random.default_rng(120 + dim)
    x = random_simplices(dim, 15, rng)
    n = x.shape[0]
    kap = rng.uniform(0.5, 2, n)
    ij, dj = geom(x)
    K = as_matrices(oracle.jacobian(dim, MASS, rule, ij, dj, constant_coef(dim, MASS, rule, kap)), dim + 1)
    base = (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / (12 if dim == 2 else 20)
    for e in range(n):
        assert np.allclose(K[e], kap[e] * vol(x[e]) * base, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_mass_matrix_textbook(dim):
    rng = np.random.default_rng(130 + dim)
    x = random_simplices(dim, 10, rng)
    n = x.shape[0]
    rule = RULES[(dim, 2)][1]
    kap = rng.uniform(0.5, 2, n)
    ij, dj = geom(x)
    K = as_matrices(oracle.jacobian(dim, MASS, rule, ij, dj, constant_coef(dim, MASS, rule, kap), order=2),
                    oracle.n_basis(dim, 2))
    for e in range(n):
        assert np.allclose(K[e], kap[e] * vol(x[e]) * textbook_mass(dim), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("rule", [mg.RULE_TRI3, mg.RULE_TRI6])
def test_p2_stiffness_reference_right_triangle(rule):
    """The textbook P2 stiffness of the right triangle (0,0), (1,0), (0,1)."""
    x = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    ij, dj = geom(x)
    K = as_matrices(oracle.jacobian(2, LAP, rule, ij, dj, constant_coef(2, LAP, rule, [1.0]), order=2), 6)[0]
    gold = np.array([[6, 1, 1, -4, -4, 0], [1, 3, 0, -4, 0, 0], [1, 0, 3, 0, -4, 0],
                     [-4, -4, 0, 16, 0, -8], [-4, 0, -4, 0, 16, -8], [0, 0, 0, -8, -8, 16]]) / 6
    assert np.allclose(K, gold, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("high", [False, True])
def test_p2_laplace_exact_integration(dim, high):
    """Constant kappa: K = kappa sum_i A_ii, A the exact integrals of products
    of physical P2 gradients (exact rational integration on the reference
    simplex, mapped by the affine geometry). Both rules are exact here."""
    rule = RULES[(dim, 2)][int(high)]
    rng = np.random.default_rng(140 + dim + 2 * high)
    x = random_simplices(dim, 8, rng)
    n = x.shape[0]
    kap = rng.uniform(0.5, 2, n)
    ij, dj = geom(x)
    K = as_matrices(oracle.jacobian(dim, LAP, rule, ij, dj, constant_coef(dim, LAP, rule, kap), order=2),
                    oracle.n_basis(dim, 2))
    I = reference_gradient_integrals(dim)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        assert np.allclose(K[e], kap[e] * np.einsum("iiab->ab", A), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_elasticity_exact_integration(dim):
    """Constant Lame coefficients, blocks (c, c'): lambda A_cc' + mu (delta_cc'
    sum_i A_ii + A_c'c), from exact integrals (the Lame energy
    lambda div u div v + 2 mu eps(u):eps(v) expanded in gradient products)."""
    rule = RULES[(dim, 2)][1]
    rng = np.random.default_rng(150 + dim)
    x = random_simplices(dim, 5, rng)
    n = x.shape[0]
    lam, mu = rng.uniform(1, 10, n), rng.uniform(0.5, 5, n)
    ij, dj = geom(x)
    K = as_matrices(oracle.jacobian(dim, EL, rule, ij, dj, constant_coef(dim, EL, rule, np.stack([lam, mu])),
                                    order=2), oracle.n_basis(dim, 2) * dim)
    I = reference_gradient_integrals(dim)
    nb = oracle.n_basis(dim, 2)
    for e in range(n):
        A = physical_gradient_integrals(x[e], I)
        ref = np.zeros((nb * dim, nb * dim))
        for c in range(dim):
            for cp in range(dim):
                ref[c::dim, cp::dim] = lam[e] * A[c, cp] + mu[e] * ((c == cp) * np.einsum("iiab->ab", A) + A[cp, c])
        assert np.allclose(K[e], ref, rtol=1e-11, atol=1e-12)


# -------------------------------------------------- consistency and structure ---

CASES = [(d, p, o, r, s) for d in (2, 3) for p in (LAP, EL, MASS) for o in (1, 2, 3) for r in RULES[(d, o)]
         for s in SPACES]


@pytest.mark.parametrize("dim,phys,order,rule,space", CASES)
def test_matrix_times_closure_is_residual(dim, phys, order, rule, space):
    """The forms are linear in u: K_e u_e equals the residual routine's R_e(u_e)
    for variable coefficients in every space."""
    rng = np.random.default_rng(hash((dim, phys, order, rule, space)) % 2 ** 32)
    n = 40
    x = random_simplices(dim, n, rng)
    ij, dj = geom(x)
    coef = coefficients(dim, phys, rule, space, n, rng)
    nbt = oracle.n_basis(dim, order) * ncomp(dim, phys)
    u = rng.uniform(-1, 1, (nbt, n))
    K = as_matrices(oracle.jacobian(dim, phys, rule, ij, dj, coef, space=space, order=order), nbt)
    R = oracle.integrate(dim, phys, rule, ij, dj, u, coef, space=space, order=order)
    Ra = oracle.integrate_abs(dim, phys, rule, ij, dj, u, coef, space=space, order=order)
    Ku = np.einsum("ers,se->re", K, u)
    assert np.all(np.abs(Ku - R) <= 1e-13 * Ra.max(axis=0) + 1e-300)
    # symmetric forms: K = K^T
    Ka = as_matrices(oracle.jacobian_abs(dim, phys, rule, ij, dj, coef, space=space, order=order), nbt)
    assert np.all(np.abs(K - np.swapaxes(K, 1, 2)) <= 1e-14 * Ka.max(axis=(1, 2))[:, None, None])
    # the absolute-value sums bound the matrix entry by entry
    assert np.all(np.abs(K) <= Ka * (1 + 1e-14))


def rigid_modes(nodes):
    """Nodal values [n_modes, N_b*d] of translations and infinitesimal rotations."""
    nb, dim = nodes.shape
    modes = []
    for c in range(dim):
        m = np.zeros((nb, dim))
        m[:, c] = 1.0
        modes.append(m.ravel())
    for a, b in itertools.combinations(range(dim), 2):
        m = np.zeros((nb, dim))
        m[:, a] = -nodes[:, b]
        m[:, b] = nodes[:, a]
        modes.append(m.ravel())
    return np.array(modes)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_null_spaces_definiteness_and_rank(dim, order):
    """Laplacian: null space = constants, rank N_b - 1. Elasticity: null space
    = the d(d+1)/2 rigid motions, rank N_bt - d(d+1)/2. Both positive
    semi-definite for positive coefficients. Mass with a rule that is exact
    for it: positive definite. No rule here integrates the P3 mass matrix
    (degree 6) exactly; with N_q < N_b points it is B^T W B of rank N_q."""
    rule = RULES[(dim, order)][0 if order == 1 else -1]
    rng = np.random.default_rng(170 + dim + 10 * order)
    n = 12
    x = random_simplices(dim, n, rng)
    ij, dj = geom(x)
    nb = oracle.n_basis(dim, order)
    for phys, nnull in ((LAP, 1), (EL, dim * (dim + 1) // 2), (MASS, 0)):
        coef = coefficients(dim, phys, rule, mg.COEF_QUAD, n, rng)
        nbt = nb * ncomp(dim, phys)
        K = as_matrices(oracle.jacobian(dim, phys, rule, ij, dj, coef, order=order), nbt)
        if phys == MASS and order == 3:
            nq = oracle.n_qpts(dim, rule)
            for e in range(n):
                sv = np.linalg.svd(K[e], compute_uv=False)
                assert np.sum(sv > 1e-12 * sv[0]) == nq
            continue
        for e in range(n):
            ev = np.linalg.eigvalsh(0.5 * (K[e] + K[e].T))
            tol = 1e-12 * ev[-1]
            assert ev[0] >= -tol
            assert np.sum(ev <= tol) == nnull, (phys, ev[:nnull + 1])
            if phys == LAP:
                assert np.abs(K[e] @ np.ones(nbt)).max() <= 1e-13 * np.abs(K[e]).max()
            if phys == EL:
                nodes = x[e] if order == 1 else (p2_nodes(x[e]) if order == 2 else p3_nodes(x[e]))
                M = rigid_modes(nodes)
                assert np.abs(K[e] @ M.T).max() <= 1e-12 * np.abs(K[e]).max() * np.abs(M).max()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("phys", [LAP, EL, MASS])
def test_coefficient_spaces_agree_on_constants(dim, order, phys):
    """A coefficient constant on the element gives the same matrix whether it
    is given at the points, as equal nodal P1 values, or as one cell value."""
    rule = RULES[(dim, order)][0]
    rng = np.random.default_rng(190 + dim + 3 * order + phys)
    n = 10
    x = random_simplices(dim, n, rng)
    ij, dj = geom(x)
    vals = coefficients(dim, phys, rule, mg.COEF_P0, n, rng)    # [N_coef, 1, n]
    ref = oracle.jacobian(dim, phys, rule, ij, dj, vals, space=mg.COEF_P0, order=order)
    quad = np.repeat(vals, oracle.n_qpts(dim, rule), axis=1)
    p1 = np.repeat(vals, dim + 1, axis=1)
    for cf, sp in ((quad, mg.COEF_QUAD), (p1, mg.COEF_P1)):
        K = oracle.jacobian(dim, phys, rule, ij, dj, cf, space=sp, order=order)
        assert np.allclose(K, ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())


def test_p1_coefficient_varies_mass_matrix_exact():
    """Mass matrix with a P1 coefficient kappa = sum_v a_v lambda_v on a
    triangle: K_ij = sum_v a_v int lam_i lam_j lam_v, and
    int lam^m = 2 |T| m_0! m_1! m_2! / (|m| + 2)! over the triangle
    (m the multiplicities of i, j, v). The integrand has degree 3, so the
    six-point degree-4 rule is exact."""
    import math
    rng = np.random.default_rng(7)
    x = random_simplices(2, 6, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    a = rng.uniform(0.5, 2, (1, 3, n))
    K = as_matrices(oracle.jacobian(2, MASS, mg.RULE_TRI6, ij, dj, a, space=mg.COEF_P1, order=1), 3)
    for e in range(n):
        T = vol(x[e])
        ref = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                for v in range(3):
                    mult = np.bincount([i, j, v], minlength=3)
                    ref[i, j] += a[0, v, e] * T * 2 * math.prod(math.factorial(m) for m in mult) / math.factorial(5)
        assert np.allclose(K[e], ref, rtol=1e-12, atol=1e-15)


def test_argument_validation():
    ij, dj = geom(random_simplices(2, 2, np.random.default_rng(0)))
    cf = np.ones((1, 3, 2))
    with pytest.raises(ValueError):
        oracle.jacobian(2, LAP, mg.RULE_TRI3, ij, dj, cf, order=4)
    with pytest.raises(ValueError):
        oracle.jacobian(2, 7, mg.RULE_TRI3, ij, dj, cf)
    with pytest.raises(ValueError):
        oracle.jacobian(2, LAP, mg.RULE_TET4, ij, dj, cf)
    with pytest.raises(ValueError):
        oracle.jacobian(2, LAP, mg.RULE_TRI3, ij, dj, cf, space=5)
    assert oracle.jacobian(2, LAP, mg.RULE_TRI3, np.zeros((4, 0)), np.zeros(0), np.zeros((1, 3, 0))).shape == (9, 0)
