"""Pins of the oracle's coefficient spaces (paper Section 4, "Variable Coefficients": an auxiliary
field on quadrature points, in the P1 space of u, or constant per cell)."""
import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg

from test_oracle_pins import (bary_gradients, cayley_menger_volume, heron_area, mesh_from_simplices,
                              random_simplices, voigt_B, voigt_D)

LAP, EL, MASS = mg.LAPLACE, mg.ELASTICITY, mg.MASS
QUAD, P1, P0 = 0, 1, 2
RULES = {2: mg.RULE_TRI3, 3: mg.RULE_TET4}


def geom(x):
    coords, conn = mesh_from_simplices(x)
    ij, dj, nd = oracle.geometry(coords, conn)
    assert nd == 0
    return ij, dj


def vol(p):
    return heron_area(p) if p.shape[1] == 2 else cayley_menger_volume(p)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("rule_kind", ["default", "centroid"])
def test_laplace_p1_and_p0_closed_forms(dim, rule_kind):
    """P1 kappa: the symmetric rules average the nodal values, so
    R = mean(kappa_b) |T| G G^T u; P0: R = kappa_e |T| G G^T u."""
    rng = np.random.default_rng(30 + dim)
    rule = RULES[dim] if rule_kind == "default" else mg.RULE_CENTROID
    x = random_simplices(dim, 25, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    u = rng.uniform(-1, 1, (dim + 1, n))
    k1 = rng.uniform(0.5, 2, (1, dim + 1, n))
    k0 = rng.uniform(0.5, 2, (1, 1, n))
    R1 = oracle.integrate(dim, LAP, rule, ij, dj, u, k1, space=P1)
    R0 = oracle.integrate(dim, LAP, rule, ij, dj, u, k0, space=P0)
    for e in range(n):
        g, V = bary_gradients(x[e])
        K = V * g @ g.T
        assert np.allclose(R1[:, e], k1[0, :, e].mean() * K @ u[:, e], rtol=1e-11, atol=1e-14)
        assert np.allclose(R0[:, e], k0[0, 0, e] * K @ u[:, e], rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_elasticity_p1_and_p0_closed_forms(dim):
    rng = np.random.default_rng(40 + dim)
    x = random_simplices(dim, 20, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    u = rng.uniform(-1, 1, ((dim + 1) * dim, n))
    c1 = np.stack([rng.uniform(1, 10, (dim + 1, n)), rng.uniform(0.5, 5, (dim + 1, n))])
    c0 = np.stack([rng.uniform(1, 10, (1, n)), rng.uniform(0.5, 5, (1, n))])
    R1 = oracle.integrate(dim, EL, RULES[dim], ij, dj, u, c1, space=P1)
    R0 = oracle.integrate(dim, EL, RULES[dim], ij, dj, u, c0, space=P0)
    for e in range(n):
        g, V = bary_gradients(x[e])
        B = voigt_B(g)
        K1 = V * B.T @ voigt_D(dim, c1[0, :, e].mean(), c1[1, :, e].mean()) @ B
        K0 = V * B.T @ voigt_D(dim, c0[0, 0, e], c0[1, 0, e]) @ B
        assert np.allclose(R1[:, e], K1 @ u[:, e], rtol=1e-10, atol=1e-13)
        assert np.allclose(R0[:, e], K0 @ u[:, e], rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_p1_coefficient_exact(dim):
    """u = 1 and a P1 kappa: R_b = int phi_b kappa = (M kappa)_b exactly
    (degree 2), which pins the node order of the P1 coefficient words."""
    rng = np.random.default_rng(50 + dim)
    x = random_simplices(dim, 20, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    k = rng.uniform(0.5, 2, (1, dim + 1, n))
    R = oracle.integrate(dim, MASS, RULES[dim], ij, dj, np.ones((dim + 1, n)), k, space=P1)
    den = 12.0 if dim == 2 else 20.0
    for e in range(n):
        M = vol(x[e]) * (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / den
        assert np.allclose(R[:, e], M @ k[0, :, e], rtol=1e-12, atol=1e-15)
    # rotating the node order of the coefficient changes the answer
    R2 = oracle.integrate(dim, MASS, RULES[dim], ij, dj, np.ones((dim + 1, n)), np.roll(k, 1, axis=1), space=P1)
    assert not np.allclose(R2, R, rtol=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("phys", [LAP, EL, MASS])
def test_linear_coefficient_same_in_every_space(dim, phys):
    """A coefficient that is linear in x is represented exactly by its P1
    nodal values and by its values at the points: both give the same R."""
    rng = np.random.default_rng(60 + dim + 3 * phys)
    x = random_simplices(dim, 20, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    nc = dim if phys == EL else 1
    ncoef = 2 if phys == EL else 1
    u = rng.uniform(-1, 1, ((dim + 1) * nc, n))
    xi, _ = oracle.rule(dim, RULES[dim])
    lam = np.concatenate([1 - xi.sum(1, keepdims=True), xi], axis=1)   # [q, b]
    xq = np.einsum("qb,nbi->nqi", lam, x)
    cq, c1 = [], []
    for m in range(ncoef):
        a = rng.normal(size=dim)
        c0 = 3.0 + m
        cq.append((xq @ a + c0).T)           # [q, n]
        c1.append((x @ a + c0).T)            # [b, n]
    Rq = oracle.integrate(dim, phys, RULES[dim], ij, dj, u, np.stack(cq), space=QUAD)
    R1 = oracle.integrate(dim, phys, RULES[dim], ij, dj, u, np.stack(c1), space=P1)
    assert np.allclose(R1, Rq, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dim,phys", [(2, LAP), (3, LAP), (2, EL), (3, EL), (2, MASS), (3, MASS)])
@pytest.mark.parametrize("space", [P1, P0])
def test_backward_central_differences_spaces(dim, phys, space):
    rng = np.random.default_rng(70 + dim + 3 * phys + space)
    x = random_simplices(dim, 16, rng)
    n = x.shape[0]
    ij, dj = geom(x)
    nc = dim if phys == EL else 1
    ncoef = 2 if phys == EL else 1
    nw = dim + 1 if space == P1 else 1
    u = rng.uniform(-1, 1, ((dim + 1) * nc, n))
    coef = rng.uniform(0.5, 2, (ncoef, nw, n))
    w = rng.uniform(-1, 1, u.shape)
    rule = RULES[dim]
    du, dc = oracle.backward(dim, phys, rule, ij, dj, u, coef, w, space=space)
    assert dc.shape == (ncoef, nw, n)

    def L(uu, cc):
        return np.sum(w * oracle.integrate(dim, phys, rule, ij, dj, uu, cc, space=space), axis=0)

    scale = max(np.abs(du).max(), np.abs(dc).max())
    for m in range(ncoef):
        for k in range(nw):
            h = 1e-3 * np.maximum(1.0, np.abs(coef[m, k]))
            cp, cm = coef.copy(), coef.copy()
            cp[m, k] += h
            cm[m, k] -= h
            fd = (L(u, cp) - L(u, cm)) / (2 * h)
            assert np.abs(fd - dc[m, k]).max() <= 1e-9 * scale
    j = 1
    h = 1e-3 * np.maximum(1.0, np.abs(u[j]))
    up, um = u.copy(), u.copy()
    up[j] += h
    um[j] -= h
    assert np.abs((L(up, coef) - L(um, coef)) / (2 * h) - du[j]).max() <= 1e-9 * scale


def test_unknown_space_rejected():
    x = random_simplices(2, 2, np.random.default_rng(1))
    ij, dj = geom(x)
    with pytest.raises(ValueError):
        oracle.integrate(2, LAP, mg.RULE_TRI3, ij, dj, np.zeros((3, 2)), np.ones((1, 3, 2)), space=7)
