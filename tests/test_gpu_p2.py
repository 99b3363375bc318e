"""GPU parity of second-order (P2) elements through the C ABI against the
FP64 oracle (order 2), with the bars of the P1 tests: scaled per-element
error and aggregate error <= 1e-5 in FP32, <= 1e-12 in FP64."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import TOL, assert_close, dev, rounded

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
KINDS = [(2, mg.LAPLACE), (3, mg.LAPLACE), (2, mg.ELASTICITY), (3, mg.ELASTICITY), (2, mg.MASS), (3, mg.MASS)]
RULES = {2: (mg.RULE_TRI3, mg.RULE_TRI6), 3: (mg.RULE_TET4, mg.RULE_TET11)}
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]


def workload(dim, phys, n_elem, rule, seed=41):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    wl = mg.make_workload(f"p2_{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed)
    return wl, mg.p2_inputs(wl, rule, mg.BASE_SEED + 3000 + seed)


def coefficients(wl, p2, space):
    if space == mg.COEF_QUAD:
        return p2.coef
    return mg.space_coefficients(wl, space, mg.BASE_SEED + 4000)


def reference(wl, p2, cf, space, dtype, u=None):
    ij, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0
    u = p2.u if u is None else u
    ur, cr = rounded(u, dtype), rounded(cf, dtype)
    R = oracle.integrate(wl.dim, wl.physics, p2.rule, ij, dj, ur, cr, space=space, order=2)
    Ra = oracle.integrate_abs(wl.dim, wl.physics, p2.rule, ij, dj, ur, cr, space=space, order=2)
    return R, Ra


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {}
    for dim, phys in KINDS:
        for rule in RULES[dim]:
            for dt in DTYPES:
                for op in (N.OP_RESIDUAL_P2, N.OP_BACKWARD_P2):
                    saved[(dim, phys, rule, dt, op)] = api.fem_get_tuning(dim, phys, rule, dt, op=op)
    yield
    for (dim, phys, rule, dt, op), t in saved.items():
        api.fem_set_tuning(dim, phys, rule, dt, op=op, **t)


def geometry(wl, dtype):
    return api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("high", [False, True])
@pytest.mark.parametrize("space", SPACES)
def test_p2_forward_matches_oracle(dim, phys, dtype, high, space):
    rule = RULES[dim][int(high)]
    wl, p2 = workload(dim, phys, 2049, rule)
    cf = coefficients(wl, p2, space)
    ij, dj = geometry(wl, dtype)
    R = api.fem_integrate_residual_p2(dim, phys, rule, ij, dj, dev(p2.u, dtype), dev(cf, dtype), coef_space=space)
    ref, ref_abs = reference(wl, p2, cf, space, dtype)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"P2 {dim}D phys {phys} rule {rule} space {space}")


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("space", SPACES)
def test_p2_backward_matches_oracle(dim, phys, dtype, space):
    rule = RULES[dim][1]
    wl, p2 = workload(dim, phys, 1025, rule, seed=43)
    cf = coefficients(wl, p2, space)
    ij, dj = geometry(wl, dtype)
    du, dc = api.fem_integrate_residual_p2_backward(dim, phys, rule, ij, dj, dev(p2.u, dtype), dev(cf, dtype),
                                                    dev(p2.w, dtype), coef_space=space)
    rij, rdj, _ = oracle.geometry(wl.coords, wl.conn)
    ur, cr, wr = rounded(p2.u, dtype), rounded(cf, dtype), rounded(p2.w, dtype)
    rdu, rdc = oracle.backward(dim, phys, rule, rij, rdj, ur, cr, wr, space=space, order=2)
    du_abs = oracle.integrate_abs(dim, phys, rule, rij, rdj, wr, cr, space=space, order=2)
    assert_close(du.cpu().numpy(), rdu, du_abs, dtype, "du")
    # dcoef scale: |w| . R_abs(u; unit coefficient word)
    nco, nw, n = rdc.shape
    dc_abs = np.zeros_like(rdc)
    for m in range(nco):
        for k in range(nw):
            unit = np.zeros_like(rdc)
            unit[m, k] = 1.0
            dc_abs[m, k] = np.sum(np.abs(wr) * oracle.integrate_abs(dim, phys, rule, rij, rdj, ur, unit,
                                                                    space=space, order=2), axis=0)
    assert_close(dc.cpu().numpy().reshape(nco * nw, n), rdc.reshape(nco * nw, n), dc_abs.reshape(nco * nw, n),
                 dtype, "dcoef")
    R_w = api.fem_integrate_residual_p2(dim, phys, rule, ij, dj, dev(p2.w, dtype), dev(cf, dtype), coef_space=space)
    assert torch.equal(du, R_w)


@pytest.mark.parametrize("dtype", DTYPES)
def test_p2_launch_shapes_bitwise(dtype):
    wl, p2 = workload(3, mg.ELASTICITY, 5003, mg.RULE_TET11)
    ij, dj = geometry(wl, dtype)
    u, cf = dev(p2.u, dtype), dev(p2.coef, dtype)
    first = None
    for waves, bpc in [(2, 0), (1, 4), (4, 0), (4, 2)]:
        api.fem_set_tuning(3, mg.ELASTICITY, mg.RULE_TET11, dtype, vec=1, waves_per_block=waves, blocks_per_cu=bpc,
                           op=N.OP_RESIDUAL_P2)
        R = api.fem_integrate_residual_p2(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, u, cf)
        first = R.clone() if first is None else first
        assert torch.equal(R, first), (waves, bpc)
    with pytest.raises(N.FemError):
        api.fem_set_tuning(3, mg.ELASTICITY, mg.RULE_TET11, dtype, vec=1, waves_per_block=8, op=N.OP_RESIDUAL_P2)


def test_p2_autograd_fd():
    dt = torch.float64
    wl, p2 = workload(2, mg.ELASTICITY, 64, mg.RULE_TRI6, seed=47)
    ij, dj = geometry(wl, dt)
    u = dev(p2.u, dt).requires_grad_(True)
    cf = dev(p2.coef, dt).requires_grad_(True)
    w = dev(p2.w, dt)
    L = (api.integrate_residual(2, mg.ELASTICITY, mg.RULE_TRI6, ij, dj, u, cf, order=2) * w).sum()
    L.backward()
    gu, gc = u.grad.cpu().numpy(), cf.grad.cpu().numpy()
    rng = np.random.default_rng(3)

    def Lof(uu, cc):
        return float((api.fem_integrate_residual_p2(2, mg.ELASTICITY, mg.RULE_TRI6, ij, dj, uu, cc) * w).sum())

    with torch.no_grad():
        for _ in range(4):
            j, e = int(rng.integers(u.shape[0])), int(rng.integers(u.shape[1]))
            up, um = u.detach().clone(), u.detach().clone()
            up[j, e] += 1e-3
            um[j, e] -= 1e-3
            assert abs((Lof(up, cf.detach()) - Lof(um, cf.detach())) / 2e-3 - gu[j, e]) <= 1e-9 * np.abs(gu).max()
            m, q = int(rng.integers(2)), int(rng.integers(6))
            cp, cm = cf.detach().clone(), cf.detach().clone()
            h = 1e-3 * max(1.0, abs(p2.coef[m, q, e]))
            cp[m, q, e] += h
            cm[m, q, e] -= h
            assert abs((Lof(u.detach(), cp) - Lof(u.detach(), cm)) / (2 * h) - gc[m, q, e]) <= 1e-9 * np.abs(gc).max()


@pytest.mark.parametrize("dtype", DTYPES)
def test_p2_full_size_laplace3d(dtype):
    """The 2^20-tetrahedron mesh with P2 nodes and the eleven-point rule."""
    wl = mg.config(2)
    p2 = mg.p2_inputs(wl, mg.RULE_TET11, mg.BASE_SEED + 5000)
    ij, dj = geometry(wl, dtype)
    R = api.fem_integrate_residual_p2(3, mg.LAPLACE, mg.RULE_TET11, ij, dj, dev(p2.u, dtype), dev(p2.coef, dtype))
    ref, ref_abs = reference(wl, p2, p2.coef, mg.COEF_QUAD, dtype)
    mx, agg = assert_close(R.cpu().numpy(), ref, ref_abs, dtype, "P2 laplace3d 2^20")
    print(f"P2 laplace3d 2^20 {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)


def test_p2_empty_and_rejected():
    e = torch.empty((9, 0), device="cuda")
    R = api.fem_integrate_residual_p2(3, mg.LAPLACE, mg.RULE_TET4, e, torch.empty(0, device="cuda"),
                                      torch.empty((10, 0), device="cuda"), torch.empty((1, 4, 0), device="cuda"))
    assert R.shape == (10, 0)
    wl, p2 = workload(2, mg.LAPLACE, 10, mg.RULE_TRI6)
    ij, dj = geometry(wl, torch.float32)
    with pytest.raises(N.FemError) as ei:
        api.fem_integrate_residual_p2(2, mg.LAPLACE, mg.RULE_CENTROID, ij, dj, dev(p2.u, torch.float32),
                                      torch.ones((1, 1, 10), device="cuda"))
    assert ei.value.status == N.FEM_ERR_UNSUPPORTED
