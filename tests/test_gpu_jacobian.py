"""GPU parity of the element matrices K_e = dR_e/du_e (fem_integrate_jacobian)
against the FP64 oracle, with the bars of the residual tests: per element,
|K_gpu - K_ref| / |K_abs| <= 1e-5 in FP32 and 1e-12 in FP64 (Euclidean
norms over the element's N_bt^2 entries, K_abs the oracle's absolute-value
sums), and the same bound for the aggregate relative error.

Also: exact symmetry of the output, K_e u_e against the residual entry
point of the same order, launch-shape independence (bitwise), NaN
containment for degenerate geometry, empty input, and the full-size meshes
(sampled elements against the oracle, properties over every element).
"""
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
RULES = {(2, 1): (mg.RULE_TRI3, mg.RULE_CENTROID), (3, 1): (mg.RULE_TET4, mg.RULE_CENTROID),
         (2, 2): (mg.RULE_TRI3, mg.RULE_TRI6), (3, 2): (mg.RULE_TET4, mg.RULE_TET11)}
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {}
    for dim, phys in KINDS:
        for order, op in ((1, N.OP_JACOBIAN), (2, N.OP_JACOBIAN_P2)):
            for rule in RULES[(dim, order)]:
                for dt in DTYPES:
                    saved[(op, dim, phys, rule, dt)] = api.fem_get_tuning(dim, phys, rule, dt, op=op)
    yield
    for (op, dim, phys, rule, dt), t in saved.items():
        api.fem_set_tuning(dim, phys, rule, dt, op=op, **t)


def workload(dim, phys, n_elem, seed=61):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    return mg.make_workload(f"jac_{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed)


def coefficients(wl, rule, space, seed=71):
    if space == mg.COEF_QUAD:
        return mg.p2_inputs(wl, rule, mg.BASE_SEED + 6000 + seed).coef
    return mg.space_coefficients(wl, space, mg.BASE_SEED + 6000 + seed)


def nbt(dim, phys, order):
    return oracle.n_basis(dim, order) * (dim if phys == mg.ELASTICITY else 1)


def reference(wl, rule, cf, space, order, dtype, cols=None):
    """Oracle matrices (and abs sums) on the FP64 geometry and the rounded coefficients."""
    ij, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0
    cr = rounded(cf, dtype)
    if cols is not None:
        ij, dj, cr = ij[:, cols], dj[cols], cr[..., cols]
    K = oracle.jacobian(wl.dim, wl.physics, rule, ij, dj, cr, space=space, order=order)
    Ka = oracle.jacobian_abs(wl.dim, wl.physics, rule, ij, dj, cr, space=space, order=order)
    return K, Ka


def geometry(wl, dtype):
    return api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_jacobian_matches_oracle(dim, phys, order, which, space, dtype):
    rule = RULES[(dim, order)][which]
    wl = workload(dim, phys, 1500 if order == 2 else 3001)
    cf = coefficients(wl, rule, space)
    ij, dj = geometry(wl, dtype)
    K = api.fem_integrate_jacobian(dim, phys, rule, ij, dj, dev(cf, dtype), coef_space=space, order=order)
    ref, ref_abs = reference(wl, rule, cf, space, order, dtype)
    assert_close(K.cpu().numpy(), ref, ref_abs, dtype, f"K {dim}D phys {phys} P{order} rule {rule} space {space}")
    m = nbt(dim, phys, order)
    Km = K.reshape(m, m, -1)
    assert torch.equal(Km, Km.transpose(0, 1)), "output not exactly symmetric"


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dtype", DTYPES)
def test_matrix_times_closure_equals_residual(dim, phys, order, dtype):
    """K_e u_e from the matrix entry point against the residual entry point of
    the same order (both on the device), relative to the oracle's
    absolute-value residual sums."""
    rule = RULES[(dim, order)][0]
    wl = workload(dim, phys, 2000, seed=63)
    cf = coefficients(wl, rule, mg.COEF_QUAD, seed=73)
    ij, dj = geometry(wl, dtype)
    m = nbt(dim, phys, order)
    u = mg.p2_inputs(wl, rule, mg.BASE_SEED + 6100).u if order == 2 else wl.u
    ud, cd = dev(u, dtype), dev(cf, dtype)
    K = api.fem_integrate_jacobian(dim, phys, rule, ij, dj, cd, order=order).reshape(m, m, -1)
    Ku = torch.einsum("rse,se->re", K.double(), ud.double()).cpu().numpy()
    if order == 1:
        R = api.fem_integrate_residual(dim, phys, rule, ij, dj, ud, cd)
    else:
        R = api.fem_integrate_residual_p2(dim, phys, rule, ij, dj, ud, cd)
    rij, rdj, _ = oracle.geometry(wl.coords, wl.conn)
    Ra = oracle.integrate_abs(dim, phys, rule, rij, rdj, rounded(u, dtype), rounded(cf, dtype), order=order)
    err = np.linalg.norm(Ku - R.double().cpu().numpy(), axis=0) / np.linalg.norm(Ra, axis=0)
    assert err.max() <= 4 * TOL[dtype], err.max()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim,phys,order", [(3, mg.ELASTICITY, 2), (2, mg.LAPLACE, 1), (3, mg.MASS, 2)])
def test_launch_shapes_bitwise(dtype, dim, phys, order):
    rule = RULES[(dim, order)][1]
    op = N.OP_JACOBIAN if order == 1 else N.OP_JACOBIAN_P2
    wl = workload(dim, phys, 4099, seed=65)
    cf = dev(coefficients(wl, rule, mg.COEF_P1, seed=75), dtype)
    ij, dj = geometry(wl, dtype)
    first = None
    for waves, bpc in [(2, 0), (1, 3), (4, 0), (4, 1)]:
        api.fem_set_tuning(dim, phys, rule, dtype, vec=1, waves_per_block=waves, blocks_per_cu=bpc, op=op)
        K = api.fem_integrate_jacobian(dim, phys, rule, ij, dj, cf, coef_space=mg.COEF_P1, order=order)
        first = K.clone() if first is None else first
        assert torch.equal(K, first), (waves, bpc)


def test_degenerate_geometry_contained():
    """Elements whose geometry is NaN (degenerate) get NaN matrices; the others
    are unaffected."""
    dt = torch.float64
    wl = workload(3, mg.ELASTICITY, 700, seed=67)
    coords = wl.coords.copy()
    conn = wl.conn.copy()
    bad = [5, 300]
    for e in bad:
        conn[e, 3] = conn[e, 2]          # two equal vertices: zero volume
    ij, dj = api.fem_geometry(dev(coords, torch.float64), dev(conn, torch.int32), dt)
    cf = coefficients(wl, mg.RULE_TET4, mg.COEF_QUAD)
    K = api.fem_integrate_jacobian(3, mg.ELASTICITY, mg.RULE_TET4, ij, dj, dev(cf, dt)).cpu().numpy()
    assert np.all(np.isnan(K[:, bad]))
    good = np.setdiff1d(np.arange(wl.n_elem), bad)
    ref, ref_abs = reference(wl, mg.RULE_TET4, cf, mg.COEF_QUAD, 1, dt, cols=good)
    assert_close(K[:, good], ref, ref_abs, dt, "good elements")


def test_empty_and_rejected():
    e = torch.empty((9, 0), device="cuda")
    K = api.fem_integrate_jacobian(3, mg.LAPLACE, mg.RULE_TET4, e, torch.empty(0, device="cuda"),
                                   torch.empty((1, 4, 0), device="cuda"))
    assert K.shape == (16, 0)
    wl = workload(2, mg.LAPLACE, 10)
    ij, dj = geometry(wl, torch.float32)
    with pytest.raises(N.FemError) as ei:
        api.fem_integrate_jacobian(2, mg.LAPLACE, mg.RULE_TRI6, ij, dj, torch.ones((1, 6, 10), device="cuda"),
                                   order=1)
    assert ei.value.status == N.FEM_ERR_UNSUPPORTED
    with pytest.raises(ValueError):   # coefficient words of another rule
        api.fem_integrate_jacobian(2, mg.LAPLACE, mg.RULE_TRI3, ij, dj, torch.ones((1, 6, 10), device="cuda"))


@pytest.mark.parametrize("cfg,order,rule", [(2, 1, mg.RULE_TET4), (2, 2, mg.RULE_TET11), ("3b", 1, mg.RULE_TET4),
                                            ("3b", 2, mg.RULE_TET11)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_meshes(cfg, order, rule, dtype):
    """The benchmark meshes (2^20 tetrahedra, Laplacian; 2^21 tetrahedra,
    elasticity) with coefficients at the points: every element is finite and
    exactly symmetric; 4096 sampled elements (including the first and last)
    match the oracle."""
    wl = mg.config(cfg)
    cf = coefficients(wl, rule, mg.COEF_QUAD, seed=77)
    ij, dj = geometry(wl, dtype)
    m = nbt(wl.dim, wl.physics, order)
    # the largest case, P2 3D elasticity in FP64, writes 900 rows of 2^21
    # elements (15.1 GB); the device holds 288 GB
    assert m * m * wl.n_elem * (4 if dtype == torch.float32 else 8) < (32 << 30)
    K = api.fem_integrate_jacobian(wl.dim, wl.physics, rule, ij, dj, dev(cf, dtype), order=order)
    Km = K.reshape(m, m, -1)
    assert bool(torch.isfinite(K).all())
    for r in range(m):  # row by row: no full-size transposed copy
        assert torch.equal(Km[r], Km[:, r]), r
    rng = np.random.default_rng(5)
    cols = np.unique(np.concatenate([[0, wl.n_elem - 1], rng.integers(0, wl.n_elem, 4094)]))
    got = K[:, torch.from_numpy(cols).to("cuda")].cpu().numpy()
    del K, Km
    ref, ref_abs = reference(wl, rule, cf, mg.COEF_QUAD, order, dtype, cols=cols)
    mx, agg = assert_close(got, ref, ref_abs, dtype, f"{wl.name} P{order}")
    print(f"jacobian {wl.name} P{order} {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)
