"""GPU: the fused from-mesh residual with run-time per-wave vertex
deduplication (FEM_STRATEGY_DEDUP) against the lane strategy of the same
entry point, bit for bit (element vectors, optional geometry outputs and the
degenerate / poor-shape counters), and against the FP64 oracle.

Cases: every P1 physics in 2D and 3D, FP32 and FP64, the three coefficient
spaces, ragged sizes (1, 63, 64, 65, 4099, 20004), four launch shapes, tiles
whose distinct vertices exceed the staging capacity (random connectivity:
up to 256 distinct vertices per 64-element tile, so part of the vertices
take the direct-gather path), degenerate elements and out-of-range indices,
and the full-size 3D Laplacian step workload."""
import numpy as np
import pytest
import torch

from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, oracle_reference

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
KINDS = [(2, mg.LAPLACE), (3, mg.LAPLACE), (2, mg.ELASTICITY), (3, mg.ELASTICITY), (2, mg.MASS), (3, mg.MASS)]
SHAPES = [(2, 0), (4, 0), (4, 2), (2, 8)]


def small_workload(dim, phys, n_elem, seed):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    return mg.make_workload(f"d{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed)


def _fused(wl, coords, conn, u, cf, dtype, strategy, waves=4, bpc=0, space=mg.COEF_QUAD, geometry=False):
    api.fem_set_tuning(wl.dim, wl.physics, wl.rule, dtype, strategy=strategy, vec=1, waves_per_block=waves,
                       blocks_per_cu=bpc, op=N.OP_RESIDUAL_MESH)
    c = torch.zeros(2, dtype=torch.int32, device="cuda")
    kw = {}
    if geometry:
        ng = wl.dim * wl.dim
        kw = dict(inv_j=torch.full((ng, conn.shape[0]), float("nan"), dtype=dtype, device="cuda"),
                  det_j=torch.full((conn.shape[0],), float("nan"), dtype=dtype, device="cuda"))
    R = api.fem_integrate_residual_mesh(wl.dim, wl.physics, wl.rule, coords, conn, u, cf, counts=c,
                                        coef_space=space, **kw)
    torch.cuda.synchronize()
    return R, c, kw


@pytest.fixture
def restore():
    saved = {}
    for dim, phys in KINDS:
        for dt in DTYPES:
            saved[(dim, phys, dt)] = api.fem_get_tuning(dim, phys, mg.default_rule(dim), dt, op=N.OP_RESIDUAL_MESH)
    yield
    for (dim, phys, dt), t in saved.items():
        api.fem_set_tuning(dim, phys, mg.default_rule(dim), dt, op=N.OP_RESIDUAL_MESH, **t)


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 63, 64, 65, 4099, 20004])
def test_dedup_bitwise_equals_lane(dim, phys, dtype, n_elem, restore):
    wl = small_workload(dim, phys, n_elem, seed=61)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
    R0, c0, g0 = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_LANE, geometry=True)
    for waves, bpc in SHAPES:
        R, c, g = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_DEDUP, waves, bpc, geometry=True)
        assert torch.equal(R, R0), f"dedup != lane at launch {(waves, bpc)}"
        assert torch.equal(g["inv_j"], g0["inv_j"]) and torch.equal(g["det_j"], g0["det_j"])
        assert torch.equal(c, c0)
        R2, _, _ = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_DEDUP, waves, bpc)
        assert torch.equal(R2, R0)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"dedup {dim}D phys {phys}")


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("space", [mg.COEF_P1, mg.COEF_P0])
@pytest.mark.parametrize("dtype", DTYPES)
def test_dedup_coefficient_spaces(dim, space, dtype, restore):
    for phys in (mg.LAPLACE, mg.ELASTICITY):
        wl = small_workload(dim, phys, 5000, seed=62)
        cfs = mg.space_coefficients(wl, space, mg.BASE_SEED + 1000)
        coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
        u, cf = dev(wl.u, dtype), dev(cfs, dtype)
        R0, _, _ = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_LANE, space=space)
        R, _, _ = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_DEDUP, space=space)
        assert torch.equal(R, R0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", DTYPES)
def test_dedup_tiles_beyond_staging_capacity(dim, dtype, restore):
    """Random connectivity over many vertices: most tiles hold more distinct
    vertices than the LDS stage, so the rest go through direct gathers."""
    rng = np.random.default_rng(mg.BASE_SEED + 63)
    n, nv = 20000, 200000
    coords = rng.uniform(-1.0, 1.0, size=(nv, dim))
    conn = rng.integers(0, nv, size=(n, dim + 1)).astype(np.int32)
    conn[::7] = conn[::7, [0] * (dim + 1)]            # some elements with repeated vertices (degenerate)
    conn[5::97, 1] = -3                               # out-of-range indices
    conn[9::89, 0] = nv + 11
    wl = small_workload(dim, mg.ELASTICITY, 10, seed=64)
    ncq = wl.coef.shape[0] * wl.coef.shape[1]
    u = dev(rng.uniform(-1, 1, size=(wl.u.shape[0], n)), dtype)
    cf = dev(rng.uniform(0.5, 2, size=(wl.coef.shape[0], wl.coef.shape[1], n)), dtype)
    assert ncq > 0
    X, C = dev(coords, torch.float64), dev(conn, torch.int32)
    R0, c0, g0 = _fused(wl, X, C, u, cf, dtype, N.STRATEGY_LANE, geometry=True)
    assert int(c0[0]) > 0
    for waves, bpc in SHAPES:
        R, c, g = _fused(wl, X, C, u, cf, dtype, N.STRATEGY_DEDUP, waves, bpc, geometry=True)
        assert torch.equal(R.nan_to_num(7.0), R0.nan_to_num(7.0))
        assert torch.equal(torch.isnan(R), torch.isnan(R0))
        assert torch.equal(g["det_j"].nan_to_num(7.0), g0["det_j"].nan_to_num(7.0))
        assert torch.equal(g["inv_j"].nan_to_num(7.0), g0["inv_j"].nan_to_num(7.0))
        assert torch.equal(c, c0)


def test_dedup_full_step_workload(restore):
    """The 2^20-tetrahedron 3D Laplacian step workload in FP32 and FP64."""
    wl = mg.config(2)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    for dtype in DTYPES:
        u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
        R0, c0, _ = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_LANE)
        R, c, _ = _fused(wl, coords, conn, u, cf, dtype, N.STRATEGY_DEDUP, 4, 0)
        assert torch.equal(R, R0) and torch.equal(c, c0)
        ref, ref_abs, _, _ = oracle_reference(wl, dtype)
        mx, agg = assert_close(R.cpu().numpy(), ref, ref_abs, dtype, "dedup full step")
        print(f"dedup full step {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)


def test_dedup_refused_elsewhere():
    with pytest.raises(N.FemError) as ei:
        api.fem_set_tuning(3, mg.LAPLACE, mg.RULE_TET4, torch.float32, strategy=N.STRATEGY_DEDUP)
    assert ei.value.status == N.FEM_ERR_INVALID_ARG
    with pytest.raises(N.FemError):
        api.fem_set_tuning(3, mg.LAPLACE, mg.RULE_TET4, torch.float32, strategy=N.STRATEGY_DEDUP, vec=2,
                           op=N.OP_RESIDUAL_MESH)
