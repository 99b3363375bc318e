"""GPU parity of the gather form (u, and a P1 coefficient, given per vertex
and gathered through the connectivity inside the fused kernel).

Checks: against the FP64 oracle on the gathered closures; bit for bit
against fem_integrate_residual_mesh on the same closures at every launch
shape; geometry outputs equal to fem_geometry; bad indices counted and
contained; empty input; the full-size 3D Laplace and elasticity workloads.
"""
import numpy as np
import pytest
import torch

from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, oracle_reference

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
KINDS = [(2, mg.LAPLACE), (3, mg.LAPLACE), (2, mg.ELASTICITY), (3, mg.ELASTICITY), (2, mg.MASS), (3, mg.MASS)]
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]


def small_workload(dim, phys, n_elem, rule=None, seed=21):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    return mg.make_workload(f"g{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed, rule=rule)


def inputs(wl, space, seed=5):
    """(per-element coefficient as the closure forms take it, coefficient as
    the gather form takes it)."""
    s = mg.BASE_SEED + 2000 + seed
    cf = mg.space_coefficients(wl, space, s)
    return cf, (mg.vertex_coefficients(wl, s) if space == mg.COEF_P1 else cf)


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {}
    for dim, phys in KINDS:
        for rule in (mg.default_rule(dim), mg.RULE_CENTROID):
            for dt in DTYPES:
                for op in (N.OP_RESIDUAL_MESH, N.OP_RESIDUAL_GATHER):
                    saved[(dim, phys, rule, dt, op)] = api.fem_get_tuning(dim, phys, rule, dt, op=op)
    yield
    for (dim, phys, rule, dt, op), t in saved.items():
        api.fem_set_tuning(dim, phys, rule, dt, op=op, **t)


def gather(wl, dtype, cg, space, **kw):
    return api.fem_integrate_residual_gather(wl.dim, wl.physics, wl.rule, dev(wl.coords, torch.float64),
                                             dev(wl.conn, torch.int32), dev(wl.u_vertex, dtype), dev(cg, dtype),
                                             coef_space=space, **kw)


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_gather_matches_oracle(dim, phys, space, dtype):
    wl = small_workload(dim, phys, 3001)
    cf, cg = inputs(wl, space)
    R = gather(wl, dtype, cg, space)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype, coef=cf, space=space)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"gather {dim}D phys {phys} space {space}")


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_gather_bitwise_equals_closure_form(dim, phys, space, dtype):
    """Same bits as the closure form at every launch shape, and the stored
    geometry equals fem_geometry's."""
    rule = mg.default_rule(dim) if (dim + phys) % 2 else mg.RULE_CENTROID
    wl = small_workload(dim, phys, 4161, rule=rule)
    cf, cg = inputs(wl, space)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    ref = api.fem_integrate_residual_mesh(dim, phys, rule, coords, conn, dev(wl.u, dtype), dev(cf, dtype),
                                          coef_space=space)
    ij, dj = api.fem_geometry(coords, conn, dtype)
    uv, cgd = dev(wl.u_vertex, dtype), dev(cg, dtype)
    for ept, waves, bpc in [(1, 1, 8), (1, 2, 0), (2, 1, 0), (2, 4, 3), (1, 8, 1), (4, 4, 0), (4, 1, 3)]:
        api.fem_set_tuning(dim, phys, rule, dtype, strategy=N.STRATEGY_LANE, vec=ept, waves_per_block=waves,
                           blocks_per_cu=bpc, op=N.OP_RESIDUAL_GATHER)
        ij2, dj2 = torch.full_like(ij, float("nan")), torch.full_like(dj, float("nan"))
        counts = torch.zeros(2, dtype=torch.int32, device="cuda")
        R = api.fem_integrate_residual_gather(dim, phys, rule, coords, conn, uv, cgd, inv_j=ij2, det_j=dj2,
                                              counts=counts, coef_space=space)
        assert torch.equal(R, ref), f"shape {(ept, waves, bpc)}"
        assert torch.equal(ij2, ij) and torch.equal(dj2, dj)
        assert int(counts[0]) == 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_bad_vertex_index_contained(dtype):
    """Indices outside [0, n_vert) make the element degenerate (NaN vector,
    counted); every other element is unaffected."""
    wl = small_workload(3, mg.ELASTICITY, 1000)
    conn = wl.conn.copy()
    bad = [3, 64, 999]
    conn[3, 1] = wl.n_vert
    conn[64, 0] = -1
    conn[999, 3] = 2 ** 31 - 1
    cf, cg = inputs(wl, mg.COEF_P1)
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    R = api.fem_integrate_residual_gather(3, mg.ELASTICITY, wl.rule, dev(wl.coords, torch.float64),
                                          dev(conn, torch.int32), dev(wl.u_vertex, dtype), dev(cg, dtype),
                                          counts=counts, coef_space=mg.COEF_P1).cpu().numpy()
    assert int(counts[0]) == len(bad)
    assert np.all(np.isnan(R[:, bad]))
    good = np.setdiff1d(np.arange(wl.n_elem), bad)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype, coef=cf, space=mg.COEF_P1)
    assert_close(R[:, good], ref[:, good], ref_abs[:, good], dtype, "good elements")


def test_empty_and_argument_errors():
    dt = torch.float32
    coords = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    conn = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    R = api.fem_integrate_residual_gather(3, mg.LAPLACE, mg.RULE_TET4, coords, conn,
                                          torch.zeros((0, 1), dtype=dt, device="cuda"),
                                          torch.zeros((1, 4, 0), dtype=dt, device="cuda"))
    assert R.shape == (4, 0)
    wl = small_workload(2, mg.LAPLACE, 10)
    with pytest.raises(ValueError):   # P1 coefficient must be per vertex in the gather form
        api.fem_integrate_residual_gather(2, mg.LAPLACE, wl.rule, dev(wl.coords, torch.float64),
                                          dev(wl.conn, torch.int32), dev(wl.u_vertex, dt),
                                          dev(mg.space_coefficients(wl, mg.COEF_P1, 1), dt), coef_space=mg.COEF_P1)
    lib = N.lib()
    assert lib.fem_integrate_residual_gather(2, mg.LAPLACE, wl.rule, 0, N.F32, 5, 0, 1, 1, 1, 1, 1, None, None,
                                             None, None) == N.FEM_ERR_INVALID_ARG


@pytest.mark.parametrize("cfg,space", [(2, mg.COEF_QUAD), (2, mg.COEF_P1), ("3b", mg.COEF_P1)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_workloads(cfg, space, dtype):
    wl = mg.config(cfg)
    cf, cg = inputs(wl, space, seed=7)
    R = gather(wl, dtype, cg, space)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype, coef=cf, space=space)
    mx, agg = assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"{wl.name} space {space}")
    print(f"gather {wl.name} space {space} {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)


def test_autotune_gather_op():
    t = api.fem_autotune(3, mg.LAPLACE, mg.RULE_TET4, torch.float32, n_elem_probe=1 << 18, op=N.OP_RESIDUAL_GATHER)
    assert t["vec"] in (1, 2, 4) and t["waves_per_block"] in (1, 2, 4, 8)
    wl = small_workload(3, mg.LAPLACE, 2000)
    cf, cg = inputs(wl, mg.COEF_QUAD)
    R = gather(wl, torch.float32, cg, mg.COEF_QUAD)
    ref, ref_abs, _, _ = oracle_reference(wl, torch.float32, coef=cf)
    assert_close(R.cpu().numpy(), ref, ref_abs, torch.float32, "after autotune")
