"""GPU parity of the matrix-core transposition for P3 tetrahedra
(FEM_STRATEGY_MFMA of fem_integrate_residual_p3; Section 3's quadrature and
basis phases with the two tabulation contractions of Eq. (2) on the matrix
cores) against the FP64 oracle at order 3, with the bars of the other
parity tests: scaled per-element error and aggregate error <= 1e-5 in FP32,
<= 1e-12 in FP64. Sizes span partial 16-element groups, several waves and a
ragged tail; every coefficient space; launch shapes give the same bits; the
benchmark mesh (2^21 tetrahedra, elasticity) is checked on sampled
elements."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, rounded

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
PHYS = [mg.LAPLACE, mg.ELASTICITY]
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]
R11 = mg.RULE_TET11


def workload(phys, n_elem, seed=181):
    grid = mg.smallest_grid(3, max(n_elem, 1))
    wl = mg.make_workload(f"p3m_{phys}", 3, phys, grid, n_elem, mg.BASE_SEED + seed)
    return wl, mg.p3_inputs(wl, R11, mg.BASE_SEED + 7000 + seed)


def coefficients(wl, p3, space):
    return p3.coef if space == mg.COEF_QUAD else mg.space_coefficients(wl, space, mg.BASE_SEED + 7500)


def reference(wl, u, cf, space, dtype, cols=None):
    ij, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0
    ur, cr = rounded(u, dtype), rounded(cf, dtype)
    if cols is not None:
        ij, dj, ur, cr = ij[:, cols], dj[cols], ur[:, cols], cr[..., cols]
    R = oracle.integrate(3, wl.physics, R11, ij, dj, ur, cr, space=space, order=3)
    Ra = oracle.integrate_abs(3, wl.physics, R11, ij, dj, ur, cr, space=space, order=3)
    return R, Ra


def set_mfma(phys, dtype, waves=4, bpc=0):
    api.fem_set_tuning(3, phys, R11, dtype, op=N.OP_RESIDUAL_P3, strategy=N.STRATEGY_MFMA, vec=1,
                       waves_per_block=waves, blocks_per_cu=bpc)


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {(p, dt): api.fem_get_tuning(3, p, R11, dt, op=N.OP_RESIDUAL_P3) for p in PHYS for dt in DTYPES}
    yield
    for (p, dt), t in saved.items():
        api.fem_set_tuning(3, p, R11, dt, op=N.OP_RESIDUAL_P3, **t)


@pytest.mark.parametrize("phys", PHYS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("n_elem", [1, 15, 16, 17, 1500, 4099])
def test_mfma_matches_oracle(phys, dtype, space, n_elem):
    print(f"p3 mfma phys {phys} {dtype} space {space} n {n_elem}", flush=True)
    wl, p3 = workload(phys, n_elem)
    cf = coefficients(wl, p3, space)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(cf, dtype)
    set_mfma(phys, dtype)
    R = api.fem_integrate_residual_p3(3, phys, R11, ij, dj, u, c, coef_space=space)
    ref, ref_abs = reference(wl, p3.u, cf, space, dtype)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"P3 MFMA phys {phys} space {space} n {n_elem}")
    # every launch shape gives the same bits
    for waves, bpc in ((1, 0), (2, 2), (4, 8), (1, 1)):
        set_mfma(phys, dtype, waves, bpc)
        R2 = api.fem_integrate_residual_p3(3, phys, R11, ij, dj, u, c, coef_space=space)
        assert torch.equal(R, R2), (waves, bpc)


@pytest.mark.parametrize("dtype", DTYPES)
def test_mfma_full_size_elasticity(dtype):
    """The 2^21-tetrahedron elasticity mesh with P3 closures: every output
    finite; 4096 sampled elements (first and last included) against the
    oracle; the lane kernel agrees within the same bar."""
    wl = mg.config("3b")
    p3 = mg.p3_inputs(wl, R11, mg.BASE_SEED + 7700)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(p3.coef, dtype)
    set_mfma(mg.ELASTICITY, dtype)
    R = api.fem_integrate_residual_p3(3, mg.ELASTICITY, R11, ij, dj, u, c)
    assert bool(torch.isfinite(R).all())
    rng = np.random.default_rng(19)
    cols = np.unique(np.concatenate([[0, wl.n_elem - 1], rng.integers(0, wl.n_elem, 4094)]))
    idx = torch.from_numpy(cols).to("cuda")
    got = R[:, idx].cpu().numpy()
    api.fem_set_tuning(3, mg.ELASTICITY, R11, dtype, op=N.OP_RESIDUAL_P3, strategy=N.STRATEGY_LANE, vec=1,
                       waves_per_block=1, blocks_per_cu=0)
    lane = api.fem_integrate_residual_p3(3, mg.ELASTICITY, R11, ij, dj, u, c)[:, idx].cpu().numpy()
    del R
    ref, ref_abs = reference(wl, p3.u, p3.coef, mg.COEF_QUAD, dtype, cols=cols)
    mx, agg = assert_close(got, ref, ref_abs, dtype, "P3 MFMA elasticity 2^21")
    assert_close(lane, ref, ref_abs, dtype, "P3 lane elasticity 2^21")
    print(f"P3 MFMA elasticity 2^21 {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)
