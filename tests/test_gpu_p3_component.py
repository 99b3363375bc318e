"""GPU parity of the component-parallel P3 elasticity kernel
(FEM_STRATEGY_COMPONENT of fem_integrate_residual_p3: three waves per
64-tetrahedron tile, one per displacement component, the stress rows
completed through LDS; Section 3's transposition split by component, Eq. (2)
at order 3) against the FP64 oracle, with the bars of the other parity tests:
scaled per-element error and aggregate error <= 1e-5 in FP32, <= 1e-12 in
FP64. Sizes cover a single element, partial and whole tiles, several
workgroups (FP32 also with two tile groups each, so groups past the end of a
range) and a ragged tail; every coefficient space; launch shapes give the
same bits; the benchmark mesh (2^21 tetrahedra) is checked on sampled
elements together with the lane kernel."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, rounded

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
SPACES = [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0]
R11 = mg.RULE_TET11
EL = mg.ELASTICITY


def workload(n_elem, seed=191):
    grid = mg.smallest_grid(3, max(n_elem, 1))
    wl = mg.make_workload("p3c", 3, EL, grid, n_elem, mg.BASE_SEED + seed)
    return wl, mg.p3_inputs(wl, R11, mg.BASE_SEED + 7100 + seed)


def coefficients(wl, p3, space):
    return p3.coef if space == mg.COEF_QUAD else mg.space_coefficients(wl, space, mg.BASE_SEED + 7600)


def reference(wl, u, cf, space, dtype, cols=None):
    ij, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0
    ur, cr = rounded(u, dtype), rounded(cf, dtype)
    if cols is not None:
        ij, dj, ur, cr = ij[:, cols], dj[cols], ur[:, cols], cr[..., cols]
    R = oracle.integrate(3, EL, R11, ij, dj, ur, cr, space=space, order=3)
    Ra = oracle.integrate_abs(3, EL, R11, ij, dj, ur, cr, space=space, order=3)
    return R, Ra


def set_strategy(dtype, strategy, waves=1, bpc=0):
    api.fem_set_tuning(3, EL, R11, dtype, op=N.OP_RESIDUAL_P3, strategy=strategy, vec=1,
                       waves_per_block=waves, blocks_per_cu=bpc)


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {dt: api.fem_get_tuning(3, EL, R11, dt, op=N.OP_RESIDUAL_P3) for dt in DTYPES}
    yield
    for dt, t in saved.items():
        api.fem_set_tuning(3, EL, R11, dt, op=N.OP_RESIDUAL_P3, **t)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("space", SPACES)
@pytest.mark.parametrize("n_elem", [1, 2, 63, 64, 65, 129, 1500, 4099])
def test_component_matches_oracle(dtype, space, n_elem):
    print(f"p3 component {dtype} space {space} n {n_elem}", flush=True)
    wl, p3 = workload(n_elem)
    cf = coefficients(wl, p3, space)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(cf, dtype)
    set_strategy(dtype, N.STRATEGY_COMPONENT)
    R = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c, coef_space=space)
    ref, ref_abs = reference(wl, p3.u, cf, space, dtype)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"P3 component space {space} n {n_elem}")
    # every launch shape gives the same bits (grid-stride over wave tiles)
    shapes = ((2, 0), (1, 2), (1, 1), (2, 8)) if dtype == torch.float32 else ((1, 2), (1, 1), (1, 8))
    for waves, bpc in shapes:
        set_strategy(dtype, N.STRATEGY_COMPONENT, waves, bpc)
        R2 = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c, coef_space=space)
        assert torch.equal(R, R2), (waves, bpc)


@pytest.mark.parametrize("dtype", DTYPES)
def test_component_writes_only_its_elements(dtype):
    """Elements past n are never written: the output rows of a larger buffer
    keep their sentinel beyond n (the tail tile clamps its loads to the last
    element and stores nothing for lanes past the end)."""
    n_elem = 43
    wl, p3 = workload(n_elem)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(p3.coef, dtype)
    set_strategy(dtype, N.STRATEGY_COMPONENT)
    R = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c)
    # the same call into a buffer one sentinel row longer than the output
    out = torch.full((61 * n_elem,), 7.25, dtype=dtype, device="cuda")
    N.check(N.lib().fem_integrate_residual_p3(3, EL, R11, mg.COEF_QUAD, api._DT[dtype], n_elem, api._ptr(ij),
                                              api._ptr(dj), api._ptr(u), api._ptr(c), api._ptr(out), api._stream()),
            "fem_integrate_residual_p3")
    torch.cuda.synchronize()
    assert torch.equal(out[:60 * n_elem].view(60, n_elem), R)
    assert bool((out[60 * n_elem:] == 7.25).all())


@pytest.mark.parametrize("dtype", DTYPES)
def test_component_full_size_elasticity(dtype):
    """The 2^21-tetrahedron elasticity mesh with P3 closures: every output
    finite; 4096 sampled elements (first and last included) against the
    oracle; the lane kernel agrees with both within the same bar."""
    wl = mg.config("3b")
    p3 = mg.p3_inputs(wl, R11, mg.BASE_SEED + 7700)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(p3.coef, dtype)
    set_strategy(dtype, N.STRATEGY_COMPONENT, 1, 0)
    R = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c)
    assert bool(torch.isfinite(R).all())
    rng = np.random.default_rng(23)
    cols = np.unique(np.concatenate([[0, wl.n_elem - 1], rng.integers(0, wl.n_elem, 4094)]))
    idx = torch.from_numpy(cols).to("cuda")
    got = R[:, idx].cpu().numpy()
    del R
    set_strategy(dtype, N.STRATEGY_LANE, 1, 0)
    lane = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c)[:, idx].cpu().numpy()
    ref, ref_abs = reference(wl, p3.u, p3.coef, mg.COEF_QUAD, dtype, cols=cols)
    mx, agg = assert_close(got, ref, ref_abs, dtype, "P3 component elasticity 2^21")
    assert_close(lane, ref, ref_abs, dtype, "P3 lane elasticity 2^21")
    # the two kernels differ only in summation order: the same bar between them
    lx, _ = assert_close(got, lane, ref_abs, dtype, "P3 component vs lane 2^21")
    print(f"P3 component elasticity 2^21 {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}, "
          f"vs lane {lx:.2e}", flush=True)


@pytest.mark.parametrize("dtype", DTYPES)
def test_autotune_p3_elasticity(dtype):
    """The autotuner weighs the lane, matrix-core and component kernels for
    P3 3D elasticity and leaves a valid configuration whose results still
    meet the oracle bar."""
    t = api.fem_autotune(3, EL, R11, dtype, 1 << 15, None, op=N.OP_RESIDUAL_P3)
    assert t["strategy"] in (N.STRATEGY_LANE, N.STRATEGY_MFMA, N.STRATEGY_COMPONENT)
    assert t["vec"] == 1 and t["waves_per_block"] in (1, 2, 4)
    if t["strategy"] == N.STRATEGY_COMPONENT:
        assert t["waves_per_block"] <= (2 if dtype == torch.float32 else 1)
    wl, p3 = workload(1500)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    R = api.fem_integrate_residual_p3(3, EL, R11, ij, dj, dev(p3.u, dtype), dev(p3.coef, dtype))
    ref, ref_abs = reference(wl, p3.u, p3.coef, mg.COEF_QUAD, dtype)
    assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"P3 elasticity after autotune {t}")


def test_default_is_the_lane_kernel():
    """3D P3 elasticity runs the lane kernel unless told otherwise (measured
    faster than the component split on a warmed-up GPU), as do the other P3
    residuals and the adjoint."""
    for dt in DTYPES:
        assert api.fem_get_tuning(3, EL, R11, dt, op=N.OP_RESIDUAL_P3)["strategy"] == N.STRATEGY_LANE
        assert api.fem_get_tuning(3, mg.LAPLACE, R11, dt, op=N.OP_RESIDUAL_P3)["strategy"] == N.STRATEGY_LANE
        assert api.fem_get_tuning(3, EL, R11, dt, op=N.OP_BACKWARD_P3)["strategy"] == N.STRATEGY_LANE


def test_component_under_graph_capture():
    """The component split (dynamic LDS, workgroup barriers) captured in a
    HIP graph through torch, beside the P3 lane kernel and the rows
    yardstick: every replay, with eager work between, equals the eager
    results."""
    dtype = torch.float32
    wl, p3 = workload(20000, seed=197)
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
    u, c = dev(p3.u, dtype), dev(p3.coef, dtype)
    R1, R2 = torch.empty_like(u), torch.empty_like(u)
    src, dst = u[:17].contiguous(), torch.empty((5, wl.n_elem), dtype=dtype, device="cuda")

    def work():
        set_strategy(dtype, N.STRATEGY_COMPONENT, 2, 2)
        api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c, out=R1)
        set_strategy(dtype, N.STRATEGY_LANE, 1, 0)
        api.fem_integrate_residual_p3(3, EL, R11, ij, dj, u, c, out=R2)
        api.fem_stream_rows(src, dst)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (R1, R2, dst)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(3):
        for t in (R1, R2, dst):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((R1, R2, dst), eager):
            assert torch.equal(a, b), f"graph replay {rep} differs"
