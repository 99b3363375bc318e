"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (see tests/_parity.py): FP32 scaled max and aggregate error <= 1e-5,
FP64 <= 1e-12; geometry in FP64 to 1e-12 relative; integer counters exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import TOL, assert_close, dcoef_abs, dev, measure, oracle_reference, rounded

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
KINDS = [(2, mg.LAPLACE), (3, mg.LAPLACE), (2, mg.ELASTICITY), (3, mg.ELASTICITY), (2, mg.MASS), (3, mg.MASS)]


def small_workload(dim, phys, n_elem, rule=None, seed=7):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    return mg.make_workload(f"t{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed, rule=rule)


def gpu_geometry(wl, dtype):
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype, counts=counts)
    return ij, dj, counts


def run_forward(wl, dtype):
    ij, dj, counts = gpu_geometry(wl, dtype)
    R = api.fem_integrate_residual(wl.dim, wl.physics, wl.rule, ij, dj, dev(wl.u, dtype), dev(wl.coef, dtype))
    torch.cuda.synchronize()
    assert int(counts[0]) == 0
    return R.cpu().numpy()


@pytest.fixture(autouse=True)
def _reset_tuning():
    saved = {}
    for dim, phys in KINDS:
        for rule in (mg.default_rule(dim), mg.RULE_CENTROID):
            for dt in DTYPES:
                saved[(dim, phys, rule, dt)] = api.fem_get_tuning(dim, phys, rule, dt)
    yield
    for (dim, phys, rule, dt), t in saved.items():
        api.fem_set_tuning(dim, phys, rule, dt, **t)


# ---------------------------------------------------------------- geometry --

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", DTYPES)
def test_geometry_matches_oracle(dim, dtype):
    wl = small_workload(dim, mg.LAPLACE, 5000)
    ij, dj, counts = gpu_geometry(wl, dtype)
    rij, rdj, nd = oracle.geometry(wl.coords, wl.conn)
    torch.cuda.synchronize()
    assert nd == 0 and int(counts[0]) == 0 and int(counts[1]) == 0
    tol = 1e-12 if dtype == torch.float64 else 2 ** -23
    gij, gdj = ij.double().cpu().numpy(), dj.double().cpu().numpy()
    assert np.all(np.abs(gdj - rdj) <= tol * np.abs(rdj))
    scale = np.abs(rij).max(axis=0)
    assert np.all(np.abs(gij - rij) <= tol * scale * 4)


def test_geometry_counters_degenerate_and_poor():
    coords = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1e-5], [0.5, 0.0]], dtype=np.float64)
    conn = np.array([[0, 1, 3],      # fine
                     [0, 1, 2],      # collinear: degenerate
                     [0, 2, 4],      # sliver: poorly shaped
                     [0, 1, 9],      # vertex index out of range: degenerate, nothing read
                     [0, 1, 3]], dtype=np.int32)
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    ij, dj = api.fem_geometry(dev(coords, torch.float64), dev(conn, torch.int32), torch.float64, counts=counts)
    torch.cuda.synchronize()
    assert counts.tolist() == [2, 1]
    d = dj.cpu().numpy()
    assert d[0] == 1.0 and d[1] == 0.0 and np.isnan(d[3]) and d[4] == 1.0
    assert np.isnan(ij.cpu().numpy()[:, 1]).all() and np.isfinite(ij.cpu().numpy()[:, 0]).all()
    # counters accumulate across calls
    api.fem_geometry(dev(coords, torch.float64), dev(conn, torch.int32), torch.float64, counts=counts)
    torch.cuda.synchronize()
    assert counts.tolist() == [4, 2]


# ----------------------------------------------------------------- forward --

@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 63, 64, 65, 1000, 4099])
def test_forward_small_and_ragged(dim, phys, dtype, n_elem):
    wl = small_workload(dim, phys, n_elem)
    R = run_forward(wl, dtype)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    assert_close(R, ref, ref_abs, dtype, f"{dim}D phys {phys} n={n_elem}")


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_forward_centroid_rule(dim, phys, dtype):
    wl = small_workload(dim, phys, 3001, rule=mg.RULE_CENTROID)
    R = run_forward(wl, dtype)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    assert_close(R, ref, ref_abs, dtype, "centroid")


LAUNCHES = [dict(strategy=N.STRATEGY_LANE, vec=v, waves_per_block=w, blocks_per_cu=b)
            for v in (1, 2, 4) for w in (1, 4, 8) for b in (0, 1, 8)]


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
def test_forward_every_launch_configuration(dim, phys, dtype):
    """Results are bitwise identical for every lane launch configuration."""
    wl = small_workload(dim, phys, 20004)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    ij, dj, _ = gpu_geometry(wl, dtype)
    u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
    first = None
    for t in LAUNCHES:
        api.fem_set_tuning(dim, phys, wl.rule, dtype, **t)
        R = api.fem_integrate_residual(dim, phys, wl.rule, ij, dj, u, cf).cpu().numpy()
        if first is None:
            first = R
            assert_close(R, ref, ref_abs, dtype, str(t))
        else:
            assert np.array_equal(R, first), f"launch {t} changed the bits"


def test_forward_unaligned_views_fall_back():
    """Rows that do not start on a 16-byte boundary use narrower accesses; the
    bits do not change (n odd, and a view at a one-word offset)."""
    dtype = torch.float32
    wl = small_workload(3, mg.LAPLACE, 1001)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    assert_close(run_forward(wl, dtype), ref, ref_abs, dtype, "n odd")
    wl = small_workload(3, mg.LAPLACE, 1000)
    R = run_forward(wl, dtype)  # aligned: 4-wide accesses
    ij, dj, _ = gpu_geometry(wl, dtype)
    big = torch.zeros(1 + wl.u.size, dtype=dtype, device="cuda")
    u_off = big[1:].view(wl.u.shape)
    u_off.copy_(dev(wl.u, dtype))
    R2 = api.fem_integrate_residual(3, mg.LAPLACE, wl.rule, ij, dj, u_off, dev(wl.coef, dtype)).cpu().numpy()
    assert np.array_equal(R2, R)


def test_forward_empty():
    dtype = torch.float32
    e = torch.empty((9, 0), dtype=dtype, device="cuda")
    R = api.fem_integrate_residual(3, mg.LAPLACE, mg.RULE_TET4, e, torch.empty(0, dtype=dtype, device="cuda"),
                                   torch.empty((4, 0), dtype=dtype, device="cuda"),
                                   torch.empty((1, 4, 0), dtype=dtype, device="cuda"))
    assert R.shape == (4, 0)


def test_forward_repeatable_bitwise():
    wl = small_workload(3, mg.ELASTICITY, 50000)
    a = run_forward(wl, torch.float32)
    b = run_forward(wl, torch.float32)
    assert np.array_equal(a, b)


def test_constant_field_gives_zero_residual():
    wl = small_workload(3, mg.LAPLACE, 4096)
    for dtype in DTYPES:
        u = np.full_like(wl.u, 0.73)
        ij, dj, _ = gpu_geometry(wl, dtype)
        R = api.fem_integrate_residual(3, mg.LAPLACE, wl.rule, ij, dj, dev(u, dtype), dev(wl.coef, dtype))
        _, ref_abs, _, _ = oracle_reference(wl, dtype, u=u)
        eps = np.finfo(np.float32 if dtype == torch.float32 else np.float64).eps
        assert np.all(np.abs(R.cpu().numpy()) <= 8 * eps * np.linalg.norm(ref_abs, axis=0))


# --------------------------------------------------------- full-size configs --

@pytest.mark.parametrize("cfg", [1, 2, "3a", "3b"])
@pytest.mark.parametrize("dtype", DTYPES)
def test_benchmark_workloads_full(cfg, dtype):
    """Every element of the benchmark workloads at their full sizes, with the
    launch configuration the benchmark uses."""
    wl = mg.config(cfg)
    R = run_forward(wl, dtype)
    ref, ref_abs, ij, dj = oracle_reference(wl, dtype)
    mx, agg = assert_close(R, ref, ref_abs, dtype, f"config {cfg}")
    # reports without a bar: the plain per-element ratio |dR_e| / |R_e| (ill-
    # conditioned where R_e is near zero) and the scaled measure against the
    # oracle on the unrounded FP64 inputs (input rounding included)
    d = np.linalg.norm(np.asarray(R, dtype=np.float64) - ref, axis=0)
    plain = d / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    exact = oracle.integrate(wl.dim, wl.physics, wl.rule, ij, dj, wl.u, wl.coef)
    mx_in, agg_in = measure(R, exact, ref_abs)
    print(f"config {cfg} {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}; plain ratio median "
          f"{np.median(plain):.2e} p99.9 {np.quantile(plain, 0.999):.2e} max {plain.max():.2e}; "
          f"unrounded inputs: scaled max {mx_in:.2e} aggregate {agg_in:.2e}", flush=True)


# ---------------------------------------------------------------- backward --

@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 65, 3001])
def test_backward_matches_oracle(dim, phys, dtype, n_elem):
    wl = small_workload(dim, phys, n_elem)
    ij, dj, _ = gpu_geometry(wl, dtype)
    du, dc = api.fem_integrate_residual_backward(dim, phys, wl.rule, ij, dj, dev(wl.u, dtype),
                                                 dev(wl.coef, dtype), dev(wl.w, dtype))
    rij, rdj, _ = oracle.geometry(wl.coords, wl.conn)
    ur, cr, wr = rounded(wl.u, dtype), rounded(wl.coef, dtype), rounded(wl.w, dtype)
    rdu, rdc = oracle.backward(dim, phys, wl.rule, rij, rdj, ur, cr, wr)
    # scales: du = R(w) is bounded by the abs residual of w; dcoef by the abs
    # bilinear form evaluated with unit coefficients
    du_abs = oracle.integrate_abs(dim, phys, wl.rule, rij, rdj, wr, cr)
    dc_abs = dcoef_abs(dim, phys, wl.rule, rij, rdj, ur, wr, rdc.shape[0], rdc.shape[1])
    assert_close(du.cpu().numpy(), rdu, du_abs, dtype, "du")
    ncq = rdc.shape[0] * rdc.shape[1]
    assert_close(dc.cpu().numpy().reshape(ncq, -1), rdc.reshape(ncq, -1), dc_abs.reshape(ncq, -1), dtype, "dcoef")


def test_backward_optional_outputs_bitwise():
    wl = small_workload(3, mg.ELASTICITY, 2048)
    dt = torch.float32
    ij, dj, _ = gpu_geometry(wl, dt)
    args = (3, mg.ELASTICITY, wl.rule, ij, dj, dev(wl.u, dt), dev(wl.coef, dt), dev(wl.w, dt))
    du, dc = api.fem_integrate_residual_backward(*args)
    du2, none = api.fem_integrate_residual_backward(*args, want_dcoef=False)
    none2, dc2 = api.fem_integrate_residual_backward(*args, want_du=False)
    assert none is None and none2 is None
    assert torch.equal(du, du2) and torch.equal(dc, dc2)
    # du is exactly the forward residual of w (same kernel arithmetic)
    R_w = api.fem_integrate_residual(3, mg.ELASTICITY, wl.rule, ij, dj, dev(wl.w, dt), dev(wl.coef, dt))
    assert torch.equal(du, R_w)


def test_autograd_function_fd_fp64():
    """The autograd wrapper against central differences of L = sum w.R on a
    512-element submesh of the adjoint workload (FP64 on the GPU)."""
    wl = mg.config(5, n_elem=512)
    dt = torch.float64
    ij, dj, _ = gpu_geometry(wl, dt)
    u = dev(wl.u, dt).requires_grad_(True)
    cf = dev(wl.coef, dt).requires_grad_(True)
    w = dev(wl.w, dt)
    L = (api.integrate_residual(3, mg.LAPLACE, wl.rule, ij, dj, u, cf) * w).sum()
    L.backward()
    gu, gc = u.grad.cpu().numpy(), cf.grad.cpu().numpy()
    rij, rdj, _ = oracle.geometry(wl.coords, wl.conn)

    def L_elem(uu, cc):
        return np.sum(wl.w * oracle.integrate(3, mg.LAPLACE, wl.rule, rij, rdj, uu, cc), axis=0)

    scale = max(np.abs(gu).max(), np.abs(gc).max())
    for j in range(wl.u.shape[0]):
        h = 1e-3 * np.maximum(1.0, np.abs(wl.u[j]))
        up, um = wl.u.copy(), wl.u.copy()
        up[j] += h
        um[j] -= h
        fd = (L_elem(up, wl.coef) - L_elem(um, wl.coef)) / (2 * h)
        assert np.abs(fd - gu[j]).max() <= 1e-9 * scale
    for q in range(wl.coef.shape[1]):
        h = 1e-3 * np.maximum(1.0, np.abs(wl.coef[0, q]))
        cp, cm = wl.coef.copy(), wl.coef.copy()
        cp[0, q] += h
        cm[0, q] -= h
        fd = (L_elem(wl.u, cp) - L_elem(wl.u, cm)) / (2 * h)
        assert np.abs(fd - gc[0, q]).max() <= 1e-9 * scale


def test_adjoint_workload_full_fp32():
    """Adjoint of the 2^21-element 3D Laplacian in FP32 against the FP64 oracle."""
    wl = mg.config(5)
    dt = torch.float32
    ij, dj, _ = gpu_geometry(wl, dt)
    du, dc = api.fem_integrate_residual_backward(3, mg.LAPLACE, wl.rule, ij, dj, dev(wl.u, dt),
                                                 dev(wl.coef, dt), dev(wl.w, dt))
    rij, rdj, _ = oracle.geometry(wl.coords, wl.conn)
    ur, cr, wr = rounded(wl.u, dt), rounded(wl.coef, dt), rounded(wl.w, dt)
    rdu, rdc = oracle.backward(3, mg.LAPLACE, wl.rule, rij, rdj, ur, cr, wr)
    du_abs = oracle.integrate_abs(3, mg.LAPLACE, wl.rule, rij, rdj, wr, cr)
    dc_abs = dcoef_abs(3, mg.LAPLACE, wl.rule, rij, rdj, ur, wr, 1, 4)
    mx1, _ = assert_close(du.cpu().numpy(), rdu, du_abs, dt, "du")
    mx2, _ = assert_close(dc.cpu().numpy()[0], rdc[0], dc_abs[0], dt, "dkappa")
    print(f"adjoint full: du {mx1:.2e} dkappa {mx2:.2e}", flush=True)


# ------------------------------------------------------------- maximum sizes --

def test_row_offsets_beyond_2_pow_31():
    """3D elasticity with 2^28 elements: 12 rows of 2^28 words put row offsets
    far beyond 2^31. The elements are 4096 distinct ones repeated, so every
    copy must equal the small computation bitwise (lane and fused kernels)."""
    dtype = torch.float32
    base = small_workload(3, mg.ELASTICITY, 4096, seed=77)
    reps = 1 << 16
    n = base.n_elem * reps
    coords = dev(base.coords, torch.float64)
    conn_s = dev(base.conn, torch.int32)
    ij_s, dj_s = api.fem_geometry(coords, conn_s, dtype)
    u_s, cf_s = dev(base.u, dtype), dev(base.coef, dtype)
    R_s = api.fem_integrate_residual(3, mg.ELASTICITY, base.rule, ij_s, dj_s, u_s, cf_s)
    u = u_s.repeat(1, reps)
    cf = cf_s.repeat(1, 1, reps)
    ij = ij_s.repeat(1, reps)
    dj = dj_s.repeat(reps)
    R = api.fem_integrate_residual(3, mg.ELASTICITY, base.rule, ij, dj, u, cf)
    del ij, dj
    torch.cuda.synchronize()
    assert R.shape == (12, n) and R.shape[0] * R.shape[1] > 2 ** 31
    for blk in (0, 1, reps // 2, reps - 1):
        sl = slice(blk * base.n_elem, (blk + 1) * base.n_elem)
        assert torch.equal(R[:, sl], R_s), f"lane kernel block {blk}"
    Rm = api.fem_integrate_residual_mesh(3, mg.ELASTICITY, base.rule, coords, conn_s.repeat(reps, 1), u, cf)
    torch.cuda.synchronize()
    for blk in (0, 7, reps // 3, reps - 1):
        sl = slice(blk * base.n_elem, (blk + 1) * base.n_elem)
        assert torch.equal(Rm[:, sl], R_s), f"fused kernel block {blk}"
    ref, ref_abs, _, _ = oracle_reference(base, dtype)
    assert_close(R_s.cpu().numpy(), ref, ref_abs, dtype, "base block")


def test_checked_calls_raise_on_degenerate_elements():
    """check=True synchronizes and raises FEM_ERR_DEGENERATE for a mesh with
    a collapsed element; the same calls unchecked return NaN for it."""
    wl = small_workload(3, mg.LAPLACE, 500)
    coords = wl.coords.copy()
    conn = wl.conn.copy()
    conn[10, 3] = conn[10, 0]                      # repeated vertex: det J = 0
    X, C = dev(coords, torch.float64), dev(conn, torch.int32)
    u, cf = dev(wl.u, torch.float32), dev(wl.coef, torch.float32)
    with pytest.raises(N.FemError) as ei:
        api.fem_geometry(X, C, torch.float32, check=True)
    assert ei.value.status == N.FEM_ERR_DEGENERATE
    with pytest.raises(N.FemError):
        api.fem_integrate_residual_mesh(3, mg.LAPLACE, wl.rule, X, C, u, cf, check=True)
    with pytest.raises(N.FemError):
        api.fem_integrate_residual_gather(3, mg.LAPLACE, wl.rule, X, C, dev(wl.u_vertex, torch.float32), cf,
                                          check=True)
    ij, dj = api.fem_geometry(X, C, torch.float32)
    assert torch.isnan(ij[:, 10]).all() and not torch.isnan(ij[:, 11]).any()
    # a caller's counter that already holds counts: only this call's are checked
    counts = torch.tensor([5, 0], dtype=torch.int32, device="cuda")
    api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), torch.float32, counts=counts,
                     check=True)
    assert int(counts[0]) == 5
