"""GPU: the thread-transposition strategy, the batched persistent launch and
its HIP graph, and the autotuner, each against the FP64 oracle and against
the lane kernel."""
import ast
import json
import os
import pathlib
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, oracle_reference

pytestmark = pytest.mark.gpu
ROOT = pathlib.Path(__file__).resolve().parents[1]

DTYPES = [torch.float32, torch.float64]
KINDS = [(2, mg.LAPLACE), (3, mg.LAPLACE), (2, mg.ELASTICITY), (3, mg.ELASTICITY), (2, mg.MASS), (3, mg.MASS)]


def small_workload(dim, phys, n_elem, rule=None, seed=11):
    grid = mg.smallest_grid(dim, max(n_elem, 1))
    return mg.make_workload(f"s{dim}{phys}", dim, phys, grid, n_elem, mg.BASE_SEED + seed, rule=rule)


def geometry(wl, dtype):
    return api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)


@pytest.fixture(autouse=True)
def _restore_tuning():
    saved = {}
    for dim, phys in KINDS:
        for rule in (mg.default_rule(dim), mg.RULE_CENTROID):
            for dt in DTYPES:
                saved[(dim, phys, rule, dt)] = api.fem_get_tuning(dim, phys, rule, dt)
    yield
    for (dim, phys, rule, dt), t in saved.items():
        api.fem_set_tuning(dim, phys, rule, dt, **t)


# ------------------------------------------------------ thread transposition --

@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 65, 1000, 20004])
@pytest.mark.parametrize("rule_kind", ["default", "centroid"])
def test_transpose_matches_oracle(dim, phys, dtype, n_elem, rule_kind):
    rule = mg.default_rule(dim) if rule_kind == "default" else mg.RULE_CENTROID
    wl = small_workload(dim, phys, n_elem, rule=rule)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    ij, dj = geometry(wl, dtype)
    u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
    first = None
    for waves in (1, 2, 4, 8):
        for bpc in (0, 2):
            api.fem_set_tuning(dim, phys, rule, dtype, strategy=N.STRATEGY_TRANSPOSE, vec=1,
                               waves_per_block=waves, blocks_per_cu=bpc)
            R = api.fem_integrate_residual(dim, phys, rule, ij, dj, u, cf).cpu().numpy()
            if first is None:
                first = R
                assert_close(R, ref, ref_abs, dtype, f"transpose {dim}D phys {phys}")
            else:
                assert np.array_equal(R, first), "transpose result depends on the launch shape"


@pytest.mark.parametrize("dim,phys", [k for k in KINDS if k[1] != mg.ELASTICITY])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 15, 17, 1000, 20004])
@pytest.mark.parametrize("rule_kind", ["default", "centroid"])
@pytest.mark.parametrize("space", [mg.COEF_QUAD, mg.COEF_P1, mg.COEF_P0])
def test_shuffle_matches_oracle(dim, phys, dtype, n_elem, rule_kind, space):
    """The transposition through quad permutations (four lanes per element,
    16 elements per wave: partial groups, several waves, a ragged tail)
    against the oracle in every coefficient space; launch shapes give the
    same bits."""
    rule = mg.default_rule(dim) if rule_kind == "default" else mg.RULE_CENTROID
    wl = small_workload(dim, phys, n_elem, rule=rule)
    cf = wl.coef if space == mg.COEF_QUAD else mg.space_coefficients(wl, space, mg.BASE_SEED + 1000)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype, coef=cf, space=space)
    ij, dj = geometry(wl, dtype)
    u, c = dev(wl.u, dtype), dev(cf, dtype)
    first = None
    for waves, bpc in ((4, 0), (1, 0), (8, 4), (2, 1)):
        api.fem_set_tuning(dim, phys, rule, dtype, strategy=N.STRATEGY_SHUFFLE, vec=1, waves_per_block=waves,
                           blocks_per_cu=bpc)
        R = api.fem_integrate_residual(dim, phys, rule, ij, dj, u, c, coef_space=space).cpu().numpy()
        if first is None:
            first = R
            assert_close(R, ref, ref_abs, dtype, f"shuffle {dim}D phys {phys} space {space}")
        else:
            assert np.array_equal(R, first), "shuffle result depends on the launch shape"


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("space", [mg.COEF_P1, mg.COEF_P0])
def test_transpose_coefficient_spaces(dim, phys, space):
    """The LDS transposition in the P1 and P0 coefficient spaces."""
    dtype = torch.float32
    rule = mg.default_rule(dim)
    wl = small_workload(dim, phys, 1000, rule=rule)
    cf = mg.space_coefficients(wl, space, mg.BASE_SEED + 1000)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype, coef=cf, space=space)
    ij, dj = geometry(wl, dtype)
    api.fem_set_tuning(dim, phys, rule, dtype, strategy=N.STRATEGY_TRANSPOSE, vec=1, waves_per_block=4,
                       blocks_per_cu=0)
    R = api.fem_integrate_residual(dim, phys, rule, ij, dj, dev(wl.u, dtype), dev(cf, dtype),
                                   coef_space=space).cpu().numpy()
    assert_close(R, ref, ref_abs, dtype, f"transpose {dim}D phys {phys} space {space}")


@pytest.mark.parametrize("cfg", [2, "3a", "3b"])
def test_transpositions_full_size(cfg):
    """Both transposition forms at the benchmark sizes (the 2^20-tet
    Laplacian, 2^22-triangle and 2^21-tet elasticity; the quad-permutation
    form only for the scalar field) against the oracle, FP32 and FP64, at the
    launch shapes the benchmark times."""
    wl = mg.config(cfg)
    for dtype in DTYPES:
        ref, ref_abs, _, _ = oracle_reference(wl, dtype)
        ij, dj = geometry(wl, dtype)
        u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
        forms = [(N.STRATEGY_TRANSPOSE, 1, 0), (N.STRATEGY_TRANSPOSE, 4, 8)]
        if wl.physics != mg.ELASTICITY:
            forms += [(N.STRATEGY_SHUFFLE, 8, 0), (N.STRATEGY_SHUFFLE, 4, 0)]
        for strategy, waves, bpc in forms:
            api.fem_set_tuning(wl.dim, wl.physics, wl.rule, dtype, strategy=strategy, vec=1,
                               waves_per_block=waves, blocks_per_cu=bpc)
            R = api.fem_integrate_residual(wl.dim, wl.physics, wl.rule, ij, dj, u, cf).cpu().numpy()
            mx, agg = assert_close(R, ref, ref_abs, dtype, f"strategy {strategy} config {cfg}")
            print(f"strategy {strategy} ({waves}, {bpc}) config {cfg} {dtype}: scaled max {mx:.2e} "
                  f"aggregate {agg:.2e}", flush=True)
        del ij, dj, u, cf


def test_shuffle_refused_for_elasticity():
    with pytest.raises(N.FemError) as ei:
        api.fem_set_tuning(3, mg.ELASTICITY, mg.RULE_TET4, torch.float32, strategy=N.STRATEGY_SHUFFLE)
    assert ei.value.status == N.FEM_ERR_UNSUPPORTED


# ------------------------------------------------------------------ batched --

def batch_meshes(dtype, sizes, rules=None):
    out, wls = [], []
    for m, ne in enumerate(sizes):
        dim, phys = mg.MESH_TYPES[m % 4] if m % 5 != 4 else (2 + m % 2, mg.MASS)
        rule = mg.default_rule(dim) if rules is None else rules[m % len(rules)](dim)
        wl = small_workload(dim, phys, ne, rule=rule, seed=100 + m)
        ij, dj = geometry(wl, dtype)
        out.append(dict(dim=dim, physics=phys, rule=rule, inv_j=ij, det_j=dj, u=dev(wl.u, dtype),
                        coef=dev(wl.coef, dtype), out=torch.full(wl.u.shape, float("nan"), dtype=dtype,
                                                                 device="cuda")))
        wls.append(wl)
    return out, wls


SIZES = [1000, 1, 4097, 257, 30000, 65, 0, 2000, 5003, 12]


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_matches_single_mesh_bitwise(dtype):
    meshes, wls = batch_meshes(dtype, SIZES, rules=[mg.default_rule, lambda d: mg.RULE_CENTROID])
    for m in meshes:  # single-mesh reference with the lane kernel
        api.fem_set_tuning(m["dim"], m["physics"], m["rule"], dtype, strategy=N.STRATEGY_LANE, vec=1)
    singles = [api.fem_integrate_residual(m["dim"], m["physics"], m["rule"], m["inv_j"], m["det_j"], m["u"],
                                          m["coef"]) for m in meshes]
    plan = api.BatchPlan(meshes)
    for waves, bpc in [(4, 8), (1, 0), (8, 1), (2, 64)]:
        for m in meshes:
            m["out"].fill_(float("nan"))
        plan.set_launch(waves, bpc)
        plan.run()
        torch.cuda.synchronize()
        for m, s, wl in zip(meshes, singles, wls):
            assert torch.equal(m["out"], s), f"batched != single for {wl.name} at launch {(waves, bpc)}"
    for m, wl in zip(meshes, wls):
        if wl.n_elem == 0:
            continue
        ref, ref_abs, _, _ = oracle_reference(wl, dtype)
        assert_close(m["out"].cpu().numpy(), ref, ref_abs, dtype, wl.name)
    plan.close()


def test_batch_graph_replays():
    dtype = torch.float32
    meshes, wls = batch_meshes(dtype, [3000, 777, 12345, 64, 999])
    plan = api.BatchPlan(meshes)
    plan.run()
    torch.cuda.synchronize()
    eager = [m["out"].clone() for m in meshes]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture()
    for rep in range(4):
        for m in meshes:
            m["out"].zero_()          # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.replay()
        s.synchronize()
        for m, e in zip(meshes, eager):
            assert torch.equal(m["out"], e), f"replay {rep} differs from the eager launch"
    # changing the launch shape drops the graph; replay must then be refused
    plan.set_launch(2, 4)
    with pytest.raises(N.FemError):
        plan.replay()
    plan.close()


def test_batch_autotune_keeps_results():
    """The batched plan's autotuner picks a valid launch shape; the results at
    that shape equal the single-mesh calls bit for bit."""
    dtype = torch.float32
    meshes, wls = batch_meshes(dtype, [3000, 777, 12345, 64, 999, 40000])
    for m in meshes:
        api.fem_set_tuning(m["dim"], m["physics"], m["rule"], dtype, strategy=N.STRATEGY_LANE, vec=1)
    singles = [api.fem_integrate_residual(m["dim"], m["physics"], m["rule"], m["inv_j"], m["det_j"], m["u"],
                                          m["coef"]) for m in meshes]
    plan = api.BatchPlan(meshes)
    t = plan.autotune()
    assert t["waves_per_block"] in (1, 2, 4, 8) and t["blocks_per_cu"] in (0, 2, 4, 8, 16)
    for m in meshes:
        m["out"].fill_(float("nan"))
    plan.run()
    torch.cuda.synchronize()
    for m, s in zip(meshes, singles):
        assert torch.equal(m["out"], s)
    plan.close()


def test_batch_plan_argument_errors():
    dtype = torch.float32
    meshes, _ = batch_meshes(dtype, [100])
    bad = dict(meshes[0])
    bad["rule"] = mg.RULE_TET4 if bad["dim"] == 2 else mg.RULE_TRI3
    with pytest.raises(N.FemError) as ei:
        api.BatchPlan([bad])
    assert ei.value.status == N.FEM_ERR_UNSUPPORTED


# --------------------------------------------------------------- autotuner --

def test_autotune_picks_a_valid_configuration(tmp_path):
    cache = tmp_path / "tune.json"
    t = api.fem_autotune(3, mg.LAPLACE, mg.RULE_TET4, torch.float32, 1 << 16, str(cache))
    assert t["strategy"] in (N.STRATEGY_LANE, N.STRATEGY_TRANSPOSE, N.STRATEGY_SHUFFLE)
    assert t["vec"] in (1, 2, 4) and t["waves_per_block"] in (1, 2, 4, 8)
    data = json.loads(cache.read_text())
    (entry,) = data["entries"]
    assert entry["arch"].startswith("gfx") and entry["op"] == 0 and entry["dim"] == 3 and entry["us"] > 0
    # a second entry is merged, the first kept
    api.fem_autotune(2, mg.ELASTICITY, mg.RULE_TRI3, torch.float64, 1 << 14, str(cache))
    assert len(json.loads(cache.read_text())["entries"]) == 2
    # loading restores the tuned configuration
    api.fem_set_tuning(3, mg.LAPLACE, mg.RULE_TET4, torch.float32, strategy=0, vec=1, waves_per_block=1,
                       blocks_per_cu=1)
    assert api.fem_load_tuning(str(cache)) == N.FEM_OK
    assert api.fem_get_tuning(3, mg.LAPLACE, mg.RULE_TET4, torch.float32) == t
    assert api.fem_load_tuning(str(tmp_path / "missing.json")) == N.FEM_ERR_NO_TUNING
    # results with the tuned configuration still match the oracle
    wl = small_workload(3, mg.LAPLACE, 5000)
    ij, dj = geometry(wl, torch.float32)
    R = api.fem_integrate_residual(3, mg.LAPLACE, wl.rule, ij, dj, dev(wl.u, torch.float32),
                                   dev(wl.coef, torch.float32)).cpu().numpy()
    ref, ref_abs, _, _ = oracle_reference(wl, torch.float32)
    assert_close(R, ref, ref_abs, torch.float32, "tuned")
    # a fresh process loads the cache named by FEM_TUNE_CACHE before its first lookup
    code = ("import torch; from paper_1607_04245_amd import api, meshgen as mg; "
            "print(api.fem_get_tuning(3, mg.LAPLACE, mg.RULE_TET4, torch.float32))")
    run = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, FEM_TUNE_CACHE=str(cache)),
                         capture_output=True, text=True, timeout=300, cwd=str(ROOT))
    assert run.returncode == 0, run.stderr
    assert ast.literal_eval(run.stdout.strip().splitlines()[-1]) == t


# ------------------------------------------------ fused geometry + residual --

def _restore_op(op, dim, phys, rule, dt):
    return api.fem_get_tuning(dim, phys, rule, dt, op=op)


@pytest.mark.parametrize("dim,phys", KINDS)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n_elem", [1, 65, 4099, 20004])
def test_residual_mesh_bitwise_equals_two_calls(dim, phys, dtype, n_elem):
    wl = small_workload(dim, phys, n_elem, seed=21)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    u, cf = dev(wl.u, dtype), dev(wl.coef, dtype)
    c_split = torch.zeros(2, dtype=torch.int32, device="cuda")
    ij, dj = api.fem_geometry(coords, conn, dtype, counts=c_split)
    R = api.fem_integrate_residual(dim, phys, wl.rule, ij, dj, u, cf)
    saved = _restore_op(N.OP_RESIDUAL_MESH, dim, phys, wl.rule, dtype)
    try:
        for ept in (1, 2, 4):
            for waves, bpc in ((1, 0), (4, 0), (2, 8)):
                api.fem_set_tuning(dim, phys, wl.rule, dtype, vec=ept, waves_per_block=waves, blocks_per_cu=bpc,
                                   op=N.OP_RESIDUAL_MESH)
                c = torch.zeros(2, dtype=torch.int32, device="cuda")
                Rm = api.fem_integrate_residual_mesh(dim, phys, wl.rule, coords, conn, u, cf, counts=c)
                ij2, dj2 = torch.empty_like(ij), torch.empty_like(dj)
                Rg = api.fem_integrate_residual_mesh(dim, phys, wl.rule, coords, conn, u, cf, inv_j=ij2, det_j=dj2)
                torch.cuda.synchronize()
                assert torch.equal(Rm, R) and torch.equal(Rg, R), f"fused != two calls (ept {ept})"
                assert torch.equal(ij2, ij) and torch.equal(dj2, dj)
                assert torch.equal(c, c_split)
    finally:
        api.fem_set_tuning(dim, phys, wl.rule, dtype, op=N.OP_RESIDUAL_MESH, **saved)
    ref, ref_abs, _, _ = oracle_reference(wl, dtype)
    assert_close(Rm.cpu().numpy(), ref, ref_abs, dtype, "fused")


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", DTYPES)
def test_geometry_launch_shapes_bitwise(dim, dtype):
    wl = small_workload(dim, mg.LAPLACE, 30011, seed=31)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    saved = _restore_op(N.OP_GEOMETRY, dim, 0, 0, dtype)
    first = None
    try:
        for ept in (1, 2, 4):
            for waves, bpc in ((1, 0), (4, 0), (8, 2)):
                api.fem_set_tuning(dim, 0, 0, dtype, vec=ept, waves_per_block=waves, blocks_per_cu=bpc,
                                   op=N.OP_GEOMETRY)
                ij, dj = api.fem_geometry(coords, conn, dtype)
                if first is None:
                    first = (ij, dj)
                else:
                    assert torch.equal(ij, first[0]) and torch.equal(dj, first[1])
    finally:
        api.fem_set_tuning(dim, 0, 0, dtype, op=N.OP_GEOMETRY, **saved)


def test_residual_mesh_degenerate_elements():
    coords = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1e-5]], dtype=np.float64)
    conn = np.array([[0, 1, 3], [0, 1, 2], [0, 2, 4], [0, 1, 7]], dtype=np.int32)
    u = np.arange(12, dtype=np.float64).reshape(3, 4)
    cf = np.ones((1, 3, 4))
    c = torch.zeros(2, dtype=torch.int32, device="cuda")
    R = api.fem_integrate_residual_mesh(2, mg.LAPLACE, mg.RULE_TRI3, dev(coords, torch.float64),
                                        dev(conn, torch.int32), dev(u, torch.float64), dev(cf, torch.float64),
                                        counts=c).cpu().numpy()
    torch.cuda.synchronize()
    assert c.tolist() == [2, 1]
    assert np.isfinite(R[:, 0]).all() and np.isnan(R[:, 1]).all() and np.isnan(R[:, 3]).all()


@pytest.mark.parametrize("cfg", [2, "3a", "3b"])
def test_residual_mesh_full_workloads(cfg):
    wl = mg.config(cfg)
    for dtype in DTYPES:
        R = api.fem_integrate_residual_mesh(wl.dim, wl.physics, wl.rule, dev(wl.coords, torch.float64),
                                            dev(wl.conn, torch.int32), dev(wl.u, dtype), dev(wl.coef, dtype))
        ref, ref_abs, _, _ = oracle_reference(wl, dtype)
        mx, agg = assert_close(R.cpu().numpy(), ref, ref_abs, dtype, f"fused config {cfg}")
        print(f"fused config {cfg} {dtype}: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)


@pytest.mark.parametrize("op,rule", [(N.OP_GEOMETRY, mg.RULE_TET4), (N.OP_RESIDUAL_MESH, mg.RULE_TET4),
                                     (N.OP_BACKWARD, mg.RULE_TET4), (N.OP_JACOBIAN, mg.RULE_TET4),
                                     (N.OP_JACOBIAN_P2, mg.RULE_TET11)])
def test_autotune_other_operations(op, rule):
    saved = api.fem_get_tuning(3, mg.LAPLACE, rule, torch.float32, op=op)
    try:
        t = api.fem_autotune(3, mg.LAPLACE, rule, torch.float32, 1 << 15, None, op=op)
        assert t["strategy"] == N.STRATEGY_LANE and t["waves_per_block"] in (1, 2, 4, 8)
        if op in (N.OP_JACOBIAN, N.OP_JACOBIAN_P2):
            assert t["vec"] == 1 and t["waves_per_block"] <= 4
    finally:
        api.fem_set_tuning(3, mg.LAPLACE, rule, torch.float32, op=op, **saved)


def test_entry_points_under_graph_capture():
    """The library's launches can be captured in a HIP graph through torch;
    every replay matches the eager results (eager work between replays)."""
    dtype = torch.float32
    wl = small_workload(3, mg.ELASTICITY, 40000, seed=41)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    u, cf, w = dev(wl.u, dtype), dev(wl.coef, dtype), dev(wl.w, dtype)
    ij, dj = torch.empty((9, wl.n_elem), dtype=dtype, device="cuda"), torch.empty(wl.n_elem, dtype=dtype, device="cuda")
    R1, R2 = torch.empty_like(u), torch.empty_like(u)
    du, dc = torch.empty_like(u), torch.empty_like(cf)

    def work():
        api.fem_geometry(coords, conn, dtype, inv_j=ij, det_j=dj)
        api.fem_integrate_residual(3, mg.ELASTICITY, wl.rule, ij, dj, u, cf, out=R1)
        api.fem_integrate_residual_mesh(3, mg.ELASTICITY, wl.rule, coords, conn, u, cf, out=R2)
        api.fem_integrate_residual_backward(3, mg.ELASTICITY, wl.rule, ij, dj, u, cf, w, du=du, dcoef=dc)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (ij, dj, R1, R2, du, dc)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(3):
        for t in (ij, dj, R1, R2, du, dc):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((ij, dj, R1, R2, du, dc), eager):
            assert torch.equal(a, b), f"graph replay {rep} differs"


def test_newer_entry_points_under_graph_capture():
    """Gather form, assembly, restriction, the P2 residual and adjoint, and
    the element matrices in one captured graph: every replay equals the eager
    results."""
    dtype = torch.float32
    wl = small_workload(3, mg.ELASTICITY, 30000, seed=43)
    p2 = mg.p2_inputs(wl, mg.RULE_TET11, mg.BASE_SEED + 77)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    uv, cf = dev(wl.u_vertex, dtype), dev(wl.coef, dtype)
    cv = dev(mg.vertex_coefficients(wl, 5), dtype)
    ij, dj = api.fem_geometry(coords, conn, dtype)
    u2, cf2, w2 = dev(p2.u, dtype), dev(p2.coef, dtype), dev(p2.w, dtype)
    plan = api.AssemblyPlan(conn, wl.n_vert)
    R = torch.empty((12, wl.n_elem), dtype=dtype, device="cuda")
    Rp = torch.empty_like(R)
    F = torch.empty((wl.n_vert, 3), dtype=dtype, device="cuda")
    C = torch.empty_like(R)
    R2 = torch.empty_like(u2)
    d2, dc2 = torch.empty_like(u2), torch.empty_like(cf2)
    K1 = torch.empty((144, wl.n_elem), dtype=dtype, device="cuda")
    K2 = torch.empty((900, wl.n_elem), dtype=dtype, device="cuda")

    def work():
        api.fem_integrate_residual_gather(3, mg.ELASTICITY, wl.rule, coords, conn, uv, cf, out=R)
        api.fem_integrate_residual_gather(3, mg.ELASTICITY, wl.rule, coords, conn, uv, cv, out=Rp,
                                          coef_space=mg.COEF_P1)
        plan.assemble(R, 3, out=F)
        api.fem_restrict(conn, F, out=C)
        api.fem_integrate_residual_p2(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, u2, cf2, out=R2)
        api.fem_integrate_residual_p2_backward(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, u2, cf2, w2, du=d2, dcoef=dc2)
        api.fem_integrate_jacobian(3, mg.ELASTICITY, wl.rule, ij, dj, cf, out=K1)
        api.fem_integrate_jacobian(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, cf2, out=K2, order=2)

    outs = (R, Rp, F, C, R2, d2, dc2, K1, K2)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = [t.clone() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(outs, eager)):
            assert torch.equal(a, b), f"graph replay {rep} differs in output {i}"


def test_batched_workload_full():
    """The 64-mesh benchmark workload (about 8.9 M elements) through one
    graph-replayed persistent launch in the benchmark's default shape:
    every mesh against the oracle, and bit for bit against its single-mesh
    lane-kernel result."""
    dtype = torch.float32
    wls = mg.batch_workloads()
    meshes = []
    for w in wls:
        ij, dj = api.fem_geometry(dev(w.coords, torch.float64), dev(w.conn, torch.int32), dtype)
        meshes.append(dict(dim=w.dim, physics=w.physics, rule=w.rule, inv_j=ij, det_j=dj, u=dev(w.u, dtype),
                           coef=dev(w.coef, dtype), out=torch.full(w.u.shape, float("nan"), dtype=dtype,
                                                                   device="cuda")))
    assert sum(w.n_elem for w in wls) > 5_000_000
    plan = api.BatchPlan(meshes)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.capture()
        plan.replay()
    torch.cuda.synchronize()
    worst = 0.0
    for m, w in zip(meshes, wls):
        single = api.fem_integrate_residual(m["dim"], m["physics"], m["rule"], m["inv_j"], m["det_j"], m["u"],
                                            m["coef"])
        assert torch.equal(m["out"], single), w.name
        ref, ref_abs, _, _ = oracle_reference(w, dtype)
        mx, _ = assert_close(m["out"].cpu().numpy(), ref, ref_abs, dtype, w.name)
        worst = max(worst, mx)
    plan.close()
    print(f"batched 64 meshes: worst scaled error {worst:.2e}", flush=True)


def test_third_order_entry_points_under_graph_capture():
    """The P3 residual, adjoint and element matrices and the planned geometry
    in one captured graph: every replay equals the eager results."""
    dtype = torch.float32
    wl = small_workload(3, mg.ELASTICITY, 20000, seed=45)
    p3 = mg.p3_inputs(wl, mg.RULE_TET11, mg.BASE_SEED + 79)
    coords, conn = dev(wl.coords, torch.float64), dev(wl.conn, torch.int32)
    ij, dj = api.fem_geometry(coords, conn, dtype)
    u3, cf3 = dev(p3.u, dtype), dev(p3.coef, dtype)
    w3 = dev(np.random.default_rng(6).uniform(-1, 1, p3.u.shape), dtype)
    mplan = api.MeshPlan(conn, wl.n_vert)
    R3, d3, dc3 = torch.empty_like(u3), torch.empty_like(u3), torch.empty_like(cf3)
    K3 = torch.empty((60 * 60, wl.n_elem), dtype=dtype, device="cuda")
    gij, gdj = torch.empty_like(ij), torch.empty_like(dj)

    def work():
        api.fem_integrate_residual_p3(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, u3, cf3, out=R3)
        api.fem_integrate_residual_p3_backward(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, u3, cf3, w3, du=d3, dcoef=dc3)
        api.fem_integrate_jacobian(3, mg.ELASTICITY, mg.RULE_TET11, ij, dj, cf3, out=K3, order=3)
        mplan.geometry(coords, dtype, inv_j=gij, det_j=gdj)

    outs = (R3, d3, dc3, K3, gij, gdj)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = [t.clone() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    for rep in range(3):
        for t in outs:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.equal(a, b), f"graph replay {rep} differs"
    mplan.close()
