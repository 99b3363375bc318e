"""The C ABI library without a GPU: it loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import pathlib

import pytest

from paper_1607_04245_amd import _native as N
from paper_1607_04245_amd import meshgen as mg

ROOT = pathlib.Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib():
    if not N.LIB_PATH.exists():
        import __graft_entry__
        __graft_entry__.build()
    return N.lib()


def test_exports_every_header_function(lib):
    names = N.header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), f"{name} declared in fem.h but not exported"
    assert set(names) == set(N.SIGNATURES), "binding signatures out of sync with fem.h"


def test_status_codes_match_header():
    text = N.HEADER.read_text()
    for code, name in N.STATUS_NAMES.items():
        assert f"#define {name} ({code})" in text or (code == 0 and f"#define {name} 0" in text)


def _v(x=0x1000):
    return ctypes.c_void_p(x)  # never dereferenced: validation fails first


@pytest.mark.parametrize("args,status", [
    ((4, 10, 10), N.FEM_ERR_INVALID_ARG),   # bad dim
    ((2, -1, 10), N.FEM_ERR_INVALID_ARG),   # negative n_elem
    ((2, 10, -1), N.FEM_ERR_INVALID_ARG),   # negative n_vert
    ((2, 10, 0), N.FEM_ERR_INVALID_ARG),    # elements without vertices
    ((2, 0, 0), N.FEM_OK),                  # empty: no launch
])
def test_geometry_validation(lib, args, status):
    dim, ne, nv = args
    st = lib.fem_geometry(dim, ne, nv, _v(), _v(), N.F32, _v(), _v(), None, None)
    assert st == status
    if status != N.FEM_OK:
        assert N.last_error()


def test_geometry_null_arrays(lib):
    assert lib.fem_geometry(2, 5, 5, None, _v(), N.F32, _v(), _v(), None, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_geometry(2, 5, 5, _v(), _v(), 7, _v(), _v(), None, None) == N.FEM_ERR_UNSUPPORTED


@pytest.mark.parametrize("combo,status", [
    ((2, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, N.F32), N.FEM_ERR_UNSUPPORTED),   # tet rule in 2D
    ((3, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, N.F32), N.FEM_ERR_UNSUPPORTED),   # triangle rule in 3D
    ((1, mg.LAPLACE, mg.RULE_CENTROID, N.COEF_QUAD, N.F32), N.FEM_ERR_UNSUPPORTED),
    ((2, 9, mg.RULE_TRI3, N.COEF_QUAD, N.F32), N.FEM_ERR_UNSUPPORTED),
    ((2, mg.LAPLACE, 9, N.COEF_QUAD, N.F32), N.FEM_ERR_UNSUPPORTED),
    ((2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, 5), N.FEM_ERR_UNSUPPORTED),
    ((2, mg.LAPLACE, mg.RULE_TRI3, 3, N.F32), N.FEM_ERR_UNSUPPORTED),            # unknown coefficient space
    ((3, mg.ELASTICITY, mg.RULE_TET4, -1, N.F64), N.FEM_ERR_UNSUPPORTED),
])
def test_residual_combo_validation(lib, combo, status):
    st = lib.fem_integrate_residual(*combo, 10, _v(), _v(), _v(), _v(), _v(), None)
    assert st == status and N.last_error()
    st = lib.fem_integrate_residual_backward(*combo, 10, _v(), _v(), _v(), _v(), _v(), _v(), _v(), None)
    assert st == status


def test_residual_sizes_and_nulls(lib):
    c = (3, mg.ELASTICITY, mg.RULE_TET4, N.COEF_P1, N.F64)
    assert lib.fem_integrate_residual(*c, -5, _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_integrate_residual(*c, 0, None, None, None, None, None, None) == N.FEM_OK
    assert lib.fem_integrate_residual(*c, 5, _v(), None, _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    # backward: no output requested is a no-op; du needs coef, dcoef needs u
    assert lib.fem_integrate_residual_backward(*c, 5, _v(), _v(), None, None, _v(), None, None, None) == N.FEM_OK
    assert lib.fem_integrate_residual_backward(*c, 5, _v(), _v(), _v(), None, _v(), _v(), None, None) \
        == N.FEM_ERR_INVALID_ARG
    assert lib.fem_integrate_residual_backward(*c, 5, _v(), _v(), None, _v(), _v(), None, _v(), None) \
        == N.FEM_ERR_INVALID_ARG


def test_stream_copy_validation(lib):
    assert lib.fem_stream_copy(_v(), _v(), 15, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_stream_copy(_v(0x1008), _v(), 16, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_stream_copy(_v(), _v(), 0, None) == N.FEM_OK


def test_tuning_roundtrip(lib):
    R = N.OP_RESIDUAL
    t = N.fem_tuning()
    assert lib.fem_get_tuning(R, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(t)) == N.FEM_OK
    assert t.strategy == N.STRATEGY_LANE and t.vec in (1, 2, 4)
    new = N.fem_tuning(N.STRATEGY_LANE, 2, 8, 4)
    assert lib.fem_set_tuning(R, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(new)) == N.FEM_OK
    got = N.fem_tuning()
    lib.fem_get_tuning(R, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(got))
    assert (got.strategy, got.vec, got.waves_per_block, got.blocks_per_cu) == (0, 2, 8, 4)
    # other operations keep their own configuration
    lib.fem_get_tuning(N.OP_BACKWARD, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(got))
    assert (got.vec, got.waves_per_block, got.blocks_per_cu) != (2, 8, 4)
    bad = N.fem_tuning(N.STRATEGY_LANE, 3, 4, 0)
    assert lib.fem_set_tuning(R, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(bad)) == N.FEM_ERR_INVALID_ARG
    bad = N.fem_tuning(N.STRATEGY_LANE, 4, 5, 0)
    assert lib.fem_set_tuning(R, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(bad)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_set_tuning(R, 2, mg.MASS, mg.RULE_TET4, N.F64, ctypes.byref(new)) == N.FEM_ERR_UNSUPPORTED
    # the transposition strategy exists only for the residual; the fused kernel takes 1, 2 or 4 elements per lane
    tt = N.fem_tuning(N.STRATEGY_TRANSPOSE, 1, 4, 0)
    assert lib.fem_set_tuning(R, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(tt)) == N.FEM_OK
    assert lib.fem_set_tuning(N.OP_BACKWARD, 2, mg.MASS, mg.RULE_CENTROID, N.F64, ctypes.byref(tt)) \
        == N.FEM_ERR_INVALID_ARG
    four = N.fem_tuning(N.STRATEGY_LANE, 4, 4, 0)
    three = N.fem_tuning(N.STRATEGY_LANE, 3, 4, 0)
    assert lib.fem_set_tuning(N.OP_RESIDUAL_MESH, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(three)) \
        == N.FEM_ERR_INVALID_ARG
    saved = N.fem_tuning()
    lib.fem_get_tuning(N.OP_RESIDUAL_MESH, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(saved))
    assert lib.fem_set_tuning(N.OP_RESIDUAL_MESH, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(four)) == N.FEM_OK
    lib.fem_set_tuning(N.OP_RESIDUAL_MESH, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(saved))
    assert lib.fem_set_tuning(N.OP_GEOMETRY, 3, 99, 99, N.F32, ctypes.byref(four)) == N.FEM_OK  # physics ignored
    assert lib.fem_set_tuning(12, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(four)) == N.FEM_ERR_UNSUPPORTED


def test_mfma_strategy_availability(lib):
    """The matrix-core strategy exists for the P3 residual of tetrahedra with
    the Laplacian or elasticity only; elsewhere fem_set_tuning refuses it."""
    P3, R11 = N.OP_RESIDUAL_P3, mg.RULE_TET11
    saved = {}
    for phys in (mg.LAPLACE, mg.ELASTICITY):
        for dt in (N.F32, N.F64):
            saved[phys, dt] = N.fem_tuning()
            lib.fem_get_tuning(P3, 3, phys, R11, dt, ctypes.byref(saved[phys, dt]))
    t = N.fem_tuning(N.STRATEGY_MFMA, 1, 4, 0)
    for phys in (mg.LAPLACE, mg.ELASTICITY):
        for dt in (N.F32, N.F64):
            assert lib.fem_set_tuning(P3, 3, phys, R11, dt, ctypes.byref(t)) == N.FEM_OK
    assert lib.fem_set_tuning(P3, 3, mg.MASS, R11, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_set_tuning(P3, 2, mg.ELASTICITY, mg.RULE_TRI6, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    for op in (N.OP_RESIDUAL, N.OP_RESIDUAL_P2, N.OP_BACKWARD_P3, N.OP_JACOBIAN_P3):
        assert lib.fem_set_tuning(op, 3, mg.LAPLACE, R11 if op != N.OP_RESIDUAL else mg.RULE_TET4, N.F32,
                                  ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
    for (phys, dt), t in saved.items():
        assert lib.fem_set_tuning(P3, 3, phys, R11, dt, ctypes.byref(t)) == N.FEM_OK


def test_stream_rows_validation(lib):
    """fem_stream_rows checks its arguments before any HIP call."""
    vp = ctypes.c_void_p(16)
    assert lib.fem_stream_rows(7, 10, 1, 1, vp, vp, None) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_stream_rows(N.F32, -1, 1, 1, vp, vp, None) == N.FEM_ERR_INVALID_ARG
    for n_in, n_out in ((0, 1), (1, 0), (257, 1), (1, 257)):
        assert lib.fem_stream_rows(N.F32, 10, n_in, n_out, vp, vp, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_stream_rows(N.F64, 10, 2, 2, None, vp, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_stream_rows(N.F64, 0, 2, 2, None, None, None) == N.FEM_OK


def test_component_strategy_availability(lib):
    """The component-parallel strategy exists for the P3 residual of
    tetrahedra with elasticity only (vec 1, one or two three-wave groups per
    workgroup in FP32, one in FP64); elsewhere fem_set_tuning refuses it."""
    P3, R11 = N.OP_RESIDUAL_P3, mg.RULE_TET11
    saved = {dt: N.fem_tuning() for dt in (N.F32, N.F64)}
    for dt in saved:
        lib.fem_get_tuning(P3, 3, mg.ELASTICITY, R11, dt, ctypes.byref(saved[dt]))
    # three-wave groups per workgroup: one or two in FP32, one in FP64
    for dt, groups in ((N.F32, (1, 2)), (N.F64, (1,))):
        for waves in groups:
            t = N.fem_tuning(N.STRATEGY_COMPONENT, 1, waves, 0)
            assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, dt, ctypes.byref(t)) == N.FEM_OK
            back = N.fem_tuning()
            lib.fem_get_tuning(P3, 3, mg.ELASTICITY, R11, dt, ctypes.byref(back))
            assert (back.strategy, back.waves_per_block) == (N.STRATEGY_COMPONENT, waves)
    t = N.fem_tuning(N.STRATEGY_COMPONENT, 1, 2, 0)
    assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, N.F64, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    t = N.fem_tuning(N.STRATEGY_COMPONENT, 1, 4, 0)
    assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    t = N.fem_tuning(N.STRATEGY_COMPONENT, 1, 8, 0)   # no P3 strategy takes eight waves
    assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, N.F32, ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
    t = N.fem_tuning(N.STRATEGY_COMPONENT, 1, 2, 0)
    for phys in (mg.LAPLACE, mg.MASS):
        assert lib.fem_set_tuning(P3, 3, phys, R11, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_set_tuning(P3, 2, mg.ELASTICITY, mg.RULE_TRI6, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
    for op in (N.OP_RESIDUAL, N.OP_RESIDUAL_P2, N.OP_BACKWARD_P3, N.OP_JACOBIAN_P3):
        assert lib.fem_set_tuning(op, 3, mg.ELASTICITY, R11 if op != N.OP_RESIDUAL else mg.RULE_TET4, N.F32,
                                  ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
    wide = N.fem_tuning(N.STRATEGY_COMPONENT, 2, 2, 0)
    assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, N.F32, ctypes.byref(wide)) == N.FEM_ERR_INVALID_ARG
    for dt in saved:
        assert lib.fem_set_tuning(P3, 3, mg.ELASTICITY, R11, dt, ctypes.byref(saved[dt])) == N.FEM_OK


def test_batch_plan_validation(lib):
    plan = ctypes.c_void_p()
    assert lib.fem_batch_plan_create(None, 1, N.F32, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_batch_plan_create(None, 0, 9, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED
    d = (N.fem_mesh_desc * 1)()
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, 10, 1, 1, 1, 1, 1)
    assert lib.fem_batch_plan_create(d, 1, N.F32, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, 5, 10, 1, 1, 1, 1, 1)
    assert lib.fem_batch_plan_create(d, 1, N.F32, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, -1, 1, 1, 1, 1, 1)
    assert lib.fem_batch_plan_create(d, 1, N.F32, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_P0, 10, 1, None, 1, 1, 1)
    assert lib.fem_batch_plan_create(d, 1, N.F32, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_batch_run(None, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_batch_replay(None, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_batch_plan_set_launch(None, 4, 8) == N.FEM_ERR_INVALID_ARG
    lib.fem_batch_plan_destroy(None)


def test_dedup_strategy_availability(lib):
    """Run-time vertex deduplication serves the fused from-mesh residual
    only, one element per lane."""
    M, R = N.OP_RESIDUAL_MESH, N.OP_RESIDUAL
    saved = N.fem_tuning()
    assert lib.fem_get_tuning(M, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(saved)) == N.FEM_OK
    try:
        for dim, rule in ((2, mg.RULE_TRI3), (3, mg.RULE_TET4)):
            for waves in (1, 8):
                t = N.fem_tuning(N.STRATEGY_DEDUP, 1, waves, 0)
                assert lib.fem_set_tuning(M, dim, mg.LAPLACE, rule, N.F32, ctypes.byref(t)) == N.FEM_ERR_UNSUPPORTED
            for waves in (2, 4):
                t = N.fem_tuning(N.STRATEGY_DEDUP, 1, waves, 0)
                assert lib.fem_set_tuning(M, dim, mg.LAPLACE, rule, N.F32, ctypes.byref(t)) == N.FEM_OK
                back = N.fem_tuning()
                assert lib.fem_get_tuning(M, dim, mg.LAPLACE, rule, N.F32, ctypes.byref(back)) == N.FEM_OK
                assert (back.strategy, back.vec, back.waves_per_block) == (N.STRATEGY_DEDUP, 1, waves)
        for op in (R, N.OP_GEOMETRY, N.OP_BACKWARD, N.OP_RESIDUAL_GATHER):
            t = N.fem_tuning(N.STRATEGY_DEDUP, 1, 4, 0)
            assert lib.fem_set_tuning(op, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
        t = N.fem_tuning(N.STRATEGY_DEDUP, 2, 4, 0)
        assert lib.fem_set_tuning(M, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
    finally:
        for dim, rule in ((2, mg.RULE_TRI3), (3, mg.RULE_TET4)):
            assert lib.fem_set_tuning(M, dim, mg.LAPLACE, rule, N.F32, ctypes.byref(saved)) == N.FEM_OK


def test_batch_noalloc_validation(lib):
    """The no-allocation batched launch rejects bad input before any HIP call."""
    run = lib.fem_batch_run_noalloc
    assert N.BATCH_NOALLOC_MAX_MESHES == 1024
    assert "#define FEM_BATCH_NOALLOC_MAX_MESHES 1024" in N.HEADER.read_text()
    assert run(None, 1, N.F32, 8, 0, None) == N.FEM_ERR_INVALID_ARG
    assert run(None, -1, N.F32, 8, 0, None) == N.FEM_ERR_INVALID_ARG
    big = (N.fem_mesh_desc * (N.BATCH_NOALLOC_MAX_MESHES + 1))()
    assert run(big, N.BATCH_NOALLOC_MAX_MESHES + 1, N.F32, 8, 0, None) == N.FEM_ERR_INVALID_ARG
    assert "limit" in N.last_error()
    d = (N.fem_mesh_desc * 1)()
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, 10, 1, 1, 1, 1, 1)
    assert run(d, 1, 9, 8, 0, None) == N.FEM_ERR_UNSUPPORTED
    assert run(d, 1, N.F32, 3, 0, None) == N.FEM_ERR_INVALID_ARG
    assert run(d, 1, N.F32, 8, 65, None) == N.FEM_ERR_INVALID_ARG
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, 10, 1, 1, 1, 1, 1)
    assert run(d, 1, N.F32, 8, 0, None) == N.FEM_ERR_UNSUPPORTED
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, -1, 1, 1, 1, 1, 1)
    assert run(d, 1, N.F32, 8, 0, None) == N.FEM_ERR_INVALID_ARG
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, 10, 1, 1, None, 1, 1)
    assert run(d, 1, N.F32, 8, 0, None) == N.FEM_ERR_INVALID_ARG
    # nothing to do: empty list and empty meshes return before any HIP call
    assert run(None, 0, N.F32, 8, 0, None) == N.FEM_OK
    d[0] = N.fem_mesh_desc(2, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, 0, None, None, None, None, None)
    assert run(d, 1, N.F32, 8, 0, None) == N.FEM_OK


def test_autotune_validation(lib):
    R = N.OP_RESIDUAL
    assert lib.fem_autotune(R, 2, mg.LAPLACE, mg.RULE_TET4, N.F32, 1 << 16, None) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_autotune(R, 2, mg.LAPLACE, mg.RULE_TRI3, N.F32, 10, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_autotune(12, 2, mg.LAPLACE, mg.RULE_TRI3, N.F32, 1 << 16, None) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_load_tuning(None) == N.FEM_ERR_INVALID_ARG


def _cache_entry(arch, op=0, dim=2, physics=2, rule=2, dtype=1, strategy=0, vec=2, waves=2, bpc=8, extra=""):
    return (f'{{"arch": "{arch}", "op": {op}, "dim": {dim}, "physics": {physics}, "rule": {rule}, '
            f'"dtype": {dtype}, "strategy": {strategy}, "vec": {vec}, "waves_per_block": {waves}, '
            f'"blocks_per_cu": {bpc}{extra}, "us": 1.0}}')


def test_load_tuning_malformed_cache(lib, tmp_path):
    """fem_load_tuning on malformed, truncated or out-of-range cache files:
    FEM_ERR_NO_TUNING, no crash, and the configuration in force unchanged.
    Every file names both the architecture of a GPU here and "unknown" (what
    the library reports with no GPU), so the valid entries apply anywhere."""
    key = (N.OP_RESIDUAL, 2, mg.MASS, mg.RULE_CENTROID, N.F64)
    base = N.fem_tuning(N.STRATEGY_LANE, 1, 4, 0)
    assert lib.fem_set_tuning(*key, ctypes.byref(base)) == N.FEM_OK

    def current():
        t = N.fem_tuning()
        assert lib.fem_get_tuning(*key, ctypes.byref(t)) == N.FEM_OK
        return (t.strategy, t.vec, t.waves_per_block, t.blocks_per_cu)

    def both(**kw):
        return ", ".join(_cache_entry(a, **kw) for a in ("unknown", "gfx950"))

    bad = {
        "empty": "",
        "not json": "\x00\xff garbage {{{ ]]] \"",
        "no entries key": '{"version": 1, "items": [' + both() + ']}',
        "truncated object": '{"version": 1, "entries": [{"arch": "unknown", "op": 0, "dim"',
        "unterminated string": '{"entries": [{"arch": "unkn',
        "array closed first": '{"entries": ]' + both() + '}',
        "value without number": '{"entries": [' + both(extra=', "vec": abc') + ']}',
        "huge numbers": '{"entries": [' + ", ".join(
            _cache_entry(a, dim="1e400", vec="-1e300", waves="nan") for a in ("unknown", "gfx950")) + ']}',
        "invalid launch shape": '{"entries": [' + both(vec=3, waves=5) + ']}',
        "unsupported op": '{"entries": [' + both(op=99) + ']}',
        "colon missing": '{"entries": [{"arch" "unknown" "op" 0}]}',
    }
    for name, text in bad.items():
        f = tmp_path / (name.replace(" ", "_") + ".json")
        f.write_text(text)
        assert lib.fem_load_tuning(str(f).encode()) == N.FEM_ERR_NO_TUNING, name
        assert current() == (0, 1, 4, 0), name
    assert lib.fem_load_tuning(str(tmp_path / "missing.json").encode()) == N.FEM_ERR_NO_TUNING
    # a malformed entry next to a valid one: the valid one is applied
    f = tmp_path / "mixed.json"
    f.write_text('{"version": 1, "entries": [' + both(vec=3) + ", " + both(vec=2, waves=2, bpc=8) + ']}')
    assert lib.fem_load_tuning(str(f).encode()) == N.FEM_OK
    assert current() == (0, 2, 2, 8)
    assert lib.fem_set_tuning(*key, ctypes.byref(base)) == N.FEM_OK


def test_residual_mesh_validation(lib):
    c = (3, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, N.F32)
    f = lib.fem_integrate_residual_mesh
    assert f(*c, 0, 0, None, None, None, None, None, None, None, None, None) == N.FEM_OK
    assert f(*c, -1, 5, _v(), _v(), _v(), _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(*c, 5, 0, _v(), _v(), _v(), _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(*c, 5, 5, _v(), None, _v(), _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    # geometry outputs: both or neither
    assert f(*c, 5, 5, _v(), _v(), _v(), _v(), _v(), _v(), None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(3, mg.LAPLACE, mg.RULE_TRI3, N.COEF_QUAD, N.F32, 5, 5, _v(), _v(), _v(), _v(), _v(), None, None, None,
             None) == N.FEM_ERR_UNSUPPORTED
    assert f(3, mg.LAPLACE, mg.RULE_TET4, 7, N.F32, 5, 5, _v(), _v(), _v(), _v(), _v(), None, None, None, None) \
        == N.FEM_ERR_UNSUPPORTED


def test_residual_gather_validation(lib):
    c = (3, mg.LAPLACE, mg.RULE_TET4, N.COEF_P1, N.F32)
    f = lib.fem_integrate_residual_gather
    assert f(*c, 0, 0, None, None, None, None, None, None, None, None, None) == N.FEM_OK
    assert f(*c, -1, 5, _v(), _v(), _v(), _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(*c, 5, 0, _v(), _v(), _v(), _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(*c, 5, 5, _v(), _v(), None, _v(), _v(), None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert f(*c, 5, 5, _v(), _v(), _v(), _v(), _v(), None, _v(), None, None) == N.FEM_ERR_INVALID_ARG
    assert f(3, mg.LAPLACE, mg.RULE_TET4, 4, N.F32, 5, 5, _v(), _v(), _v(), _v(), _v(), None, None, None, None) \
        == N.FEM_ERR_UNSUPPORTED
    three = N.fem_tuning(N.STRATEGY_LANE, 3, 4, 0)
    assert lib.fem_set_tuning(N.OP_RESIDUAL_GATHER, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(three)) \
        == N.FEM_ERR_INVALID_ARG


def test_assembly_validation(lib):
    plan = ctypes.c_void_p()
    f = lib.fem_assembly_plan_create
    assert f(2, 5, 5, _v(), None, None) == N.FEM_ERR_INVALID_ARG            # out is NULL
    assert f(4, 5, 5, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED
    assert f(2, -1, 5, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert f(2, 5, 0, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert f(2, 5, 5, None, None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert f(3, 2 ** 30, 5, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED  # 4 * 2^30 slots
    assert not plan.value
    assert lib.fem_assemble(None, 1, N.F32, _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    r = lib.fem_restrict
    assert r(2, 1, N.F32, 0, 0, None, None, None, None) == N.FEM_OK
    assert r(2, 4, N.F32, 5, 5, _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED
    assert r(2, 1, 9, 5, 5, _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED
    assert r(5, 1, N.F32, 5, 5, _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED
    assert r(2, 1, N.F32, 5, 0, _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    assert r(2, 1, N.F32, 5, 5, _v(), None, _v(), None) == N.FEM_ERR_INVALID_ARG
    lib.fem_assembly_plan_destroy(None)


def test_p2_validation(lib):
    f, b = lib.fem_integrate_residual_p2, lib.fem_integrate_residual_p2_backward
    ok = (3, mg.ELASTICITY, mg.RULE_TET11, N.COEF_QUAD, N.F32)
    assert f(*ok, 0, None, None, None, None, None, None) == N.FEM_OK
    assert f(*ok, -1, _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    assert f(*ok, 5, _v(), None, _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    for bad in [(3, mg.LAPLACE, mg.RULE_CENTROID, 0, N.F32), (2, mg.LAPLACE, mg.RULE_TET11, 0, N.F32),
                (3, mg.LAPLACE, mg.RULE_TRI6, 0, N.F32), (3, 7, mg.RULE_TET4, 0, N.F32),
                (3, mg.LAPLACE, mg.RULE_TET4, 5, N.F32), (3, mg.LAPLACE, mg.RULE_TET4, 0, 3)]:
        assert f(*bad, 5, _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED, bad
        assert b(*bad, 5, _v(), _v(), _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED, bad
    assert b(*ok, 5, _v(), _v(), None, None, _v(), None, None, None) == N.FEM_OK            # nothing wanted
    assert b(*ok, 5, _v(), _v(), None, _v(), _v(), None, _v(), None) == N.FEM_ERR_INVALID_ARG  # dcoef needs u
    # the degree-4 rules exist only for the second-order entry points
    assert lib.fem_integrate_residual(2, mg.LAPLACE, mg.RULE_TRI6, 0, N.F32, 5, _v(), _v(), _v(), _v(), _v(),
                                      None) == N.FEM_ERR_UNSUPPORTED
    t = N.fem_tuning(N.STRATEGY_LANE, 1, 8, 0)
    assert lib.fem_set_tuning(N.OP_RESIDUAL_P2, 3, mg.LAPLACE, mg.RULE_TET11, N.F32, ctypes.byref(t)) \
        == N.FEM_ERR_INVALID_ARG
    t = N.fem_tuning(N.STRATEGY_LANE, 2, 4, 0)
    assert lib.fem_set_tuning(N.OP_BACKWARD_P2, 3, mg.LAPLACE, mg.RULE_TET11, N.F32, ctypes.byref(t)) \
        == N.FEM_ERR_INVALID_ARG


def test_p3_validation(lib):
    f = lib.fem_integrate_residual_p3
    ok = (3, mg.ELASTICITY, mg.RULE_TET11, N.COEF_P1, N.F64)
    assert f(*ok, 0, None, None, None, None, None, None) == N.FEM_OK
    assert f(*ok, -1, _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
    assert f(*ok, 5, _v(), _v(), _v(), None, _v(), None) == N.FEM_ERR_INVALID_ARG
    for bad in [(3, mg.LAPLACE, mg.RULE_TET4, 0, N.F32), (2, mg.LAPLACE, mg.RULE_TRI3, 0, N.F32),
                (2, mg.LAPLACE, mg.RULE_TET11, 0, N.F32), (3, mg.LAPLACE, mg.RULE_CENTROID, 0, N.F32),
                (3, 7, mg.RULE_TET11, 0, N.F32), (3, mg.LAPLACE, mg.RULE_TET11, 5, N.F32),
                (3, mg.LAPLACE, mg.RULE_TET11, 0, 3), (4, mg.LAPLACE, mg.RULE_TET11, 0, N.F32)]:
        assert f(*bad, 5, _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED, bad
    b = lib.fem_integrate_residual_p3_backward
    for bad in [(3, mg.LAPLACE, mg.RULE_TET4, 0, N.F32), (2, mg.LAPLACE, mg.RULE_TRI3, 0, N.F32),
                (3, mg.LAPLACE, mg.RULE_TET11, 5, N.F32)]:
        assert b(*bad, 5, _v(), _v(), _v(), _v(), _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED, bad
    assert b(*ok, 5, _v(), _v(), None, None, _v(), None, None, None) == N.FEM_OK            # nothing wanted
    assert b(*ok, 5, _v(), _v(), None, _v(), _v(), None, _v(), None) == N.FEM_ERR_INVALID_ARG  # dcoef needs u
    assert b(*ok, 5, _v(), _v(), _v(), None, _v(), _v(), None, None) == N.FEM_ERR_INVALID_ARG  # du needs coef
    t = N.fem_tuning(N.STRATEGY_LANE, 1, 8, 0)   # at most four waves per block
    for op in (N.OP_RESIDUAL_P3, N.OP_BACKWARD_P3):
        assert lib.fem_set_tuning(op, 3, mg.LAPLACE, mg.RULE_TET11, N.F32, ctypes.byref(t)) == N.FEM_ERR_INVALID_ARG
    t = N.fem_tuning(N.STRATEGY_LANE, 1, 4, 0)
    assert lib.fem_set_tuning(N.OP_RESIDUAL_P3, 3, mg.LAPLACE, mg.RULE_TET4, N.F32, ctypes.byref(t)) \
        == N.FEM_ERR_UNSUPPORTED


def test_mesh_plan_validation(lib):
    plan = ctypes.c_void_p()
    assert lib.fem_mesh_plan_create(2, 10, 10, _v(), None, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_mesh_plan_create(4, 10, 10, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_mesh_plan_create(3, -1, 10, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_mesh_plan_create(3, 10, 10, None, None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_mesh_plan_create(3, 10, 0, _v(), None, ctypes.byref(plan)) == N.FEM_ERR_INVALID_ARG
    assert not plan.value
    for f in (lib.fem_integrate_residual_planned, lib.fem_integrate_residual_gather_planned):
        assert f(None, mg.LAPLACE, mg.RULE_TET4, 0, N.F32, _v(), _v(), _v(), _v(), None, None, None,
                 None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_mesh_plan_info(None, None, None, None, None, None) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_geometry_planned(None, _v(), N.F32, _v(), _v(), None, None) == N.FEM_ERR_INVALID_ARG
    lib.fem_mesh_plan_destroy(None)


def test_batch_autotune_validation(lib):
    w, b = ctypes.c_int(), ctypes.c_int()
    assert lib.fem_batch_plan_autotune(None, None, ctypes.byref(w), ctypes.byref(b)) == N.FEM_ERR_INVALID_ARG
    assert N.last_error()


def test_jacobian_validation(lib):
    f = lib.fem_integrate_jacobian
    # (dim, physics, rule, coef_space, order, dtype)
    ok1 = (3, mg.ELASTICITY, mg.RULE_CENTROID, N.COEF_P1, 1, N.F64)
    ok2 = (2, mg.MASS, mg.RULE_TRI6, N.COEF_P0, 2, N.F32)
    ok3 = (3, mg.ELASTICITY, mg.RULE_TET11, N.COEF_P1, 3, N.F64)
    for ok in (ok1, ok2, ok3):
        assert f(*ok, 0, None, None, None, None, None) == N.FEM_OK
        assert f(*ok, -1, _v(), _v(), _v(), _v(), None) == N.FEM_ERR_INVALID_ARG
        for k in range(4):
            arrs = [_v(), _v(), _v(), _v()]
            arrs[k] = None
            assert f(*ok, 5, *arrs, None) == N.FEM_ERR_INVALID_ARG, k
    for bad in [(2, mg.LAPLACE, mg.RULE_TRI6, 0, 1, N.F32),       # degree-4 rule with order 1
                (3, mg.LAPLACE, mg.RULE_CENTROID, 0, 2, N.F32),   # centroid with order 2
                (2, mg.LAPLACE, mg.RULE_TET4, 0, 1, N.F32),       # tet rule in 2D
                (3, mg.LAPLACE, mg.RULE_TET4, 0, 3, N.F32),       # order 3 with a degree-2 rule
                (3, mg.LAPLACE, mg.RULE_TET11, 0, 4, N.F32),      # order 4
                (3, 9, mg.RULE_TET4, 0, 1, N.F32), (3, mg.LAPLACE, mg.RULE_TET4, 4, 1, N.F32),
                (3, mg.LAPLACE, mg.RULE_TET4, 0, 1, 2), (4, mg.LAPLACE, mg.RULE_TET4, 0, 1, N.F32)]:
        assert f(*bad, 5, _v(), _v(), _v(), _v(), None) == N.FEM_ERR_UNSUPPORTED, bad
        assert N.last_error()
    t = N.fem_tuning(N.STRATEGY_LANE, 1, 4, 2)
    for op, rule in ((N.OP_JACOBIAN, mg.RULE_CENTROID), (N.OP_JACOBIAN_P2, mg.RULE_TET11),
                     (N.OP_JACOBIAN_P3, mg.RULE_TET11)):
        assert lib.fem_set_tuning(op, 3, mg.LAPLACE, rule, N.F32, ctypes.byref(t)) == N.FEM_OK
        for bad_t in (N.fem_tuning(N.STRATEGY_LANE, 2, 4, 0), N.fem_tuning(N.STRATEGY_LANE, 1, 8, 0)):
            assert lib.fem_set_tuning(op, 3, mg.LAPLACE, rule, N.F32, ctypes.byref(bad_t)) == N.FEM_ERR_INVALID_ARG
    assert lib.fem_set_tuning(N.OP_JACOBIAN, 3, mg.LAPLACE, mg.RULE_TET11, N.F32, ctypes.byref(t)) \
        == N.FEM_ERR_UNSUPPORTED
    assert lib.fem_set_tuning(N.OP_JACOBIAN_P2, 3, mg.LAPLACE, mg.RULE_CENTROID, N.F32, ctypes.byref(t)) \
        == N.FEM_ERR_UNSUPPORTED


@pytest.mark.parametrize("std", ["c99", "c11"])
def test_header_is_plain_c(tmp_path, std):
    """include/fem.h compiles as ISO C with warnings as errors (no C++, no HIP headers)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_fem.c"
    src.write_text('#include "fem.h"\nint main(void) { fem_tuning t = {0, 1, 2, 0}; (void)t; return FEM_OK; }\n')
    inc = pathlib.Path(__file__).resolve().parents[1] / "include"
    r = subprocess.run(["gcc", f"-std={std}", "-Wall", "-Wextra", "-pedantic", "-Werror", f"-I{inc}", "-fsyntax-only",
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_no_device_gives_hip_error_not_a_crash(lib):
    """On a host without a GPU a call that passes validation fails with
    FEM_ERR_HIP and the runtime's message; nothing is launched. (Skipped where
    a GPU is visible: there the placeholder pointers would be dereferenced.)"""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible; this case needs a host without one")
    ptr = [0x1000 * (k + 1) for k in range(8)]
    st = lib.fem_integrate_residual(3, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, N.F32, 1000, *ptr[:5], None)
    assert st == N.FEM_ERR_HIP and "fem_integrate_residual" in N.last_error()
    st = lib.fem_geometry(3, 1000, 500, ptr[0], ptr[1], N.F32, ptr[2], ptr[3], None, None)
    assert st == N.FEM_ERR_HIP and "fem_geometry" in N.last_error()
    d = (N.fem_mesh_desc * 1)()
    d[0] = N.fem_mesh_desc(3, mg.LAPLACE, mg.RULE_TET4, N.COEF_QUAD, 10, *ptr[:5])
    assert lib.fem_batch_run_noalloc(d, 1, N.F32, 8, 0, None) == N.FEM_ERR_HIP
    assert "fem_batch_run_noalloc" in N.last_error()


def test_env_tuning_cache_unusable_keeps_defaults(tmp_path):
    """FEM_TUNE_CACHE naming a missing or malformed file leaves the default
    tunings (compared with a fresh process without the variable) and no error."""
    import os
    import subprocess
    import sys
    root = pathlib.Path(__file__).resolve().parents[1]
    code = ("from paper_1607_04245_amd import api, _native as N, meshgen as mg; "
            "print([api.fem_get_tuning(3, mg.LAPLACE, mg.RULE_TET4, 0, op=o) for o in range(5)], "
            "repr(N.last_error()))")
    def run(extra):
        env = {k: v for k, v in os.environ.items() if k != "FEM_TUNE_CACHE"}
        env.update(extra)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300,
                           cwd=str(root))
        assert r.returncode == 0, r.stderr
        return r.stdout.strip().splitlines()[-1]
    bad = tmp_path / "bad.json"
    bad.write_text("{ not json")
    base = run({})
    assert run({"FEM_TUNE_CACHE": str(tmp_path / "missing.json")}) == base
    assert run({"FEM_TUNE_CACHE": str(bad)}) == base
