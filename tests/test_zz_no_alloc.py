"""GPU: the no-allocation batched launch (fem_batch_run_noalloc), called
through the C ABI, against the plan-based batched launch (fem_batch_plan_create
+ fem_batch_run) on the same meshes: bitwise equal element vectors, on two
calls in a row, the second with fewer and smaller meshes, in FP32 and FP64
and at several launch shapes. The first call's outputs are checked to stay
untouched by the second, and one mesh of each call against the FP64 oracle."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1607_04245_amd import api, meshgen as mg
from paper_1607_04245_amd import _native as N

from _parity import assert_close, dev, oracle_reference

pytestmark = pytest.mark.gpu


def _meshes(dtype, sizes, seed0):
    out, wls = [], []
    for m, ne in enumerate(sizes):
        dim, phys = mg.MESH_TYPES[m % 4]
        rule = mg.default_rule(dim) if m % 3 else mg.RULE_CENTROID
        grid = mg.smallest_grid(dim, max(ne, 1))
        wl = mg.make_workload(f"na{m}", dim, phys, grid, ne, mg.BASE_SEED + seed0 + m, rule=rule)
        ij, dj = api.fem_geometry(dev(wl.coords, torch.float64), dev(wl.conn, torch.int32), dtype)
        out.append(dict(dim=dim, physics=phys, rule=rule, inv_j=ij, det_j=dj, u=dev(wl.u, dtype),
                        coef=dev(wl.coef, dtype),
                        out=torch.full(wl.u.shape, float("nan"), dtype=dtype, device="cuda")))
        wls.append(wl)
    return out, wls


def _descs(meshes):
    d = (N.fem_mesh_desc * len(meshes))()
    for i, m in enumerate(meshes):
        d[i] = N.fem_mesh_desc(m["dim"], m["physics"], m["rule"], N.COEF_QUAD, m["det_j"].shape[0],
                               m["inv_j"].data_ptr(), m["det_j"].data_ptr(), m["u"].data_ptr(),
                               m["coef"].data_ptr(), m["out"].data_ptr())
    return d


def _plan_outputs(meshes, dtype, waves, bpc):
    """Element vectors of the existing plan-based entry point."""
    lib = N.lib()
    d = _descs(meshes)
    plan = ctypes.c_void_p()
    N.check(lib.fem_batch_plan_create(d, len(meshes), N.F32 if dtype == torch.float32 else N.F64,
                                      ctypes.byref(plan)), "fem_batch_plan_create")
    try:
        N.check(lib.fem_batch_plan_set_launch(plan, waves, bpc), "fem_batch_plan_set_launch")
        for m in meshes:
            m["out"].fill_(float("nan"))
        N.check(lib.fem_batch_run(plan, None), "fem_batch_run")
        torch.cuda.synchronize()
        return [m["out"].clone() for m in meshes]
    finally:
        lib.fem_batch_plan_destroy(plan)


def _noalloc(meshes, dtype, waves, bpc):
    for m in meshes:
        m["out"].fill_(float("nan"))
    torch.cuda.synchronize()
    d = _descs(meshes)
    N.check(N.lib().fem_batch_run_noalloc(d, len(meshes), N.F32 if dtype == torch.float32 else N.F64,
                                          waves, bpc, None), "fem_batch_run_noalloc")
    torch.cuda.synchronize()
    return [m["out"].clone() for m in meshes]


FIRST = [3000, 1, 4097, 0, 30000, 65, 2000, 5003, 12, 777, 12345]
SECOND = [500, 64, 129]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("waves,bpc", [(8, 0), (4, 8), (1, 2)])
def test_noalloc_matches_plan_two_calls(dtype, waves, bpc):
    torch.cuda.set_device(0)
    first, wl1 = _meshes(dtype, FIRST, 300)
    second, wl2 = _meshes(dtype, SECOND, 400)
    ref1 = _plan_outputs(first, dtype, waves, bpc)
    ref2 = _plan_outputs(second, dtype, waves, bpc)
    got1 = _noalloc(first, dtype, waves, bpc)
    for g, r, wl in zip(got1, ref1, wl1):
        assert torch.equal(g, r), f"first call: {wl.name} ({wl.n_elem} elements) differs from the plan"
    got2 = _noalloc(second, dtype, waves, bpc)
    for g, r, wl in zip(got2, ref2, wl2):
        assert torch.equal(g, r), f"second call: {wl.name} ({wl.n_elem} elements) differs from the plan"
    # the smaller second call left the first call's outputs alone
    for m, g in zip(first, got1):
        assert torch.equal(m["out"], g)
    # parity with the oracle on one mesh of each call
    for wl, g in ((wl1[4], got1[4]), (wl2[0], got2[0])):
        ref, ref_abs, _, _ = oracle_reference(wl, dtype)
        assert_close(g.cpu().numpy(), ref, ref_abs, dtype, f"noalloc {wl.name}")


def test_noalloc_many_meshes_chunked_upload():
    """More meshes than one descriptor upload carries (32): 70 meshes, some
    empty, against the plan; then 33 meshes in a second call."""
    dtype = torch.float32
    rng = np.random.default_rng(mg.BASE_SEED + 310)
    sizes = [int(x) for x in rng.integers(0, 3000, size=70)]
    sizes[5] = sizes[40] = 0
    meshes, wls = _meshes(dtype, sizes, 600)
    ref = _plan_outputs(meshes, dtype, 4, 0)
    got = _noalloc(meshes, dtype, 4, 0)
    for g, r, wl in zip(got, ref, wls):
        assert torch.equal(g, r), f"{wl.name} ({wl.n_elem} elements) differs from the plan"
    fewer = meshes[:33]
    ref2 = _plan_outputs(fewer, dtype, 2, 4)
    got2 = _noalloc(fewer, dtype, 2, 4)
    for g, r in zip(got2, ref2):
        assert torch.equal(g, r)


def test_noalloc_python_binding_and_limit():
    dtype = torch.float32
    meshes, _ = _meshes(dtype, [1000, 2000], 500)
    ref = _plan_outputs(meshes, dtype, 8, 0)
    for m in meshes:
        m["out"].fill_(float("nan"))
    api.batch_run_noalloc(meshes)
    torch.cuda.synchronize()
    for m, r in zip(meshes, ref):
        assert torch.equal(m["out"], r)
    with pytest.raises(N.FemError) as ei:
        api.batch_run_noalloc([meshes[0]] * (N.BATCH_NOALLOC_MAX_MESHES + 1))
    assert ei.value.status == N.FEM_ERR_INVALID_ARG
