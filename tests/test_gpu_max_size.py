"""Element counts above 2^31: the kernels index SoA rows with 64-bit offsets.

Inputs are drawn on the device (about 120 GB per case, within the 288 GB of
one MI355X); sampled elements, among them those on either side of 2^31 and
the ragged tail, are copied back and checked against the FP64 oracle with
the FP32 bars of the other parity tests.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_04245_amd import api, meshgen as mg

from _parity import assert_close

pytestmark = pytest.mark.gpu

N_BIG = (1 << 31) + 4097


def _need_memory(gib):
    total = torch.cuda.get_device_properties(0).total_memory
    if total < gib * (1 << 30):
        pytest.skip(f"needs {gib} GiB of device memory")


def _samples(n, rng, k=2048):
    around = np.arange((1 << 31) - 70, (1 << 31) + 70)
    tail = np.arange(n - 70, n)
    return np.unique(np.concatenate([[0, 1, 63, 64], around[around < n], tail, rng.integers(0, n, k)]))


def _uniform(shape, lo, hi, gen):
    t = torch.empty(shape, dtype=torch.float32, device="cuda")
    t.uniform_(lo, hi, generator=gen)
    return t


def test_integrate_above_2p31_elements():
    _need_memory(160)
    n = N_BIG
    gen = torch.Generator(device="cuda")
    gen.manual_seed(mg.BASE_SEED + 900)
    rule = mg.RULE_TRI3
    ij = _uniform((4, n), -1.5, 1.5, gen)
    dj = _uniform((n,), 0.5, 2.0, gen)
    u = _uniform((3, n), -1.0, 1.0, gen)
    cf = _uniform((1, 3, n), 0.5, 2.0, gen)
    R = api.fem_integrate_residual(2, mg.LAPLACE, rule, ij, dj, u, cf)
    torch.cuda.synchronize()
    cols = _samples(n, np.random.default_rng(3))
    ci = torch.from_numpy(cols).to("cuda")
    got = R[:, ci].cpu().numpy()
    ij_s, dj_s = ij[:, ci].cpu().double().numpy(), dj[ci].cpu().double().numpy()
    u_s, cf_s = u[:, ci].cpu().double().numpy(), cf[:, :, ci].cpu().double().numpy()
    del R, ij, dj, u, cf
    torch.cuda.empty_cache()
    ref = oracle.integrate(2, mg.LAPLACE, rule, ij_s, dj_s, u_s, cf_s)
    ref_abs = oracle.integrate_abs(2, mg.LAPLACE, rule, ij_s, dj_s, u_s, cf_s)
    mx, agg = assert_close(got, ref, ref_abs, torch.float32, "2^31 + 4097 elements")
    print(f"integrate, {n} elements: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)


def _grid_connectivity(nx, ny, n_elem):
    """Triangles of an nx x ny grid of cells, two per cell ((v00, v10, v11) and
    (v00, v11, v01)), first n_elem, built on the device in chunks."""
    conn = torch.empty((n_elem, 3), dtype=torch.int32, device="cuda")
    chunk = 1 << 27
    for s in range(0, n_elem, chunk):
        e = torch.arange(s, min(s + chunk, n_elem), dtype=torch.int64, device="cuda")
        cell, t = e // 2, e % 2
        i, j = cell // ny, cell % ny
        v00 = i * (ny + 1) + j
        v10, v01 = v00 + (ny + 1), v00 + 1
        v11 = v10 + 1
        conn[s:s + e.numel(), 0] = v00.to(torch.int32)
        conn[s:s + e.numel(), 1] = torch.where(t == 0, v10, v11).to(torch.int32)
        conn[s:s + e.numel(), 2] = torch.where(t == 0, v11, v01).to(torch.int32)
        del e, cell, t, i, j, v00, v10, v01, v11
    return conn


def test_fused_mesh_above_2p31_elements():
    _need_memory(160)
    nx = ny = 32769                       # 2 * 32769^2 = 2^31 + 131074 triangles
    n = N_BIG
    assert 2 * nx * ny >= n
    nvx, nvy = nx + 1, ny + 1
    n_vert = nvx * nvy                    # about 1.07e9 vertices, int32 indices
    h = 1.0 / nx
    gen = torch.Generator(device="cuda")
    gen.manual_seed(mg.BASE_SEED + 901)
    coords = torch.empty((n_vert, 2), dtype=torch.float64, device="cuda")
    chunk = 1 << 27
    for s in range(0, n_vert, chunk):
        v = torch.arange(s, min(s + chunk, n_vert), dtype=torch.int64, device="cuda")
        coords[s:s + v.numel(), 0] = (v // nvy).double() * h
        coords[s:s + v.numel(), 1] = (v % nvy).double() * h
        del v
    conn = _grid_connectivity(nx, ny, n)
    rule = mg.RULE_TRI3
    u = _uniform((3, n), -1.0, 1.0, gen)
    cf = _uniform((1, 3, n), 0.5, 2.0, gen)
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    R = api.fem_integrate_residual_mesh(2, mg.LAPLACE, rule, coords, conn, u, cf, counts=counts)
    torch.cuda.synchronize()
    assert int(counts[0]) == 0
    cols = _samples(n, np.random.default_rng(4))
    ci = torch.from_numpy(cols).to("cuda")
    got = R[:, ci].cpu().numpy()
    conn_s = conn[ci].cpu().numpy().astype(np.int64)
    x_s = coords[torch.from_numpy(conn_s.ravel()).to("cuda")].cpu().numpy()
    u_s, cf_s = u[:, ci].cpu().double().numpy(), cf[:, :, ci].cpu().double().numpy()
    del R, u, cf, conn, coords
    torch.cuda.empty_cache()
    # the sampled elements as a disconnected mesh of their own
    local = np.arange(3 * cols.size, dtype=np.int32).reshape(-1, 3)
    ref, nd = oracle.residual(2, mg.LAPLACE, rule, x_s, local, u_s, cf_s)
    assert nd == 0
    ij, dj, _ = oracle.geometry(x_s, local)
    ref_abs = oracle.integrate_abs(2, mg.LAPLACE, rule, ij, dj, u_s, cf_s)
    mx, agg = assert_close(got, ref, ref_abs, torch.float32, "fused, 2^31 + 4097 elements")
    print(f"fused mesh, {n} elements: scaled max {mx:.2e} aggregate {agg:.2e}", flush=True)
