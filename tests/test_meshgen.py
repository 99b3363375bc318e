"""The synthetic workloads: sizes, seeding, orientation and layouts."""
import numpy as np
import pytest

import oracle
from paper_1607_04245_amd import meshgen as mg


@pytest.mark.parametrize("cfg,ne,nv", [(1, 8192, 4225), (2, 1 << 20, 274625),
                                        ("3a", 1 << 22, 2102500), ("3b", 1 << 21, 373248),
                                        (5, 1 << 21, 373248)])
def test_config_sizes_and_orientation(cfg, ne, nv):
    wl = mg.config(cfg)
    assert wl.n_elem == ne and wl.n_vert == nv
    assert wl.conn.dtype == np.int32 and wl.conn.flags.c_contiguous
    assert wl.u.shape == ((wl.dim + 1) * wl.n_comp, ne)
    assert wl.coef.shape == ((2 if wl.physics == mg.ELASTICITY else 1), wl.n_q, ne)
    assert wl.w.shape == wl.u.shape
    # every element positively oriented after jitter (fail loudly, never patch)
    _, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0 and dj.min() > 0


def test_value_ranges():
    lap = mg.config(1)
    assert lap.coef.min() >= 0.5 and lap.coef.max() <= 2.0
    assert np.abs(lap.u_vertex).max() <= 1.0
    el = mg.config("3b", n_elem=4096)
    assert el.coef[0].min() >= 1 and el.coef[0].max() <= 10
    assert el.coef[1].min() >= 0.5 and el.coef[1].max() <= 5
    assert np.abs(el.u_vertex).max() <= 1e-2


def test_jitter_only_interior():
    wl = mg.config(1)
    n = 64
    idx = np.stack(np.unravel_index(np.arange(wl.n_vert), (n + 1, n + 1)), axis=1)
    grid = idx / n
    moved = np.any(wl.coords != grid, axis=1)
    boundary = np.any((idx == 0) | (idx == n), axis=1)
    assert not moved[boundary].any()
    assert moved[~boundary].all()
    assert np.abs(wl.coords - grid).max() <= 0.2 / n + 1e-15


def test_seeded_and_deterministic():
    a, b = mg.config(1), mg.config(1)
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.coef, b.coef)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.w, b.w)


def test_closure_layout():
    wl = mg.config(2, n_elem=100)
    for e in (0, 17, 99):
        for b in range(4):
            assert wl.u[b, e] == wl.u_vertex[wl.conn[e, b], 0]


def test_tet_split_covers_cube():
    coords, conn = mg.tet_grid(3)
    _, dj, nd = oracle.geometry(coords, conn)
    assert nd == 0 and dj.min() > 0
    # six tetrahedra per cell fill the cube exactly: total volume 1
    assert np.sum(dj) / 6.0 == pytest.approx(1.0, rel=1e-14)
    coords, conn = mg.tri_grid(5)
    _, dj, _ = oracle.geometry(coords, conn)
    assert np.sum(dj) / 2.0 == pytest.approx(1.0, rel=1e-14)


def test_smallest_grid():
    for dim in (2, 3):
        for ne in (1, 5, 1000, 12345, 999999):
            n = mg.smallest_grid(dim, ne)
            per = 2 if dim == 2 else 6
            assert per * n ** dim >= ne
            assert n == 1 or per * (n - 1) ** dim < ne


def test_batch_workloads_small():
    meshes = mg.batch_workloads(n_mesh=8, lo=2.0, hi=3.0)
    assert len(meshes) == 8
    for m, wl in enumerate(meshes):
        assert (wl.dim, wl.physics) == mg.MESH_TYPES[m % 4]
        _, dj, nd = oracle.geometry(wl.coords, wl.conn)
        assert nd == 0 and dj.min() > 0
    sizes = mg.batch_sizes()
    assert len(sizes) == 64 and min(sizes) >= 1000 and max(sizes) < 10 ** 6


def test_empty_workload():
    for dim, phys in mg.MESH_TYPES:
        wl = mg.make_workload("empty", dim, phys, 1, 0, mg.BASE_SEED)
        assert wl.n_elem == 0 and wl.u.shape == ((dim + 1) * wl.n_comp, 0)
        assert wl.coef.shape[-1] == 0 and wl.w.shape == wl.u.shape
