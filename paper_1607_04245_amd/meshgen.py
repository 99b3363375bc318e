"""Seeded synthetic inputs for P1 element integration.

This module only builds inputs: jittered structured simplex meshes, random
coefficients at quadrature points, random nodal values and random upstream
weights. It holds none of the integration method's arithmetic (no Jacobians,
no determinants, no tabulation, no quadrature), so that both the FP64 oracle
and the HIP path can be fed from it without sharing any of the method.

The paper benchmarks unstructured meshes of the unit square and unit cube made
by external mesh generators (Section "Benchmarks"); structured grids with
jittered interior vertices stand in for them here.

Random streams: ``SeedSequence(seed).spawn(4)`` gives, in order, the streams
for [vertex jitter, coefficients, nodal values, upstream weights].
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

BASE_SEED = 160704245

# Physics / rule / coefficient-space codes; the numeric values match include/fem.h.
LAPLACE, ELASTICITY, MASS = 0, 1, 2
RULE_TRI3, RULE_TET4, RULE_CENTROID, RULE_TRI6, RULE_TET11 = 0, 1, 2, 3, 4
COEF_QUAD, COEF_P1, COEF_P0 = 0, 1, 2

PHYSICS_NAMES = {LAPLACE: "laplace", ELASTICITY: "elasticity", MASS: "mass"}


def n_comp(dim: int, physics: int) -> int:
    """Field components: 1 for the scalar forms, dim for elasticity."""
    return dim if physics == ELASTICITY else 1


def n_coef(physics: int) -> int:
    """Coefficient fields per quadrature point: kappa, or (lambda, mu)."""
    return 2 if physics == ELASTICITY else 1


def n_qpts(dim: int, rule: int) -> int:
    if rule == RULE_TRI6:
        return 6
    if rule == RULE_TET11:
        return 11
    if rule == RULE_CENTROID:
        return 1
    return dim + 1


def default_rule(dim: int) -> int:
    return RULE_TRI3 if dim == 2 else RULE_TET4


def streams(seed: int):
    """The four independent generators [jitter, coef, u, w]."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------

def _jitter(coords: np.ndarray, interior: np.ndarray, h: float, amount: float,
            rng: np.random.Generator) -> np.ndarray:
    """Move interior vertices by U[-amount*h, amount*h] in each coordinate."""
    d = rng.uniform(-amount * h, amount * h, size=coords.shape)
    return coords + d * interior[:, None]


def tri_grid(n: int, n_elem: int | None = None, rng: np.random.Generator | None = None,
             jitter: float = 0.2):
    """Unit square, n x n cells, two triangles per cell.

    Vertex (i, j) sits at (i/n, j/n) and has index i*(n+1)+j. Cell (i, j),
    i slowest, with corners v00, v10, v01, v11 is split into (v00, v10, v11)
    and (v00, v11, v01); both are counter-clockwise on the undistorted grid.
    The first ``n_elem`` triangles in that order are kept (all if None).
    Returns (coords[N_v, 2] float64, conn[N_e, 3] int32).
    """
    h = 1.0 / n
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    coords = np.stack([i.ravel() * h, j.ravel() * h], axis=1).astype(np.float64)
    interior = ((i > 0) & (i < n) & (j > 0) & (j < n)).ravel().astype(np.float64)
    if rng is not None and jitter > 0:
        coords = _jitter(coords, interior, h, jitter, rng)
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    v00 = ci * (n + 1) + cj
    v10 = (ci + 1) * (n + 1) + cj
    v01 = ci * (n + 1) + cj + 1
    v11 = (ci + 1) * (n + 1) + cj + 1
    t0 = np.stack([v00, v10, v11], axis=1)
    t1 = np.stack([v00, v11, v01], axis=1)
    conn = np.stack([t0, t1], axis=1).reshape(-1, 3)
    if n_elem is not None:
        if n_elem > conn.shape[0]:
            raise ValueError(f"grid {n}^2 has only {conn.shape[0]} triangles, asked {n_elem}")
        conn = conn[:n_elem]
    return coords, np.ascontiguousarray(conn, dtype=np.int32)


# Axis permutations in lexicographic order, with their parity (+1 even, -1 odd).
_PERMS = [(p, (1 if sum(1 for a, b in itertools.combinations(p, 2) if a > b) % 2 == 0 else -1))
          for p in itertools.permutations(range(3))]


def tet_grid(n: int, n_elem: int | None = None, rng: np.random.Generator | None = None,
             jitter: float = 0.2):
    """Unit cube, n^3 cells, six tetrahedra per cell (Kuhn split).

    Vertex (i, j, k) sits at (i/n, j/n, k/n) and has index ((i*(n+1))+j)*(n+1)+k.
    Cell (i, j, k), i slowest. For each axis permutation p in lexicographic
    order, the tetrahedron is the path v000, v000+e_p0, v000+e_p0+e_p1, v111.
    Its orientation on the undistorted grid is the parity of p, so for odd p
    the last two vertices are swapped: every tetrahedron is positively oriented
    before jitter. The first ``n_elem`` tetrahedra are kept (all if None).
    Returns (coords[N_v, 3] float64, conn[N_e, 4] int32).
    """
    h = 1.0 / n
    m = n + 1
    i, j, k = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([i.ravel() * h, j.ravel() * h, k.ravel() * h], axis=1).astype(np.float64)
    interior = ((i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)).ravel().astype(np.float64)
    if rng is not None and jitter > 0:
        coords = _jitter(coords, interior, h, jitter, rng)
    n_cells = n ** 3
    n_keep = 6 * n_cells if n_elem is None else n_elem
    if n_keep > 6 * n_cells:
        raise ValueError(f"grid {n}^3 has only {6 * n_cells} tetrahedra, asked {n_keep}")
    cells_needed = -(-n_keep // 6)
    cell = np.arange(cells_needed)
    ci, rem = np.divmod(cell, n * n)
    cj, ck = np.divmod(rem, n)
    base = np.stack([ci, cj, ck], axis=1)

    def vid(off):
        v = base + np.asarray(off)[None, :]
        return (v[:, 0] * m + v[:, 1]) * m + v[:, 2]

    tets = []
    for p, parity in _PERMS:
        e0 = [0, 0, 0]
        e0[p[0]] = 1
        e01 = list(e0)
        e01[p[1]] = 1
        a, b, c, d = vid((0, 0, 0)), vid(e0), vid(e01), vid((1, 1, 1))
        if parity < 0:
            c, d = d, c
        tets.append(np.stack([a, b, c, d], axis=1))
    conn = np.stack(tets, axis=1).reshape(-1, 4)[:n_keep]
    return coords, np.ascontiguousarray(conn, dtype=np.int32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One mesh with its fields, every array in the library's layouts.

    coords   [N_v, dim]              float64
    conn     [N_e, dim+1]            int32
    u_vertex [N_v, N_comp]           float64
    u        [N_b*N_comp, N_e]       float64, closure; row b*N_comp + c
    coef     [N_coef, N_q, N_e]      float64
    w        [N_b*N_comp, N_e]       float64, upstream weights for the adjoint
    """
    name: str
    dim: int
    physics: int
    rule: int
    coords: np.ndarray
    conn: np.ndarray
    u_vertex: np.ndarray
    u: np.ndarray
    coef: np.ndarray
    w: np.ndarray

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_comp(self) -> int:
        return n_comp(self.dim, self.physics)

    @property
    def n_q(self) -> int:
        return n_qpts(self.dim, self.rule)

    def subset(self, n: int) -> "Workload":
        """The first n elements, same vertices."""
        return dataclasses.replace(
            self, name=f"{self.name}[:{n}]", conn=self.conn[:n].copy(),
            u=np.ascontiguousarray(self.u[:, :n]), coef=np.ascontiguousarray(self.coef[:, :, :n]),
            w=np.ascontiguousarray(self.w[:, :n]))


def closure(conn: np.ndarray, u_vertex: np.ndarray) -> np.ndarray:
    """Gather nodal values per element: out[b*N_comp + c, e] = u_vertex[conn[e, b], c]."""
    g = u_vertex[conn]                       # [N_e, N_b, N_comp]
    return np.ascontiguousarray(g.reshape(conn.shape[0], conn.shape[1] * u_vertex.shape[1]).T)


def _draw_fields(dim, physics, rule, conn, n_vert, rngs):
    _, r_coef, r_u, r_w = rngs
    ne = conn.shape[0]
    nq = n_qpts(dim, rule)
    nc = n_comp(dim, physics)
    if physics == ELASTICITY:
        lam = r_coef.uniform(1.0, 10.0, size=(nq, ne))
        mu = r_coef.uniform(0.5, 5.0, size=(nq, ne))
        coef = np.stack([lam, mu], axis=0)
        u_vertex = r_u.uniform(-1e-2, 1e-2, size=(n_vert, nc))
    else:
        coef = r_coef.uniform(0.5, 2.0, size=(1, nq, ne))
        u_vertex = r_u.uniform(-1.0, 1.0, size=(n_vert, nc))
    w = r_w.uniform(-1.0, 1.0, size=((dim + 1) * nc, ne))
    return np.ascontiguousarray(coef), u_vertex, np.ascontiguousarray(w)


def _coef_draw(physics, rng, shape):
    if physics == ELASTICITY:
        return np.stack([rng.uniform(1.0, 10.0, size=shape), rng.uniform(0.5, 5.0, size=shape)], axis=0)
    return rng.uniform(0.5, 2.0, size=(1,) + shape)


def vertex_coefficients(wl: "Workload", seed: int) -> np.ndarray:
    """The vertex field behind space_coefficients(wl, COEF_P1, seed):
    [N_v, N_coef] float64, coefficient m of vertex v at [v, m]."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_coef_draw(wl.physics, rng, (wl.n_vert,)).T)


def space_coefficients(wl: "Workload", space: int, seed: int) -> np.ndarray:
    """Coefficients of ``wl`` in another space, [N_coef, N_w, N_e] float64.

    COEF_QUAD returns the workload's own values at the points. COEF_P1 draws a
    vertex field (one value per mesh vertex and coefficient, the distribution
    of the point values) and gathers its closure, so neighbouring elements
    share vertex values as an auxiliary P1 field does. COEF_P0 draws one value
    per cell.
    """
    if space == COEF_QUAD:
        return wl.coef
    if space == COEF_P1:
        vert = vertex_coefficients(wl, seed)                       # [N_v, N_coef]
        return np.ascontiguousarray(np.stack([closure(wl.conn, vert[:, m:m + 1]) for m in range(vert.shape[1])]))
    rng = np.random.default_rng(seed)
    if space == COEF_P0:
        return np.ascontiguousarray(_coef_draw(wl.physics, rng, (1, wl.n_elem)))
    raise ValueError(f"unknown coefficient space {space}")


def make_workload(name: str, dim: int, physics: int, grid_n: int, n_elem: int | None,
                  seed: int, rule: int | None = None, jitter: float = 0.2) -> Workload:
    rngs = streams(seed)
    rule = default_rule(dim) if rule is None else rule
    if dim == 2:
        coords, conn = tri_grid(grid_n, n_elem, rngs[0], jitter)
    elif dim == 3:
        coords, conn = tet_grid(grid_n, n_elem, rngs[0], jitter)
    else:
        raise ValueError("dim must be 2 or 3")
    coef, u_vertex, w = _draw_fields(dim, physics, rule, conn, coords.shape[0], rngs)
    return Workload(name=name, dim=dim, physics=physics, rule=rule, coords=coords, conn=conn,
                    u_vertex=u_vertex, u=closure(conn, u_vertex), coef=coef, w=w)


def smallest_grid(dim: int, n_elem: int) -> int:
    """Smallest n whose n^d grid holds at least n_elem simplices."""
    per = 2 if dim == 2 else 6
    n = max(1, int(math.ceil((n_elem / per) ** (1.0 / dim))))
    while per * n ** dim < n_elem:
        n += 1
    while n > 1 and per * (n - 1) ** dim >= n_elem:
        n -= 1
    return n


# The five benchmark workloads (sizes in elements).
CONFIGS = {
    1: dict(name="laplace2d_8192", dim=2, physics=LAPLACE, grid_n=64, n_elem=8192),
    2: dict(name="laplace3d_2p20", dim=3, physics=LAPLACE, grid_n=64, n_elem=1 << 20),
    "3a": dict(name="elasticity2d_2p22", dim=2, physics=ELASTICITY, grid_n=1449, n_elem=1 << 22),
    "3b": dict(name="elasticity3d_2p21", dim=3, physics=ELASTICITY, grid_n=71, n_elem=1 << 21),
    5: dict(name="laplace3d_2p21_adjoint", dim=3, physics=LAPLACE, grid_n=71, n_elem=1 << 21),
}
_CONFIG_NUMBER = {1: 1, 2: 2, "3a": 3, "3b": 3, 5: 5}


def config(cfg, n_elem: int | None = None) -> Workload:
    """Workload of benchmark configuration ``cfg`` (1, 2, '3a', '3b', 5).

    ``n_elem`` truncates to the first elements of the same mesh and draws.
    """
    c = dict(CONFIGS[cfg])
    seed = BASE_SEED + _CONFIG_NUMBER[cfg] + (100 if cfg == "3b" else 0)
    wl = make_workload(c["name"], c["dim"], c["physics"], c["grid_n"], c["n_elem"], seed)
    if n_elem is not None and n_elem < wl.n_elem:
        wl = wl.subset(n_elem)
    return wl


MESH_TYPES = [(2, LAPLACE), (3, LAPLACE), (2, ELASTICITY), (3, ELASTICITY)]


def batch_sizes(seed: int = BASE_SEED + 4, n_mesh: int = 64, lo: float = 3.0, hi: float = 6.0):
    """Element counts floor(10^U(lo, hi)) of the batched workload."""
    rng = np.random.default_rng(seed)
    return [int(math.floor(10.0 ** x)) for x in rng.uniform(lo, hi, size=n_mesh)]


def batch_workloads(n_mesh: int = 64, lo: float = 3.0, hi: float = 6.0,
                    seed: int = BASE_SEED + 4) -> list[Workload]:
    """Independent meshes of mixed type: mesh m has type MESH_TYPES[m % 4].

    Each mesh is the smallest square/cube grid with enough simplices,
    truncated, with the per-type distributions of the single-mesh workloads.
    Mesh m draws from ``SeedSequence(seed).spawn(n_mesh)[m]``.
    """
    sizes = batch_sizes(seed, n_mesh, lo, hi)
    children = np.random.SeedSequence(seed).spawn(n_mesh)
    out = []
    for m, ne in enumerate(sizes):
        dim, phys = MESH_TYPES[m % 4]
        g = smallest_grid(dim, ne)
        rngs = [np.random.default_rng(s) for s in children[m].spawn(4)]
        rule = default_rule(dim)
        if dim == 2:
            coords, conn = tri_grid(g, ne, rngs[0])
        else:
            coords, conn = tet_grid(g, ne, rngs[0])
        coef, u_vertex, w = _draw_fields(dim, phys, rule, conn, coords.shape[0], rngs)
        out.append(Workload(name=f"batch{m}_{PHYSICS_NAMES[phys]}{dim}d_{ne}", dim=dim,
                            physics=phys, rule=rule, coords=coords, conn=conn,
                            u_vertex=u_vertex, u=closure(conn, u_vertex), coef=coef, w=w))
    return out


# ------------------------------------------------------ second-order inputs --

P2_EDGES = {2: [(0, 1), (0, 2), (1, 2)], 3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}


def p2_connectivity(conn: np.ndarray, n_vert: int):
    """P2 node numbering of a simplex mesh: vertices keep their numbers, each
    edge gets one node n_vert + k (k in order of the sorted vertex pair).
    Returns (conn2 [N_e, N_b] int64 with vertices then lexicographic edges,
    number of nodes)."""
    dim = conn.shape[1] - 1
    ei = np.array([i for i, _ in P2_EDGES[dim]])
    ej = np.array([j for _, j in P2_EDGES[dim]])
    a, b = conn[:, ei].astype(np.int64), conn[:, ej].astype(np.int64)
    key = np.minimum(a, b) * n_vert + np.maximum(a, b)
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    conn2 = np.concatenate([conn.astype(np.int64), n_vert + inv.reshape(key.shape)], axis=1)
    return conn2, n_vert + uniq.size


@dataclasses.dataclass
class P2Inputs:
    """Second-order inputs on the mesh of a Workload (same vertices and
    elements): node field, its closure, coefficients at the rule's points
    and upstream weights.

    conn2  [N_e, N_b] int64, N_b = (d+1)(d+2)/2
    u_node [N_nodes, N_comp]
    u, w   [N_b*N_comp, N_e]   closure rows b*N_comp + c
    coef   [N_coef, N_q, N_e]
    """
    rule: int
    conn2: np.ndarray
    n_nodes: int
    u_node: np.ndarray
    u: np.ndarray
    coef: np.ndarray
    w: np.ndarray


def p2_inputs(wl: "Workload", rule: int, seed: int) -> P2Inputs:
    """P2 inputs with the per-physics distributions of the P1 workloads,
    drawn from ``SeedSequence(seed).spawn(3)`` = [coef, u, w]."""
    r_coef, r_u, r_w = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3)]
    conn2, n_nodes = p2_connectivity(wl.conn, wl.n_vert)
    nc, nq, ne = wl.n_comp, n_qpts(wl.dim, rule), wl.n_elem
    coef = np.ascontiguousarray(_coef_draw(wl.physics, r_coef, (nq, ne)))
    lo, hi = (-1e-2, 1e-2) if wl.physics == ELASTICITY else (-1.0, 1.0)
    u_node = r_u.uniform(lo, hi, size=(n_nodes, nc))
    u = closure(conn2, u_node)
    w = np.ascontiguousarray(r_w.uniform(-1.0, 1.0, size=u.shape))
    return P2Inputs(rule=rule, conn2=conn2, n_nodes=n_nodes, u_node=u_node, u=u, coef=coef, w=w)


@dataclasses.dataclass
class P3Inputs:
    rule: int
    u: np.ndarray          # [N_b * N_comp, N_e] closure rows, N_b = 10 (2D) or 20 (3D)
    coef: np.ndarray       # [N_coef, N_q, N_e] values at the rule's points


def p3_inputs(wl: "Workload", rule: int, seed: int) -> P3Inputs:
    """Third-order inputs with the per-physics distributions of the P1
    workloads, drawn from ``SeedSequence(seed).spawn(2)`` = [coef, u]. The
    closure rows are drawn per element (the integration reads closure rows;
    continuity of the field across elements does not enter it)."""
    r_coef, r_u = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(2)]
    nb = (wl.dim + 1) * (wl.dim + 2) * (wl.dim + 3) // 6
    nq, ne = n_qpts(wl.dim, rule), wl.n_elem
    coef = np.ascontiguousarray(_coef_draw(wl.physics, r_coef, (nq, ne)))
    lo, hi = (-1e-2, 1e-2) if wl.physics == ELASTICITY else (-1.0, 1.0)
    u = np.ascontiguousarray(r_u.uniform(lo, hi, size=(nb * wl.n_comp, ne)))
    return P3Inputs(rule=rule, u=u, coef=coef)
