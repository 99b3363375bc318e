"""Python binding of the libfemq C ABI (include/fem.h): argument marshalling.

The ``fem_*`` functions mirror the C entry points one to one and take torch
tensors on the GPU; every step of the computation runs in the HIP library on
the current torch stream. Output tensors may be passed in (no allocation) or
are allocated with torch (plumbing only).
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _native as N
from .meshgen import ELASTICITY

_DT = {torch.float32: N.F32, torch.float64: N.F64}
_TORCH_DT = {N.F32: torch.float32, N.F64: torch.float64}


def n_comp(dim: int, physics: int) -> int:
    return dim if physics == ELASTICITY else 1


def n_coef(physics: int) -> int:
    return 2 if physics == ELASTICITY else 1


def n_qpts(dim: int, rule: int) -> int:
    return {2: 1, 3: 6, 4: 11}.get(rule, dim + 1)


def n_basis(dim: int, order: int = 1) -> int:
    """Lagrange nodes per element: d+1 (P1), (d+1)(d+2)/2 (P2) or
    (d+1)(d+2)(d+3)/6 (P3)."""
    if order not in (1, 2, 3):
        raise ValueError(f"no Lagrange elements of order {order}")
    return math.comb(dim + order, order)


def n_coef_words(dim: int, rule: int, coef_space: int = N.COEF_QUAD) -> int:
    """Words per coefficient and element: N_q values at the points, the
    N_b = d+1 vertex values of a P1 field, or one cell value (Section 4)."""
    if coef_space == N.COEF_QUAD:
        return n_qpts(dim, rule)
    if coef_space == N.COEF_P1:
        return dim + 1
    if coef_space == N.COEF_P0:
        return 1
    raise ValueError(f"unknown coefficient space {coef_space}")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (libfemq has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _checked_counts(counts, check, device):
    """The counter array to pass: the caller's, or a zeroed one when checking."""
    if counts is None and check:
        counts = torch.zeros(2, dtype=torch.int32, device=device)
    return counts


def _raise_if_degenerate(counts, base, what):
    """Synchronizes on the counters and raises for degenerate elements
    counted by this call (``base``: the count before it)."""
    nd = int(counts[0]) - base
    if nd:
        raise N.FemError(N.FEM_ERR_DEGENERATE, f"{what}: {nd} degenerate element(s) (det J = 0, non-finite, "
                                               f"or a vertex index out of range)")


def fem_geometry(coords: torch.Tensor, conn: torch.Tensor, dtype=torch.float32, inv_j=None, det_j=None,
                 counts=None, *, check=False):
    """(inv_j [d*d, n], det_j [n]) from coords [n_vert, d] float64 and conn [n, d+1] int32.

    ``counts`` (int32 [2] on the GPU, added to) receives the number of
    degenerate and of poorly shaped elements. ``check=True`` synchronizes
    after the launch and raises FemError(FEM_ERR_DEGENERATE) if any element
    is degenerate (the unchecked call never synchronizes).
    """
    _need(coords, "coords", torch.float64)
    dim = coords.shape[1]
    _need(conn, "conn", torch.int32)
    if conn.dim() != 2 or conn.shape[1] != dim + 1:
        raise ValueError(f"conn must be [n_elem, {dim + 1}]")
    n = conn.shape[0]
    if inv_j is None:
        inv_j = torch.empty((dim * dim, n), dtype=dtype, device=coords.device)
    if det_j is None:
        det_j = torch.empty((n,), dtype=dtype, device=coords.device)
    _need(inv_j, "inv_j", dtype, (dim * dim, n))
    _need(det_j, "det_j", dtype, (n,))
    base = int(counts[0]) if (check and counts is not None) else 0
    counts = _checked_counts(counts, check, coords.device)
    if counts is not None:
        _need(counts, "counts", torch.int32, (2,))
    N.check(N.lib().fem_geometry(dim, n, coords.shape[0], _ptr(coords), _ptr(conn), _DT[dtype], _ptr(inv_j),
                                 _ptr(det_j), _ptr(counts), _stream()), "fem_geometry")
    if check:
        _raise_if_degenerate(counts, base, "fem_geometry")
    return inv_j, det_j


def _shapes(dim, physics, rule, n, coef_space=N.COEF_QUAD, order=1):
    nbt = n_basis(dim, order) * n_comp(dim, physics)
    return (dim * dim, n), (n,), (nbt, n), (n_coef(physics), n_coef_words(dim, rule, coef_space), n)


def fem_integrate_residual(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, out=None, *,
                           coef_space=N.COEF_QUAD):
    """Element residuals R [N_bt, n] (paper Eq. (2), before assembly).

    coef is [N_coef, N_w, n] with N_w given by ``coef_space`` (n_coef_words)."""
    dtype = det_j.dtype
    if dtype not in _DT:
        raise TypeError("geometry must be float32 or float64")
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(u, "u", dtype, su)
    _need(coef, "coef", dtype, scf)
    if out is None:
        out = torch.empty(su, dtype=dtype, device=u.device)
    _need(out, "out", dtype, su)
    N.check(N.lib().fem_integrate_residual(dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j), _ptr(u),
                                           _ptr(coef), _ptr(out), _stream()), "fem_integrate_residual")
    return out


def fem_integrate_residual_mesh(dim: int, physics: int, rule: int, coords, conn, u, coef, out=None,
                                inv_j=None, det_j=None, counts=None, *, coef_space=N.COEF_QUAD, check=False):
    """Element residuals straight from coordinates and connectivity (geometry
    fused into the integration; bitwise equal to fem_geometry followed by
    fem_integrate_residual). Pass inv_j and det_j to also receive the geometry."""
    dtype = u.dtype
    if dtype not in _DT:
        raise TypeError("u must be float32 or float64")
    _need(coords, "coords", torch.float64)
    _need(conn, "conn", torch.int32)
    if coords.dim() != 2 or coords.shape[1] != dim or conn.dim() != 2 or conn.shape[1] != dim + 1:
        raise ValueError(f"coords must be [n_vert, {dim}] and conn [n_elem, {dim + 1}]")
    n = conn.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space)
    _need(u, "u", dtype, su)
    _need(coef, "coef", dtype, scf)
    if out is None:
        out = torch.empty(su, dtype=dtype, device=u.device)
    _need(out, "out", dtype, su)
    if (inv_j is None) != (det_j is None):
        raise ValueError("pass both inv_j and det_j, or neither")
    if inv_j is not None:
        _need(inv_j, "inv_j", dtype, sij)
        _need(det_j, "det_j", dtype, sdj)
    base = int(counts[0]) if (check and counts is not None) else 0
    counts = _checked_counts(counts, check, u.device)
    if counts is not None:
        _need(counts, "counts", torch.int32, (2,))
    N.check(N.lib().fem_integrate_residual_mesh(dim, physics, rule, coef_space, _DT[dtype], n, coords.shape[0], _ptr(coords),
                                                _ptr(conn), _ptr(u), _ptr(coef), _ptr(out), _ptr(inv_j),
                                                _ptr(det_j), _ptr(counts), _stream()),
            "fem_integrate_residual_mesh")
    if check:
        _raise_if_degenerate(counts, base, "fem_integrate_residual_mesh")
    return out


def fem_integrate_residual_gather(dim: int, physics: int, rule: int, coords, conn, u_vertex, coef, out=None,
                                  inv_j=None, det_j=None, counts=None, *, coef_space=N.COEF_QUAD, check=False):
    """Element residuals from the mesh with u given per vertex, u_vertex
    [n_vert, N_comp]; the closure is gathered in the kernel. A P1 coefficient
    is given per vertex too, [n_vert, N_coef]; point and cell coefficients
    per element as for fem_integrate_residual. Bitwise equal to
    fem_integrate_residual_mesh on the gathered closures."""
    dtype = u_vertex.dtype
    if dtype not in _DT:
        raise TypeError("u_vertex must be float32 or float64")
    _need(coords, "coords", torch.float64)
    _need(conn, "conn", torch.int32)
    if coords.dim() != 2 or coords.shape[1] != dim or conn.dim() != 2 or conn.shape[1] != dim + 1:
        raise ValueError(f"coords must be [n_vert, {dim}] and conn [n_elem, {dim + 1}]")
    n, nv = conn.shape[0], coords.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space)
    _need(u_vertex, "u_vertex", dtype, (nv, n_comp(dim, physics)))
    _need(coef, "coef", dtype, (nv, n_coef(physics)) if coef_space == N.COEF_P1 else scf)
    if out is None:
        out = torch.empty(su, dtype=dtype, device=u_vertex.device)
    _need(out, "out", dtype, su)
    if (inv_j is None) != (det_j is None):
        raise ValueError("pass both inv_j and det_j, or neither")
    if inv_j is not None:
        _need(inv_j, "inv_j", dtype, sij)
        _need(det_j, "det_j", dtype, sdj)
    base = int(counts[0]) if (check and counts is not None) else 0
    counts = _checked_counts(counts, check, u_vertex.device)
    if counts is not None:
        _need(counts, "counts", torch.int32, (2,))
    N.check(N.lib().fem_integrate_residual_gather(dim, physics, rule, coef_space, _DT[dtype], n, nv, _ptr(coords),
                                                  _ptr(conn), _ptr(u_vertex), _ptr(coef), _ptr(out), _ptr(inv_j),
                                                  _ptr(det_j), _ptr(counts), _stream()),
            "fem_integrate_residual_gather")
    if check:
        _raise_if_degenerate(counts, base, "fem_integrate_residual_gather")
    return out


def fem_integrate_residual_backward(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, w,
                                    want_du=True, want_dcoef=True, du=None, dcoef=None, *, coef_space=N.COEF_QUAD):
    """(du [N_bt, n] or None, dcoef [N_coef, N_w, n] or None) for L = sum w . R."""
    dtype = det_j.dtype
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(w, "w", dtype, su)
    if want_du:
        _need(coef, "coef", dtype, scf)
        if du is None:
            du = torch.empty(su, dtype=dtype, device=w.device)
        _need(du, "du", dtype, su)
    else:
        du = None
    if want_dcoef:
        _need(u, "u", dtype, su)
        if dcoef is None:
            dcoef = torch.empty(scf, dtype=dtype, device=w.device)
        _need(dcoef, "dcoef", dtype, scf)
    else:
        dcoef = None
    N.check(N.lib().fem_integrate_residual_backward(
        dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j), _ptr(u) if want_dcoef else None,
        _ptr(coef) if want_du else None, _ptr(w), _ptr(du), _ptr(dcoef), _stream()),
        "fem_integrate_residual_backward")
    return du, dcoef


def fem_integrate_residual_p2(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, out=None, *,
                              coef_space=N.COEF_QUAD):
    """Element residuals of second-order (P2) elements, R [N_b*N_comp, n] with
    N_b = (d+1)(d+2)/2 (vertices, then edges in lexicographic order), from
    precomputed affine geometry."""
    dtype = det_j.dtype
    if dtype not in _DT:
        raise TypeError("geometry must be float32 or float64")
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space, order=2)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(u, "u", dtype, su)
    _need(coef, "coef", dtype, scf)
    if out is None:
        out = torch.empty(su, dtype=dtype, device=u.device)
    _need(out, "out", dtype, su)
    N.check(N.lib().fem_integrate_residual_p2(dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j),
                                              _ptr(u), _ptr(coef), _ptr(out), _stream()), "fem_integrate_residual_p2")
    return out


def fem_integrate_residual_p3(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, out=None, *,
                              coef_space=N.COEF_QUAD):
    """Element residuals of third-order (P3) elements, R [N_b*N_comp, n] with
    N_b = 10 (2D) or 20 (3D): vertices, two nodes per lexicographic edge
    (the one nearer its first vertex first), then the faces; rule is the
    degree-4 rule of the dimension."""
    dtype = det_j.dtype
    if dtype not in _DT:
        raise TypeError("geometry must be float32 or float64")
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space, order=3)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(u, "u", dtype, su)
    _need(coef, "coef", dtype, scf)
    if out is None:
        out = torch.empty(su, dtype=dtype, device=u.device)
    _need(out, "out", dtype, su)
    N.check(N.lib().fem_integrate_residual_p3(dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j),
                                              _ptr(u), _ptr(coef), _ptr(out), _stream()), "fem_integrate_residual_p3")
    return out


def fem_integrate_residual_p3_backward(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, w,
                                       want_du=True, want_dcoef=True, du=None, dcoef=None, *, coef_space=N.COEF_QUAD):
    """(du, dcoef) of L = sum w.R for P3 elements (see fem_integrate_residual_p3)."""
    dtype = det_j.dtype
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space, order=3)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(w, "w", dtype, su)
    if want_du:
        _need(coef, "coef", dtype, scf)
        du = torch.empty(su, dtype=dtype, device=w.device) if du is None else du
        _need(du, "du", dtype, su)
    else:
        du = None
    if want_dcoef:
        _need(u, "u", dtype, su)
        dcoef = torch.empty(scf, dtype=dtype, device=w.device) if dcoef is None else dcoef
        _need(dcoef, "dcoef", dtype, scf)
    else:
        dcoef = None
    N.check(N.lib().fem_integrate_residual_p3_backward(
        dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j), _ptr(u) if want_dcoef else None,
        _ptr(coef) if want_du else None, _ptr(w), _ptr(du), _ptr(dcoef), _stream()),
        "fem_integrate_residual_p3_backward")
    return du, dcoef


def fem_integrate_jacobian(dim: int, physics: int, rule: int, inv_j, det_j, coef, out=None, *,
                           coef_space=N.COEF_QUAD, order=1):
    """Element matrices K = dR_e/du_e [N_bt*N_bt, n] (row r*N_bt + s: test
    function r = b*N_comp + c, trial function s), for P1 (order 1), P2
    (order 2) or P3 (order 3) elements from precomputed affine geometry. For
    these linear forms K_e u_e is the element residual."""
    dtype = det_j.dtype
    if dtype not in _DT:
        raise TypeError("geometry must be float32 or float64")
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space, order=order)
    smat = (su[0] * su[0], n)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(coef, "coef", dtype, scf)
    if out is None:
        out = torch.empty(smat, dtype=dtype, device=det_j.device)
    _need(out, "out", dtype, smat)
    N.check(N.lib().fem_integrate_jacobian(dim, physics, rule, coef_space, order, _DT[dtype], n, _ptr(inv_j),
                                           _ptr(det_j), _ptr(coef), _ptr(out), _stream()), "fem_integrate_jacobian")
    return out


def fem_integrate_residual_p2_backward(dim: int, physics: int, rule: int, inv_j, det_j, u, coef, w,
                                       want_du=True, want_dcoef=True, du=None, dcoef=None, *, coef_space=N.COEF_QUAD):
    """(du, dcoef) of L = sum w.R for P2 elements (see fem_integrate_residual_p2)."""
    dtype = det_j.dtype
    n = det_j.shape[0]
    sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space, order=2)
    _need(inv_j, "inv_j", dtype, sij)
    _need(det_j, "det_j", dtype, sdj)
    _need(w, "w", dtype, su)
    if want_du:
        _need(coef, "coef", dtype, scf)
        du = torch.empty(su, dtype=dtype, device=w.device) if du is None else du
        _need(du, "du", dtype, su)
    else:
        du = None
    if want_dcoef:
        _need(u, "u", dtype, su)
        dcoef = torch.empty(scf, dtype=dtype, device=w.device) if dcoef is None else dcoef
        _need(dcoef, "dcoef", dtype, scf)
    else:
        dcoef = None
    N.check(N.lib().fem_integrate_residual_p2_backward(
        dim, physics, rule, coef_space, _DT[dtype], n, _ptr(inv_j), _ptr(det_j), _ptr(u) if want_dcoef else None,
        _ptr(coef) if want_du else None, _ptr(w), _ptr(du), _ptr(dcoef), _stream()),
        "fem_integrate_residual_p2_backward")
    return du, dcoef


def fem_stream_copy(src: torch.Tensor, dst: torch.Tensor):
    _need(src, "src")
    _need(dst, "dst")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    N.check(N.lib().fem_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream()), "fem_stream_copy")


def fem_stream_rows(src: torch.Tensor, dst: torch.Tensor):
    """The SoA streaming yardstick: src [n_in, n] and dst [n_out, n] of one
    float dtype; dst[w] = src.sum(0) (in row order) + w."""
    _need(src, "src")
    _need(dst, "dst")
    if src.dim() != 2 or dst.dim() != 2 or src.shape[1] != dst.shape[1] or src.dtype != dst.dtype:
        raise ValueError("src [n_in, n] and dst [n_out, n] of one dtype")
    if src.dtype not in _DT:
        raise TypeError("float32 or float64")
    N.check(N.lib().fem_stream_rows(_DT[src.dtype], src.shape[1], src.shape[0], dst.shape[0], _ptr(src), _ptr(dst),
                                    _stream()), "fem_stream_rows")


# ------------------------------------------------------------------ tuning --

def fem_get_tuning(dim, physics, rule, dtype, op=N.OP_RESIDUAL) -> dict:
    t = N.fem_tuning()
    N.check(N.lib().fem_get_tuning(op, dim, physics, rule, _DT.get(dtype, dtype), ctypes.byref(t)), "fem_get_tuning")
    return dict(strategy=t.strategy, vec=t.vec, waves_per_block=t.waves_per_block, blocks_per_cu=t.blocks_per_cu)


def fem_set_tuning(dim, physics, rule, dtype, strategy=N.STRATEGY_LANE, vec=1, waves_per_block=2,
                   blocks_per_cu=0, op=N.OP_RESIDUAL):
    t = N.fem_tuning(strategy, vec, waves_per_block, blocks_per_cu)
    N.check(N.lib().fem_set_tuning(op, dim, physics, rule, _DT.get(dtype, dtype), ctypes.byref(t)),
            "fem_set_tuning")


def fem_autotune(dim, physics, rule, dtype, n_elem_probe=1 << 20, cache_path=None, op=N.OP_RESIDUAL) -> dict:
    cp = cache_path.encode() if cache_path else None
    N.check(N.lib().fem_autotune(op, dim, physics, rule, _DT.get(dtype, dtype), n_elem_probe, cp), "fem_autotune")
    return fem_get_tuning(dim, physics, rule, dtype, op=op)


def fem_load_tuning(cache_path: str) -> int:
    return N.lib().fem_load_tuning(cache_path.encode())


# ----------------------------------------------------------------- batched --

def _mesh_descs(meshes: list[dict]):
    """Checked descriptor array of a mesh list (see BatchPlan) and its dtype."""
    if not meshes:
        raise ValueError("no meshes")
    dtype = meshes[0]["det_j"].dtype
    descs = (N.fem_mesh_desc * len(meshes))()
    for i, m in enumerate(meshes):
        n = m["det_j"].shape[0]
        space = m.get("coef_space", N.COEF_QUAD)
        sij, sdj, su, scf = _shapes(m["dim"], m["physics"], m["rule"], n, space)
        _need(m["inv_j"], "inv_j", dtype, sij)
        _need(m["det_j"], "det_j", dtype, sdj)
        _need(m["u"], "u", dtype, su)
        _need(m["coef"], "coef", dtype, scf)
        _need(m["out"], "out", dtype, su)
        descs[i] = N.fem_mesh_desc(m["dim"], m["physics"], m["rule"], space, n, m["inv_j"].data_ptr(),
                                   m["det_j"].data_ptr(), m["u"].data_ptr(), m["coef"].data_ptr(),
                                   m["out"].data_ptr())
    return descs, dtype


def batch_run_noalloc(meshes: list[dict], waves_per_block: int = 8, blocks_per_cu: int = 0):
    """The batched launch without a plan and without any device allocation
    (fem_batch_run_noalloc): the descriptor table goes to the library's fixed
    per-GPU array. Mesh dicts as for BatchPlan; at most
    BATCH_NOALLOC_MAX_MESHES meshes. Calls that overlap on one GPU race."""
    descs, dtype = _mesh_descs(meshes)
    N.check(N.lib().fem_batch_run_noalloc(descs, len(meshes), _DT[dtype], waves_per_block, blocks_per_cu,
                                          _stream()), "fem_batch_run_noalloc")


class BatchPlan:
    """Many meshes (mixed dim/physics) integrated by one persistent launch.

    ``meshes`` is a list of dicts with keys dim, physics, rule, inv_j, det_j,
    u, coef and out (torch tensors, one dtype for all), and optionally
    coef_space (default: values at the points). The tensors must stay alive
    while the plan is used.
    """

    def __init__(self, meshes: list[dict]):
        self._plan = ctypes.c_void_p()
        descs, dtype = _mesh_descs(meshes)
        self._keep = list(meshes)
        N.check(N.lib().fem_batch_plan_create(descs, len(meshes), _DT[dtype], ctypes.byref(self._plan)),
                "fem_batch_plan_create")

    def set_launch(self, waves_per_block=8, blocks_per_cu=0):
        N.check(N.lib().fem_batch_plan_set_launch(self._plan, waves_per_block, blocks_per_cu),
                "fem_batch_plan_set_launch")

    def autotune(self) -> dict:
        """Time every launch shape on this plan's meshes (their element
        vectors are written) and keep the fastest; returns it."""
        w, b = ctypes.c_int(), ctypes.c_int()
        N.check(N.lib().fem_batch_plan_autotune(self._plan, _stream(), ctypes.byref(w), ctypes.byref(b)),
                "fem_batch_plan_autotune")
        return dict(waves_per_block=w.value, blocks_per_cu=b.value)

    def run(self):
        N.check(N.lib().fem_batch_run(self._plan, _stream()), "fem_batch_run")

    def capture(self):
        N.check(N.lib().fem_batch_capture(self._plan, _stream()), "fem_batch_capture")

    def replay(self):
        N.check(N.lib().fem_batch_replay(self._plan, _stream()), "fem_batch_replay")

    def close(self):
        if self._plan:
            N.lib().fem_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- assembly --

def fem_restrict(conn, vertex_vec, out=None):
    """Closure of a vertex field: out[b*N_comp + c, e] = vertex_vec[conn[e, b], c]
    (the element restriction, adjoint of assembly)."""
    _need(conn, "conn", torch.int32)
    dtype = vertex_vec.dtype
    if dtype not in _DT:
        raise TypeError("vertex_vec must be float32 or float64")
    if conn.dim() != 2 or conn.shape[1] not in (3, 4) or vertex_vec.dim() != 2:
        raise ValueError("conn must be [n_elem, dim+1] and vertex_vec [n_vert, n_comp]")
    dim, n = conn.shape[1] - 1, conn.shape[0]
    nv, nc = vertex_vec.shape
    _need(vertex_vec, "vertex_vec", dtype)
    if out is None:
        out = torch.empty(((dim + 1) * nc, n), dtype=dtype, device=vertex_vec.device)
    _need(out, "out", dtype, ((dim + 1) * nc, n))
    N.check(N.lib().fem_restrict(dim, nc, _DT[dtype], n, nv, _ptr(conn), _ptr(vertex_vec), _ptr(out), _stream()),
            "fem_restrict")
    return out


class MeshPlan:
    """Distinct vertices of every 64-element tile of a mesh
    (fem_mesh_plan_create), for repeated from-mesh residuals. Building it
    copies the connectivity to the host once and synchronizes the stream.
    It pays on tetrahedral meshes; on triangles the unplanned entry points
    measured faster."""

    def __init__(self, conn: torch.Tensor, n_vert: int):
        _need(conn, "conn", torch.int32)
        if conn.dim() != 2 or conn.shape[1] not in (3, 4):
            raise ValueError("conn must be [n_elem, dim+1]")
        self.dim, self.n_elem, self.n_vert = conn.shape[1] - 1, conn.shape[0], int(n_vert)
        self._plan = ctypes.c_void_p()
        N.check(N.lib().fem_mesh_plan_create(self.dim, self.n_elem, self.n_vert, _ptr(conn), _stream(),
                                             ctypes.byref(self._plan)), "fem_mesh_plan_create")

    def info(self) -> dict:
        d, ne, nv, mx = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        tot = ctypes.c_int64()
        N.check(N.lib().fem_mesh_plan_info(self._plan, ctypes.byref(d), ctypes.byref(ne), ctypes.byref(nv),
                                           ctypes.byref(mx), ctypes.byref(tot)), "fem_mesh_plan_info")
        return dict(dim=d.value, n_elem=ne.value, n_vert=nv.value, max_tile_vertices=mx.value,
                    tile_vertices=tot.value)

    def geometry(self, coords, dtype=torch.float32, inv_j=None, det_j=None, counts=None):
        """fem_geometry through the plan (bitwise the same): (inv_j, det_j)."""
        if dtype not in _DT:
            raise TypeError("dtype must be float32 or float64")
        dim, n = self.dim, self.n_elem
        _need(coords, "coords", torch.float64, (self.n_vert, dim))
        if inv_j is None:
            inv_j = torch.empty((dim * dim, n), dtype=dtype, device=coords.device)
        if det_j is None:
            det_j = torch.empty((n,), dtype=dtype, device=coords.device)
        _need(inv_j, "inv_j", dtype, (dim * dim, n))
        _need(det_j, "det_j", dtype, (n,))
        if counts is not None:
            _need(counts, "counts", torch.int32, (2,))
        N.check(N.lib().fem_geometry_planned(self._plan, _ptr(coords), _DT[dtype], _ptr(inv_j), _ptr(det_j),
                                             _ptr(counts), _stream()), "fem_geometry_planned")
        return inv_j, det_j

    def _run(self, fn, name, physics, rule, coords, u, coef, out, counts, coef_space, per_vertex, inv_j, det_j):
        dtype = u.dtype
        if dtype not in _DT:
            raise TypeError("u must be float32 or float64")
        dim, n = self.dim, self.n_elem
        _need(coords, "coords", torch.float64, (self.n_vert, dim))
        sij, sdj, su, scf = _shapes(dim, physics, rule, n, coef_space)
        if per_vertex:
            _need(u, "u_vertex", dtype, (self.n_vert, n_comp(dim, physics)))
            _need(coef, "coef", dtype, (self.n_vert, n_coef(physics)) if coef_space == N.COEF_P1 else scf)
        else:
            _need(u, "u", dtype, su)
            _need(coef, "coef", dtype, scf)
        if out is None:
            out = torch.empty(su, dtype=dtype, device=u.device)
        _need(out, "out", dtype, su)
        if counts is not None:
            _need(counts, "counts", torch.int32, (2,))
        if (inv_j is None) != (det_j is None):
            raise ValueError("pass both inv_j and det_j, or neither")
        if inv_j is not None:
            _need(inv_j, "inv_j", dtype, sij)
            _need(det_j, "det_j", dtype, sdj)
        N.check(fn(self._plan, physics, rule, coef_space, _DT[dtype], _ptr(coords), _ptr(u), _ptr(coef), _ptr(out),
                   _ptr(inv_j), _ptr(det_j), _ptr(counts), _stream()), name)
        return out

    def integrate(self, physics, rule, coords, u, coef, out=None, counts=None, *, coef_space=N.COEF_QUAD,
                  inv_j=None, det_j=None):
        """fem_integrate_residual_mesh through the plan (bitwise the same)."""
        return self._run(N.lib().fem_integrate_residual_planned, "fem_integrate_residual_planned", physics, rule,
                         coords, u, coef, out, counts, coef_space, False, inv_j, det_j)

    def gather(self, physics, rule, coords, u_vertex, coef, out=None, counts=None, *, coef_space=N.COEF_QUAD,
               inv_j=None, det_j=None):
        """fem_integrate_residual_gather through the plan (bitwise the same)."""
        return self._run(N.lib().fem_integrate_residual_gather_planned, "fem_integrate_residual_gather_planned",
                         physics, rule, coords, u_vertex, coef, out, counts, coef_space, True, inv_j, det_j)

    def close(self):
        if self._plan:
            N.lib().fem_mesh_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AssemblyPlan:
    """Vertex-to-slot index of a mesh for deterministic assembly
    (fem_assembly_plan_create). Building it synchronizes the current stream."""

    def __init__(self, conn: torch.Tensor, n_vert: int):
        _need(conn, "conn", torch.int32)
        if conn.dim() != 2 or conn.shape[1] not in (3, 4):
            raise ValueError("conn must be [n_elem, dim+1]")
        self.dim, self.n_elem, self.n_vert = conn.shape[1] - 1, conn.shape[0], int(n_vert)
        self._plan = ctypes.c_void_p()
        N.check(N.lib().fem_assembly_plan_create(self.dim, self.n_elem, self.n_vert, _ptr(conn), _stream(),
                                                 ctypes.byref(self._plan)), "fem_assembly_plan_create")

    def assemble(self, elem_vec: torch.Tensor, n_comp: int, out=None):
        """Global residual [n_vert, n_comp] = sum_e E_e^T R_e (Section 2)."""
        dtype = elem_vec.dtype
        if dtype not in _DT:
            raise TypeError("elem_vec must be float32 or float64")
        _need(elem_vec, "elem_vec", dtype, ((self.dim + 1) * n_comp, self.n_elem))
        if out is None:
            out = torch.empty((self.n_vert, n_comp), dtype=dtype, device=elem_vec.device)
        _need(out, "out", dtype, (self.n_vert, n_comp))
        N.check(N.lib().fem_assemble(self._plan, n_comp, _DT[dtype], _ptr(elem_vec), _ptr(out), _stream()),
                "fem_assemble")
        return out

    def close(self):
        if self._plan:
            N.lib().fem_assembly_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Assemble(torch.autograd.Function):
    """F = sum_e E_e^T R_e; the gradient with respect to R is the closure of
    the gradient with respect to F."""

    @staticmethod
    def forward(ctx, plan, conn, elem_vec, n_comp):
        ctx.plan, ctx.conn = plan, conn
        return plan.assemble(elem_vec.contiguous(), n_comp)

    @staticmethod
    def backward(ctx, grad_f):
        return None, None, fem_restrict(ctx.conn, grad_f.contiguous()), None


class Restrict(torch.autograd.Function):
    """Closure of a vertex field; the gradient is the assembly of the
    gradient with respect to the closure."""

    @staticmethod
    def forward(ctx, plan, conn, vertex_vec):
        ctx.plan, ctx.n_comp = plan, vertex_vec.shape[1]
        return fem_restrict(conn, vertex_vec.contiguous())

    @staticmethod
    def backward(ctx, grad_e):
        return None, None, ctx.plan.assemble(grad_e.contiguous(), ctx.n_comp)


def assemble(plan, conn, elem_vec, n_comp):
    """Differentiable assembly (see Assemble)."""
    return Assemble.apply(plan, conn, elem_vec, n_comp)


def restrict(plan, conn, vertex_vec):
    """Differentiable restriction (see Restrict)."""
    return Restrict.apply(plan, conn, vertex_vec)


# ---------------------------------------------------------------- autograd --

class IntegrateResidual(torch.autograd.Function):
    """R = integrate(u, coef) with gradients for u and coef from the adjoint
    kernel. Geometry is treated as a constant."""

    @staticmethod
    def forward(ctx, dim, physics, rule, inv_j, det_j, u, coef, coef_space, order):
        ctx.save_for_backward(inv_j, det_j, u, coef)
        ctx.meta = (dim, physics, rule, coef_space, order)
        fwd = {1: fem_integrate_residual, 2: fem_integrate_residual_p2, 3: fem_integrate_residual_p3}[order]
        return fwd(dim, physics, rule, inv_j, det_j, u.contiguous(), coef.contiguous(), coef_space=coef_space)

    @staticmethod
    def backward(ctx, grad_r):
        inv_j, det_j, u, coef = ctx.saved_tensors
        dim, physics, rule, coef_space, order = ctx.meta
        bwd = {1: fem_integrate_residual_backward, 2: fem_integrate_residual_p2_backward,
               3: fem_integrate_residual_p3_backward}[order]
        du, dcoef = bwd(dim, physics, rule, inv_j, det_j, u.contiguous(), coef.contiguous(), grad_r.contiguous(),
                        want_du=ctx.needs_input_grad[5], want_dcoef=ctx.needs_input_grad[6], coef_space=coef_space)
        return None, None, None, None, None, du, dcoef, None, None


def integrate_residual(dim, physics, rule, inv_j, det_j, u, coef, coef_space=N.COEF_QUAD, order=1):
    """Differentiable element residuals (see IntegrateResidual); order 1 (P1), 2 (P2) or 3 (P3)."""
    if order not in (1, 2, 3):
        raise ValueError("order must be 1, 2 or 3")
    return IntegrateResidual.apply(dim, physics, rule, inv_j, det_j, u, coef, coef_space, order)
