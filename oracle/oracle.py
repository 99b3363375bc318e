"""ctypes front end of the FP64 reference integrator (fem_oracle.c).

TEST INFRASTRUCTURE: see the package docstring. Arrays use the library's
structure-of-arrays layouts: inv_j [d*d][n], det_j [n], u/w/R [N_bt][n],
coef [N_coef][N_q][n]; coords [n_vert][d] and conn [n][d+1].
"""
from __future__ import annotations

import ctypes
import math
import os
import pathlib

import numpy as np

_LIB = None
_HERE = pathlib.Path(__file__).resolve().parent

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def load():
    global _LIB
    if _LIB is None:
        # FEMQ_ORACLE_LIB names another build of fem_oracle.c (the sanitized
        # one of the test suite); by default the library next to this file
        alt = os.environ.get("FEMQ_ORACLE_LIB")
        path = pathlib.Path(alt) if alt else _HERE / "liboracle.so"
        if not path.exists() and not alt:
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(str(path))
        lib.fem_oracle_n_qpts.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.fem_oracle_n_qpts.restype = ctypes.c_int
        lib.fem_oracle_rule.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        lib.fem_oracle_rule.restype = ctypes.c_int
        lib.fem_oracle_geometry.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _dp, _ip, _dp, _dp]
        lib.fem_oracle_geometry.restype = ctypes.c_int64
        lib.fem_oracle_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.fem_oracle_integrate.restype = ctypes.c_int
        lib.fem_oracle_residual.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int64, ctypes.c_int64, _dp, _ip, _dp, _dp, _dp]
        lib.fem_oracle_residual.restype = ctypes.c_int64
        lib.fem_oracle_backward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.fem_oracle_backward.restype = ctypes.c_int
        lib.fem_oracle_integrate_p.argtypes = [ctypes.c_int] + lib.fem_oracle_integrate.argtypes
        lib.fem_oracle_integrate_p.restype = ctypes.c_int
        lib.fem_oracle_backward_p.argtypes = [ctypes.c_int] + lib.fem_oracle_backward.argtypes
        lib.fem_oracle_backward_p.restype = ctypes.c_int
        lib.fem_oracle_jacobian_p.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.fem_oracle_jacobian_p.restype = ctypes.c_int
        for name in ("fem_oracle_assemble", "fem_oracle_restrict"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _ip, _dp, _dp]
            f.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _ncomp(dim, physics):
    return dim if physics == 1 else 1


def _ncoef(physics):
    return 2 if physics == 1 else 1


def coef_words(dim, rule_id, space):
    """Words of one coefficient field per element: N_q, d+1 (P1) or 1."""
    return {0: n_qpts(dim, rule_id), 1: dim + 1, 2: 1}[space]


def n_basis(dim, order):
    """Lagrange basis functions per element: d+1 (order 1), (d+1)(d+2)/2
    (order 2), (d+1)(d+2)(d+3)/6 (order 3)."""
    if order not in (1, 2, 3):
        raise ValueError(f"no Lagrange elements of order {order}")
    return math.comb(dim + order, order)


def n_qpts(dim: int, rule: int) -> int:
    n = load().fem_oracle_n_qpts(dim, rule)
    if n < 0:
        raise ValueError(f"no rule {rule} in {dim}D")
    return n


def rule(dim: int, rule_id: int):
    """(xi[N_q, dim], weights[N_q]) of a quadrature rule on the unit simplex."""
    nq = n_qpts(dim, rule_id)
    xi = np.zeros((nq, dim))
    w = np.zeros(nq)
    load().fem_oracle_rule(dim, rule_id, _p(xi), _p(w))
    return xi, w


def geometry(coords, conn):
    """(inv_j[d*d, n], det_j[n], n_degenerate) in FP64."""
    coords, conn = _f64(coords), _i32(conn)
    dim = coords.shape[1]
    n = conn.shape[0]
    inv_j = np.zeros((dim * dim, n))
    det_j = np.zeros(n)
    r = load().fem_oracle_geometry(dim, n, coords.shape[0], _p(coords), _p(conn, _ip), _p(inv_j), _p(det_j))
    if r < 0:
        raise ValueError("oracle geometry: bad arguments or vertex index out of range")
    return inv_j, det_j, int(r)


def _integrate(dim, physics, rule_id, inv_j, det_j, u, coef, absmode, space, order):
    inv_j, det_j, u, coef = _f64(inv_j), _f64(det_j), _f64(u), _f64(coef)
    n = det_j.shape[0]
    nb = n_basis(dim, order)
    R = np.zeros((nb * _ncomp(dim, physics), n))
    r = load().fem_oracle_integrate_p(order, dim, physics, rule_id, space, n, _p(inv_j), _p(det_j), _p(u),
                                      _p(coef), _p(R), int(absmode))
    if r != 0:
        raise ValueError("oracle integrate: bad arguments")
    return R


def integrate(dim, physics, rule_id, inv_j, det_j, u, coef, space=0, order=1):
    """Element residuals R[N_bt, n] from precomputed geometry (Eq. (2) bracket).
    ``space``: 0 coefficients on quadrature points, 1 P1 nodal, 2 P0;
    ``order``: 1 (P1), 2 (P2, vertices then edges in lexicographic order) or
    3 (P3: vertices, two nodes per lexicographic edge (i, j), the one nearer
    i first, then the faces (i, j, k) in lexicographic order)."""
    return _integrate(dim, physics, rule_id, inv_j, det_j, u, coef, False, space, order)


def integrate_abs(dim, physics, rule_id, inv_j, det_j, u, coef, space=0, order=1):
    """Same sums with |.| on every factor: the scale of the rounding measure."""
    return _integrate(dim, physics, rule_id, inv_j, det_j, u, coef, True, space, order)


def residual(dim, physics, rule_id, coords, conn, u, coef, space=0):
    """Coordinates/connectivity to residuals R[N_bt, n]; returns (R, n_degenerate)."""
    coords, conn, u, coef = _f64(coords), _i32(conn), _f64(u), _f64(coef)
    n = conn.shape[0]
    R = np.zeros(((dim + 1) * _ncomp(dim, physics), n))
    r = load().fem_oracle_residual(dim, physics, rule_id, space, n, coords.shape[0], _p(coords), _p(conn, _ip),
                                   _p(u), _p(coef), _p(R))
    if r < 0:
        raise ValueError("oracle residual: bad arguments")
    return R, int(r)


def backward(dim, physics, rule_id, inv_j, det_j, u, coef, w, want_du=True, want_dcoef=True, space=0, order=1):
    """Adjoint of L = sum w.R: (du[N_bt, n] or None, dcoef[N_coef, N_w, n] or None)."""
    inv_j, det_j, u, coef, w = _f64(inv_j), _f64(det_j), _f64(u), _f64(coef), _f64(w)
    n = det_j.shape[0]
    nw = coef_words(dim, rule_id, space)
    du = np.zeros((n_basis(dim, order) * _ncomp(dim, physics), n)) if want_du else None
    dcoef = np.zeros((_ncoef(physics), nw, n)) if want_dcoef else None
    r = load().fem_oracle_backward_p(order, dim, physics, rule_id, space, n, _p(inv_j), _p(det_j), _p(u),
                                     _p(coef), _p(w), _p(du), _p(dcoef))
    if r != 0:
        raise ValueError("oracle backward: bad arguments")
    return du, dcoef


def _jacobian(dim, physics, rule_id, inv_j, det_j, coef, absmode, space, order):
    inv_j, det_j, coef = _f64(inv_j), _f64(det_j), _f64(coef)
    n = det_j.shape[0]
    nbt = n_basis(dim, order) * _ncomp(dim, physics)
    K = np.zeros((nbt * nbt, n))
    r = load().fem_oracle_jacobian_p(order, dim, physics, rule_id, space, n, _p(inv_j), _p(det_j), _p(coef),
                                     _p(K), int(absmode))
    if r != 0:
        raise ValueError("oracle jacobian: bad arguments")
    return K


def jacobian(dim, physics, rule_id, inv_j, det_j, coef, space=0, order=1):
    """Element matrices K[N_bt*N_bt, n] = dR_e/du_e (row r*N_bt + s: test
    function r = b*N_comp + c, trial function s), from the pointwise
    derivatives of f0 and f1 (Section 2, Eq. (2) differentiated)."""
    return _jacobian(dim, physics, rule_id, inv_j, det_j, coef, False, space, order)


def jacobian_abs(dim, physics, rule_id, inv_j, det_j, coef, space=0, order=1):
    """Same sums with |.| on every factor: the scale of the rounding measure."""
    return _jacobian(dim, physics, rule_id, inv_j, det_j, coef, True, space, order)


def assemble(dim, n_comp, n_vert, conn, elem_vec):
    """Global residual F[n_vert, n_comp] = sum_e E_e^T R_e (Section 2)."""
    conn, elem_vec = _i32(conn), _f64(elem_vec)
    n = conn.shape[0]
    F = np.zeros((n_vert, n_comp))
    if load().fem_oracle_assemble(dim, n_comp, n, n_vert, _p(conn, _ip), _p(elem_vec), _p(F)) != 0:
        raise ValueError("oracle assemble: bad arguments or vertex index out of range")
    return F


def restrict(dim, n_comp, conn, vert):
    """Closure R[(d+1)*n_comp, n] of a vertex field vert[n_vert, n_comp]."""
    conn, vert = _i32(conn), _f64(vert)
    n = conn.shape[0]
    out = np.zeros(((dim + 1) * n_comp, n))
    if load().fem_oracle_restrict(dim, n_comp, n, vert.shape[0], _p(conn, _ip), _p(vert), _p(out)) != 0:
        raise ValueError("oracle restrict: bad arguments or vertex index out of range")
    return out
