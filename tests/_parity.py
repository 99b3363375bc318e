"""Shared helpers of the GPU parity tests: inputs on the device, the oracle
on the same (rounded) inputs, and the error measures.

Error measure for a floating-point path (per element e, Euclidean norms over
the element vector):  err_e = |R_gpu,e - R_ref,e| / |R_abs,e|, where R_abs is
the oracle evaluated with |.| on every factor. R_abs bounds every partial sum
of the computation, so err_e measures rounding relative to the magnitudes
actually summed; the plain ratio |dR|/|R| is ill-conditioned when u is nearly
constant on an element. The oracle consumes the device inputs rounded to the
device precision and widened to FP64, so the measure isolates arithmetic
error. Bars: FP32 max err_e <= 1e-5 and aggregate |dR|_F/|R|_F <= 1e-5;
FP64 both <= 1e-12.
"""
import numpy as np
import torch

import oracle

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rounded(a, dtype):
    """a rounded to the device dtype, widened back to float64."""
    return np.asarray(a, dtype=np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def measure(got, ref, ref_abs):
    got = np.asarray(got, dtype=np.float64)
    d = np.linalg.norm(got - ref, axis=0)
    s = np.linalg.norm(ref_abs, axis=0)
    per = d / np.maximum(s, 1e-300)
    agg = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    return float(per.max()) if per.size else 0.0, float(agg)


def assert_close(got, ref, ref_abs, dtype, what=""):
    mx, agg = measure(got, ref, ref_abs)
    tol = TOL[dtype]
    assert np.all(np.isfinite(np.asarray(got))), f"{what}: non-finite output"
    assert mx <= tol and agg <= tol, f"{what}: scaled max {mx:.3e}, aggregate {agg:.3e} > {tol:.0e}"
    return mx, agg


def oracle_reference(wl, dtype, u=None, coef=None, space=0):
    """(R, R_abs, inv_j, det_j) of the oracle on the rounded inputs."""
    u = wl.u if u is None else u
    coef = wl.coef if coef is None else coef
    ij, dj, nd = oracle.geometry(wl.coords, wl.conn)
    assert nd == 0
    ur, cr = rounded(u, dtype), rounded(coef, dtype)
    R = oracle.integrate(wl.dim, wl.physics, wl.rule, ij, dj, ur, cr, space=space)
    Ra = oracle.integrate_abs(wl.dim, wl.physics, wl.rule, ij, dj, ur, cr, space=space)
    return R, Ra, ij, dj


def dcoef_abs(dim, physics, rule, inv_j, det_j, u, w, n_coef, n_w, space=0):
    """Scale of the coefficient adjoint: |w| . R_abs(u; unit coefficient)."""
    n = det_j.shape[0]
    out = np.zeros((n_coef, n_w, n))
    for m in range(n_coef):
        for k in range(n_w):
            unit = np.zeros((n_coef, n_w, n))
            unit[m, k] = 1.0
            Ra = oracle.integrate_abs(dim, physics, rule, inv_j, det_j, u, unit, space=space)
            out[m, k] = np.sum(np.abs(w) * Ra, axis=0)
    return out
