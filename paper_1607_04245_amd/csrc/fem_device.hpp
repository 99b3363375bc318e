// fem_device.hpp -- device-side building blocks of libfemq (gfx950).
//
// Element traits, the quadrature rules and P1 tabulation as compile-time
// constants (the paper loads the tabulation once per thread block, Section 3;
// here it is folded into the instruction stream), the pointwise physics
// functors f0/f1 (paper Eq. (1) and Section 6), and the per-element
// arithmetic of the residual and its adjoint.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem.h"
#include "fem_scheme.hpp"

namespace femq {

// Fused multiply-add, written out: the library is compiled with FMA
// contraction off, so every fusion in the element arithmetic is explicit and
// the operation sequence of an element is the same in every kernel.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- traits --

// RULE is a scheme (fem_scheme.hpp): quadrature rule and coefficient space.
template <int DIM, int PHYS, int RULE>
struct Elem {
    static_assert(DIM == 2 || DIM == 3, "dim");
    static constexpr int D = DIM;
    static constexpr int NB = DIM + 1;                              // P1 basis functions
    static constexpr int NC = (PHYS == FEM_ELASTICITY) ? DIM : 1;   // field components
    static constexpr int NBT = NB * NC;                             // closure / element-vector length
    static constexpr int NQ = (rule_of(RULE) == FEM_RULE_CENTROID) ? 1 : DIM + 1;
    static constexpr int SPACE = space_of(RULE);                    // coefficient space
    static constexpr int NW = SPACE == FEM_COEF_QUAD ? NQ : SPACE == FEM_COEF_P1 ? NB : 1;
    static constexpr int NCOEF = (PHYS == FEM_ELASTICITY) ? 2 : 1;
    static constexpr int NCQ = NCOEF * NW;                          // coefficient words per element
    static constexpr int NG = DIM * DIM;                            // inverse-Jacobian words
};

// ------------------------------------------------------- quadrature rules --
// Points are given by barycentric coordinates; point q has the large weight
// at vertex q. Both degree-2 rules have equal weights, which sum to 1/dim!.

template <int DIM, int SCHEME>
struct Rule {
    static constexpr int R = rule_of(SCHEME);
    static constexpr int NQ = (R == FEM_RULE_CENTROID) ? 1 : DIM + 1;
    // weight of every point
    static constexpr double W = (R == FEM_RULE_TRI3)   ? 1.0 / 6.0
                              : (R == FEM_RULE_TET4)   ? 1.0 / 24.0
                              : (DIM == 2)             ? 0.5
                                                       : 1.0 / 6.0;
    // barycentric value of point q at its own vertex, and at the others
    static constexpr double LA = (R == FEM_RULE_TRI3)  ? 2.0 / 3.0
                               : (R == FEM_RULE_TET4)  ? 0.58541019662496845446137605030969143531609
                                                       : 1.0 / (DIM + 1);
    static constexpr double LB = (R == FEM_RULE_TRI3)  ? 1.0 / 6.0
                               : (R == FEM_RULE_TET4)  ? 0.13819660112501051517954131656343618822797
                                                       : 1.0 / (DIM + 1);
    // B[q][b] = phi_b(xi_q): for P1 the basis functions are the barycentric coordinates
    __host__ __device__ static constexpr double B(int q, int b) { return q == b ? LA : LB; }
};

// --------------------------------------------------------------- physics --
// Each functor evaluates f0 (NC values) and f1 (NC x DIM values) at one
// quadrature point from the field value uq[NC], its gradient g[NC][DIM]
// (g[c][i] = d u_c / d x_i) and the coefficients a[NCOEF] at that point.
// All three are linear in the coefficients and symmetric in (u, test), which
// the adjoint relies on.

template <int PHYS> struct Physics;

template <> struct Physics<FEM_LAPLACE> {
    static constexpr bool HAS_F0 = false, HAS_F1 = true, NEEDS_U = false;
    template <int DIM, typename Real>
    __device__ static __forceinline__ void point(const Real* uq, const Real (&g)[1][DIM],
                                                 const Real* a, Real* f0, Real (&f1)[1][DIM]) {
        (void)uq; (void)f0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) f1[0][i] = a[0] * g[0][i];
    }
};

template <> struct Physics<FEM_ELASTICITY> {
    static constexpr bool HAS_F0 = false, HAS_F1 = true, NEEDS_U = false;
    template <int DIM, typename Real>
    __device__ static __forceinline__ void point(const Real* uq, const Real (&g)[DIM][DIM],
                                                 const Real* a, Real* f0, Real (&f1)[DIM][DIM]) {
        (void)uq; (void)f0;
        const Real half = Real(0.5);
        Real tr = Real(0);
#pragma unroll
        for (int i = 0; i < DIM; ++i) tr += g[i][i];
        const Real lam_tr = a[0] * tr;
        const Real two_mu = a[1] + a[1];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const Real eps = half * (g[c][i] + g[i][c]);
                f1[c][i] = c == i ? fmadd(two_mu, eps, lam_tr) : two_mu * eps;
            }
    }
};

template <> struct Physics<FEM_MASS> {
    static constexpr bool HAS_F0 = true, HAS_F1 = false, NEEDS_U = true;
    template <int DIM, typename Real>
    __device__ static __forceinline__ void point(const Real* uq, const Real (&g)[1][DIM],
                                                 const Real* a, Real* f0, Real (&f1)[1][DIM]) {
        (void)g; (void)f1;
        f0[0] = a[0] * uq[0];
    }
};

// ------------------------------------------------- per-element arithmetic --
// Inputs of one element:
//   ij[k*DIM+i] = d xi_k / d x_i, dj = det J, u[b*NC+c], cf[m*NQ+q]
// Output: r[b*NC+c].
//
// P1 on an affine element: the reference gradients of the basis are
// constant (grad phi_0 = -1, grad phi_k = e_k), so D^T u is a difference of
// nodal values and grad u is the same at every quadrature point; the basis
// gradients G_b = J^{-T} grad phi_b do not depend on q either, so
//   sum_q G_b . (w_q |J| f1_q) = G_b . F,  F = sum_q w_q |J| f1_q,
// and F is pulled back to reference coordinates once (Fh = J^{-1} F) before
// the D^T contraction. f0/f1 are still evaluated at every quadrature point.

// Coefficient m at quadrature point q from the element's coefficient words
// cf[m*NW + k] in their space: the value at the point, the P1 interpolant
// sum_b phi_b(xi_q) a_b, or the cell value.
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ Real coef_at(const Real* cf, int m, int q) {
    using E = Elem<DIM, PHYS, RULE>;
    using Q = Rule<DIM, RULE>;
    if constexpr (E::SPACE == FEM_COEF_QUAD) {
        return cf[m * E::NW + q];
    } else if constexpr (E::SPACE == FEM_COEF_P1) {
        Real v = Real(Q::B(q, 0)) * cf[m * E::NW];
#pragma unroll
        for (int b = 1; b < E::NB; ++b) v = fmadd(Real(Q::B(q, b)), cf[m * E::NW + b], v);
        return v;
    } else {
        return cf[m];
    }
}

template <int DIM, int NC, typename Real>
__device__ __forceinline__ void physical_gradient(const Real* ij, const Real* u, Real (&g)[NC][DIM]) {
    // reference gradient gh[c][k] = u_{k+1,c} - u_{0,c}; then g = J^{-T} gh
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Real gh[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gh[k] = u[(k + 1) * NC + c] - u[c];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            Real s = ij[0 * DIM + i] * gh[0];
#pragma unroll
            for (int k = 1; k < DIM; ++k) s = fmadd(ij[k * DIM + i], gh[k], s);
            g[c][i] = s;
        }
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void element_residual(const Real* ij, Real dj, const Real* u,
                                                 const Real* cf, Real* r) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    constexpr int NC = E::NC, NB = E::NB, NQ = E::NQ;

    Real g[NC][DIM];
    physical_gradient<DIM, NC>(ij, u, g);
    const Real s = Real(Q::W) * fabs(dj);  // w_q |det J| (equal weights)

    Real F[NC][DIM];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < DIM; ++i) F[c][i] = Real(0);
#pragma unroll
    for (int b = 0; b < NB * NC; ++b) r[b] = Real(0);

    // quadrature phase: pointwise physics at every point, weighted
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Real uq[NC];
        if constexpr (P::NEEDS_U) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Real v = Real(Q::B(q, 0)) * u[c];
#pragma unroll
                for (int b = 1; b < NB; ++b) v = fmadd(Real(Q::B(q, b)), u[b * NC + c], v);
                uq[c] = v;
            }
        }
        Real a[E::NCOEF];
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) a[m] = coef_at<DIM, PHYS, RULE, Real>(cf, m, q);
        Real f0[NC], f1[NC][DIM];
        P::template point<DIM, Real>(uq, g, a, f0, f1);
        if constexpr (P::HAS_F1) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < DIM; ++i) F[c][i] = fmadd(s, f1[c][i], F[c][i]);
        }
        if constexpr (P::HAS_F0) {
            // B^T W f0: phi_b(xi_q) times the weighted f0
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const Real t = s * f0[c];
#pragma unroll
                for (int b = 0; b < NB; ++b) r[b * NC + c] = fmadd(Real(Q::B(q, b)), t, r[b * NC + c]);
            }
        }
    }

    // basis phase: D^T (J^{-T})^T F = grad(phi_b) . Fh with Fh = J^{-1} F
    if constexpr (P::HAS_F1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Real sum = Real(0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                Real fh = ij[k * DIM + 0] * F[c][0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) fh = fmadd(ij[k * DIM + i], F[c][i], fh);
                r[(k + 1) * NC + c] += fh;
                sum += fh;
            }
            r[c] -= sum;
        }
    }
}

// Adjoint of L = w . R for one element. du = R(w) (symmetric forms); the
// derivative with respect to coefficient m at point q is
// w_q |J| [ w^q . f0(e_m) + grad w : f1(e_m) ] with f0/f1 evaluated at unit
// coefficient e_m (the forms are linear in coefficients); it is stored as is
// (points), or summed onto the nodal values with weights phi_b(xi_q) (P1),
// or onto the cell value (P0), by the chain rule.
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void element_dcoef(const Real* ij, Real dj, const Real* u,
                                              const Real* w, Real* dcf) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    constexpr int NC = E::NC, NB = E::NB, NQ = E::NQ;

    Real gu[NC][DIM], gw[NC][DIM];
    if constexpr (P::HAS_F1) {
        physical_gradient<DIM, NC>(ij, u, gu);
        physical_gradient<DIM, NC>(ij, w, gw);
    }
    const Real s = Real(Q::W) * fabs(dj);
#pragma unroll
    for (int k = 0; k < E::NCQ; ++k) dcf[k] = Real(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Real uq[NC], wq[NC];
        if constexpr (P::NEEDS_U) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Real vu = Real(Q::B(q, 0)) * u[c];
                Real vw = Real(Q::B(q, 0)) * w[c];
#pragma unroll
                for (int b = 1; b < NB; ++b) {
                    vu = fmadd(Real(Q::B(q, b)), u[b * NC + c], vu);
                    vw = fmadd(Real(Q::B(q, b)), w[b * NC + c], vw);
                }
                uq[c] = vu;
                wq[c] = vw;
            }
        }
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) {
            Real a[E::NCOEF];
#pragma unroll
            for (int mm = 0; mm < E::NCOEF; ++mm) a[mm] = Real(mm == m ? 1 : 0);
            Real f0[NC], f1[NC][DIM];
            P::template point<DIM, Real>(uq, gu, a, f0, f1);
            Real acc = Real(0);
            if constexpr (P::HAS_F0) {
#pragma unroll
                for (int c = 0; c < NC; ++c) acc = fmadd(wq[c], f0[c], acc);
            }
            if constexpr (P::HAS_F1) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int i = 0; i < DIM; ++i) acc = fmadd(gw[c][i], f1[c][i], acc);
            }
            const Real dq = s * acc;
            if constexpr (E::SPACE == FEM_COEF_QUAD) {
                dcf[m * E::NW + q] = dq;
            } else if constexpr (E::SPACE == FEM_COEF_P1) {
#pragma unroll
                for (int b = 0; b < NB; ++b) dcf[m * E::NW + b] = fmadd(Real(Q::B(q, b)), dq, dcf[m * E::NW + b]);
            } else {
                dcf[m] += dq;
            }
        }
    }
}

// ---------------------------------------------------------------- geometry --
// Affine geometry of one element in FP64: J[i][k] = (x_k - x_0)_i, det J, and
// inv[k][i] = (J^{-1})[k][i] = d xi_k / d x_i. Shared by the geometry kernel
// and the fused mesh kernel, so both produce the same bits.

// Poor shape: |det J| below this fraction of the product of edge lengths,
// tested on squares (det^2 < 1e-6 prod |J[:,k]|^2) so no square root is taken.
constexpr double kPoorShape2 = 1e-6;

template <int DIM>
__device__ __forceinline__ double element_geometry(const double (&x)[DIM + 1][DIM], double (&inv)[DIM][DIM],
                                                   double& edge_product2) {
    double J[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int k = 0; k < DIM; ++k) J[i][k] = x[k + 1][i] - x[0][i];
    double det;
    if constexpr (DIM == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double r = 1.0 / det;
        inv[0][0] = J[1][1] * r;
        inv[0][1] = -J[0][1] * r;
        inv[1][0] = -J[1][0] * r;
        inv[1][1] = J[0][0] * r;
    } else {
        // cofactors C[i][k]; J^{-1}[k][i] = C[i][k] / det
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        const double r = 1.0 / det;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i) inv[k][i] = C[i][k] * r;
    }
    double len2 = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) s += J[i][k] * J[i][k];
        len2 *= s;
    }
    edge_product2 = len2;
    return det;
}

// Loads the dim+1 vertex indices of element e (one 16-byte load for
// tetrahedra when the array is 16-byte aligned). Validation is a separate
// step (conn_ok) so that a caller can issue further loads before it needs
// the indices: testing them right after the load would make the wave wait
// for every load it has in flight.
template <int DIM, bool VEC_CONN>
__device__ __forceinline__ void load_conn(const int32_t* __restrict__ conn, int64_t e, int32_t (&v)[DIM + 1]) {
    if constexpr (VEC_CONN && DIM == 3) {
        typedef int32_t I4 __attribute__((ext_vector_type(4)));
        const I4 c = __builtin_nontemporal_load(reinterpret_cast<const I4*>(conn + e * 4));
        v[0] = c[0]; v[1] = c[1]; v[2] = c[2]; v[3] = c[3];
    } else {
#pragma unroll
        for (int b = 0; b <= DIM; ++b) v[b] = __builtin_nontemporal_load(conn + e * (DIM + 1) + b);
    }
}

// Whether all vertex indices lie in [0, nv). Bitwise, not short-circuit, so
// that it compiles to compares and no branches.
template <int DIM>
__device__ __forceinline__ bool conn_ok(const int32_t (&v)[DIM + 1], int64_t nv) {
    bool ok = true;
#pragma unroll
    for (int b = 0; b <= DIM; ++b) ok &= (v[b] >= 0) & ((int64_t)v[b] < nv);
    return ok;
}

// Gathers the vertex coordinates. Indices are clamped into [0, nv), so an
// element with a bad index (flagged degenerate by the caller) never reads
// outside the array; the clamp is branch-free, which keeps all the gathers of
// an element together in the instruction stream. (Wider loads, e.g. a
// 16-byte pair plus one word per FP64 vertex, measured no faster.)
// Largest valid vertex index as an int32 (connectivity indices are int32, so
// vertices past INT32_MAX are unreachable anyway).
__device__ __forceinline__ int32_t vertex_hi(int64_t nv) {
    return nv - 1 > (int64_t)INT32_MAX ? INT32_MAX : (int32_t)(nv - 1);
}

template <int DIM>
__device__ __forceinline__ void gather_coords(const double* __restrict__ X, const int32_t (&v)[DIM + 1], int64_t nv,
                                              double (&x)[DIM + 1][DIM]) {
    const int32_t hi = vertex_hi(nv);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        const int64_t vi = (int64_t)min(max(v[b], 0), hi);
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[b][i] = X[vi * DIM + i];
    }
}

// Classifies the element and replaces the geometry of a degenerate one by NaN.
// Returns 1 for degenerate, 2 for poorly shaped, 0 otherwise.
template <int DIM>
// Selects only (no branches), so a caller's arithmetic is never moved into a
// conditional block.
__device__ __forceinline__ int finish_geometry(bool ok, double& det, double (&inv)[DIM][DIM], double edge_product2) {
    const bool degenerate = !ok | (det == 0.0) | !isfinite(det);
    const double nan = __builtin_nan("");
    det = ok ? det : nan;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i < DIM; ++i) inv[k][i] = degenerate ? nan : inv[k][i];
    const bool poor = det * det < kPoorShape2 * edge_product2;
    return degenerate ? 1 : (poor ? 2 : 0);
}

// Geometry of one element from its vertices, classified, and stored (rounded
// once to the output type) when valid: the epilogue of every kernel that
// writes the geometry alone.
template <int DIM, typename Out>
__device__ __forceinline__ void geometry_finish(bool valid, int64_t e, int64_t n, bool ok,
                                                const double (&x)[DIM + 1][DIM], Out* __restrict__ inv_j,
                                                Out* __restrict__ det_j, int& ndeg, int& npoor) {
    double inv[DIM][DIM], ep2;
    double det = element_geometry<DIM>(x, inv, ep2);
    const int flag = finish_geometry<DIM>(ok, det, inv, ep2);
    ndeg += (int)(valid & (flag == 1));
    npoor += (int)(valid & (flag == 2));
    if (valid) {
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int i = 0; i < DIM; ++i)
                __builtin_nontemporal_store(static_cast<Out>(inv[k][i]), inv_j + (int64_t)(k * DIM + i) * n + e);
        __builtin_nontemporal_store(static_cast<Out>(det), det_j + e);
    }
}

// XCD-aware work split for kernels that gather vertices. Workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2; numbering the
// workgroups so that XCD k holds a contiguous run of logical indices, and
// giving each logical workgroup a contiguous range of element tiles, keeps
// the vertices an XCD gathers in a compact slice of the mesh, which fits its
// L2 instead of spilling to the shared last-level cache.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t g) {
    const int64_t per = (g + kXcds - 1) / kXcds;  // logical blocks of the fuller XCDs
    const int64_t rem = g % kXcds;                // XCDs holding `per` blocks (all, if 0)
    const int64_t xcd = b % kXcds, slot = b / kXcds;
    const int64_t start = (rem == 0 || xcd < rem) ? xcd * per : rem * per + (xcd - rem) * (per - 1);
    return start + slot;
}

// The wave-tile range [begin, end) of this workgroup; its waves take tiles
// begin + wave, begin + wave + waves_per_block, ...
__device__ __forceinline__ void block_tile_range(int64_t n_tiles, int64_t& begin, int64_t& end) {
    const int64_t L = xcd_logical_block(blockIdx.x, gridDim.x);
    begin = L * n_tiles / gridDim.x;
    end = (L + 1) * n_tiles / gridDim.x;
}

// Adds per-wave sums of the two counters (every lane of the wave active).
__device__ __forceinline__ void add_counts(int32_t* counts, int ndeg, int npoor) {
    if (counts == nullptr) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ndeg += __shfl_xor(ndeg, off, 64);
        npoor += __shfl_xor(npoor, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (ndeg) atomicAdd(&counts[0], ndeg);
        if (npoor) atomicAdd(&counts[1], npoor);
    }
}

// --------------------------------------------------- vector memory access --

template <typename Real, int V> struct VecT;
template <> struct VecT<float, 1> { typedef float T; };
template <> struct VecT<float, 2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct VecT<float, 4> { typedef float T __attribute__((ext_vector_type(4))); };
template <> struct VecT<double, 1> { typedef double T; };
template <> struct VecT<double, 2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct VecT<double, 4> { typedef double T __attribute__((ext_vector_type(4))); };

// Load V consecutive elements of one SoA row (p must be aligned to V words).
template <typename Real, int V>
__device__ __forceinline__ void ld_row(const Real* __restrict__ p, Real (&out)[V]) {
    typedef typename VecT<Real, V>::T T;
    const T x = __builtin_nontemporal_load(reinterpret_cast<const T*>(p));
    if constexpr (V == 1) {
        out[0] = x;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = x[v];
    }
}

template <typename Real, int V>
__device__ __forceinline__ void st_row(Real* __restrict__ p, const Real (&in)[V]) {
    typedef typename VecT<Real, V>::T T;
    T x;
    if constexpr (V == 1) {
        x = in[0];
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = in[v];
    }
    __builtin_nontemporal_store(x, reinterpret_cast<T*>(p));
}

}  // namespace femq
