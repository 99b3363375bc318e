// p2_device.hpp -- element arithmetic of second-order (P2) Lagrange
// elements on affine simplices: the quadrature and basis phases of Eq. (2)
// with the P2 basis, evaluated with the barycentric structure of the basis.
//
// Basis (node order: vertices v = 0..d, then edges (i, j), i < j,
// lexicographic): phi_v = lam_v (2 lam_v - 1), phi_ij = 4 lam_i lam_j, with
// lam_0 = 1 - sum xi, lam_k = xi_k. With g_v the physical gradients of the
// barycentric coordinates (g_{k+1} = row k of J^{-1}, g_0 = -sum), the
// gradient of a P2 field is affine in the barycentric coordinates:
//   grad u(x) = sum_w lam_w(x) B_w,   B_w = sum_v (4 U_vw - u_v) g_v,
// U_vv = u_v and U_vw = u on the edge (v, w); so B is formed once per element
// and the gradient at a point costs d+1 multiply-adds per entry. The basis
// phase is its transpose: with the weighted flux F_q = w_q |J| f1(x_q) and
// its moments M_w = sum_q lam_w(x_q) F_q (and M = sum_w M_w = sum_q F_q),
//   r_v = g_v . (4 M_v - M),   r_ij = 4 (g_i . M_j + g_j . M_i),
// so each point only adds d+1 scaled copies of its flux. f0 and f1 are
// still evaluated at every point; the f0 term is summed directly with the
// basis values. The geometry is affine, as for P1, and a P1 coefficient
// keeps its d+1 vertex values and the P1 basis.
#pragma once

#include "fem_device.hpp"

namespace femq {

// Quadrature rules for P2: the degree-2 rules of the P1 path (TRI3, TET4)
// and degree-4 rules (TRI6, TET11), as barycentric coordinates and weights.
template <int DIM, int RULE>
struct RuleP2;

template <>
struct RuleP2<2, FEM_RULE_TRI3> {
    static constexpr int NQ = 3;
    __host__ __device__ static constexpr double lam(int q, int v) { return q == v ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double w(int) { return 1.0 / 6.0; }
};

template <>
struct RuleP2<3, FEM_RULE_TET4> {
    static constexpr int NQ = 4;
    __host__ __device__ static constexpr double lam(int q, int v) {
        return q == v ? 0.58541019662496845446137605030969143531609 : 0.13819660112501051517954131656343618822797;
    }
    __host__ __device__ static constexpr double w(int) { return 1.0 / 24.0; }
};

// Six points in two orbits; point q (and q + 3) has the distinguished value
// at vertex q.
template <>
struct RuleP2<2, FEM_RULE_TRI6> {
    static constexpr int NQ = 6;
    static constexpr double A1 = 0.108103018168070227363341492234, B1 = 0.5 * (1.0 - A1);
    static constexpr double A2 = 0.816847572980458513080857073195, B2 = 0.5 * (1.0 - A2);
    __host__ __device__ static constexpr double lam(int q, int v) {
        return q < 3 ? (q == v ? A1 : B1) : (q - 3 == v ? A2 : B2);
    }
    __host__ __device__ static constexpr double w(int q) {
        return q < 3 ? 0.5 * 0.223381589678011465944710768628 : 0.5 * 0.109951743655321867388622564704;
    }
};

// Eleven points: the centroid (negative weight), four points with 11/14 at
// one vertex, six with (1 + sqrt(5/14))/4 at both vertices of an edge
// (edges lexicographic).
template <>
struct RuleP2<3, FEM_RULE_TET11> {
    static constexpr int NQ = 11;
    static constexpr double A = 0.39940357616679920499610214746996;  // (1 + sqrt(5/14)) / 4
    static constexpr double B = 0.10059642383320079500389785253004;  // (1 - sqrt(5/14)) / 4
    __host__ __device__ static constexpr int edge_i(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
    __host__ __device__ static constexpr int edge_j(int k) { return k < 3 ? k + 1 : (k < 5 ? k - 1 : 3); }
    __host__ __device__ static constexpr double lam(int q, int v) {
        return q == 0 ? 0.25
             : q < 5  ? (q - 1 == v ? 11.0 / 14.0 : 1.0 / 14.0)
                      : ((v == edge_i(q - 5) || v == edge_j(q - 5)) ? A : B);
    }
    __host__ __device__ static constexpr double w(int q) {
        return q == 0 ? -148.0 / 1875.0 / 6.0 : (q < 5 ? 343.0 / 7500.0 / 6.0 : 56.0 / 375.0 / 6.0);
    }
};

template <int DIM, int PHYS, int RULE, int SPACE>
struct ElemP2 {
    static constexpr int D = DIM;
    static constexpr int NV = DIM + 1;                              // vertices
    static constexpr int NE = DIM == 2 ? 3 : 6;                     // edges
    static constexpr int NB = NV + NE;                              // P2 basis functions
    static constexpr int NC = (PHYS == FEM_ELASTICITY) ? DIM : 1;
    static constexpr int NBT = NB * NC;
    static constexpr int NQ = RuleP2<DIM, RULE>::NQ;
    static constexpr int NW = SPACE == FEM_COEF_QUAD ? NQ : SPACE == FEM_COEF_P1 ? NV : 1;
    static constexpr int NCOEF = (PHYS == FEM_ELASTICITY) ? 2 : 1;
    static constexpr int NCQ = NCOEF * NW;
    static constexpr int NG = DIM * DIM;
    // edge k = (ei(k), ej(k)), lexicographic
    __host__ __device__ static constexpr int ei(int k) {
        return DIM == 2 ? (k < 2 ? 0 : 1) : (k < 3 ? 0 : (k < 5 ? 1 : 2));
    }
    __host__ __device__ static constexpr int ej(int k) {
        return DIM == 2 ? (k < 2 ? k + 1 : 2) : (k < 3 ? k + 1 : (k < 5 ? k - 1 : 3));
    }
    // index of the edge joining vertices a != b
    __host__ __device__ static constexpr int edge_of(int a, int b) {
        return DIM == 2 ? ((a < b ? a : b) == 0 ? (a < b ? b : a) - 1 : 2)
                        : ((a < b ? a : b) == 0 ? (a < b ? b : a) - 1
                                                : ((a < b ? a : b) == 1 ? (a < b ? b : a) + 1 : 5));
    }
};

// Coefficient m at point q from the element's words cf[m*NW + k].
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ Real coef_at_p2(const Real* cf, int m, int q) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    if constexpr (SPACE == FEM_COEF_QUAD) {
        return cf[m * E::NW + q];
    } else if constexpr (SPACE == FEM_COEF_P1) {
        Real v = Real(Q::lam(q, 0)) * cf[m * E::NW];
#pragma unroll
        for (int b = 1; b < E::NV; ++b) v = fmadd(Real(Q::lam(q, b)), cf[m * E::NW + b], v);
        return v;
    } else {
        return cf[m];
    }
}

// Physical gradients of the barycentric coordinates: g[k+1] = row k of
// J^{-1}, g[0] = -(g[1] + ... + g[d]).
template <int DIM, typename Real>
__device__ __forceinline__ void p2_bary_grads(const Real* ij, Real (&g)[DIM + 1][DIM]) {
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        Real s = ij[i];
        g[1][i] = ij[i];
#pragma unroll
        for (int k = 1; k < DIM; ++k) {
            g[k + 1][i] = ij[k * DIM + i];
            s += ij[k * DIM + i];
        }
        g[0][i] = -s;
    }
}

// Gradient coefficients of the field u[b*NC + c]: grad u_c(x) =
// sum_w lam_w(x) B[c][w][i].
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void p2_grad_coeffs(const Real* u, const Real (&g)[DIM + 1][DIM],
                                               Real (&B)[ElemP2<DIM, PHYS, RULE, SPACE>::NC][DIM + 1][DIM]) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    constexpr int NC = E::NC, NV = E::NV;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int w = 0; w < NV; ++w) {
            Real d[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const Real U = v == w ? u[v * NC + c] : u[(NV + E::edge_of(v, w)) * NC + c];
                d[v] = fmadd(Real(4), U, -u[v * NC + c]);
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                Real s = d[0] * g[0][i];
#pragma unroll
                for (int v = 1; v < NV; ++v) s = fmadd(d[v], g[v][i], s);
                B[c][w][i] = s;
            }
        }
}

// Physical gradient at point q from the gradient coefficients.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void p2_grad_at(int q, const Real (&B)[ElemP2<DIM, PHYS, RULE, SPACE>::NC][DIM + 1][DIM],
                                           Real (&gq)[ElemP2<DIM, PHYS, RULE, SPACE>::NC][DIM]) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
#pragma unroll
    for (int c = 0; c < E::NC; ++c)
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            Real s = Real(Q::lam(q, 0)) * B[c][0][i];
#pragma unroll
            for (int w = 1; w < E::NV; ++w) s = fmadd(Real(Q::lam(q, w)), B[c][w][i], s);
            gq[c][i] = s;
        }
}

// Value of the field at point q: sum_b phi_b(x_q) u_b.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void p2_value_at(int q, const Real* u, Real (&uq)[ElemP2<DIM, PHYS, RULE, SPACE>::NC]) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    constexpr int NC = E::NC, NV = E::NV;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Real s = Real(Q::lam(q, 0) * (2.0 * Q::lam(q, 0) - 1.0)) * u[c];
#pragma unroll
        for (int v = 1; v < NV; ++v) s = fmadd(Real(Q::lam(q, v) * (2.0 * Q::lam(q, v) - 1.0)), u[v * NC + c], s);
#pragma unroll
        for (int k = 0; k < E::NE; ++k)
            s = fmadd(Real(4.0 * Q::lam(q, E::ei(k)) * Q::lam(q, E::ej(k))), u[(NV + k) * NC + c], s);
        uq[c] = s;
    }
}

// Residual of one P2 element: r[b*NC + c], from invJ ij[k*DIM + i], det J,
// closure u[b*NC + c] and coefficient words cf.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void element_residual_p2(const Real* ij, Real dj, const Real* u, const Real* cf, Real* r) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int NC = E::NC, NV = E::NV;
#pragma unroll
    for (int b = 0; b < E::NBT; ++b) r[b] = Real(0);
    const Real adj = fabs(dj);
    Real g[NV][DIM];
    p2_bary_grads<DIM, Real>(ij, g);
    Real B[NC][NV][DIM];
    if constexpr (P::HAS_F1) p2_grad_coeffs<DIM, PHYS, RULE, SPACE, Real>(u, g, B);
    Real M[NC][NV][DIM];  // flux moments
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int w = 0; w < NV; ++w)
#pragma unroll
            for (int i = 0; i < DIM; ++i) M[c][w][i] = Real(0);
#pragma unroll
    for (int q = 0; q < E::NQ; ++q) {
        Real uq[NC], gq[NC][DIM];
        if constexpr (P::NEEDS_U) p2_value_at<DIM, PHYS, RULE, SPACE, Real>(q, u, uq);
        if constexpr (P::HAS_F1) p2_grad_at<DIM, PHYS, RULE, SPACE, Real>(q, B, gq);
        Real a[E::NCOEF];
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) a[m] = coef_at_p2<DIM, PHYS, RULE, SPACE, Real>(cf, m, q);
        Real f0[NC], f1[NC][DIM];
        P::template point<DIM, Real>(uq, gq, a, f0, f1);
        const Real s = Real(Q::w(q)) * adj;
        if constexpr (P::HAS_F1) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    const Real F = s * f1[c][i];
#pragma unroll
                    for (int w = 0; w < NV; ++w) M[c][w][i] = fmadd(Real(Q::lam(q, w)), F, M[c][w][i]);
                }
        }
        if constexpr (P::HAS_F0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const Real sf = s * f0[c];
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    r[v * NC + c] = fmadd(Real(Q::lam(q, v) * (2.0 * Q::lam(q, v) - 1.0)), sf, r[v * NC + c]);
#pragma unroll
                for (int k = 0; k < E::NE; ++k)
                    r[(NV + k) * NC + c] =
                        fmadd(Real(4.0 * Q::lam(q, E::ei(k)) * Q::lam(q, E::ej(k))), sf, r[(NV + k) * NC + c]);
            }
        }
    }
    if constexpr (P::HAS_F1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Real Mt[DIM];  // sum over the points of the weighted flux
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                Real t = M[c][0][i];
#pragma unroll
                for (int w = 1; w < NV; ++w) t += M[c][w][i];
                Mt[i] = t;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Real t = g[v][0] * fmadd(Real(4), M[c][v][0], -Mt[0]);
#pragma unroll
                for (int i = 1; i < DIM; ++i) t = fmadd(g[v][i], fmadd(Real(4), M[c][v][i], -Mt[i]), t);
                r[v * NC + c] += t;
            }
#pragma unroll
            for (int k = 0; k < E::NE; ++k) {
                const int a = E::ei(k), b = E::ej(k);
                Real t = g[a][0] * M[c][b][0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) t = fmadd(g[a][i], M[c][b][i], t);
#pragma unroll
                for (int i = 0; i < DIM; ++i) t = fmadd(g[b][i], M[c][a][i], t);
                r[(NV + k) * NC + c] += Real(4) * t;
            }
        }
    }
}

// Derivative of L = w . R with respect to the coefficient words (the forms
// are linear in the coefficients): at point q, w_q |J| [w^q . f0(u; e_m) +
// grad w : f1(u; e_m)], mapped onto the coefficient's space.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void element_dcoef_p2(const Real* ij, Real dj, const Real* u, const Real* w, Real* dcf) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int NC = E::NC;
#pragma unroll
    for (int k = 0; k < E::NCQ; ++k) dcf[k] = Real(0);
    const Real adj = fabs(dj);
    constexpr int NV = E::NV;
    Real g[NV][DIM];
    p2_bary_grads<DIM, Real>(ij, g);
    Real Bu[NC][NV][DIM], Bw[NC][NV][DIM];
    if constexpr (P::HAS_F1) {
        p2_grad_coeffs<DIM, PHYS, RULE, SPACE, Real>(u, g, Bu);
        p2_grad_coeffs<DIM, PHYS, RULE, SPACE, Real>(w, g, Bw);
    }
#pragma unroll
    for (int q = 0; q < E::NQ; ++q) {
        Real uq[NC], gu[NC][DIM], wq[NC], gw[NC][DIM];
        if constexpr (P::NEEDS_U) p2_value_at<DIM, PHYS, RULE, SPACE, Real>(q, u, uq);
        if constexpr (P::HAS_F0) p2_value_at<DIM, PHYS, RULE, SPACE, Real>(q, w, wq);
        if constexpr (P::HAS_F1) {
            p2_grad_at<DIM, PHYS, RULE, SPACE, Real>(q, Bu, gu);
            p2_grad_at<DIM, PHYS, RULE, SPACE, Real>(q, Bw, gw);
        }
        const Real s = Real(Q::w(q)) * adj;
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) {
            Real a[E::NCOEF];
#pragma unroll
            for (int mm = 0; mm < E::NCOEF; ++mm) a[mm] = Real(mm == m ? 1 : 0);
            Real f0[NC], f1[NC][DIM];
            P::template point<DIM, Real>(uq, gu, a, f0, f1);
            Real acc = Real(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (P::HAS_F0) acc = fmadd(wq[c], f0[c], acc);
                if constexpr (P::HAS_F1) {
#pragma unroll
                    for (int i = 0; i < DIM; ++i) acc = fmadd(gw[c][i], f1[c][i], acc);
                }
            }
            const Real dq = s * acc;
            if constexpr (SPACE == FEM_COEF_QUAD) {
                dcf[m * E::NW + q] = dq;
            } else if constexpr (SPACE == FEM_COEF_P1) {
#pragma unroll
                for (int b = 0; b < E::NV; ++b) dcf[m * E::NW + b] = fmadd(Real(Q::lam(q, b)), dq, dcf[m * E::NW + b]);
            } else {
                dcf[m] += dq;
            }
        }
    }
}

}  // namespace femq
