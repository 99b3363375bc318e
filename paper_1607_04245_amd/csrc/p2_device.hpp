// p2_device.hpp -- element arithmetic of second-order (P2) Lagrange
// elements on affine simplices: the quadrature and basis phases of Eq. (2)
// with the P2 basis, evaluated with the barycentric structure of the basis.
//
// Basis (node order: vertices v = 0..d, then edges (i, j), i < j,
// lexicographic): phi_v = lam_v (2 lam_v - 1), phi_ij = 4 lam_i lam_j, with
// lam_0 = 1 - sum xi, lam_k = xi_k, grad lam_0 = -1, grad lam_k = e_k. Hence
// at a point
//   grad_xi u = sum_v c_v grad lam_v,
//   c_v = u_v (4 lam_v - 1) + 4 sum_{edges (v, j)} u_vj lam_j,
// so the reference gradient is (c_1 - c_0, ..., c_d - c_0); and with
// t_v = grad lam_v . fh (t_0 = -sum_k fh_k, t_k = fh_{k-1}) the basis phase
// is r_v += (4 lam_v - 1) t_v, r_ij += 4 (lam_i t_j + lam_j t_i). No
// multiplication by a tabulated zero is executed. The geometry is affine, as
// for P1, and a P1 coefficient keeps its d+1 vertex values and the P1 basis.
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

// Value and physical gradient of the field at point q: uq[c], g[c][i].
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void p2_field_at(int q, const Real* ij, const Real* u, Real (&uq)[ElemP2<DIM, PHYS, RULE, SPACE>::NC],
                                            Real (&g)[ElemP2<DIM, PHYS, RULE, SPACE>::NC][DIM], bool need_value) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    constexpr int NC = E::NC, NV = E::NV;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Real cv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) cv[v] = Real(4.0 * Q::lam(q, v) - 1.0) * u[v * NC + c];
#pragma unroll
        for (int k = 0; k < E::NE; ++k) {
            const Real ue = Real(4) * u[(NV + k) * NC + c];
            const int i = E::ei(k), j = E::ej(k);
            cv[i] = fmadd(Real(Q::lam(q, j)), ue, cv[i]);
            cv[j] = fmadd(Real(Q::lam(q, i)), ue, cv[j]);
        }
        Real gh[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gh[k] = cv[k + 1] - cv[0];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            Real s = gh[0] * ij[i];
#pragma unroll
            for (int k = 1; k < DIM; ++k) s = fmadd(gh[k], ij[k * DIM + i], s);
            g[c][i] = s;
        }
        if (need_value) {
            Real s = Real(Q::lam(q, 0) * (2.0 * Q::lam(q, 0) - 1.0)) * u[c];
#pragma unroll
            for (int v = 1; v < NV; ++v) s = fmadd(Real(Q::lam(q, v) * (2.0 * Q::lam(q, v) - 1.0)), u[v * NC + c], s);
#pragma unroll
            for (int k = 0; k < E::NE; ++k)
                s = fmadd(Real(4.0 * Q::lam(q, E::ei(k)) * Q::lam(q, E::ej(k))), u[(NV + k) * NC + c], s);
            uq[c] = s;
        } else {
            uq[c] = Real(0);
        }
    }
}

// Adds the weighted point contribution s*f0[c] phi_b + G_b . (s*f1[c]) to r.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void p2_basis_add(int q, const Real* ij, Real s, const Real (&f0)[ElemP2<DIM, PHYS, RULE, SPACE>::NC],
                                             const Real (&f1)[ElemP2<DIM, PHYS, RULE, SPACE>::NC][DIM], bool has_f0,
                                             bool has_f1, Real* r) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    constexpr int NC = E::NC, NV = E::NV;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (has_f1) {
            // reference flux fh = J^{-1} (s f1)
            Real fh[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                Real t = ij[k * DIM] * f1[c][0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) t = fmadd(ij[k * DIM + i], f1[c][i], t);
                fh[k] = s * t;
            }
            Real tv[NV];
            Real sum = fh[0];
#pragma unroll
            for (int k = 1; k < DIM; ++k) sum += fh[k];
            tv[0] = -sum;
#pragma unroll
            for (int k = 0; k < DIM; ++k) tv[k + 1] = fh[k];
#pragma unroll
            for (int v = 0; v < NV; ++v) r[v * NC + c] = fmadd(Real(4.0 * Q::lam(q, v) - 1.0), tv[v], r[v * NC + c]);
#pragma unroll
            for (int k = 0; k < E::NE; ++k) {
                const int i = E::ei(k), j = E::ej(k);
                Real t = fmadd(Real(4.0 * Q::lam(q, i)), tv[j], r[(NV + k) * NC + c]);
                r[(NV + k) * NC + c] = fmadd(Real(4.0 * Q::lam(q, j)), tv[i], t);
            }
        }
        if (has_f0) {
            const Real sf = s * f0[c];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                r[v * NC + c] = fmadd(Real(Q::lam(q, v) * (2.0 * Q::lam(q, v) - 1.0)), sf, r[v * NC + c]);
#pragma unroll
            for (int k = 0; k < E::NE; ++k)
                r[(NV + k) * NC + c] = fmadd(Real(4.0 * Q::lam(q, E::ei(k)) * Q::lam(q, E::ej(k))), sf, r[(NV + k) * NC + c]);
        }
    }
}

// Residual of one P2 element: r[b*NC + c], from invJ ij[k*DIM + i], det J,
// closure u[b*NC + c] and coefficient words cf.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void element_residual_p2(const Real* ij, Real dj, const Real* u, const Real* cf, Real* r) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    using Q = RuleP2<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int NC = E::NC;
#pragma unroll
    for (int b = 0; b < E::NBT; ++b) r[b] = Real(0);
    const Real adj = fabs(dj);
#pragma unroll
    for (int q = 0; q < E::NQ; ++q) {
        Real uq[NC], g[NC][DIM];
        p2_field_at<DIM, PHYS, RULE, SPACE, Real>(q, ij, u, uq, g, P::NEEDS_U);
        Real a[E::NCOEF];
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) a[m] = coef_at_p2<DIM, PHYS, RULE, SPACE, Real>(cf, m, q);
        Real f0[NC], f1[NC][DIM];
        P::template point<DIM, Real>(uq, g, a, f0, f1);
        p2_basis_add<DIM, PHYS, RULE, SPACE, Real>(q, ij, Real(Q::w(q)) * adj, f0, f1, P::HAS_F0, P::HAS_F1, r);
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
#pragma unroll
    for (int q = 0; q < E::NQ; ++q) {
        Real uq[NC], gu[NC][DIM], wq[NC], gw[NC][DIM];
        p2_field_at<DIM, PHYS, RULE, SPACE, Real>(q, ij, u, uq, gu, P::NEEDS_U);
        p2_field_at<DIM, PHYS, RULE, SPACE, Real>(q, ij, w, wq, gw, P::HAS_F0);
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
