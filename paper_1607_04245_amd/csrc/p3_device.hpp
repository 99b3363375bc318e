// p3_device.hpp -- element arithmetic of third-order (P3) Lagrange elements
// on affine simplices: the quadrature and basis phases of Eq. (2) with the
// P3 basis tabulated at the points (Section 3's B and D), one lane per
// element.
//
// Basis (node order: vertices v = 0..d; per edge (i, j), i < j,
// lexicographic, the node at 2/3 of lam_i then the node at 2/3 of lam_j; per
// face (i, j, k), lexicographic, its centroid):
//   vertex  lam_v (3 lam_v - 1)(3 lam_v - 2) / 2,
//   edge    (9/2) lam_a lam_o (3 lam_a - 1)   (a the nearer vertex),
//   face    27 lam_i lam_j lam_k.
// Each function's derivatives with respect to the barycentric coordinates
// at a quadrature point are compile-time constants (the points are), so a
// physical gradient is sum_v dphi/dlam_v g_v with g_v the gradients of the
// barycentric coordinates, and the tabulation costs no memory traffic: the
// quadrature phase forms U_v = sum_b dphi_b/dlam_v u_b (zero entries
// dropped at compile time), grad u = sum_v U_v g_v, and the basis phase
// adds dphi_b/dlam_v (g_v . w_q |J| f1) to every r_b. The rules are the
// degree-4 rules of the P2 path, which integrate a P3 stiffness entry with
// a constant coefficient exactly.
#pragma once

#include "p2_device.hpp"

namespace femq {

template <int DIM, int PHYS, int RULE, int SPACE>
struct ElemP3 {
    static constexpr int NV = DIM + 1;                              // vertices
    static constexpr int NE = DIM == 2 ? 3 : 6;                     // edges, two nodes each
    static constexpr int NF = DIM == 2 ? 1 : 4;                     // faces, one node each
    static constexpr int NB = NV + 2 * NE + NF;                     // 10 or 20
    static constexpr int NC = (PHYS == FEM_ELASTICITY) ? DIM : 1;
    static constexpr int NBT = NB * NC;
    static constexpr int NQ = RuleP2<DIM, RULE>::NQ;
    static constexpr int NW = SPACE == FEM_COEF_QUAD ? NQ : SPACE == FEM_COEF_P1 ? NV : 1;
    static constexpr int NCOEF = (PHYS == FEM_ELASTICITY) ? 2 : 1;
    static constexpr int NCQ = NCOEF * NW;
    static constexpr int NG = DIM * DIM;
};

// The P3 basis and its barycentric derivatives at point q of RULE.
template <int DIM, int RULE>
struct P3Basis {
    using Q = RuleP2<DIM, RULE>;
    static constexpr int NV = DIM + 1, NE = DIM == 2 ? 3 : 6;
    // edge k = (ei(k), ej(k)) and face f = (fa, fb, fc), lexicographic
    __host__ __device__ static constexpr int ei(int k) { return ElemP2<DIM, 0, RULE, 0>::ei(k); }
    __host__ __device__ static constexpr int ej(int k) { return ElemP2<DIM, 0, RULE, 0>::ej(k); }
    __host__ __device__ static constexpr int fa(int f) { return DIM == 2 ? 0 : (f < 3 ? 0 : 1); }
    __host__ __device__ static constexpr int fb(int f) { return DIM == 2 ? 1 : (f < 2 ? 1 : 2); }
    __host__ __device__ static constexpr int fc(int f) { return DIM == 2 ? 2 : (f == 0 ? 2 : 3); }

    __host__ __device__ static constexpr double phi(int q, int b) {
        if (b < NV) {
            const double l = Q::lam(q, b);
            return 0.5 * l * (3.0 * l - 1.0) * (3.0 * l - 2.0);
        }
        if (b < NV + 2 * NE) {
            const int k = (b - NV) / 2, s = (b - NV) % 2;
            const int a = s == 0 ? ei(k) : ej(k), o = s == 0 ? ej(k) : ei(k);
            return 4.5 * Q::lam(q, a) * Q::lam(q, o) * (3.0 * Q::lam(q, a) - 1.0);
        }
        const int f = b - NV - 2 * NE;
        return 27.0 * Q::lam(q, fa(f)) * Q::lam(q, fb(f)) * Q::lam(q, fc(f));
    }

    // d phi_b / d lam_v at point q
    __host__ __device__ static constexpr double dl(int q, int b, int v) {
        if (b < NV) {
            const double l = Q::lam(q, b);
            return v == b ? 0.5 * (27.0 * l * l - 18.0 * l + 2.0) : 0.0;
        }
        if (b < NV + 2 * NE) {
            const int k = (b - NV) / 2, s = (b - NV) % 2;
            const int a = s == 0 ? ei(k) : ej(k), o = s == 0 ? ej(k) : ei(k);
            const double la = Q::lam(q, a), lo = Q::lam(q, o);
            return v == a ? 4.5 * lo * (6.0 * la - 1.0) : (v == o ? 4.5 * la * (3.0 * la - 1.0) : 0.0);
        }
        const int f = b - NV - 2 * NE;
        const int i = fa(f), j = fb(f), k = fc(f);
        const double li = Q::lam(q, i), lj = Q::lam(q, j), lk = Q::lam(q, k);
        return v == i ? 27.0 * lj * lk : (v == j ? 27.0 * li * lk : (v == k ? 27.0 * li * lj : 0.0));
    }
};

// The basis values and barycentric derivatives at the points as a table,
// for lookups with a run-time (wave-uniform) function index.
template <int DIM, int RULE>
struct P3Table {
    static constexpr int NQ = RuleP2<DIM, RULE>::NQ, NB = ElemP3<DIM, 0, RULE, 0>::NB, NV = DIM + 1;
    double phi[NQ][NB];
    double dl[NQ][NB][NV];
    constexpr P3Table() : phi(), dl() {
        for (int q = 0; q < NQ; ++q)
            for (int b = 0; b < NB; ++b) {
                phi[q][b] = P3Basis<DIM, RULE>::phi(q, b);
                for (int v = 0; v < NV; ++v) dl[q][b][v] = P3Basis<DIM, RULE>::dl(q, b, v);
            }
    }
};

// Calls f(std::integral_constant<int, i>) for i = B .. E-1, so the basis
// values at a point are constant expressions: zero entries drop out at
// compile time and no loop is left to the optimizer's unrolling limits.
template <int B, int E, typename F>
__device__ __forceinline__ void unroll_for(const F& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        unroll_for<B + 1, E>(f);
    }
}

// The coefficient words of element e turned into values at the points: the
// space is a uniform run-time branch (one kernel per dimension, physics and
// type), the arithmetic after it is the same for every space. STREAM: the
// loads bypass the caches' retention (each word is read once); kernels whose
// tiles share cache lines read through the caches.
template <int DIM, int PHYS, int RULE, typename Real, bool STREAM = true>
__device__ __forceinline__ void p3_coef_points(int space, const Real* __restrict__ coef, int64_t n, int64_t e,
                                               Real (&aq)[ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>::NCQ]) {
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    auto load = [](const Real* p) {
        if constexpr (STREAM) return __builtin_nontemporal_load(p);
        else return *p;
    };
    if (space == FEM_COEF_QUAD) {
#pragma unroll
        for (int f = 0; f < E::NCQ; ++f) aq[f] = load(coef + f * n + e);
    } else if (space == FEM_COEF_P1) {
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) {
            Real c[E::NV];
#pragma unroll
            for (int v = 0; v < E::NV; ++v) c[v] = load(coef + (m * E::NV + v) * n + e);
#pragma unroll
            for (int q = 0; q < E::NQ; ++q) {
                Real t = Real(Q::lam(q, 0)) * c[0];
#pragma unroll
                for (int v = 1; v < E::NV; ++v) t = fmadd(Real(Q::lam(q, v)), c[v], t);
                aq[m * E::NQ + q] = t;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) {
            const Real c = load(coef + m * n + e);
#pragma unroll
            for (int q = 0; q < E::NQ; ++q) aq[m * E::NQ + q] = c;
        }
    }
}

// Residual of one P3 element: r[b*NC + c], from invJ ij[k*DIM + i], det J,
// closure u[b*NC + c] and the coefficient values at the points
// aq[m*NQ + q].
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void element_residual_p3(const Real* ij, Real dj, const Real* u, const Real* aq, Real* r) {
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    using T = P3Basis<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int NC = E::NC, NV = E::NV, NB = E::NB;
#pragma unroll
    for (int b = 0; b < E::NBT; ++b) r[b] = Real(0);
    const Real adj = fabs(dj);
    Real g[NV][DIM];
    p2_bary_grads<DIM, Real>(ij, g);
    unroll_for<0, E::NQ>([&](auto q_c) {
        constexpr int q = decltype(q_c)::value;
        Real uq[NC], gq[NC][DIM];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (P::NEEDS_U) {
                Real s = Real(0);
                unroll_for<0, NB>([&](auto b_c) {
                    constexpr int b = decltype(b_c)::value;
                    s = fmadd(Real(T::phi(q, b)), u[b * NC + c], s);
                });
                uq[c] = s;
            }
            if constexpr (P::HAS_F1) {
                Real U[NV];
                unroll_for<0, NV>([&](auto v_c) {
                    constexpr int v = decltype(v_c)::value;
                    Real s = Real(0);
                    unroll_for<0, NB>([&](auto b_c) {
                        constexpr int b = decltype(b_c)::value;
                        constexpr double d = T::dl(q, b, v);
                        if constexpr (d != 0.0) s = fmadd(Real(d), u[b * NC + c], s);
                    });
                    U[v] = s;
                });
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    Real s = U[0] * g[0][i];
#pragma unroll
                    for (int v = 1; v < NV; ++v) s = fmadd(U[v], g[v][i], s);
                    gq[c][i] = s;
                }
            }
        }
        Real a[E::NCOEF];
#pragma unroll
        for (int m = 0; m < E::NCOEF; ++m) a[m] = aq[m * E::NQ + q];
        Real f0[NC], f1[NC][DIM];
        P::template point<DIM, Real>(uq, gq, a, f0, f1);
        const Real s = Real(Q::w(q)) * adj;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (P::HAS_F1) {
                Real h[NV];  // g_v . (w_q |J| f1)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Real t = g[v][0] * f1[c][0];
#pragma unroll
                    for (int i = 1; i < DIM; ++i) t = fmadd(g[v][i], f1[c][i], t);
                    h[v] = s * t;
                }
                unroll_for<0, NB>([&](auto b_c) {
                    constexpr int b = decltype(b_c)::value;
                    unroll_for<0, NV>([&](auto v_c) {
                        constexpr int v = decltype(v_c)::value;
                        constexpr double d = T::dl(q, b, v);
                        if constexpr (d != 0.0) r[b * NC + c] = fmadd(Real(d), h[v], r[b * NC + c]);
                    });
                });
            }
            if constexpr (P::HAS_F0) {
                const Real sf = s * f0[c];
                unroll_for<0, NB>([&](auto b_c) {
                    constexpr int b = decltype(b_c)::value;
                    r[b * NC + c] = fmadd(Real(T::phi(q, b)), sf, r[b * NC + c]);
                });
            }
        }
    });
}

// Derivative of L = w . R with respect to the coefficient values at the
// points (the forms are linear in the coefficients): dq[m*NQ + q] =
// w_q |J| [w^q . f0(u; e_m) + grad w : f1(u; e_m)].
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void element_dcoef_points_p3(const Real* ij, Real dj, const Real* u, const Real* w,
                                                        Real* dq) {
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    using T = P3Basis<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int NC = E::NC, NV = E::NV, NB = E::NB;
    const Real adj = fabs(dj);
    Real g[NV][DIM];
    p2_bary_grads<DIM, Real>(ij, g);
    // value and physical gradient of a field at point q
    auto field_at = [&](auto q_c, const Real* f, Real (&fq)[NC], Real (&gf)[NC][DIM]) {
        constexpr int q = decltype(q_c)::value;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (P::HAS_F0) {
                Real s = Real(0);
                unroll_for<0, NB>([&](auto b_c) {
                    constexpr int b = decltype(b_c)::value;
                    s = fmadd(Real(T::phi(q, b)), f[b * NC + c], s);
                });
                fq[c] = s;
            }
            if constexpr (P::HAS_F1) {
                Real U[NV];
                unroll_for<0, NV>([&](auto v_c) {
                    constexpr int v = decltype(v_c)::value;
                    Real s = Real(0);
                    unroll_for<0, NB>([&](auto b_c) {
                        constexpr int b = decltype(b_c)::value;
                        constexpr double d = T::dl(q, b, v);
                        if constexpr (d != 0.0) s = fmadd(Real(d), f[b * NC + c], s);
                    });
                    U[v] = s;
                });
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    Real s = U[0] * g[0][i];
#pragma unroll
                    for (int v = 1; v < NV; ++v) s = fmadd(U[v], g[v][i], s);
                    gf[c][i] = s;
                }
            }
        }
    };
    unroll_for<0, E::NQ>([&](auto q_c) {
        constexpr int q = decltype(q_c)::value;
        Real uq[NC], gu[NC][DIM], wq[NC], gw[NC][DIM];
        field_at(q_c, u, uq, gu);
        field_at(q_c, w, wq, gw);
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
            dq[m * E::NQ + q] = s * acc;
        }
    });
}

}  // namespace femq
