// jacobian.hip -- element matrices K_e = dR_e / du_e of the forms of Eq. (1)
// for P1 and P2 Lagrange elements, from precomputed affine geometry.
//
// Differentiating the bracket of Eq. (2) with respect to the closure puts
// the pointwise derivatives of f0 and f1 between the basis values and
// physical gradients:
//   K[(b,c),(b',c')] = sum_q w_q |J| ( phi_b g0 phi_b'
//                      + sum_ij G_b,i g3[c][i][c'][j] G_b',j ),
// Laplacian g3 = kappa delta_ij, elasticity g3 = lambda delta_ci delta_c'j
// + mu (delta_cc' delta_ij + delta_cj delta_ic'), mass g0 = kappa.
//
// One lane per element; every SoA row is one coalesced access per wave, and
// the output (N_bt^2 rows) dominates the traffic. The rule and coefficient
// space only enter the moments below, so they are uniform run-time
// arguments of one kernel per (dim, physics, order, dtype). The gradient terms use the
// barycentric structure of the basis: grad phi_b = sum_v alpha_bv grad lam_v
// with alpha_bv affine in the barycentric coordinates (P1: alpha = delta;
// P2 vertex v: 4 lam_v - 1; P2 edge (i, j): 4 lam_j at i and 4 lam_i at j).
// The quadrature sum then reduces to weighted moments of the coefficient,
//   m0 = sum_q k_q, m1_v = sum_q k_q lam_v, m2_vw = sum_q k_q lam_v lam_w,
// k_q = w_q |J| a(x_q), computed once per element, and each matrix entry is
// a short combination of moments and the products g_v . g_w of the physical
// barycentric gradients. The mass term (products of basis values) is summed
// over the points directly. The matrix is written exactly symmetric: each
// entry below the diagonal is a copy of its mirror.
#include "fem_internal.hpp"
#include "p2_device.hpp"

namespace femq {

// Quadrature rules of both orders as barycentric points: the degree-2 and
// degree-4 rules, and the one-point centroid rule.
template <int DIM, int RULE>
struct RuleBary : RuleP2<DIM, RULE> {};

template <int DIM>
struct RuleBary<DIM, FEM_RULE_CENTROID> {
    static constexpr int NQ = 1;
    __host__ __device__ static constexpr double lam(int, int) { return 1.0 / (DIM + 1); }
    __host__ __device__ static constexpr double w(int) { return DIM == 2 ? 0.5 : 1.0 / 6.0; }
};

// alpha = a0 + a1 * lam_u (u < 0: constant)
struct Aff {
    double a0;
    int u;
    double a1;
};

// Lagrange basis of order 1 or 2; node order: vertices, then edges (i, j),
// i < j, lexicographic.
template <int DIM, int ORDER>
struct LagBasis {
    static constexpr int NV = DIM + 1;
    static constexpr int NE = DIM == 2 ? 3 : 6;
    static constexpr int NB = ORDER == 1 ? NV : NV + NE;
    __host__ __device__ static constexpr int ei(int k) {
        return DIM == 2 ? (k < 2 ? 0 : 1) : (k < 3 ? 0 : (k < 5 ? 1 : 2));
    }
    __host__ __device__ static constexpr int ej(int k) {
        return DIM == 2 ? (k < 2 ? k + 1 : 2) : (k < 3 ? k + 1 : (k < 5 ? k - 1 : 3));
    }
    // barycentric gradients in grad phi_b: one (vertex functions) or two (edges)
    __host__ __device__ static constexpr int nsupp(int b) { return (ORDER == 1 || b < NV) ? 1 : 2; }
    __host__ __device__ static constexpr int supp(int b, int s) {
        return (ORDER == 1 || b < NV) ? b : (s == 0 ? ei(b - NV) : ej(b - NV));
    }
    __host__ __device__ static constexpr Aff alpha(int b, int s) {
        return ORDER == 1 ? Aff{1.0, -1, 0.0}
             : b < NV     ? Aff{-1.0, b, 4.0}
             : s == 0     ? Aff{0.0, ej(b - NV), 4.0}
                          : Aff{0.0, ei(b - NV), 4.0};
    }
    // phi_b at a point with barycentric coordinates lam(v)
    template <typename L>
    __host__ __device__ static constexpr double value(int b, const L& lam) {
        return ORDER == 1 ? lam(b)
             : b < NV     ? lam(b) * (2.0 * lam(b) - 1.0)
                          : 4.0 * lam(ei(b - NV)) * lam(ej(b - NV));
    }
};

// Calls f(std::integral_constant<int, i>) for i = B .. E-1: loops whose
// bounds depend on an outer index stay compile-time constants.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(const F& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for<B + 1, E>(f);
    }
}

template <int NV, typename Real>
struct Moments {
    Real m0;
    Real m1[NV];
    Real m2[NV][NV];
};

// sum_q k_q alpha_A(q) alpha_B(q) from the moments; constant factors fold at
// compile time once the callers' loops are unrolled.
template <int NV, typename Real>
__device__ __forceinline__ Real moment(const Moments<NV, Real>& M, Aff A, Aff B) {
    const int ua = A.u < 0 ? 0 : A.u, ub = B.u < 0 ? 0 : B.u;
    Real s = Real(0);
    if (A.a0 != 0.0 && B.a0 != 0.0) s = Real(A.a0 * B.a0) * M.m0;
    if (A.a0 != 0.0 && B.a1 != 0.0) s = fmadd(Real(A.a0 * B.a1), M.m1[ub], s);
    if (A.a1 != 0.0 && B.a0 != 0.0) s = fmadd(Real(A.a1 * B.a0), M.m1[ua], s);
    if (A.a1 != 0.0 && B.a1 != 0.0) s = fmadd(Real(A.a1 * B.a1), M.m2[ua][ub], s);
    return s;
}

// Coefficient at the points of the rule, weighted: k[m][q] = w_q |J| a_m(x_q)
// from the element's words in their space.
template <int DIM, int RULE, int SPACE, int NCOEF, typename Real>
__device__ __forceinline__ void weighted_coef(const Real* __restrict__ coef, int64_t n, int64_t e, Real dj,
                                              Real (&k)[NCOEF][RuleBary<DIM, RULE>::NQ]) {
    using Q = RuleBary<DIM, RULE>;
    constexpr int NV = DIM + 1, NQ = Q::NQ;
    constexpr int NW = SPACE == FEM_COEF_QUAD ? NQ : SPACE == FEM_COEF_P1 ? NV : 1;
#pragma unroll
    for (int m = 0; m < NCOEF; ++m) {
        Real cf[NW];
#pragma unroll
        for (int f = 0; f < NW; ++f) cf[f] = __builtin_nontemporal_load(coef + (int64_t)(m * NW + f) * n + e);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            Real a;
            if constexpr (SPACE == FEM_COEF_QUAD) {
                a = cf[q];
            } else if constexpr (SPACE == FEM_COEF_P1) {
                a = Real(Q::lam(q, 0)) * cf[0];
#pragma unroll
                for (int v = 1; v < NV; ++v) a = fmadd(Real(Q::lam(q, v)), cf[v], a);
            } else {
                a = cf[0];
            }
            k[m][q] = (Real(Q::w(q)) * dj) * a;
        }
    }
}

// Moments of the weighted coefficients (m1, m2 only for second order).
template <int DIM, int RULE, int SPACE, int NCOEF, int ORDER, typename Real>
__device__ __forceinline__ void coef_moments(const Real* __restrict__ coef, int64_t n, int64_t e, Real dj,
                                             Moments<DIM + 1, Real> (&M)[NCOEF]) {
    using Q = RuleBary<DIM, RULE>;
    constexpr int NV = DIM + 1, NQ = Q::NQ;
    Real k[NCOEF][NQ];
    weighted_coef<DIM, RULE, SPACE, NCOEF, Real>(coef, n, e, dj, k);
#pragma unroll
    for (int m = 0; m < NCOEF; ++m) {
        Real s = k[m][0];
#pragma unroll
        for (int q = 1; q < NQ; ++q) s += k[m][q];
        M[m].m0 = s;
        if constexpr (ORDER == 2) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Real s1 = Real(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) s1 = fmadd(Real(Q::lam(q, v)), k[m][q], s1);
                M[m].m1[v] = s1;
#pragma unroll
                for (int w = 0; w < NV; ++w) {
                    if (w < v) continue;
                    Real s2 = Real(0);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) s2 = fmadd(Real(Q::lam(q, v) * Q::lam(q, w)), k[m][q], s2);
                    M[m].m2[v][w] = s2;
                    M[m].m2[w][v] = s2;
                }
            }
        }
    }
}

// Mass matrix K_bb' = sum_q k_q phi_b(x_q) phi_b'(x_q), stored directly.
template <int DIM, int ORDER, int RULE, int SPACE, typename Real>
__device__ __forceinline__ void mass_matrix(const Real* __restrict__ coef, int64_t n, int64_t e, Real dj,
                                            Real* __restrict__ out) {
    using Q = RuleBary<DIM, RULE>;
    using Bs = LagBasis<DIM, ORDER>;
    constexpr int NB = Bs::NB, NQ = Q::NQ;
    Real k[1][NQ];
    weighted_coef<DIM, RULE, SPACE, 1, Real>(coef, n, e, dj, k);
    static_for<0, NB>([&](auto b_c) {
        constexpr int b = decltype(b_c)::value;
        static_for<b, NB>([&](auto bp_c) {
            constexpr int bp = decltype(bp_c)::value;
            Real s = Real(0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                auto lam = [q](int v) { return Q::lam(q, v); };
                s = fmadd(Real(Bs::value(b, lam) * Bs::value(bp, lam)), k[0][q], s);
            }
            __builtin_nontemporal_store(s, out + (int64_t)(b * NB + bp) * n + e);
            if constexpr (bp != b) __builtin_nontemporal_store(s, out + (int64_t)(bp * NB + b) * n + e);
        });
    });
}

// Calls f(rule constant, space constant) for the element's (rule, space):
// order 1 takes the degree-2 rule or the centroid, order 2 the degree-2 or
// the degree-4 rule. The host validates the pair; the arguments are uniform
// over the grid, so the branch is scalar.
template <int DIM, int ORDER, typename F>
__device__ __forceinline__ void with_scheme(int rule, int space, const F& f) {
    constexpr int LOW = DIM == 2 ? FEM_RULE_TRI3 : FEM_RULE_TET4;
    constexpr int OTHER = ORDER == 1 ? FEM_RULE_CENTROID : (DIM == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11);
    auto by_space = [&](auto rule_c) {
        if (space == FEM_COEF_QUAD) f(rule_c, std::integral_constant<int, FEM_COEF_QUAD>());
        else if (space == FEM_COEF_P1) f(rule_c, std::integral_constant<int, FEM_COEF_P1>());
        else f(rule_c, std::integral_constant<int, FEM_COEF_P0>());
    };
    if (rule == LOW) by_space(std::integral_constant<int, LOW>());
    else by_space(std::integral_constant<int, OTHER>());
}

template <int DIM, int PHYS, int ORDER, typename Real>
__global__ void __launch_bounds__(256)
jacobian_kernel(int64_t n, int rule, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                const Real* __restrict__ coef, Real* __restrict__ out) {
    using Bs = LagBasis<DIM, ORDER>;
    constexpr int NV = DIM + 1, NB = Bs::NB;
    constexpr int NC = PHYS == FEM_ELASTICITY ? DIM : 1, NBT = NB * NC;
    constexpr int NCOEF = PHYS == FEM_ELASTICITY ? 2 : 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const Real dj = fabs(__builtin_nontemporal_load(det_j + e));
        if constexpr (PHYS == FEM_MASS) {
            with_scheme<DIM, ORDER>(rule, space, [&](auto rule_c, auto space_c) {
                mass_matrix<DIM, ORDER, decltype(rule_c)::value, decltype(space_c)::value, Real>(coef, n, e, dj, out);
            });
        } else {
            Moments<NV, Real> M[NCOEF];
            with_scheme<DIM, ORDER>(rule, space, [&](auto rule_c, auto space_c) {
                coef_moments<DIM, decltype(rule_c)::value, decltype(space_c)::value, NCOEF, ORDER, Real>(coef, n, e,
                                                                                                        dj, M);
            });
            Real ij[DIM * DIM];
#pragma unroll
            for (int f = 0; f < DIM * DIM; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
            // physical barycentric gradients: g_{k+1} = row k of J^{-1}, g_0 = -sum
            Real g[NV][DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                Real s = Real(0);
#pragma unroll
                for (int kk = 0; kk < DIM; ++kk) {
                    g[kk + 1][i] = ij[kk * DIM + i];
                    s += ij[kk * DIM + i];
                }
                g[0][i] = -s;
            }
            Real P[NV][NV];  // g_v . g_w
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int w = 0; w < NV; ++w) {
                    if (w < v) continue;
                    Real s = g[v][0] * g[w][0];
#pragma unroll
                    for (int i = 1; i < DIM; ++i) s = fmadd(g[v][i], g[w][i], s);
                    P[v][w] = s;
                    P[w][v] = s;
                }
            static_for<0, NB>([&](auto b_c) {
                constexpr int b = decltype(b_c)::value;
                static_for<b, NB>([&](auto bp_c) {
                    constexpr int bp = decltype(bp_c)::value;
                    Real blk[NC][NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int cp = 0; cp < NC; ++cp) blk[c][cp] = Real(0);
#pragma unroll
                    for (int s = 0; s < Bs::nsupp(b); ++s)
#pragma unroll
                        for (int t = 0; t < Bs::nsupp(bp); ++t) {
                            const int v = Bs::supp(b, s), w = Bs::supp(bp, t);
                            const Aff A = Bs::alpha(b, s), B = Bs::alpha(bp, t);
                            if constexpr (PHYS == FEM_LAPLACE) {
                                blk[0][0] = fmadd(moment(M[0], A, B), P[v][w], blk[0][0]);
                            } else {
                                const Real lm = moment(M[0], A, B), mu = moment(M[1], A, B);
#pragma unroll
                                for (int c = 0; c < NC; ++c)
#pragma unroll
                                    for (int cp = 0; cp < NC; ++cp) {
                                        if (bp == b && cp < c) continue;
                                        Real x = fmadd(lm * g[v][c], g[w][cp], blk[c][cp]);
                                        x = fmadd(mu, g[v][cp] * g[w][c], x);
                                        if (c == cp) x = fmadd(mu, P[v][w], x);
                                        blk[c][cp] = x;
                                    }
                            }
                        }
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int cp = 0; cp < NC; ++cp) {
                            if (bp == b && cp < c) continue;
                            const int r = b * NC + c, s = bp * NC + cp;
                            __builtin_nontemporal_store(blk[c][cp], out + (int64_t)(r * NBT + s) * n + e);
                            if (s != r) __builtin_nontemporal_store(blk[c][cp], out + (int64_t)(s * NBT + r) * n + e);
                        }
                });
            });
        }
    }
}

template <int DIM, int PHYS, int ORDER, typename Real>
static hipError_t launch_jac(int rule, int space, const JacobianArgs& a, const Launch& l) {
    hipLaunchKernelGGL((jacobian_kernel<DIM, PHYS, ORDER, Real>), dim3(l.grid), dim3(l.block), 0, l.stream, a.n, rule,
                       space, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

// Runtime (dim, physics, order, dtype) to a kernel instance; (rule, space)
// are kernel arguments. Rules: order 1 takes the degree-2 rule of its
// dimension or the centroid, order 2 the degree-2 or the degree-4 rule.
hipError_t launch_jacobian(int dim, int phys, int order, int rule, int space, int dtype, const JacobianArgs& a,
                           const Launch& l) {
    const int low = dim == 2 ? FEM_RULE_TRI3 : FEM_RULE_TET4, high = dim == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11;
    const bool rule_ok = rule == low || (order == 1 && rule == FEM_RULE_CENTROID) || (order == 2 && rule == high);
    const bool space_ok = space == FEM_COEF_QUAD || space == FEM_COEF_P1 || space == FEM_COEF_P0;
    if (!rule_ok || !space_ok || (dtype != FEM_F32 && dtype != FEM_F64)) return hipErrorInvalidValue;
    auto go = [&](auto dim_c, auto phys_c, auto order_c) -> hipError_t {
        constexpr int D = decltype(dim_c)::value, P = decltype(phys_c)::value, O = decltype(order_c)::value;
        return dtype == FEM_F32 ? launch_jac<D, P, O, float>(rule, space, a, l)
                                : launch_jac<D, P, O, double>(rule, space, a, l);
    };
    auto by_order = [&](auto dim_c, auto phys_c) -> hipError_t {
        if (order == 1) return go(dim_c, phys_c, std::integral_constant<int, 1>());
        if (order == 2) return go(dim_c, phys_c, std::integral_constant<int, 2>());
        return hipErrorInvalidValue;
    };
    auto by_phys = [&](auto dim_c) -> hipError_t {
        switch (phys) {
        case FEM_LAPLACE: return by_order(dim_c, std::integral_constant<int, FEM_LAPLACE>());
        case FEM_ELASTICITY: return by_order(dim_c, std::integral_constant<int, FEM_ELASTICITY>());
        case FEM_MASS: return by_order(dim_c, std::integral_constant<int, FEM_MASS>());
        default: return hipErrorInvalidValue;
        }
    };
    if (dim == 2) return by_phys(std::integral_constant<int, 2>());
    if (dim == 3) return by_phys(std::integral_constant<int, 3>());
    return hipErrorInvalidValue;
}

}  // namespace femq
