// residual_p3.hip -- element residuals of third-order (P3) Lagrange elements,
// their adjoint and element matrices from precomputed affine geometry.
//
// One lane per element, as the P1 and P2 lane kernels: every SoA row
// (inverse Jacobian, det J, the N_b * N_comp closure rows, the coefficient
// rows) is one coalesced access per wave, and the quadrature and basis
// phases run in registers with the basis tabulated at compile time
// (p3_device.hpp). Workgroups hold at most four waves, so the largest
// elements (3D elasticity in FP64, 60 closure and 60 output words) may use
// the accumulation registers too instead of spilling to memory.
#include "fem_internal.hpp"
#include "p3_device.hpp"

namespace femq {

template <int DIM, int PHYS, typename Real>
__global__ void __launch_bounds__(256)
residual_p3_kernel(int64_t n, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                   const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    constexpr int RULE = DIM == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11;
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        Real ij[E::NG], uu[E::NBT], aq[E::NCQ], r[E::NBT];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
        const Real dj = __builtin_nontemporal_load(det_j + e);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) uu[f] = __builtin_nontemporal_load(u + f * n + e);
        p3_coef_points<DIM, PHYS, RULE, Real>(space, coef, n, e, aq);
        element_residual_p3<DIM, PHYS, RULE, Real>(ij, dj, uu, aq, r);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], out + f * n + e);
    }
}

// du = R(w) (the forms are symmetric) and dcoef, the derivative with respect
// to the coefficient words: the point values mapped back onto the space
// (the transpose of p3_coef_points). Either output may be skipped
// (uniform flags); u is read only for dcoef.
template <int DIM, int PHYS, typename Real>
__global__ void __launch_bounds__(256)
backward_p3_kernel(int64_t n, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                   const Real* __restrict__ u, const Real* __restrict__ coef, const Real* __restrict__ w,
                   Real* __restrict__ du, Real* __restrict__ dcoef) {
    constexpr int RULE = DIM == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11;
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        Real ij[E::NG], ww[E::NBT];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
        const Real dj = __builtin_nontemporal_load(det_j + e);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) ww[f] = __builtin_nontemporal_load(w + f * n + e);
        if (du != nullptr) {
            Real aq[E::NCQ], r[E::NBT];
            p3_coef_points<DIM, PHYS, RULE, Real>(space, coef, n, e, aq);
            element_residual_p3<DIM, PHYS, RULE, Real>(ij, dj, ww, aq, r);
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], du + f * n + e);
        }
        if (dcoef != nullptr) {
            Real uu[E::NBT], dq[E::NCQ];
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) uu[f] = __builtin_nontemporal_load(u + f * n + e);
            element_dcoef_points_p3<DIM, PHYS, RULE, Real>(ij, dj, uu, ww, dq);
            if (space == FEM_COEF_QUAD) {
#pragma unroll
                for (int f = 0; f < E::NCQ; ++f) __builtin_nontemporal_store(dq[f], dcoef + f * n + e);
            } else if (space == FEM_COEF_P1) {
#pragma unroll
                for (int m = 0; m < E::NCOEF; ++m)
#pragma unroll
                    for (int v = 0; v < E::NV; ++v) {
                        Real t = Real(0);
#pragma unroll
                        for (int q = 0; q < E::NQ; ++q) t = fmadd(Real(Q::lam(q, v)), dq[m * E::NQ + q], t);
                        __builtin_nontemporal_store(t, dcoef + (m * E::NV + v) * n + e);
                    }
            } else {
#pragma unroll
                for (int m = 0; m < E::NCOEF; ++m) {
                    Real t = Real(0);
#pragma unroll
                    for (int q = 0; q < E::NQ; ++q) t += dq[m * E::NQ + q];
                    __builtin_nontemporal_store(t, dcoef + m * n + e);
                }
            }
        }
    }
}

// Element matrices: the three forms are linear in u, so column s of K_e is
// R_e(e_s), the residual of the unit closure e_s = (basis function b_s,
// component c_s). Its value and gradient at a point are phi_{b_s} and
// sum_v dphi_{b_s}/dlam_v g_v in component c_s alone, read from a table
// with the wave-uniform index b_s; the basis phase is the residual's, over
// the rows r <= s only. Column s stores those entries at (r, s) and (s, r),
// so the matrix is exactly symmetric. Columns run in a loop (the arithmetic
// is inlined once).
__constant__ P3Table<2, FEM_RULE_TRI6> kP3Table2;
__constant__ P3Table<3, FEM_RULE_TET11> kP3Table3;

template <int DIM>
__device__ __forceinline__ const auto& p3_table() {
    if constexpr (DIM == 2) return kP3Table2;
    else return kP3Table3;
}

template <int DIM, int PHYS, typename Real>
__global__ void __launch_bounds__(256)
jacobian_p3_kernel(int64_t n, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                   const Real* __restrict__ coef, Real* __restrict__ out) {
    constexpr int RULE = DIM == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11;
    using E = ElemP3<DIM, PHYS, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    using T = P3Basis<DIM, RULE>;
    using P = Physics<PHYS>;
    constexpr int M = E::NBT, NC = E::NC, NV = E::NV, NB = E::NB;
    const auto& tab = p3_table<DIM>();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        Real ij[E::NG], aq[E::NCQ];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
        const Real adj = fabs(__builtin_nontemporal_load(det_j + e));
        p3_coef_points<DIM, PHYS, RULE, Real>(space, coef, n, e, aq);
        Real g[NV][DIM];
        p2_bary_grads<DIM, Real>(ij, g);
#pragma unroll 1
        for (int s = 0; s < M; ++s) {
            const int bs = s / NC, cs = s - bs * NC;
            Real r[M];
#pragma unroll
            for (int f = 0; f < M; ++f) r[f] = Real(0);
            unroll_for<0, E::NQ>([&](auto q_c) {
                constexpr int q = decltype(q_c)::value;
                Real uq[NC], gq[NC][DIM];
                if constexpr (P::NEEDS_U) {
                    const Real ph = Real(tab.phi[q][bs]);
#pragma unroll
                    for (int c = 0; c < NC; ++c) uq[c] = c == cs ? ph : Real(0);
                }
                if constexpr (P::HAS_F1) {
                    Real gs[DIM];
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        Real t = Real(tab.dl[q][bs][0]) * g[0][i];
#pragma unroll
                        for (int v = 1; v < NV; ++v) t = fmadd(Real(tab.dl[q][bs][v]), g[v][i], t);
                        gs[i] = t;
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int i = 0; i < DIM; ++i) gq[c][i] = c == cs ? gs[i] : Real(0);
                }
                Real a[E::NCOEF];
#pragma unroll
                for (int m = 0; m < E::NCOEF; ++m) a[m] = aq[m * E::NQ + q];
                Real f0[NC], f1[NC][DIM];
                P::template point<DIM, Real>(uq, gq, a, f0, f1);
                const Real w = Real(Q::w(q)) * adj;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if constexpr (P::HAS_F1) {
                        Real h[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            Real t = g[v][0] * f1[c][0];
#pragma unroll
                            for (int i = 1; i < DIM; ++i) t = fmadd(g[v][i], f1[c][i], t);
                            h[v] = w * t;
                        }
                        unroll_for<0, NB>([&](auto b_c) {
                            constexpr int b = decltype(b_c)::value;
                            if (b * NC + c <= s) {
                                unroll_for<0, NV>([&](auto v_c) {
                                    constexpr int v = decltype(v_c)::value;
                                    constexpr double d = T::dl(q, b, v);
                                    if constexpr (d != 0.0) r[b * NC + c] = fmadd(Real(d), h[v], r[b * NC + c]);
                                });
                            }
                        });
                    }
                    if constexpr (P::HAS_F0) {
                        const Real sf = w * f0[c];
                        unroll_for<0, NB>([&](auto b_c) {
                            constexpr int b = decltype(b_c)::value;
                            if (b * NC + c <= s) r[b * NC + c] = fmadd(Real(T::phi(q, b)), sf, r[b * NC + c]);
                        });
                    }
                }
            });
#pragma unroll
            for (int f = 0; f < M; ++f) {
                if (f <= s) {
                    __builtin_nontemporal_store(r[f], out + (int64_t)(f * M + s) * n + e);
                    __builtin_nontemporal_store(r[f], out + (int64_t)(s * M + f) * n + e);
                }
            }
        }
    }
}

template <int DIM, int PHYS, typename Real>
static hipError_t launch_jac(int space, const JacobianArgs& a, const Launch& l) {
    hipLaunchKernelGGL((jacobian_p3_kernel<DIM, PHYS, Real>), dim3(l.grid), dim3(l.block), 0, l.stream, a.n, space,
                       static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

template <int DIM, int PHYS, typename Real>
static hipError_t launch_bwd(int space, const BackwardArgs& a, const Launch& l) {
    hipLaunchKernelGGL((backward_p3_kernel<DIM, PHYS, Real>), dim3(l.grid), dim3(l.block), 0, l.stream, a.n, space,
                       static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<const Real*>(a.w),
                       static_cast<Real*>(a.du), static_cast<Real*>(a.dcoef));
    return hipGetLastError();
}

template <int DIM, int PHYS, typename Real>
static hipError_t launch_fwd(int space, const ResidualArgs& a, const Launch& l) {
    hipLaunchKernelGGL((residual_p3_kernel<DIM, PHYS, Real>), dim3(l.grid), dim3(l.block), 0, l.stream, a.n, space,
                       static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

// Runtime (dim, physics, dtype) to a kernel instance; the rule is the
// degree-4 rule of the dimension (checked by the caller), the space a
// kernel argument.
template <typename F>
static hipError_t p3_dispatch(int dim, int phys, int space, int dtype, const F& f) {
    if (space != FEM_COEF_QUAD && space != FEM_COEF_P1 && space != FEM_COEF_P0) return hipErrorInvalidValue;
    auto by_phys = [&](auto dim_c) -> hipError_t {
        constexpr int D = decltype(dim_c)::value;
        auto go = [&](auto phys_c) -> hipError_t {
            constexpr int P = decltype(phys_c)::value;
            return dtype == FEM_F32 ? f.template operator()<D, P, float>() : f.template operator()<D, P, double>();
        };
        switch (phys) {
        case FEM_LAPLACE: return go(std::integral_constant<int, FEM_LAPLACE>());
        case FEM_ELASTICITY: return go(std::integral_constant<int, FEM_ELASTICITY>());
        case FEM_MASS: return go(std::integral_constant<int, FEM_MASS>());
        default: return hipErrorInvalidValue;
        }
    };
    if (dim == 2) return by_phys(std::integral_constant<int, 2>());
    if (dim == 3) return by_phys(std::integral_constant<int, 3>());
    return hipErrorInvalidValue;
}

struct P3Fwd {
    int space;
    const ResidualArgs& a;
    const Launch& l;
    template <int D, int P, typename Real>
    hipError_t operator()() const { return launch_fwd<D, P, Real>(space, a, l); }
};

struct P3Bwd {
    int space;
    const BackwardArgs& a;
    const Launch& l;
    template <int D, int P, typename Real>
    hipError_t operator()() const { return launch_bwd<D, P, Real>(space, a, l); }
};

struct P3Jac {
    int space;
    const JacobianArgs& a;
    const Launch& l;
    template <int D, int P, typename Real>
    hipError_t operator()() const { return launch_jac<D, P, Real>(space, a, l); }
};

hipError_t launch_jacobian_p3(int dim, int phys, int space, int dtype, const JacobianArgs& a, const Launch& l) {
    return p3_dispatch(dim, phys, space, dtype, P3Jac{space, a, l});
}

hipError_t launch_residual_p3(int dim, int phys, int space, int dtype, const ResidualArgs& a, const Launch& l) {
    return p3_dispatch(dim, phys, space, dtype, P3Fwd{space, a, l});
}

hipError_t launch_backward_p3(int dim, int phys, int space, int dtype, const BackwardArgs& a, const Launch& l) {
    return p3_dispatch(dim, phys, space, dtype, P3Bwd{space, a, l});
}

}  // namespace femq
