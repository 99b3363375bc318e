// residual_p2.hip -- element residuals and their adjoint for second-order
// (P2) Lagrange elements from precomputed affine geometry.
//
// One lane per element, as the P1 lane kernel: every SoA row (inverse
// Jacobian, det J, the N_b * N_comp closure rows, the coefficient rows) is
// one coalesced access per wave; the quadrature and basis phases run in
// registers with the barycentric structure of the P2 basis (p2_device.hpp).
// Workgroups hold at most four waves, so the largest elements (3D
// elasticity in FP64) may use the accumulation registers too instead of
// spilling to memory.
#include "fem_internal.hpp"
#include "p2_device.hpp"

namespace femq {

template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__global__ void __launch_bounds__(256)
residual_p2_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                   const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        Real ij[E::NG], uu[E::NBT], cf[E::NCQ], r[E::NBT];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
        const Real dj = __builtin_nontemporal_load(det_j + e);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) uu[f] = __builtin_nontemporal_load(u + f * n + e);
#pragma unroll
        for (int f = 0; f < E::NCQ; ++f) cf[f] = __builtin_nontemporal_load(coef + f * n + e);
        element_residual_p2<DIM, PHYS, RULE, SPACE, Real>(ij, dj, uu, cf, r);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], out + f * n + e);
    }
}

// du = R(w) (symmetric forms), dcoef from element_dcoef_p2; either may be
// skipped (wave-uniform flags), and u is read only for dcoef.
template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
__global__ void __launch_bounds__(256)
backward_p2_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                   const Real* __restrict__ u, const Real* __restrict__ coef, const Real* __restrict__ w,
                   Real* __restrict__ du, Real* __restrict__ dcoef) {
    using E = ElemP2<DIM, PHYS, RULE, SPACE>;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        Real ij[E::NG], ww[E::NBT];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(inv_j + f * n + e);
        const Real dj = __builtin_nontemporal_load(det_j + e);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) ww[f] = __builtin_nontemporal_load(w + f * n + e);
        if (du != nullptr) {
            Real cf[E::NCQ], r[E::NBT];
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) cf[f] = __builtin_nontemporal_load(coef + f * n + e);
            element_residual_p2<DIM, PHYS, RULE, SPACE, Real>(ij, dj, ww, cf, r);
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], du + f * n + e);
        }
        if (dcoef != nullptr) {
            Real uu[E::NBT], d[E::NCQ];
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) uu[f] = __builtin_nontemporal_load(u + f * n + e);
            element_dcoef_p2<DIM, PHYS, RULE, SPACE, Real>(ij, dj, uu, ww, d);
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) __builtin_nontemporal_store(d[f], dcoef + f * n + e);
        }
    }
}

template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
static hipError_t launch_fwd(const ResidualArgs& a, const Launch& l) {
    hipLaunchKernelGGL((residual_p2_kernel<DIM, PHYS, RULE, SPACE, Real>), dim3(l.grid), dim3(l.block), 0, l.stream,
                       a.n, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

template <int DIM, int PHYS, int RULE, int SPACE, typename Real>
static hipError_t launch_bwd(const BackwardArgs& a, const Launch& l) {
    hipLaunchKernelGGL((backward_p2_kernel<DIM, PHYS, RULE, SPACE, Real>), dim3(l.grid), dim3(l.block), 0, l.stream,
                       a.n, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<const Real*>(a.w),
                       static_cast<Real*>(a.du), static_cast<Real*>(a.dcoef));
    return hipGetLastError();
}

// Runtime (dim, physics, rule, space, dtype) to a kernel instance.
template <typename F>
static hipError_t p2_dispatch(int dim, int phys, int rule, int space, int dtype, const F& f) {
    auto by_space = [&](auto dim_c, auto phys_c, auto rule_c) -> hipError_t {
        constexpr int D = decltype(dim_c)::value, P = decltype(phys_c)::value, RU = decltype(rule_c)::value;
        auto go = [&](auto sp_c) -> hipError_t {
            constexpr int S = decltype(sp_c)::value;
            return dtype == FEM_F32 ? f.template operator()<D, P, RU, S, float>()
                                    : f.template operator()<D, P, RU, S, double>();
        };
        switch (space) {
        case FEM_COEF_QUAD: return go(std::integral_constant<int, FEM_COEF_QUAD>());
        case FEM_COEF_P1: return go(std::integral_constant<int, FEM_COEF_P1>());
        case FEM_COEF_P0: return go(std::integral_constant<int, FEM_COEF_P0>());
        default: return hipErrorInvalidValue;
        }
    };
    auto by_rule = [&](auto dim_c, auto phys_c) -> hipError_t {
        constexpr int D = decltype(dim_c)::value;
        if constexpr (D == 2) {
            if (rule == FEM_RULE_TRI3) return by_space(dim_c, phys_c, std::integral_constant<int, FEM_RULE_TRI3>());
            if (rule == FEM_RULE_TRI6) return by_space(dim_c, phys_c, std::integral_constant<int, FEM_RULE_TRI6>());
        } else {
            if (rule == FEM_RULE_TET4) return by_space(dim_c, phys_c, std::integral_constant<int, FEM_RULE_TET4>());
            if (rule == FEM_RULE_TET11) return by_space(dim_c, phys_c, std::integral_constant<int, FEM_RULE_TET11>());
        }
        return hipErrorInvalidValue;
    };
    auto by_phys = [&](auto dim_c) -> hipError_t {
        switch (phys) {
        case FEM_LAPLACE: return by_rule(dim_c, std::integral_constant<int, FEM_LAPLACE>());
        case FEM_ELASTICITY: return by_rule(dim_c, std::integral_constant<int, FEM_ELASTICITY>());
        case FEM_MASS: return by_rule(dim_c, std::integral_constant<int, FEM_MASS>());
        default: return hipErrorInvalidValue;
        }
    };
    if (dim == 2) return by_phys(std::integral_constant<int, 2>());
    if (dim == 3) return by_phys(std::integral_constant<int, 3>());
    return hipErrorInvalidValue;
}

struct P2Fwd {
    const ResidualArgs& a;
    const Launch& l;
    template <int D, int P, int RU, int S, typename Real>
    hipError_t operator()() const { return launch_fwd<D, P, RU, S, Real>(a, l); }
};

struct P2Bwd {
    const BackwardArgs& a;
    const Launch& l;
    template <int D, int P, int RU, int S, typename Real>
    hipError_t operator()() const { return launch_bwd<D, P, RU, S, Real>(a, l); }
};

hipError_t launch_residual_p2(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                              const Launch& l) {
    return p2_dispatch(dim, phys, rule, space, dtype, P2Fwd{a, l});
}

hipError_t launch_backward_p2(int dim, int phys, int rule, int space, int dtype, const BackwardArgs& a,
                              const Launch& l) {
    return p2_dispatch(dim, phys, rule, space, dtype, P2Bwd{a, l});
}

}  // namespace femq
