// backward_lane.hip -- adjoint of the element residual, one lane per element.
//
// For L = sum_e w_e . R_e: du_e = R_e(u := w_e) because every supported form
// is a symmetric bilinear form in (u, test function), and dcoef at each
// quadrature point is the weighted pointwise derivative of f0/f1 with respect
// to the coefficient (the forms are linear in the coefficients). Same
// coalesced V-wide SoA access as the forward kernel; du and dcoef are
// optional (wave-uniform branches), and u is only read when dcoef is wanted.
#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

template <int DIM, int PHYS, int RULE, typename Real, int V>
__global__ void __launch_bounds__(512)
backward_lane_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                     const Real* __restrict__ u, const Real* __restrict__ coef,
                     const Real* __restrict__ w, Real* __restrict__ du, Real* __restrict__ dcoef) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t nchunk = n / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool want_du = du != nullptr;
    const bool want_dc = dcoef != nullptr;
    for (int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nchunk; ch += stride) {
        const int64_t e0 = ch * V;
        Real rij[E::NG][V], rdj[V], rw[E::NBT][V];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ld_row<Real, V>(inv_j + f * n + e0, rij[f]);
        ld_row<Real, V>(det_j + e0, rdj);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) ld_row<Real, V>(w + f * n + e0, rw[f]);
        if (want_du) {
            Real rcf[E::NCQ][V], rr[E::NBT][V];
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) ld_row<Real, V>(coef + f * n + e0, rcf[f]);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                Real ij[E::NG], ww[E::NBT], cf[E::NCQ], r[E::NBT];
#pragma unroll
                for (int f = 0; f < E::NG; ++f) ij[f] = rij[f][v];
#pragma unroll
                for (int f = 0; f < E::NBT; ++f) ww[f] = rw[f][v];
#pragma unroll
                for (int f = 0; f < E::NCQ; ++f) cf[f] = rcf[f][v];
                element_residual<DIM, PHYS, RULE, Real>(ij, rdj[v], ww, cf, r);
#pragma unroll
                for (int f = 0; f < E::NBT; ++f) rr[f][v] = r[f];
            }
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) st_row<Real, V>(du + f * n + e0, rr[f]);
        }
        if (want_dc) {
            Real ru[E::NBT][V], rd[E::NCQ][V];
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) ld_row<Real, V>(u + f * n + e0, ru[f]);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                Real ij[E::NG], uu[E::NBT], ww[E::NBT], d[E::NCQ];
#pragma unroll
                for (int f = 0; f < E::NG; ++f) ij[f] = rij[f][v];
#pragma unroll
                for (int f = 0; f < E::NBT; ++f) {
                    uu[f] = ru[f][v];
                    ww[f] = rw[f][v];
                }
                element_dcoef<DIM, PHYS, RULE, Real>(ij, rdj[v], uu, ww, d);
#pragma unroll
                for (int f = 0; f < E::NCQ; ++f) rd[f][v] = d[f];
            }
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) st_row<Real, V>(dcoef + f * n + e0, rd[f]);
        }
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_v(const BackwardArgs& a, const Launch& l) {
    const Real* ij = static_cast<const Real*>(a.inv_j);
    const Real* dj = static_cast<const Real*>(a.det_j);
    const Real* u = static_cast<const Real*>(a.u);
    const Real* cf = static_cast<const Real*>(a.coef);
    const Real* w = static_cast<const Real*>(a.w);
    Real* du = static_cast<Real*>(a.du);
    Real* dc = static_cast<Real*>(a.dcoef);
    switch (l.vec) {
    case 1:
        hipLaunchKernelGGL((backward_lane_kernel<DIM, PHYS, RULE, Real, 1>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, w, du, dc);
        break;
    case 2:
        hipLaunchKernelGGL((backward_lane_kernel<DIM, PHYS, RULE, Real, 2>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, w, du, dc);
        break;
    case 4:
        hipLaunchKernelGGL((backward_lane_kernel<DIM, PHYS, RULE, Real, 4>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, w, du, dc);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DIM, int PHYS, int RULE>
static hipError_t launch_t(int dtype, const BackwardArgs& a, const Launch& l) {
    return dtype == FEM_F32 ? launch_v<DIM, PHYS, RULE, float>(a, l) : launch_v<DIM, PHYS, RULE, double>(a, l);
}

struct BackwardDispatch {
    int dtype;
    const BackwardArgs& a;
    const Launch& l;
    template <int D, int P, int S>
    hipError_t operator()() const { return launch_t<D, P, S>(dtype, a, l); }
};

hipError_t launch_backward_lane(int dim, int phys, int rule, int space, int dtype, const BackwardArgs& a,
                               const Launch& l) {
    const BackwardDispatch f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
