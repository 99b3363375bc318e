// residual_lane.hip -- element residual kernels, one lane per element.
//
// Each lane owns V consecutive elements. Every structure-of-arrays row is
// read with one V-wide vector load per lane, so a wavefront reads 64*V
// consecutive words of a row at once (fully coalesced, 16-byte accesses for
// V*sizeof(Real) = 16). The quadrature phase (pointwise f0/f1 at every
// point) and the basis phase (sum back onto the basis functions) run in
// registers, so no value crosses lanes and no reduction is needed; the paper's
// concern about per-thread storage (Section 1) does not bind on gfx950, whose
// lanes hold up to 512 VGPRs. Grid-stride over chunks of V elements.
#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

template <int DIM, int PHYS, int RULE, typename Real, int V>
__global__ void __launch_bounds__(512)
residual_lane_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                     const Real* __restrict__ u, const Real* __restrict__ coef,
                     Real* __restrict__ out) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t nchunk = n / V;  // the host guarantees V divides n
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nchunk; ch += stride) {
        const int64_t e0 = ch * V;
        Real rij[E::NG][V], rdj[V], ru[E::NBT][V], rcf[E::NCQ][V], rr[E::NBT][V];
#pragma unroll
        for (int f = 0; f < E::NG; ++f) ld_row<Real, V>(inv_j + f * n + e0, rij[f]);
        ld_row<Real, V>(det_j + e0, rdj);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) ld_row<Real, V>(u + f * n + e0, ru[f]);
#pragma unroll
        for (int f = 0; f < E::NCQ; ++f) ld_row<Real, V>(coef + f * n + e0, rcf[f]);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            Real ij[E::NG], uu[E::NBT], cf[E::NCQ], r[E::NBT];
#pragma unroll
            for (int f = 0; f < E::NG; ++f) ij[f] = rij[f][v];
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) uu[f] = ru[f][v];
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) cf[f] = rcf[f][v];
            element_residual<DIM, PHYS, RULE, Real>(ij, rdj[v], uu, cf, r);
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) rr[f][v] = r[f];
        }
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) st_row<Real, V>(out + f * n + e0, rr[f]);
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_v(const ResidualArgs& a, const Launch& l) {
    const Real* ij = static_cast<const Real*>(a.inv_j);
    const Real* dj = static_cast<const Real*>(a.det_j);
    const Real* u = static_cast<const Real*>(a.u);
    const Real* cf = static_cast<const Real*>(a.coef);
    Real* out = static_cast<Real*>(a.out);
    switch (l.vec) {
    case 1:
        hipLaunchKernelGGL((residual_lane_kernel<DIM, PHYS, RULE, Real, 1>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, out);
        break;
    case 2:
        hipLaunchKernelGGL((residual_lane_kernel<DIM, PHYS, RULE, Real, 2>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, out);
        break;
    case 4:
        hipLaunchKernelGGL((residual_lane_kernel<DIM, PHYS, RULE, Real, 4>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, ij, dj, u, cf, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DIM, int PHYS, int RULE>
static hipError_t launch_t(int dtype, const ResidualArgs& a, const Launch& l) {
    return dtype == FEM_F32 ? launch_v<DIM, PHYS, RULE, float>(a, l) : launch_v<DIM, PHYS, RULE, double>(a, l);
}

struct LaneDispatch {
    int dtype;
    const ResidualArgs& a;
    const Launch& l;
    template <int D, int P, int S>
    hipError_t operator()() const { return launch_t<D, P, S>(dtype, a, l); }
};

hipError_t launch_residual_lane(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                               const Launch& l) {
    const LaneDispatch f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
