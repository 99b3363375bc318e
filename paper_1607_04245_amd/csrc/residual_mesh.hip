// residual_mesh.hip -- element residuals straight from coordinates and
// connectivity: geometry and integration fused in one pass.
//
// The paper's kernel reads precomputed J^{-1} and det J (Section 3,
// Appendix); storing them and reading them back costs (d^2+1) words per
// element twice. Here each lane computes its elements' geometry in FP64 from
// the gathered vertices, rounds it to the working precision exactly as
// fem_geometry stores it, and integrates from those rounded values with the
// same element arithmetic as fem_integrate_residual, so the element vectors
// are bitwise equal to the two-call path. Writing the geometry out as well is
// optional. Wave tiles of 64*EPT elements, lane l owning elements l, l+64,
// ...; the closure and coefficient rows do not depend on the connectivity and
// are requested before the vertex gathers, so both streams are in flight
// together.
#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool STORE_GEOM, bool VEC>
__global__ void __launch_bounds__(512)
residual_mesh_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                     const Real* __restrict__ u, const Real* __restrict__ coef,
                     Real* __restrict__ out, Real* __restrict__ inv_j, Real* __restrict__ det_j,
                     int32_t* __restrict__ counts) {
    using E = Elem<DIM, PHYS, RULE>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    const int64_t n_tiles = (n + 64 * EPT - 1) / (64 * EPT);
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    int ndeg = 0, npoor = 0;
    for (int64_t tile = t_begin + wave; tile < t_end; tile += waves) {
        int64_t e[EPT];
        bool ok[EPT];
        int32_t v[EPT][DIM + 1];
        Real uu[EPT][E::NBT], cf[EPT][E::NCQ];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            e[j] = tile * (64 * EPT) + j * 64 + lane;
            ok[j] = false;
            if (e[j] < n)
                ok[j] = load_conn<DIM, VEC>(conn, e[j], nv, v[j]);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (e[j] >= n) continue;
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) uu[j][f] = __builtin_nontemporal_load(u + f * n + e[j]);
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) cf[j][f] = __builtin_nontemporal_load(coef + f * n + e[j]);
        }
        double x[EPT][DIM + 1][DIM];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (e[j] < n) gather_coords<DIM, VEC>(X, v[j], ok[j], x[j]);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (e[j] >= n) continue;
            double inv[DIM][DIM], ep;
            double det = element_geometry<DIM>(x[j], inv, ep);
            const int flag = finish_geometry<DIM>(ok[j], det, inv, ep);
            ndeg += flag == 1;
            npoor += flag == 2;
            Real ij[E::NG], r[E::NBT];
#pragma unroll
            for (int k = 0; k < DIM; ++k)
#pragma unroll
                for (int i = 0; i < DIM; ++i) ij[k * DIM + i] = static_cast<Real>(inv[k][i]);
            const Real dj = static_cast<Real>(det);
            if constexpr (STORE_GEOM) {
#pragma unroll
                for (int f = 0; f < E::NG; ++f) __builtin_nontemporal_store(ij[f], inv_j + f * n + e[j]);
                __builtin_nontemporal_store(dj, det_j + e[j]);
            }
            element_residual<DIM, PHYS, RULE, Real>(ij, dj, uu[j], cf[j], r);
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], out + f * n + e[j]);
        }
    }
    add_counts(counts, ndeg, npoor);
}

template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool VEC>
static hipError_t launch_s(const MeshArgs& a, const Launch& l) {
    const Real* u = static_cast<const Real*>(a.u);
    const Real* cf = static_cast<const Real*>(a.coef);
    Real* out = static_cast<Real*>(a.out);
    Real* ij = static_cast<Real*>(a.inv_j);
    Real* dj = static_cast<Real*>(a.det_j);
    if (ij != nullptr)
        hipLaunchKernelGGL((residual_mesh_kernel<DIM, PHYS, RULE, Real, EPT, true, VEC>), dim3(l.grid), dim3(l.block),
                           0, l.stream, a.n, a.n_vert, a.coords, a.conn, u, cf, out, ij, dj, a.counts);
    else
        hipLaunchKernelGGL((residual_mesh_kernel<DIM, PHYS, RULE, Real, EPT, false, VEC>), dim3(l.grid), dim3(l.block),
                           0, l.stream, a.n, a.n_vert, a.coords, a.conn, u, cf, out, ij, dj, a.counts);
    return hipGetLastError();
}

// The wide-access variant needs 16-byte aligned coordinates (and, for
// tetrahedra, connectivity); torch allocations always are.
template <int DIM, int PHYS, int RULE, typename Real, int EPT>
static hipError_t launch_a(const MeshArgs& a, const Launch& l) {
    const bool vec = (reinterpret_cast<uintptr_t>(a.coords) % 16) == 0 &&
                     (DIM == 2 || (reinterpret_cast<uintptr_t>(a.conn) % 16) == 0);
    return vec ? launch_s<DIM, PHYS, RULE, Real, EPT, true>(a, l) : launch_s<DIM, PHYS, RULE, Real, EPT, false>(a, l);
}

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_v(const MeshArgs& a, const Launch& l) {
    switch (l.vec) {
    case 1: return launch_a<DIM, PHYS, RULE, Real, 1>(a, l);
    case 2: return launch_a<DIM, PHYS, RULE, Real, 2>(a, l);
    default: return hipErrorInvalidValue;
    }
}

template <int DIM, int PHYS, int RULE>
static hipError_t launch_t(int dtype, const MeshArgs& a, const Launch& l) {
    return dtype == FEM_F32 ? launch_v<DIM, PHYS, RULE, float>(a, l) : launch_v<DIM, PHYS, RULE, double>(a, l);
}

template <int DIM, int PHYS>
static hipError_t launch_r(int rule, int dtype, const MeshArgs& a, const Launch& l) {
    if (rule == FEM_RULE_CENTROID) return launch_t<DIM, PHYS, FEM_RULE_CENTROID>(dtype, a, l);
    if constexpr (DIM == 2) {
        if (rule == FEM_RULE_TRI3) return launch_t<DIM, PHYS, FEM_RULE_TRI3>(dtype, a, l);
    } else {
        if (rule == FEM_RULE_TET4) return launch_t<DIM, PHYS, FEM_RULE_TET4>(dtype, a, l);
    }
    return hipErrorInvalidValue;
}

template <int DIM>
static hipError_t launch_p(int phys, int rule, int dtype, const MeshArgs& a, const Launch& l) {
    switch (phys) {
    case FEM_LAPLACE: return launch_r<DIM, FEM_LAPLACE>(rule, dtype, a, l);
    case FEM_ELASTICITY: return launch_r<DIM, FEM_ELASTICITY>(rule, dtype, a, l);
    case FEM_MASS: return launch_r<DIM, FEM_MASS>(rule, dtype, a, l);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_residual_mesh(int dim, int phys, int rule, int dtype, const MeshArgs& a, const Launch& l) {
    if (dim == 2) return launch_p<2>(phys, rule, dtype, a, l);
    if (dim == 3) return launch_p<3>(phys, rule, dtype, a, l);
    return hipErrorInvalidValue;
}

}  // namespace femq
