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
// are requested together with it, ahead of the vertex gathers.
#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

// The loads of one element that do not depend on other loads: vertex
// indices, closure and coefficients.
template <int NBT, int NCQ, typename Real>
struct MeshStage {
    int32_t v[4];
    Real u[NBT], cf[NCQ];
};

// Issues the loads of element e without any condition: an index past the end
// is clamped to the last element (its data is then ignored), so the number of
// loads in flight is the same on every path and the compiler can wait for
// exactly the ones it needs.
template <int DIM, int PHYS, int RULE, typename Real, bool VEC>
__device__ __forceinline__ void mesh_stage_load(MeshStage<Elem<DIM, PHYS, RULE>::NBT, Elem<DIM, PHYS, RULE>::NCQ, Real>& st,
                                                int64_t e, int64_t n, const int32_t* __restrict__ conn,
                                                const Real* __restrict__ u, const Real* __restrict__ coef) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t ec = e < n ? e : n - 1;
    int32_t vv[DIM + 1];
    load_conn<DIM, VEC>(conn, ec, vv);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) st.v[b] = vv[b];
#pragma unroll
    for (int f = 0; f < E::NBT; ++f) st.u[f] = __builtin_nontemporal_load(u + f * n + ec);
#pragma unroll
    for (int f = 0; f < E::NCQ; ++f) st.cf[f] = __builtin_nontemporal_load(coef + f * n + ec);
}

// Vertex gathers of a loaded stage; an element past the end or with a bad
// index gathers vertex 0 (always in bounds) and is not ok.
template <int DIM, int NBT, int NCQ, typename Real>
__device__ __forceinline__ bool mesh_stage_gather(const MeshStage<NBT, NCQ, Real>& st, int64_t e, int64_t n,
                                                  int64_t nv, const double* __restrict__ X,
                                                  double (&x)[DIM + 1][DIM]) {
    int32_t vv[DIM + 1];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) vv[b] = st.v[b];
    gather_coords<DIM>(X, vv, nv, x);
    return e < n && conn_ok<DIM>(vv, nv);
}

// Geometry, integration and stores of one element whose vertices are in x.
// The arithmetic runs for every lane; only the stores and the counters are
// predicated on `valid`, so no load feeding it can be moved into a branch.
template <int DIM, int PHYS, int RULE, typename Real, bool STORE_GEOM>
__device__ __forceinline__ void mesh_element_finish(bool valid, int64_t e, int64_t n, bool ok,
                                                    const double (&x)[DIM + 1][DIM], const Real* uu, const Real* cf,
                                                    Real* __restrict__ out, Real* __restrict__ inv_j,
                                                    Real* __restrict__ det_j, int& ndeg, int& npoor) {
    using E = Elem<DIM, PHYS, RULE>;
    double inv[DIM][DIM], ep2;
    double det = element_geometry<DIM>(x, inv, ep2);
    const int flag = finish_geometry<DIM>(ok, det, inv, ep2);
    ndeg += valid && flag == 1;
    npoor += valid && flag == 2;
    Real ij[E::NG], r[E::NBT];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i < DIM; ++i) ij[k * DIM + i] = static_cast<Real>(inv[k][i]);
    const Real dj = static_cast<Real>(det);
    element_residual<DIM, PHYS, RULE, Real>(ij, dj, uu, cf, r);
    if (valid) {
        if constexpr (STORE_GEOM) {
#pragma unroll
            for (int f = 0; f < E::NG; ++f) __builtin_nontemporal_store(ij[f], inv_j + f * n + e);
            __builtin_nontemporal_store(dj, det_j + e);
        }
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], out + f * n + e);
    }
}

// EPT = 1: software-pipelined. While the vertex gathers and the arithmetic of
// tile k run, the connectivity, closure and coefficient loads of the wave's
// next tile are already in flight, so a wave pays roughly one memory latency
// per tile instead of two. EPT = 2: two elements per lane, no pipelining.
template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool STORE_GEOM, bool VEC>
__global__ void __launch_bounds__(512)
residual_mesh_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                     const Real* __restrict__ u, const Real* __restrict__ coef,
                     Real* __restrict__ out, Real* __restrict__ inv_j, Real* __restrict__ det_j,
                     int32_t* __restrict__ counts) {
    using E = Elem<DIM, PHYS, RULE>;
    using Stage = MeshStage<E::NBT, E::NCQ, Real>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    const int64_t n_tiles = (n + 64 * EPT - 1) / (64 * EPT);
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    int ndeg = 0, npoor = 0;
    int64_t tile = t_begin + wave;
    if constexpr (EPT == 1) {
        // ping-pong between two stages: no register copies between iterations
        Stage a, b;
        mesh_stage_load<DIM, PHYS, RULE, Real, VEC>(a, tile < t_end ? tile * 64 + lane : n, n, conn, u, coef);
        while (tile < t_end) {
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                const bool ok = mesh_stage_gather<DIM>(a, e, n, nv, X, x);
                // keep every gather ahead of the prefetch (no load may move
                // across), so the wait for them leaves the prefetched loads in flight
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC>(b, next < t_end ? next * 64 + lane : n, n, conn, u, coef);
                mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e < n, e, n, ok, x, a.u, a.cf, out, inv_j,
                                                                       det_j, ndeg, npoor);
                tile = next;
            }
            if (tile >= t_end) break;
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                const bool ok = mesh_stage_gather<DIM>(b, e, n, nv, X, x);
                // keep every gather ahead of the prefetch (no load may move
                // across), so the wait for them leaves the prefetched loads in flight
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC>(a, next < t_end ? next * 64 + lane : n, n, conn, u, coef);
                mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e < n, e, n, ok, x, b.u, b.cf, out, inv_j,
                                                                       det_j, ndeg, npoor);
                tile = next;
            }
        }
    } else {
        for (; tile < t_end; tile += waves) {
            Stage st[EPT];
            int64_t e[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                e[j] = tile * (64 * EPT) + j * 64 + lane;
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC>(st[j], e[j], n, conn, u, coef);
            }
            double x[EPT][DIM + 1][DIM];
            bool ok[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) ok[j] = mesh_stage_gather<DIM>(st[j], e[j], n, nv, X, x[j]);
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e[j] < n, e[j], n, ok[j], x[j], st[j].u,
                                                                       st[j].cf, out, inv_j, det_j, ndeg, npoor);
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

// The wide-access variant (one 16-byte connectivity load per tetrahedron)
// needs 16-byte aligned connectivity; torch allocations always are.
template <int DIM, int PHYS, int RULE, typename Real, int EPT>
static hipError_t launch_a(const MeshArgs& a, const Launch& l) {
    const bool vec = DIM == 3 && (reinterpret_cast<uintptr_t>(a.conn) % 16) == 0;
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

struct MeshDispatch {
    int dtype;
    const MeshArgs& a;
    const Launch& l;
    template <int D, int P, int S>
    hipError_t operator()() const { return launch_t<D, P, S>(dtype, a, l); }
};

hipError_t launch_residual_mesh(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                               const Launch& l) {
    const MeshDispatch f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
