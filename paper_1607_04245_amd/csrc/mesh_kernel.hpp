// mesh_kernel.hpp -- the fused from-mesh element kernel: geometry and
// integration in one pass, from coordinates and connectivity.
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
//
// Two forms share this code: u given as per-element closure rows (the
// paper's kernel input), or u given per vertex and gathered through the
// connectivity (the closure built in the kernel, with a P1 coefficient also
// gathered from its vertex values). Both run identical element arithmetic
// on identical values, so they agree bit for bit.
#pragma once

#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {


// The loads of one element that do not depend on other loads (vertex
// indices, and closure and coefficient rows when they are given per
// element), and the slots the vertex gathers fill in.
template <int NBT, int NCQ, typename Real>
struct MeshStage {
    int32_t v[4];
    Real u[NBT], cf[NCQ];
};

// Whether the coefficient is gathered from vertex values: only P1
// coefficients in the gather form.
template <int DIM, int PHYS, int RULE, bool GATHER>
constexpr bool coef_per_vertex() { return GATHER && Elem<DIM, PHYS, RULE>::SPACE == FEM_COEF_P1; }

// Issues the loads of element e without any condition: an index past the end
// is clamped to the last element (its data is then ignored), so the number of
// loads in flight is the same on every path and the compiler can wait for
// exactly the ones it needs.
template <int DIM, int PHYS, int RULE, typename Real, bool VEC, bool GATHER>
__device__ __forceinline__ void mesh_stage_load(MeshStage<Elem<DIM, PHYS, RULE>::NBT, Elem<DIM, PHYS, RULE>::NCQ, Real>& st,
                                                int64_t e, int64_t n, const int32_t* __restrict__ conn,
                                                const Real* __restrict__ u, const Real* __restrict__ coef) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t ec = e < n ? e : n - 1;
    int32_t vv[DIM + 1];
    load_conn<DIM, VEC>(conn, ec, vv);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) st.v[b] = vv[b];
    if constexpr (!GATHER) {
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) st.u[f] = __builtin_nontemporal_load(u + f * n + ec);
    }
    if constexpr (!coef_per_vertex<DIM, PHYS, RULE, GATHER>()) {
#pragma unroll
        for (int f = 0; f < E::NCQ; ++f) st.cf[f] = __builtin_nontemporal_load(coef + f * n + ec);
    }
}

// Vertex gathers of a loaded stage: coordinates, and in the gather form the
// vertex values of u (and of a P1 coefficient) into the closure slots, entry
// b*N_comp + c (coefficient m*N_b + b). An element past the end or with a
// bad index gathers clamped, in-bounds vertices and is not ok.
template <int DIM, int PHYS, int RULE, typename Real, bool GATHER>
__device__ __forceinline__ bool mesh_stage_gather(MeshStage<Elem<DIM, PHYS, RULE>::NBT, Elem<DIM, PHYS, RULE>::NCQ, Real>& st,
                                                  int64_t e, int64_t n, int64_t nv, const double* __restrict__ X,
                                                  const Real* __restrict__ u_vert, const Real* __restrict__ coef_vert,
                                                  double (&x)[DIM + 1][DIM]) {
    using E = Elem<DIM, PHYS, RULE>;
    int32_t vv[DIM + 1];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) vv[b] = st.v[b];
    gather_coords<DIM>(X, vv, nv, x);
    if constexpr (GATHER) {
        const int32_t hi = vertex_hi(nv);
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            const int64_t vi = (int64_t)min(max(vv[b], 0), hi);
#pragma unroll
            for (int c = 0; c < E::NC; ++c) st.u[b * E::NC + c] = u_vert[vi * E::NC + c];
            if constexpr (coef_per_vertex<DIM, PHYS, RULE, GATHER>()) {
#pragma unroll
                for (int m = 0; m < E::NCOEF; ++m) st.cf[m * E::NB + b] = coef_vert[vi * E::NCOEF + m];
            }
        }
    }
    return (e < n) & conn_ok<DIM>(vv, nv);
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
    ndeg += (int)(valid & (flag == 1));
    npoor += (int)(valid & (flag == 2));
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
// per tile instead of two. (A three-deep pipeline, with the gathers of tile
// k+1 also in flight during the arithmetic of tile k, measured slower at
// every launch shape.) EPT = 2 or 4: that many elements per lane, no
// pipelining.
// GATHER: u (and a P1 coefficient) are vertex arrays gathered through the
// connectivity instead of per-element closure rows.
template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool STORE_GEOM, bool VEC, bool GATHER>
__global__ void __launch_bounds__(512)
residual_mesh_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                     const Real* __restrict__ u, const Real* __restrict__ coef,
                     Real* __restrict__ out, Real* __restrict__ inv_j, Real* __restrict__ det_j,
                     int32_t* __restrict__ counts) {
    using E = Elem<DIM, PHYS, RULE>;
    using Stage = MeshStage<E::NBT, E::NCQ, Real>;
    const int lane = threadIdx.x & 63;
    // wave-uniform (readfirstlane): the tile loop is then scalar control flow
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), waves = blockDim.x >> 6;
    const int64_t n_tiles = (n + 64 * EPT - 1) / (64 * EPT);
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    int ndeg = 0, npoor = 0;
    int64_t tile = t_begin + wave;
    if constexpr (EPT == 1) {
        // ping-pong between two stages: no register copies between iterations
        Stage a, b;
        mesh_stage_load<DIM, PHYS, RULE, Real, VEC, GATHER>(a, tile < t_end ? tile * 64 + lane : n, n, conn, u, coef);
        while (tile < t_end) {
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                const bool ok = mesh_stage_gather<DIM, PHYS, RULE, Real, GATHER>(a, e, n, nv, X, u, coef, x);
                // keep every gather ahead of the prefetch (no load may move
                // across), so the wait for them leaves the prefetched loads in flight
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC, GATHER>(b, next < t_end ? next * 64 + lane : n, n, conn, u, coef);
                mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e < n, e, n, ok, x, a.u, a.cf, out, inv_j,
                                                                       det_j, ndeg, npoor);
                tile = next;
            }
            if (tile >= t_end) break;
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                const bool ok = mesh_stage_gather<DIM, PHYS, RULE, Real, GATHER>(b, e, n, nv, X, u, coef, x);
                // keep every gather ahead of the prefetch (no load may move
                // across), so the wait for them leaves the prefetched loads in flight
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC, GATHER>(a, next < t_end ? next * 64 + lane : n, n, conn, u, coef);
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
                mesh_stage_load<DIM, PHYS, RULE, Real, VEC, GATHER>(st[j], e[j], n, conn, u, coef);
            }
            double x[EPT][DIM + 1][DIM];
            bool ok[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) ok[j] = mesh_stage_gather<DIM, PHYS, RULE, Real, GATHER>(st[j], e[j], n, nv, X, u, coef, x[j]);
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e[j] < n, e[j], n, ok[j], x[j], st[j].u,
                                                                       st[j].cf, out, inv_j, det_j, ndeg, npoor);
        }
    }
    add_counts(counts, ndeg, npoor);
}

template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool VEC, bool GATHER>
static hipError_t launch_s(const MeshArgs& a, const Launch& l) {
    const Real* u = static_cast<const Real*>(a.u);
    const Real* cf = static_cast<const Real*>(a.coef);
    Real* out = static_cast<Real*>(a.out);
    Real* ij = static_cast<Real*>(a.inv_j);
    Real* dj = static_cast<Real*>(a.det_j);
    if (ij != nullptr)
        hipLaunchKernelGGL((residual_mesh_kernel<DIM, PHYS, RULE, Real, EPT, true, VEC, GATHER>), dim3(l.grid), dim3(l.block),
                           0, l.stream, a.n, a.n_vert, a.coords, a.conn, u, cf, out, ij, dj, a.counts);
    else
        hipLaunchKernelGGL((residual_mesh_kernel<DIM, PHYS, RULE, Real, EPT, false, VEC, GATHER>), dim3(l.grid), dim3(l.block),
                           0, l.stream, a.n, a.n_vert, a.coords, a.conn, u, cf, out, ij, dj, a.counts);
    return hipGetLastError();
}

// The wide-access variant (one 16-byte connectivity load per tetrahedron)
// needs 16-byte aligned connectivity; torch allocations always are.
template <int DIM, int PHYS, int RULE, typename Real, int EPT, bool GATHER>
static hipError_t launch_a(const MeshArgs& a, const Launch& l) {
    const bool vec = DIM == 3 && (reinterpret_cast<uintptr_t>(a.conn) % 16) == 0;
    return vec ? launch_s<DIM, PHYS, RULE, Real, EPT, true, GATHER>(a, l)
               : launch_s<DIM, PHYS, RULE, Real, EPT, false, GATHER>(a, l);
}

template <int DIM, int PHYS, int RULE, typename Real, bool GATHER>
static hipError_t launch_v(const MeshArgs& a, const Launch& l) {
    switch (l.vec) {
    case 1: return launch_a<DIM, PHYS, RULE, Real, 1, GATHER>(a, l);
    case 2: return launch_a<DIM, PHYS, RULE, Real, 2, GATHER>(a, l);
    case 4: return launch_a<DIM, PHYS, RULE, Real, 4, GATHER>(a, l);
    default: return hipErrorInvalidValue;
    }
}

template <int DIM, int PHYS, int RULE, bool GATHER>
static hipError_t launch_t(int dtype, const MeshArgs& a, const Launch& l) {
    return dtype == FEM_F32 ? launch_v<DIM, PHYS, RULE, float, GATHER>(a, l)
                            : launch_v<DIM, PHYS, RULE, double, GATHER>(a, l);
}

// Calls launch_t for a runtime (dim, physics, rule, space, dtype).
template <bool GATHER>
struct MeshDispatch {
    int dtype;
    const MeshArgs& a;
    const Launch& l;
    template <int D, int P, int S>
    hipError_t operator()() const { return launch_t<D, P, S, GATHER>(dtype, a, l); }
};

}  // namespace femq
