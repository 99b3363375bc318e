// residual_dedup.hip -- the fused from-mesh residual with each wave's vertex
// records gathered once per tile, deduplicated in LDS at run time.
//
// In the fused kernel (mesh_kernel.hpp) every lane gathers the d+1 vertex
// records of its own element, although the 64 elements of a wave tile of a
// conforming mesh share most of their vertices (about 47 distinct vertices
// for 256 references on a tetrahedral grid). The per-lane gathers, not the
// bytes, bound that kernel. A mesh plan (mesh_plan.hip) removes the
// duplicates ahead of time; this kernel removes them on the fly, with no
// precomputed data, from the connectivity the caller passes:
//
//   insert   every lane enters its element's d+1 vertex indices into a
//            per-wave open-addressing hash table in LDS (compare-and-swap,
//            linear probing); the lane whose swap fills a slot owns it
//   number   ballots over the owners give every distinct vertex a dense
//            position; owners record it in the slot and list the vertex
//   stage    the wave loads the listed vertices' coordinates, one component
//            per lane (three contiguous lanes per vertex record), into LDS;
//            the next tile's connectivity, closure and coefficient loads are
//            issued behind these gathers and stay in flight
//   read     every lane reads its element's vertices from LDS
//   reset    the lanes clear the slots they used, for the next tile
//
// Vertices beyond the staging capacity (a tile of almost unshared elements)
// are gathered by their lanes directly. The element arithmetic is that of the
// fused kernel on the same FP64 coordinates, so the element vectors (and the
// optional geometry outputs and counters) are bitwise those of
// fem_integrate_residual_mesh with the lane strategy.
#include "mesh_kernel.hpp"

namespace femq {

constexpr int kDedupSlots = 256;     // hash slots per wave (power of two, >= 4 x 64 indices)
constexpr int kDedupCap = 96;        // distinct vertices staged per tile
constexpr uint8_t kNotStaged = 0xFF;

template <int DIM>
struct DedupSlab {
    int32_t key[kDedupSlots];          // vertex index, -1 = empty
    uint8_t pos[kDedupSlots];          // dense position of the slot's vertex, kNotStaged beyond the capacity
    int32_t ids[kDedupCap];            // vertex of each dense position
    double x[kDedupCap * DIM];         // its coordinates
};

__device__ __forceinline__ void dd_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t dd_hash(int32_t v) { return ((uint32_t)v * 0x9E3779B1u) >> 24; }

// Stage 1 and 2 for one tile: slots of the element's vertices (-1 if the
// table had no room, which cannot happen with 4 x 64 <= 256 indices), and the
// number of distinct vertices.
template <int DIM>
__device__ __forceinline__ int dd_insert(DedupSlab<DIM>& S, const int32_t (&vi)[DIM + 1], int (&slot)[DIM + 1]) {
    bool won[DIM + 1];
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        uint32_t h = dd_hash(vi[b]);
        slot[b] = -1;
        won[b] = false;
        for (int probe = 0; probe < kDedupSlots; ++probe) {
            const int32_t old = atomicCAS(&S.key[h], -1, vi[b]);
            if (old == -1 || old == vi[b]) {
                slot[b] = (int)h;
                won[b] = old == -1;
                break;
            }
            h = (h + 1) & (kDedupSlots - 1);
        }
    }
    int base = 0;
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        const uint64_t m = __ballot(won[b]);
        if (won[b]) {
            const int d = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            S.pos[slot[b]] = d < kDedupCap ? (uint8_t)d : kNotStaged;
            if (d < kDedupCap) S.ids[d] = vi[b];
        }
        base += __popcll(m);
    }
    return base;
}

template <int DIM, int PHYS, int RULE, typename Real, bool STORE_GEOM, bool VEC, int WPB>
__global__ void __launch_bounds__(64 * WPB)
residual_dedup_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                      const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out,
                      Real* __restrict__ inv_j, Real* __restrict__ det_j, int32_t* __restrict__ counts) {
    using E = Elem<DIM, PHYS, RULE>;
    using Stage = MeshStage<E::NBT, E::NCQ, Real>;
    constexpr int ROUNDS = (kDedupCap * DIM + 63) / 64;   // staging loads per lane
    __shared__ DedupSlab<DIM> slabs[WPB];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    DedupSlab<DIM>& S = slabs[wave];
    for (int k = lane; k < kDedupSlots; k += 64) S.key[k] = -1;

    const int64_t n_tiles = (n + 63) / 64;
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    const int32_t hi = vertex_hi(nv);
    int ndeg = 0, npoor = 0;
    int64_t tile = t_begin + wave;
    Stage a, b;
    mesh_stage_load<DIM, PHYS, RULE, Real, VEC, false>(a, tile < t_end ? tile * 64 + lane : n, n, conn, u, coef);
    // the two stages alternate roles; one body, called with (a, b) then (b, a)
    auto step = [&](Stage& cur, Stage& nxt) {
        const int64_t e = tile * 64 + lane;
        int32_t vi[DIM + 1];
#pragma unroll
        for (int k = 0; k <= DIM; ++k) vi[k] = min(max(cur.v[k], 0), hi);
        dd_wave_sync();   // the previous tile's slots are clear
        int slot[DIM + 1];
        const int distinct = dd_insert<DIM>(S, vi, slot);
        const int staged = min(distinct, kDedupCap);
        dd_wave_sync();
        double xr[ROUNDS];
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int j = lane + 64 * r;
            xr[r] = 0.0;
            if (j < staged * DIM) {
                const int d = j / DIM;
                xr[r] = X[(int64_t)S.ids[d] * DIM + (j - d * DIM)];
            }
        }
        // keep the gathers ahead of the prefetch, so that waiting for them
        // leaves the prefetched loads in flight
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        const int64_t next = tile + WPB;
        mesh_stage_load<DIM, PHYS, RULE, Real, VEC, false>(nxt, next < t_end ? next * 64 + lane : n, n, conn, u,
                                                           coef);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int j = lane + 64 * r;
            if (j < staged * DIM) S.x[j] = xr[r];
        }
        dd_wave_sync();
        double x[DIM + 1][DIM];
#pragma unroll
        for (int k = 0; k <= DIM; ++k) {
            const int p = slot[k] >= 0 ? (int)S.pos[slot[k]] : (int)kNotStaged;
            if (p != kNotStaged) {
#pragma unroll
                for (int i = 0; i < DIM; ++i) x[k][i] = S.x[p * DIM + i];
            } else {
#pragma unroll
                for (int i = 0; i < DIM; ++i) x[k][i] = X[(int64_t)vi[k] * DIM + i];
            }
        }
        dd_wave_sync();   // every lane has read its slots before they are cleared
#pragma unroll
        for (int k = 0; k <= DIM; ++k)
            if (slot[k] >= 0) S.key[slot[k]] = -1;
        int32_t v0[DIM + 1];
#pragma unroll
        for (int k = 0; k <= DIM; ++k) v0[k] = cur.v[k];
        const bool ok = (e < n) & conn_ok<DIM>(v0, nv);
        mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e < n, e, n, ok, x, cur.u, cur.cf, out, inv_j, det_j,
                                                               ndeg, npoor);
        tile = next;
    };
    while (tile < t_end) {
        step(a, b);
        if (tile >= t_end) break;
        step(b, a);
    }
    add_counts(counts, ndeg, npoor);
}

template <int DIM, int PHYS, int RULE, typename Real, int WPB>
static hipError_t launch_dd_w(const MeshArgs& a, const Launch& l) {
    const Real* u = static_cast<const Real*>(a.u);
    const Real* cf = static_cast<const Real*>(a.coef);
    Real* out = static_cast<Real*>(a.out);
    Real* ij = static_cast<Real*>(a.inv_j);
    Real* dj = static_cast<Real*>(a.det_j);
#define FEMQ_DD(SG, V)                                                                                     \
    hipLaunchKernelGGL((residual_dedup_kernel<DIM, PHYS, RULE, Real, SG, V, WPB>), dim3(l.grid), dim3(l.block), 0, \
                       l.stream, a.n, a.n_vert, a.coords, a.conn, u, cf, out, ij, dj, a.counts)
    // one 16-byte connectivity load per tetrahedron when the array allows it
    if constexpr (DIM == 3) {
        const bool vec = (reinterpret_cast<uintptr_t>(a.conn) % 16) == 0;
        if (ij != nullptr) {
            if (vec) FEMQ_DD(true, true); else FEMQ_DD(true, false);
        } else {
            if (vec) FEMQ_DD(false, true); else FEMQ_DD(false, false);
        }
    } else {
        if (ij != nullptr) FEMQ_DD(true, false); else FEMQ_DD(false, false);
    }
#undef FEMQ_DD
    return hipGetLastError();
}

struct DedupDispatch {
    int dtype;
    const MeshArgs& a;
    const Launch& l;
    template <int D, int P, int S>
    hipError_t operator()() const {
        if (dtype == FEM_F32) return by_waves<D, P, S, float>();
        return by_waves<D, P, S, double>();
    }
    template <int D, int P, int S, typename Real>
    hipError_t by_waves() const {
        switch (l.block) {   // two or four waves per workgroup (the measured best shapes)
        case 128: return launch_dd_w<D, P, S, Real, 2>(a, l);
        case 256: return launch_dd_w<D, P, S, Real, 4>(a, l);
        default: return hipErrorInvalidValue;
        }
    }
};

hipError_t launch_residual_dedup(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                 const Launch& l) {
    const DedupDispatch f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
