// geometry.hip -- affine element geometry: det J and J^{-1} per element.
//
// The paper's integration kernel reads precomputed Jacobian inverses and
// determinants (Section 3 and the Appendix); this kernel produces them from
// vertex coordinates and connectivity. One lane per element: gather the
// dim+1 vertices (FP64), form J[i][k] = (x_k - x_0)_i, and write det J and
// J^{-1} (row-major) in structure-of-arrays order, so a wavefront writes 64
// consecutive words of every output row. The arithmetic is FP64 for both
// output types, so nearly degenerate elements get an FP64 inverse even when
// the outputs are FP32 (rounded once, at the store).
#include <math.h>

#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

// Each wave owns tiles of 64*EPT consecutive elements; lane l handles
// elements l, l+64, ..., so every load and store instruction of the wave
// covers 64 consecutive elements. Workgroups own contiguous tile ranges laid
// out XCD by XCD (block_tile_range). Connectivity loads are unconditional
// (indices past the end are clamped, their results ignored) and validated
// only after the next loads are issued, so the wave never waits for more
// than it needs. EPT = 1 is software-pipelined: the next tile's connectivity
// is in flight while the current tile's vertices are gathered and processed.
// EPT > 1 gives each lane EPT independent gather chains instead.
template <int DIM, typename Out, int EPT, bool VEC>
__global__ void __launch_bounds__(512)
geometry_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                Out* __restrict__ inv_j, Out* __restrict__ det_j, int32_t* __restrict__ counts) {
    const int lane = threadIdx.x & 63;
    // wave-uniform (readfirstlane): the tile loop is then scalar control flow
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), waves = blockDim.x >> 6;
    const int64_t n_tiles = (n + 64 * EPT - 1) / (64 * EPT);
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    int ndeg = 0, npoor = 0;
    int64_t tile = t_begin + wave;
    auto clamp = [&](int64_t e) { return e < n ? e : n - 1; };
    if constexpr (EPT == 1) {
        int32_t va[DIM + 1], vb[DIM + 1];
        load_conn<DIM, VEC>(conn, clamp(tile < t_end ? tile * 64 + lane : n), va);
        while (tile < t_end) {
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                gather_coords<DIM>(X, va, nv, x);
                const bool ok = (e < n) & conn_ok<DIM>(va, nv);
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                load_conn<DIM, VEC>(conn, clamp(next < t_end ? next * 64 + lane : n), vb);
                geometry_finish<DIM, Out>(e < n, e, n, ok, x, inv_j, det_j, ndeg, npoor);
                tile = next;
            }
            if (tile >= t_end) break;
            {
                const int64_t e = tile * 64 + lane;
                double x[DIM + 1][DIM];
                gather_coords<DIM>(X, vb, nv, x);
                const bool ok = (e < n) & conn_ok<DIM>(vb, nv);
                __asm__ volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const int64_t next = tile + waves;
                load_conn<DIM, VEC>(conn, clamp(next < t_end ? next * 64 + lane : n), va);
                geometry_finish<DIM, Out>(e < n, e, n, ok, x, inv_j, det_j, ndeg, npoor);
                tile = next;
            }
        }
    } else {
        for (; tile < t_end; tile += waves) {
            int64_t e[EPT];
            int32_t v[EPT][DIM + 1];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                e[j] = tile * (64 * EPT) + j * 64 + lane;
                load_conn<DIM, VEC>(conn, clamp(e[j]), v[j]);
            }
            double x[EPT][DIM + 1][DIM];
#pragma unroll
            for (int j = 0; j < EPT; ++j) gather_coords<DIM>(X, v[j], nv, x[j]);
#pragma unroll
            for (int j = 0; j < EPT; ++j)
                geometry_finish<DIM, Out>(e[j] < n, e[j], n, (e[j] < n) & conn_ok<DIM>(v[j], nv), x[j], inv_j, det_j,
                                          ndeg, npoor);
        }
    }
    add_counts(counts, ndeg, npoor);
}

template <int DIM, typename Out, bool VEC>
static hipError_t launch_e(int64_t n, int64_t nv, const double* X, const int32_t* conn, Out* ij, Out* dj,
                           int32_t* counts, const Launch& l) {
    switch (l.vec) {
    case 1:
        hipLaunchKernelGGL((geometry_kernel<DIM, Out, 1, VEC>), dim3(l.grid), dim3(l.block), 0, l.stream, n, nv, X,
                           conn, ij, dj, counts);
        break;
    case 2:
        hipLaunchKernelGGL((geometry_kernel<DIM, Out, 2, VEC>), dim3(l.grid), dim3(l.block), 0, l.stream, n, nv, X,
                           conn, ij, dj, counts);
        break;
    case 4:
        hipLaunchKernelGGL((geometry_kernel<DIM, Out, 4, VEC>), dim3(l.grid), dim3(l.block), 0, l.stream, n, nv, X,
                           conn, ij, dj, counts);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The wide-access variant (one 16-byte connectivity load per tetrahedron)
// needs 16-byte aligned connectivity; torch allocations always are.
template <int DIM, typename Out>
static hipError_t launch_d(int64_t n, int64_t nv, const double* X, const int32_t* conn, void* ij, void* dj,
                           int32_t* counts, const Launch& l) {
    const bool vec = DIM == 3 && (reinterpret_cast<uintptr_t>(conn) % 16) == 0;
    Out* o_ij = static_cast<Out*>(ij);
    Out* o_dj = static_cast<Out*>(dj);
    return vec ? launch_e<DIM, Out, true>(n, nv, X, conn, o_ij, o_dj, counts, l)
               : launch_e<DIM, Out, false>(n, nv, X, conn, o_ij, o_dj, counts, l);
}

hipError_t launch_geometry(int dim, int dtype, int64_t n_elem, int64_t n_vert, const double* coords,
                           const int32_t* conn, void* inv_j, void* det_j, int32_t* counts, const Launch& l) {
    if (dim == 2)
        return dtype == FEM_F32 ? launch_d<2, float>(n_elem, n_vert, coords, conn, inv_j, det_j, counts, l)
                                : launch_d<2, double>(n_elem, n_vert, coords, conn, inv_j, det_j, counts, l);
    if (dim == 3)
        return dtype == FEM_F32 ? launch_d<3, float>(n_elem, n_vert, coords, conn, inv_j, det_j, counts, l)
                                : launch_d<3, double>(n_elem, n_vert, coords, conn, inv_j, det_j, counts, l);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------ stream copy --
// Plain 16-byte streaming copy: the achievable-bandwidth yardstick and the
// calibration kernel for hardware byte counters.
__global__ void __launch_bounds__(512)
stream_copy_kernel(int64_t n16, const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
    typedef int32_t I4 __attribute__((ext_vector_type(4)));
    const I4* s = reinterpret_cast<const I4*>(src);
    I4* d = reinterpret_cast<I4*>(dst);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
    }
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t n_bytes, const Launch& l) {
    hipLaunchKernelGGL(stream_copy_kernel, dim3(l.grid), dim3(l.block), 0, l.stream, n_bytes / 16,
                       static_cast<const int32_t*>(src), static_cast<int32_t*>(dst));
    return hipGetLastError();
}

}  // namespace femq
