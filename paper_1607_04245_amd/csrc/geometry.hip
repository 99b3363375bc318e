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

// Poor shape: |det J| below this fraction of the product of edge lengths.
constexpr double kPoorShape = 1e-3;

template <int DIM, typename Out, bool VEC_CONN>
__global__ void __launch_bounds__(512)
geometry_kernel(int64_t n, int64_t nv, const double* __restrict__ X, const int32_t* __restrict__ conn,
                Out* __restrict__ inv_j, Out* __restrict__ det_j, int32_t* __restrict__ counts) {
    int ndeg = 0, npoor = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        int32_t v[DIM + 1];
        if constexpr (VEC_CONN && DIM == 3) {
            typedef int32_t I4 __attribute__((ext_vector_type(4)));
            const I4 c = __builtin_nontemporal_load(reinterpret_cast<const I4*>(conn + e * 4));
            v[0] = c[0]; v[1] = c[1]; v[2] = c[2]; v[3] = c[3];
        } else {
#pragma unroll
            for (int b = 0; b <= DIM; ++b) v[b] = conn[e * (DIM + 1) + b];
        }
        bool ok = true;
#pragma unroll
        for (int b = 0; b <= DIM; ++b) ok = ok && v[b] >= 0 && (int64_t)v[b] < nv;
        double x[DIM + 1][DIM];
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            const int64_t vi = ok ? (int64_t)v[b] : 0;  // never read outside coords
#pragma unroll
            for (int i = 0; i < DIM; ++i) x[b][i] = X[vi * DIM + i];
        }
        double J[DIM][DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int k = 0; k < DIM; ++k) J[i][k] = x[k + 1][i] - x[0][i];
        double det, inv[DIM][DIM];
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double r = 1.0 / det;
            inv[0][0] = J[1][1] * r;
            inv[0][1] = -J[0][1] * r;
            inv[1][0] = -J[1][0] * r;
            inv[1][1] = J[0][0] * r;
        } else {
            // cofactors C[i][k]; J^{-1}[k][i] = C[i][k] / det
            double C[3][3];
            C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
            const double r = 1.0 / det;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int i = 0; i < 3; ++i) inv[k][i] = C[i][k] * r;
        }
        const bool degenerate = !ok || det == 0.0 || !isfinite(det);
        if (degenerate) {
            const double nan = __builtin_nan("");
            if (!ok) det = nan;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
#pragma unroll
                for (int i = 0; i < DIM; ++i) inv[k][i] = nan;
            ++ndeg;
        } else {
            double len = 1.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) s += J[i][k] * J[i][k];
                len *= sqrt(s);
            }
            if (fabs(det) < kPoorShape * len) ++npoor;
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int i = 0; i < DIM; ++i) inv_j[(int64_t)(k * DIM + i) * n + e] = static_cast<Out>(inv[k][i]);
        det_j[e] = static_cast<Out>(det);
    }
    if (counts != nullptr) {
        // wave-level sums (every lane of the wave is active here), one atomic per wave
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            ndeg += __shfl_xor(ndeg, off, 64);
            npoor += __shfl_xor(npoor, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            if (ndeg) atomicAdd(&counts[0], ndeg);
            if (npoor) atomicAdd(&counts[1], npoor);
        }
    }
}

template <int DIM, typename Out>
static hipError_t launch_d(int64_t n, int64_t nv, const double* X, const int32_t* conn, void* ij, void* dj,
                           int32_t* counts, const Launch& l) {
    const bool vec = DIM == 3 && (reinterpret_cast<uintptr_t>(conn) % 16) == 0;
    if (vec)
        hipLaunchKernelGGL((geometry_kernel<DIM, Out, true>), dim3(l.grid), dim3(l.block), 0, l.stream, n, nv, X,
                           conn, static_cast<Out*>(ij), static_cast<Out*>(dj), counts);
    else
        hipLaunchKernelGGL((geometry_kernel<DIM, Out, false>), dim3(l.grid), dim3(l.block), 0, l.stream, n, nv,
                           X, conn, static_cast<Out*>(ij), static_cast<Out*>(dj), counts);
    return hipGetLastError();
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
