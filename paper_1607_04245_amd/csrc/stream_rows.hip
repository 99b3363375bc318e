// stream_rows.hip -- the structure-of-arrays streaming yardstick.
//
// A kernel that reads its element data as R rows of n words and writes R'
// rows streams at a rate that depends on how many rows are in flight, not
// only on the byte count: the rows are separate address streams. This
// kernel has exactly that row structure and no arithmetic beyond a sum that
// keeps every load live, so it measures the rate any element kernel with
// the same rows can reach. One lane per column.
#include "fem_internal.hpp"

namespace femq {

// Every row of a chunk is requested before any is summed, so a lane has up
// to CHUNK loads in flight; CHUNK is the smallest of 16, 32, 64 and 128 that
// covers the rows (more rows run as successive chunks of 128).
template <typename T, int CHUNK>
__global__ void __launch_bounds__(256)
stream_rows_kernel(int64_t n, int n_in, int n_out, const T* __restrict__ src, T* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        T s = T(0);
        for (int r0 = 0; r0 < n_in; r0 += CHUNK) {
            T v[CHUNK];
#pragma unroll
            for (int k = 0; k < CHUNK; ++k)
                v[k] = r0 + k < n_in ? __builtin_nontemporal_load(src + (int64_t)(r0 + k) * n + e) : T(0);
#pragma unroll
            for (int k = 0; k < CHUNK; ++k) s += v[k];
        }
        for (int w = 0; w < n_out; ++w) __builtin_nontemporal_store(s + T(w), dst + (int64_t)w * n + e);
    }
}

template <typename T>
static hipError_t launch_rows(int64_t n, int n_in, int n_out, const void* src, void* dst, const Launch& l) {
    const T* s = static_cast<const T*>(src);
    T* d = static_cast<T*>(dst);
    if (n_in <= 16)
        hipLaunchKernelGGL((stream_rows_kernel<T, 16>), dim3(l.grid), dim3(l.block), 0, l.stream, n, n_in, n_out, s, d);
    else if (n_in <= 32)
        hipLaunchKernelGGL((stream_rows_kernel<T, 32>), dim3(l.grid), dim3(l.block), 0, l.stream, n, n_in, n_out, s, d);
    else if (n_in <= 64)
        hipLaunchKernelGGL((stream_rows_kernel<T, 64>), dim3(l.grid), dim3(l.block), 0, l.stream, n, n_in, n_out, s, d);
    else
        hipLaunchKernelGGL((stream_rows_kernel<T, 128>), dim3(l.grid), dim3(l.block), 0, l.stream, n, n_in, n_out, s, d);
    return hipGetLastError();
}

hipError_t launch_stream_rows(int dtype, int64_t n, int n_in, int n_out, const void* src, void* dst,
                              const Launch& l) {
    if (dtype == FEM_F32) return launch_rows<float>(n, n_in, n_out, src, dst, l);
    if (dtype == FEM_F64) return launch_rows<double>(n, n_in, n_out, src, dst, l);
    return hipErrorInvalidValue;
}

}  // namespace femq
