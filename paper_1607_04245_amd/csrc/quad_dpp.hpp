// quad_dpp.hpp -- broadcasts within a quad of lanes (lanes 4k .. 4k+3) by DPP
// quad permutations: no LDS, one move per 32-bit word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace femq {

// Value of lane (quad base + K) in every lane of the quad.
template <int K>
__device__ __forceinline__ float quad_bcast(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), K * 0x55, 0xF, 0xF, false));
}
template <int K>
__device__ __forceinline__ double quad_bcast(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, K * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), K * 0x55, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Every lane of the quad receives the values x of lanes 0..N-1 in out[0..N-1].
template <int N, typename Real, int M>
__device__ __forceinline__ void quad_gather(Real x, Real (&out)[M]) {
    static_assert(N <= M && N <= 4, "at most the quad's four lanes");
    if constexpr (N > 0) out[0] = quad_bcast<0>(x);
    if constexpr (N > 1) out[1] = quad_bcast<1>(x);
    if constexpr (N > 2) out[2] = quad_bcast<2>(x);
    if constexpr (N > 3) out[3] = quad_bcast<3>(x);
}

}  // namespace femq
