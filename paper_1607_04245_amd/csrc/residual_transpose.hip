// residual_transpose.hip -- element residual with the paper's thread
// transposition (Section 3, Fig. 1 and 3): the quadrature phase runs one lane
// per (element, quadrature point, component), the basis phase one lane per
// (element, basis function, component), and the weighted f0/f1 values pass
// between the two phases through LDS, so every output sum is formed by a
// single lane in a fixed order and no cross-lane reduction is needed.
//
// Redesign for gfx950 (wave64, LDS): each wavefront owns a private LDS slab
// and a tile of 64 elements. Only wave-level synchronization is needed, so
// the waves of a workgroup never wait for each other.
//   load phase     lane = element, one coalesced word per SoA row -> LDS
//   quadrature     item (e, q, c), e-major over the tile; reads geometry,
//                  closure and its coefficient from LDS, evaluates f0/f1 at
//                  point q, weights by w_q |det J| and pulls f1 back to
//                  reference coordinates -> LDS flux tile
//   basis          item (e, b, c); sums over q in order -> LDS
//   store phase    lane = element, one coalesced word per SoA row
// The per-element strides of the flux and output tiles are odd so that the
// lanes of a half-wave hit distinct LDS banks.
#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DIM, int PHYS, int RULE>
struct TTLayout {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    static constexpr int TILE = 64;
    static constexpr int IN_ROWS = E::NG + 1 + E::NBT + E::NCQ;    // [row][TILE]
    static constexpr int OFF_DJ = E::NG, OFF_U = E::NG + 1, OFF_CF = E::NG + 1 + E::NBT;
    static constexpr int NFX = (P::HAS_F1 ? DIM : 0) + (P::HAS_F0 ? 1 : 0);  // per (q, c)
    static constexpr int FX_WORDS = E::NQ * E::NC * NFX;
    static constexpr int FX_STRIDE = FX_WORDS | 1;                  // per element, odd
    static constexpr int OUT_STRIDE = E::NBT | 1;                   // per element, odd
    static constexpr int WAVE_WORDS = IN_ROWS * TILE + FX_STRIDE * TILE;
    static_assert(OUT_STRIDE * TILE <= IN_ROWS * TILE, "output tile aliases the input tile");
};

template <int DIM, int PHYS, int RULE, typename Real>
__global__ void __launch_bounds__(512)
residual_transpose_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                          const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    using L = TTLayout<DIM, PHYS, RULE>;
    constexpr int T = L::TILE, NC = E::NC, NQ = E::NQ, NB = E::NB;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    Real* in_s = reinterpret_cast<Real*>(smem_raw) + (size_t)wave * L::WAVE_WORDS;
    Real* fx_s = in_s + L::IN_ROWS * T;
    Real* out_s = in_s;  // the input tile is dead after the quadrature phase

    const int64_t n_tiles = (n + T - 1) / T;
    for (int64_t tile = (int64_t)blockIdx.x * waves + wave; tile < n_tiles; tile += (int64_t)gridDim.x * waves) {
        const int64_t e0 = tile * T;
        const int64_t e = e0 + lane;
        const bool valid = e < n;

        // ---- load phase: coalesced rows into the wave's LDS slab
#pragma unroll
        for (int f = 0; f < E::NG; ++f) in_s[f * T + lane] = valid ? inv_j[f * n + e] : Real(0);
        in_s[L::OFF_DJ * T + lane] = valid ? det_j[e] : Real(0);
#pragma unroll
        for (int f = 0; f < E::NBT; ++f) in_s[(L::OFF_U + f) * T + lane] = valid ? u[f * n + e] : Real(0);
#pragma unroll
        for (int f = 0; f < E::NCQ; ++f) in_s[(L::OFF_CF + f) * T + lane] = valid ? coef[f * n + e] : Real(0);
        wave_sync();

        // ---- quadrature phase: one item per (element, point, component)
#pragma unroll
        for (int k = 0; k < NQ * NC; ++k) {
            const int it = k * T + lane;
            const int el = it / (NQ * NC);
            const int qc = it - el * (NQ * NC);
            const int q = qc / NC, c = qc - q * NC;
            Real ij[E::NG], uu[E::NBT], a[E::NCOEF];
#pragma unroll
            for (int f = 0; f < E::NG; ++f) ij[f] = in_s[f * T + el];
            const Real dj = in_s[L::OFF_DJ * T + el];
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) uu[f] = in_s[(L::OFF_U + f) * T + el];
            Real cfl[E::NCQ];
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) cfl[f] = in_s[(L::OFF_CF + f) * T + el];
#pragma unroll
            for (int m = 0; m < E::NCOEF; ++m) a[m] = coef_at<DIM, PHYS, RULE, Real>(cfl, m, q);
            Real g[NC][DIM];
            physical_gradient<DIM, NC>(ij, uu, g);
            Real uq[NC];
            if constexpr (P::NEEDS_U) {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    // phi_b at point q: LA at vertex q, LB elsewhere
                    Real v = Real(0);
#pragma unroll
                    for (int b = 0; b < NB; ++b) v = fmadd(b == q ? Real(Q::LA) : Real(Q::LB), uu[b * NC + cc], v);
                    uq[cc] = v;
                }
            }
            Real f0[NC], f1[NC][DIM];
            P::template point<DIM, Real>(uq, g, a, f0, f1);
            const Real s = Real(Q::W) * fabs(dj);
            Real* fx = fx_s + el * L::FX_STRIDE + qc * L::NFX;
            if constexpr (P::HAS_F1) {
                Real t[DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i) t[i] = s * f1[c][i];
#pragma unroll
                for (int kk = 0; kk < DIM; ++kk) {
                    Real fh = ij[kk * DIM + 0] * t[0];
#pragma unroll
                    for (int i = 1; i < DIM; ++i) fh = fmadd(ij[kk * DIM + i], t[i], fh);
                    fx[kk] = fh;
                }
            }
            if constexpr (P::HAS_F0) fx[L::NFX - 1] = s * f0[c];
        }
        wave_sync();

        // ---- basis phase: one item per (element, basis function, component)
#pragma unroll
        for (int k = 0; k < E::NBT; ++k) {
            const int it = k * T + lane;
            const int el = it / E::NBT;
            const int bc = it - el * E::NBT;
            const int b = bc / NC, c = bc - b * NC;
            const Real* fx = fx_s + el * L::FX_STRIDE;
            Real r = Real(0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const Real* f = fx + (q * NC + c) * L::NFX;
                if constexpr (P::HAS_F1) {
                    if (b > 0) {
                        r += f[b - 1];
                    } else {
                        Real sum = f[0];
#pragma unroll
                        for (int kk = 1; kk < DIM; ++kk) sum += f[kk];
                        r -= sum;
                    }
                }
                if constexpr (P::HAS_F0) r = fmadd(b == q ? Real(Q::LA) : Real(Q::LB), f[L::NFX - 1], r);
            }
            out_s[el * L::OUT_STRIDE + bc] = r;
        }
        wave_sync();

        // ---- store phase: coalesced rows
        if (valid) {
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) out[f * n + e] = out_s[lane * L::OUT_STRIDE + f];
        }
        wave_sync();  // the next tile's loads overwrite the slab
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
static size_t tt_bytes_per_wave() {
    return (size_t)TTLayout<DIM, PHYS, RULE>::WAVE_WORDS * sizeof(Real);
}

constexpr size_t kMaxLdsPerBlock = 64 * 1024;

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_tt(const ResidualArgs& a, const Launch& l) {
    const size_t lds = (size_t)(l.block / 64) * tt_bytes_per_wave<DIM, PHYS, RULE, Real>();
    if (lds > kMaxLdsPerBlock || l.block % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((residual_transpose_kernel<DIM, PHYS, RULE, Real>), dim3(l.grid), dim3(l.block), lds,
                       l.stream, a.n, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

// Dispatch helper: calls f.template operator()<DIM, PHYS, SCHEME, Real>() for a
// runtime combination; returns fallback for an unknown one.
template <typename F, typename R>
struct TTByType {
    const F& f;
    int dtype;
    template <int D, int P, int S>
    R operator()() const {
        return dtype == FEM_F32 ? f.template operator()<D, P, S, float>() : f.template operator()<D, P, S, double>();
    }
};

template <typename F, typename R>
static R tt_dispatch(int dim, int phys, int rule, int space, int dtype, const F& f, R fallback) {
    const TTByType<F, R> g{f, dtype};
    return dispatch_element(dim, phys, rule, space, g, fallback);
}

struct TTLaunch {
    const ResidualArgs& a;
    const Launch& l;
    template <int D, int P, int RU, typename Real>
    hipError_t operator()() const { return launch_tt<D, P, RU, Real>(a, l); }
};

struct TTBytes {
    template <int D, int P, int RU, typename Real>
    size_t operator()() const { return tt_bytes_per_wave<D, P, RU, Real>(); }
};

hipError_t launch_residual_transpose(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                     const Launch& l) {
    return tt_dispatch(dim, phys, rule, space, dtype, TTLaunch{a, l}, hipErrorInvalidValue);
}

int transpose_block_threads(int dim, int phys, int rule, int space, int dtype, int waves_per_block) {
    const size_t per_wave = tt_dispatch(dim, phys, rule, space, dtype, TTBytes{}, (size_t)0);
    if (per_wave == 0) return 0;
    int w = waves_per_block;
    while (w > 1 && (size_t)w * per_wave > kMaxLdsPerBlock) w >>= 1;
    return (size_t)w * per_wave <= kMaxLdsPerBlock ? 64 * w : 0;
}

}  // namespace femq
