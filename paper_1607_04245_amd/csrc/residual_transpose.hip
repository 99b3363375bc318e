// residual_transpose.hip -- element residuals with the paper's thread
// transposition (Section 3, Fig. 1 and 3): the quadrature phase runs one lane
// per (element, quadrature point), the basis phase one lane per (element,
// basis function, component), and the weighted, pulled-back f0/f1
// values pass from the first phase to the second, so every output sum is
// formed by a single lane in a fixed order and no reduction is needed.
//
// Two exchanges, two kernels:
//
// LDS (FEM_STRATEGY_TRANSPOSE, every P1 combination). Each wavefront owns a
// private LDS slab and a tile of 64 elements; only wave-level
// synchronization is needed, so the waves of a workgroup never wait for
// each other.
//   load phase     lane = element, one coalesced word per SoA row; the lane
//                  forms what every point of its element shares (the
//                  physical gradient of u, the weighted measure w |det J|)
//                  and stages it with J^{-1} and the coefficient words
//   quadrature     item (e, q), e-major over the tile: f0/f1 at point q
//                  from the staged words (every component: the stress of
//                  elasticity couples them), weighted and pulled back to
//                  reference coordinates -> flux tile
//   basis          item (e, b, c): sums over q in order -> output tile
//   store phase    lane = element, one coalesced word per SoA row
// The next tile's rows are requested before the current tile's LDS phases,
// so a wave waits for memory only when it runs ahead of the stream.
// Per-element strides of the flux and output tiles are odd, so the lanes of
// a half-wave hit distinct LDS banks. The slab size per workgroup is checked
// against the device's LDS per workgroup.
//
// Cross-lane (FEM_STRATEGY_SHUFFLE, scalar fields: Laplacian and mass, any
// P1 rule). Four consecutive lanes (a quad) share an element, lane r of the
// quad being point r in the quadrature phase and basis function r in the
// basis phase (N_q, N_b <= 4). Each lane loads a quarter of its element's
// geometry words, its own closure value and its own point's coefficient;
// quad broadcasts (DPP quad permutations, no LDS) give every lane the shared
// words, and after the quadrature phase they give basis lane b the pulled-
// back flux of every point, which it sums in point order.
#include "fem_device.hpp"
#include "fem_internal.hpp"
#include "quad_dpp.hpp"

namespace femq {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------- LDS --

template <int DIM, int PHYS, int RULE>
struct TTLayout {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    static constexpr int TILE = 64;
    // staged per element, [word][TILE]
    static constexpr int N_IJ = P::HAS_F1 ? E::NG : 0;          // J^{-1} for the pull-back
    static constexpr int N_GRAD = P::HAS_F1 ? E::NC * DIM : 0;  // physical gradient g[c][i]
    static constexpr int N_U = P::NEEDS_U ? E::NBT : 0;         // nodal values for f0
    static constexpr int OFF_IJ = 0, OFF_S = N_IJ, OFF_G = OFF_S + 1, OFF_U = OFF_G + N_GRAD,
                         OFF_CF = OFF_U + N_U;
    static constexpr int IN_ROWS = OFF_CF + E::NCQ;
    // per (q, c): the pulled-back flux (DIM words) and their sum, then the
    // weighted f0
    static constexpr int NFX = (P::HAS_F1 ? DIM + 1 : 0) + (P::HAS_F0 ? 1 : 0);
    static constexpr int OUT_STRIDE = E::NBT | 1;                   // per element, odd
    // Vector fields on a four-point rule: the four point items of an element
    // are the four lanes of a quad, which sum the pulled-back flux over the
    // points by quad broadcasts (each lane the same sums, in point order) and
    // write the element vector straight to the output tile; no flux tile,
    // no basis phase. The output tile then takes the flux tile's place (the
    // staged words are still being read while it is written).
    static constexpr bool QUAD_SUM = E::NQ == 4 && E::NC > 1 && P::HAS_F1 && !P::HAS_F0;
    static constexpr int FX_WORDS = E::NQ * E::NC * NFX;
    static constexpr int FX_STRIDE = QUAD_SUM ? OUT_STRIDE : (FX_WORDS | 1);  // per element, odd
    static constexpr int WAVE_WORDS = IN_ROWS * TILE + FX_STRIDE * TILE;
    static_assert(OUT_STRIDE <= IN_ROWS, "the output tile reuses the staged words");
};

// The per-element words of one tile: what the load phase reads.
template <int DIM, int PHYS, int RULE, typename Real>
struct TTStage {
    using E = Elem<DIM, PHYS, RULE>;
    Real ij[E::NG], dj, uu[E::NBT], cf[E::NCQ];
};

// Requests the words of element e without a condition: an index past the end
// is clamped to the last element (n >= 1), whose data then fills the unused
// slots of the tail tile and is never stored.
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void tt_load(TTStage<DIM, PHYS, RULE, Real>& st, int64_t e, int64_t n,
                                        const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                                        const Real* __restrict__ u, const Real* __restrict__ coef) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t ec = e < n ? e : n - 1;
#pragma unroll
    for (int f = 0; f < E::NG; ++f) st.ij[f] = __builtin_nontemporal_load(inv_j + f * n + ec);
    st.dj = __builtin_nontemporal_load(det_j + ec);
#pragma unroll
    for (int f = 0; f < E::NBT; ++f) st.uu[f] = __builtin_nontemporal_load(u + f * n + ec);
#pragma unroll
    for (int f = 0; f < E::NCQ; ++f) st.cf[f] = __builtin_nontemporal_load(coef + f * n + ec);
}

// Quadrature phase of one tile: item (element, point), e-major over the
// tile; the item evaluates f0/f1 at its point once and writes the record of
// every component. It reads only the staged words and writes only the flux
// tile (restrict: the compiler may overlap one item's reads with another's
// arithmetic and stores).
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void tt_quadrature(const Real* __restrict__ in_s, Real* __restrict__ fx_s, int lane) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    using L = TTLayout<DIM, PHYS, RULE>;
    constexpr int T = L::TILE, NC = E::NC, NQ = E::NQ, NB = E::NB;
    // scalar fields: every item unrolled (their LDS reads overlap); vector
    // fields: one item at a time (an item holds the whole stress tensor)
    constexpr int UNROLL = NC > 1 ? 1 : NQ;
#pragma unroll UNROLL
    for (int k = 0; k < NQ; ++k) {
        const int it = k * T + lane;
        const int el = it / NQ;
        const int q = it - el * NQ;
        Real a[E::NCOEF];
        if constexpr (E::SPACE == FEM_COEF_QUAD) {
            // the item's own point: one staged word per coefficient
#pragma unroll
            for (int m = 0; m < E::NCOEF; ++m) a[m] = in_s[(L::OFF_CF + m * E::NW + q) * T + el];
        } else {
            Real cfl[E::NCQ];
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) cfl[f] = in_s[(L::OFF_CF + f) * T + el];
#pragma unroll
            for (int m = 0; m < E::NCOEF; ++m) a[m] = coef_at<DIM, PHYS, RULE, Real>(cfl, m, q);
        }
        Real g[NC][DIM];
        if constexpr (P::HAS_F1) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                for (int i = 0; i < DIM; ++i) g[cc][i] = in_s[(L::OFF_G + cc * DIM + i) * T + el];
        }
        Real uq[NC];
        if constexpr (P::NEEDS_U) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                // phi_b at point q: LA at vertex q, LB elsewhere
                Real v = Real(0);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    v = fmadd(b == q ? Real(Q::LA) : Real(Q::LB), in_s[(L::OFF_U + b * NC + cc) * T + el], v);
                uq[cc] = v;
            }
        }
        Real f0[NC], f1[NC][DIM];
        P::template point<DIM, Real>(uq, g, a, f0, f1);
        const Real s = in_s[L::OFF_S * T + el];
        Real ij[P::HAS_F1 ? E::NG : 1];
        if constexpr (P::HAS_F1) {
#pragma unroll
            for (int f = 0; f < E::NG; ++f) ij[f] = in_s[(L::OFF_IJ + f) * T + el];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            [[maybe_unused]] Real* fx = fx_s + el * L::FX_STRIDE + (q * NC + c) * L::NFX;
            if constexpr (P::HAS_F1) {
                Real t[DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i) t[i] = s * f1[c][i];
                Real fh[DIM];
#pragma unroll
                for (int kk = 0; kk < DIM; ++kk) {
                    fh[kk] = ij[kk * DIM] * t[0];
#pragma unroll
                    for (int i = 1; i < DIM; ++i) fh[kk] = fmadd(ij[kk * DIM + i], t[i], fh[kk]);
                    if constexpr (!L::QUAD_SUM) fx[kk] = fh[kk];
                }
                // the vertex at the origin takes minus the sum (its reference
                // gradient is -(1, ..., 1)): formed once here, not by every
                // basis lane
                Real sum = fh[0];
#pragma unroll
                for (int kk = 1; kk < DIM; ++kk) sum += fh[kk];
                if constexpr (L::QUAD_SUM) {
                    // R_{b,c} = sum over the points, in point order, of entry
                    // b - 1 (b > 0) or minus the sum (b = 0): the basis
                    // phase's arithmetic, on values gathered from the quad
                    Real rb[DIM + 1];
#pragma unroll
                    for (int j = 0; j <= DIM; ++j) {
                        Real v[4];
                        quad_gather<4>(j < DIM ? fh[j] : sum, v);
                        Real r = Real(0);
#pragma unroll
                        for (int qq = 0; qq < 4; ++qq) r = j < DIM ? r + v[qq] : r - v[qq];
                        rb[j < DIM ? j + 1 : 0] = r;
                    }
                    // lane q of the quad stores basis function q
                    Real mine = rb[0];
#pragma unroll
                    for (int b = 1; b <= DIM; ++b) mine = q == b ? rb[b] : mine;
                    fx_s[el * L::OUT_STRIDE + q * NC + c] = mine;
                } else {
                    fx[DIM] = sum;
                }
            }
            if constexpr (P::HAS_F0) fx[L::NFX - 1] = s * f0[c];
        }
    }
}

// Basis phase of one tile: item (element, basis function, component), the
// sum over the points in order. Reads only the flux tile, writes only the
// output tile.
template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void tt_basis(const Real* __restrict__ fx_s, Real* __restrict__ out_s, int lane) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    using L = TTLayout<DIM, PHYS, RULE>;
    constexpr int T = L::TILE, NC = E::NC, NQ = E::NQ;
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
                // the pulled-back flux dotted with the reference gradient
                // of phi_b: entry b - 1, or minus the stored sum for the
                // vertex at the origin (one word per lane, no branch: b
                // differs between the lanes of a wave)
                const Real fb = f[b > 0 ? b - 1 : DIM];
                r = b > 0 ? r + fb : r - fb;
            }
            if constexpr (P::HAS_F0) r = fmadd(b == q ? Real(Q::LA) : Real(Q::LB), f[L::NFX - 1], r);
        }
        out_s[el * L::OUT_STRIDE + bc] = r;
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
__global__ void __launch_bounds__(512)
residual_transpose_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                          const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    using L = TTLayout<DIM, PHYS, RULE>;
    constexpr int T = L::TILE, NC = E::NC;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    Real* in_s = reinterpret_cast<Real*>(smem_raw) + (size_t)wave * L::WAVE_WORDS;
    Real* fx_s = in_s + L::IN_ROWS * T;
    // the staged words are dead after the quadrature phase, unless the
    // quadrature phase writes the element vectors itself
    Real* out_s = L::QUAD_SUM ? fx_s : in_s;

    const int64_t n_tiles = (n + T - 1) / T;
    const int64_t step = (int64_t)gridDim.x * waves;
    int64_t tile = (int64_t)blockIdx.x * waves + wave;
    // software pipeline: the next tile's words are in flight while this tile
    // goes through its LDS phases
    TTStage<DIM, PHYS, RULE, Real> nxt;
    if (tile < n_tiles) tt_load<DIM, PHYS, RULE, Real>(nxt, tile * T + lane, n, inv_j, det_j, u, coef);
    for (; tile < n_tiles; tile += step) {
        const int64_t e0 = tile * T;
        const int64_t e = e0 + lane;
        const bool valid = e < n;
        const TTStage<DIM, PHYS, RULE, Real> cur = nxt;
        if (tile + step < n_tiles)
            tt_load<DIM, PHYS, RULE, Real>(nxt, (tile + step) * T + lane, n, inv_j, det_j, u, coef);

        // ---- load phase: coalesced rows; per-element shared quantities
        {
            in_s[L::OFF_S * T + lane] = Real(Q::W) * fabs(cur.dj);
            if constexpr (P::HAS_F1) {
                Real g[NC][DIM];
                physical_gradient<DIM, NC>(cur.ij, cur.uu, g);
#pragma unroll
                for (int f = 0; f < E::NG; ++f) in_s[(L::OFF_IJ + f) * T + lane] = cur.ij[f];
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int i = 0; i < DIM; ++i) in_s[(L::OFF_G + c * DIM + i) * T + lane] = g[c][i];
            }
            if constexpr (P::NEEDS_U) {
#pragma unroll
                for (int f = 0; f < E::NBT; ++f) in_s[(L::OFF_U + f) * T + lane] = cur.uu[f];
            }
#pragma unroll
            for (int f = 0; f < E::NCQ; ++f) in_s[(L::OFF_CF + f) * T + lane] = cur.cf[f];
        }
        wave_sync();

        // ---- quadrature phase: one item per (element, point)
        tt_quadrature<DIM, PHYS, RULE, Real>(in_s, fx_s, lane);
        wave_sync();

        // ---- basis phase: one item per (element, basis function, component)
        if constexpr (!L::QUAD_SUM) {
            tt_basis<DIM, PHYS, RULE, Real>(fx_s, out_s, lane);
            wave_sync();
        }

        // ---- store phase: coalesced rows
        if (valid) {
#pragma unroll
            for (int f = 0; f < E::NBT; ++f) out[f * n + e] = out_s[lane * L::OUT_STRIDE + f];
        }
        wave_sync();  // the next tile's staging overwrites the slab
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
static size_t tt_bytes_per_wave() {
    return (size_t)TTLayout<DIM, PHYS, RULE>::WAVE_WORDS * sizeof(Real);
}

// LDS a workgroup may use on the current device (read once per device).
static size_t lds_per_block() {
    static size_t cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cached[dev] = (size_t)v;
    }
    return cached[dev];
}

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_tt(const ResidualArgs& a, const Launch& l) {
    const size_t lds = (size_t)(l.block / 64) * tt_bytes_per_wave<DIM, PHYS, RULE, Real>();
    if (lds > lds_per_block() || l.block % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((residual_transpose_kernel<DIM, PHYS, RULE, Real>), dim3(l.grid), dim3(l.block), lds,
                       l.stream, a.n, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                       static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef), static_cast<Real*>(a.out));
    return hipGetLastError();
}

// ----------------------------------------------------------- cross-lane --

template <int DIM, int PHYS, int RULE, typename Real>
__global__ void __launch_bounds__(512)
residual_shuffle_kernel(int64_t n, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                        const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    using E = Elem<DIM, PHYS, RULE>;
    using P = Physics<PHYS>;
    using Q = Rule<DIM, RULE>;
    constexpr int NQ = E::NQ, NB = E::NB, NG = E::NG, NW = E::NW;
    static_assert(E::NC == 1 && NQ <= 4 && NB <= 4, "one scalar field, at most four points and basis functions");
    constexpr int NGEO = NG + 1;                 // J^{-1} words and det J
    constexpr int GEO_PER_LANE = (NGEO + 3) / 4; // geometry words loaded per lane

    const int lane = threadIdx.x & 63, r = lane & 3;
    const int64_t n_groups = (n + 15) >> 4;     // 16 elements per wave
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); grp < n_groups; grp += waves) {
        const int64_t e = grp * 16 + (lane >> 2);
        const bool valid = e < n;
        const int64_t ec = valid ? e : n - 1;
        // ---- loads: a quarter of the geometry, the own closure value, the
        // coefficient words of the own point (or the shared ones)
        Real geo[GEO_PER_LANE];
#pragma unroll
        for (int t = 0; t < GEO_PER_LANE; ++t) {
            const int w = r + 4 * t;
            const Real* p = w < NG ? inv_j + (int64_t)w * n : det_j;
            geo[t] = w <= NG ? __builtin_nontemporal_load(p + ec) : Real(0);
        }
        const Real ur = r < NB ? __builtin_nontemporal_load(u + (int64_t)(r < NB ? r : 0) * n + ec) : Real(0);
        Real cw = Real(0);
        if constexpr (E::SPACE == FEM_COEF_P0) {
            cw = __builtin_nontemporal_load(coef + ec);
        } else {
            constexpr int NCW = E::SPACE == FEM_COEF_QUAD ? NQ : NW;
            cw = r < NCW ? __builtin_nontemporal_load(coef + (int64_t)(r < NCW ? r : 0) * n + ec) : Real(0);
        }

        // ---- quad broadcasts: every lane gets the element's shared words
        Real ij[NG], dj;
        {
            Real g0[4], g1[4], g2[4];
            quad_gather<4>(geo[0], g0);
            if constexpr (GEO_PER_LANE > 1) quad_gather<4>(geo[1], g1);
            if constexpr (GEO_PER_LANE > 2) quad_gather<4>(geo[2], g2);
#pragma unroll
            for (int w = 0; w <= NG; ++w) {
                const Real x = w < 4 ? g0[w] : (w < 8 ? g1[w - 4] : g2[w - 8]);
                if (w < NG) ij[w] = x; else dj = x;
            }
        }
        Real ub[4];
        quad_gather<NB>(ur, ub);
        const Real s = Real(Q::W) * fabs(dj);

        // ---- quadrature phase: lane r is point r
        Real a;
        if constexpr (E::SPACE == FEM_COEF_P1) {
            Real av[4];
            quad_gather<NB>(cw, av);
            // the P1 interpolant at this lane's point: LA at vertex r, LB elsewhere
            a = Real(0);
#pragma unroll
            for (int b = 0; b < NB; ++b) a = fmadd(b == r ? Real(Q::LA) : Real(Q::LB), av[b], a);
        } else {
            a = cw;
        }
        Real fx[DIM + 1];   // pulled-back weighted f1, then weighted f0
        if constexpr (P::HAS_F1) {
            Real g[1][DIM];
            physical_gradient<DIM, 1>(ij, ub, g);
            Real uq[1], f0[1], f1[1][DIM], am[1] = {a};
            P::template point<DIM, Real>(uq, g, am, f0, f1);
            Real t[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) t[i] = s * f1[0][i];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                Real fh = ij[k * DIM] * t[0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) fh = fmadd(ij[k * DIM + i], t[i], fh);
                fx[k] = fh;
            }
        }
        if constexpr (P::HAS_F0) {
            Real uq = Real(0);
#pragma unroll
            for (int b = 0; b < NB; ++b) uq = fmadd(b == r ? Real(Q::LA) : Real(Q::LB), ub[b], uq);
            Real f0[1], f1[1][DIM], am[1] = {a}, uqa[1] = {uq}, g[1][DIM];
            P::template point<DIM, Real>(uqa, g, am, f0, f1);
            fx[DIM] = s * f0[0];
        }

        // ---- basis phase: lane r is basis function r; the points' values
        // come from the quad's lanes, summed in point order
        Real res = Real(0);
        if constexpr (P::HAS_F1) {
            Real fq[DIM][4];
#pragma unroll
            for (int k = 0; k < DIM; ++k) quad_gather<NQ>(fx[k], fq[k]);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                Real sum = fq[0][q];
#pragma unroll
                for (int k = 1; k < DIM; ++k) sum += fq[k][q];
                Real pick = fq[0][q];
#pragma unroll
                for (int k = 1; k < DIM; ++k) pick = r == k + 1 ? fq[k][q] : pick;
                res = r == 0 ? res - sum : res + pick;
            }
        }
        if constexpr (P::HAS_F0) {
            Real f0q[4];
            quad_gather<NQ>(fx[DIM], f0q);
#pragma unroll
            for (int q = 0; q < NQ; ++q) res = fmadd(r == q ? Real(Q::LA) : Real(Q::LB), f0q[q], res);
        }
        if (valid && r < NB) __builtin_nontemporal_store(res, out + (int64_t)r * n + e);
    }
}

template <int DIM, int PHYS, int RULE, typename Real>
static hipError_t launch_shuffle(const ResidualArgs& a, const Launch& l) {
    if constexpr (Elem<DIM, PHYS, RULE>::NC != 1) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((residual_shuffle_kernel<DIM, PHYS, RULE, Real>), dim3(l.grid), dim3(l.block), 0,
                           l.stream, a.n, static_cast<const Real*>(a.inv_j), static_cast<const Real*>(a.det_j),
                           static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef),
                           static_cast<Real*>(a.out));
        return hipGetLastError();
    }
}

// ------------------------------------------------------------- dispatch --

// Calls f.template operator()<DIM, PHYS, SCHEME, Real>() for a runtime
// combination; returns fallback for an unknown one.
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

struct ShuffleLaunch {
    const ResidualArgs& a;
    const Launch& l;
    template <int D, int P, int RU, typename Real>
    hipError_t operator()() const { return launch_shuffle<D, P, RU, Real>(a, l); }
};

struct TTBytes {
    template <int D, int P, int RU, typename Real>
    size_t operator()() const { return tt_bytes_per_wave<D, P, RU, Real>(); }
};

hipError_t launch_residual_transpose(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                     const Launch& l) {
    return tt_dispatch(dim, phys, rule, space, dtype, TTLaunch{a, l}, hipErrorInvalidValue);
}

hipError_t launch_residual_shuffle(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                   const Launch& l) {
    if (phys == FEM_ELASTICITY) return hipErrorInvalidValue;
    return tt_dispatch(dim, phys, rule, space, dtype, ShuffleLaunch{a, l}, hipErrorInvalidValue);
}

int transpose_block_threads(int dim, int phys, int rule, int space, int dtype, int waves_per_block) {
    const size_t per_wave = tt_dispatch(dim, phys, rule, space, dtype, TTBytes{}, (size_t)0);
    if (per_wave == 0) return 0;
    const size_t cap = lds_per_block();
    int w = waves_per_block;
    while (w > 1 && (size_t)w * per_wave > cap) w >>= 1;
    return (size_t)w * per_wave <= cap ? 64 * w : 0;
}

}  // namespace femq
