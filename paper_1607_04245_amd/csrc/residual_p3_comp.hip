// residual_p3_comp.hip -- P3 tetrahedral elasticity residuals with each
// element's work split over three waves, one per displacement component.
//
// The lane kernel keeps an element's 60 closure words and 60 output sums in
// one lane, which leaves two waves per SIMD in FP32 and one in FP64 to
// overlap the memory stream with the arithmetic. Here a group of three
// waves takes a tile of 64 elements, lane l of wave c holding component c of
// element l: its 20 closure words, its 20 sums and the barycentric
// gradients. Section 3's thread transposition splits an element's work over
// threads by quadrature point and by basis function; for a vector field the
// components split it without any table depending on the thread, so every
// basis value stays a compile-time constant, as in the lane kernel, and
// every access of a wave is one coalesced row of 64 elements.
//
// The quadrature phase: at every point q wave c forms
// U_v = sum_b dphi_b/dlam_v u_{b,c} and G_k = sum_v U_v g_v[(c + k) mod 3],
// the gradient of u_c with its axes rotated so that entry 0 is axis c, and
// writes it to LDS. One barrier, and then the stress phase: row c of the
// stress,
//   f1_ci = lambda tr(grad u) delta_ci + 2 mu (du_c/dx_i + du_i/dx_c) / 2,
// needs three words of the other two waves: their diagonal entries (the
// trace) and, from each, the entry that pairs with one of its own
// (du_i/dx_c). In rotated axes these are the same entries for every wave
// (entry 0 of both, entry 2 of wave c + 1 and entry 1 of wave c + 2), so
// the reads are uniform. The basis phase adds
// dphi_b/dlam_v (g_v . w_q |J| f1_c) to the wave's 20 sums. The closure
// words are dead after the quadrature phase and the sums live only in the
// second, so a lane holds at most one of them with the gradients and
// coefficient values, and a tile takes two barriers (one per phase).
// FP64 runs one group per workgroup (its gradients take 49.5 KB of LDS).
//
// Results agree with the lane kernel to rounding (the trace and the dot
// products g_v . f1_c are summed in rotated order, and the quadrature weight
// scales lambda and mu instead of the flux). Measured against the lane
// kernel with both timed on a warmed-up GPU it is 5-10 % slower: in FP32
// both are bound by the vector arithmetic, of which the split issues about
// 5 % more, and in FP64 three groups per CU (the LDS bound) keep fewer bytes
// in flight than the lane kernel's single wave per SIMD with all its
// element's loads issued at once.
#include "fem_internal.hpp"
#include "p3_device.hpp"

namespace femq {

namespace {

constexpr int kCompMaxGroups = 2;   // three-wave groups per workgroup

// LDS of one three-wave group: every point's rotated gradient of every
// component, [point][component][rotated entry][lane] (a wave's 64 lanes
// read one entry as 64 consecutive words: no bank conflicts).
template <typename Real>
struct CompShared {
    static constexpr int NQ = RuleP2<3, FEM_RULE_TET11>::NQ;
    Real grad[NQ][3][3][64];
};

}  // namespace

int comp_max_groups(int dtype) { return dtype == FEM_F32 ? kCompMaxGroups : 1; }

size_t p3_comp_shared_bytes(int dtype, int groups) {
    return (size_t)groups * (dtype == FEM_F32 ? sizeof(CompShared<float>) : sizeof(CompShared<double>));
}

template <typename Real>
__global__ void __launch_bounds__(192 * kCompMaxGroups)
residual_p3_comp_kernel(int64_t n, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                        const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    constexpr int DIM = 3, RULE = FEM_RULE_TET11;
    using E = ElemP3<DIM, FEM_ELASTICITY, RULE, FEM_COEF_QUAD>;
    using Q = RuleP2<DIM, RULE>;
    using T = P3Basis<DIM, RULE>;
    constexpr int NB = E::NB, NV = E::NV, NQ = E::NQ;
    extern __shared__ __align__(16) unsigned char comp_lds[];
    const int lane = threadIdx.x & 63;
    // wave-uniform (readfirstlane): group, component and the loops below are
    // scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = w / DIM, c = w - DIM * grp;
    const int c1 = c == 2 ? 0 : c + 1;   // (c + 1) mod 3
    const int c2 = c == 0 ? 2 : c - 1;   // (c + 2) mod 3
    const int groups = blockDim.x / (64 * DIM);
    CompShared<Real>& sh = reinterpret_cast<CompShared<Real>*>(comp_lds)[grp];
    const int64_t n_tiles = (n + 63) / 64;
    int64_t t_begin, t_end;
    block_tile_range(n_tiles, t_begin, t_end);
    // every wave of the workgroup runs the same number of rounds (and so of
    // barriers); a group past the range computes a clamped tile and stores
    // nothing
    const int64_t rounds = (t_end - t_begin + groups - 1) / groups;
    const int64_t row_stride = DIM * n;
    for (int64_t rd = 0; rd < rounds; ++rd) {
        const int64_t t = t_begin + rd * groups + grp;
        const int64_t e0 = t * 64 + lane;
        const bool valid = (t < t_end) & (e0 < n);
        const int64_t e = e0 < n ? e0 : n - 1;
        // The three waves read the same geometry and coefficient words (cached
        // loads: the second and third reads hit the CU's cache) and their own
        // closure and output rows (streaming).
        // barycentric gradients g_v, axes rotated: g[v][k] is along axis (c + k) mod 3
        Real g[NV][DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int ax = c + k < DIM ? c + k : c + k - DIM;
#pragma unroll
            for (int v = 1; v < NV; ++v)
                g[v][k] = inv_j[(int64_t)((v - 1) * DIM + ax) * n + e];
            Real s = g[1][k];
            s += g[2][k];
            s += g[3][k];
            g[0][k] = -s;
        }
        const Real adj = fabs(det_j[e]);
        Real uc[NB];
        const Real* ub = u + (int64_t)c * n + e;
#pragma unroll
        for (int b = 0; b < NB; ++b) uc[b] = __builtin_nontemporal_load(ub + b * row_stride);
        Real aq[E::NCQ];
        p3_coef_points<DIM, FEM_ELASTICITY, RULE, Real, false>(space, coef, n, e, aq);
        // every wave has finished reading the previous tile's gradients
        __syncthreads();
        // quadrature phase: the gradient of u_c at every point, to LDS
        unroll_for<0, NQ>([&](auto q_c) {
            constexpr int q = decltype(q_c)::value;
            Real U[NV];
            unroll_for<0, NV>([&](auto v_c) {
                constexpr int v = decltype(v_c)::value;
                Real s = Real(0);
                unroll_for<0, NB>([&](auto b_c) {
                    constexpr int b = decltype(b_c)::value;
                    constexpr double d = T::dl(q, b, v);
                    if constexpr (d != 0.0) s = fmadd(Real(d), uc[b], s);
                });
                U[v] = s;
            });
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                Real s = U[0] * g[0][k];
#pragma unroll
                for (int v = 1; v < NV; ++v) s = fmadd(U[v], g[v][k], s);
                sh.grad[q][c][k][lane] = s;
            }
        });
        __syncthreads();
        // stress rows and basis phase
        Real r[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) r[b] = Real(0);
        unroll_for<0, NQ>([&](auto q_c) {
            constexpr int q = decltype(q_c)::value;
            Real G[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) G[k] = sh.grad[q][c][k][lane];
            // du_{c+1}/dx_{c+1} and du_{c+1}/dx_c from wave c + 1;
            // du_{c+2}/dx_{c+2} and du_{c+2}/dx_c from wave c + 2
            const Real d1 = sh.grad[q][c1][0][lane], o1 = sh.grad[q][c1][2][lane];
            const Real d2 = sh.grad[q][c2][0][lane], o2 = sh.grad[q][c2][1][lane];
            // w_q |J| times row c of f1 in rotated axes: lambda tr delta_ci +
            // mu (du_c/dx_i + du_i/dx_c), the weight folded into lambda and mu
            const Real sw = Real(Q::w(q)) * adj;
            const Real lam = aq[q] * sw, mu = aq[NQ + q] * sw;
            Real f[DIM];
            f[0] = fmadd(mu + mu, G[0], lam * ((G[0] + d1) + d2));
            f[1] = mu * (G[1] + o1);
            f[2] = mu * (G[2] + o2);
            Real h[NV];   // g_v . (w_q |J| f1_c)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Real s = g[v][0] * f[0];
                s = fmadd(g[v][1], f[1], s);
                h[v] = fmadd(g[v][2], f[2], s);
            }
            unroll_for<0, NB>([&](auto b_c) {
                constexpr int b = decltype(b_c)::value;
                unroll_for<0, NV>([&](auto v_c) {
                    constexpr int v = decltype(v_c)::value;
                    constexpr double d = T::dl(q, b, v);
                    if constexpr (d != 0.0) r[b] = fmadd(Real(d), h[v], r[b]);
                });
            });
        });
        // the sums are complete here in every lane: without this the compiler
        // moves the arithmetic after the exchanges into the store branch, and
        // every point's gradients and partner words are live at once
#pragma unroll
        for (int b = 0; b < NB; ++b) __asm__ volatile("" : "+v"(r[b]));
        if (valid) {
            Real* ob = out + (int64_t)c * n + e;
#pragma unroll
            for (int b = 0; b < NB; ++b) __builtin_nontemporal_store(r[b], ob + b * row_stride);
        }
    }
}

hipError_t launch_residual_p3_comp(int space, int dtype, const ResidualArgs& a, const Launch& l) {
    if (l.block % 192 != 0 || l.block / 192 > comp_max_groups(dtype)) return hipErrorInvalidValue;
    const size_t lds = p3_comp_shared_bytes(dtype, l.block / 192);
    if (dtype == FEM_F32)
        hipLaunchKernelGGL((residual_p3_comp_kernel<float>), dim3(l.grid), dim3(l.block), lds, l.stream, a.n, space,
                           static_cast<const float*>(a.inv_j), static_cast<const float*>(a.det_j),
                           static_cast<const float*>(a.u), static_cast<const float*>(a.coef),
                           static_cast<float*>(a.out));
    else if (dtype == FEM_F64)
        hipLaunchKernelGGL((residual_p3_comp_kernel<double>), dim3(l.grid), dim3(l.block), lds, l.stream, a.n, space,
                           static_cast<const double*>(a.inv_j), static_cast<const double*>(a.det_j),
                           static_cast<const double*>(a.u), static_cast<const double*>(a.coef),
                           static_cast<double*>(a.out));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace femq
