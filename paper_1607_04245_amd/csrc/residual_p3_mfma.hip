// residual_p3_mfma.hip -- third-order (P3) residuals of tetrahedra with the
// paper's thread transposition (Section 3, Fig. 1 and 3), the two
// tabulation contractions of Eq. (2) carried out by the matrix cores.
//
// Four lanes share an element. A wave works on 16 elements at a time: lane
// l = 16 g + j serves element j of the group in lane group g.
//
//  quadrature phase  (point-parallel) lane group g owns the points
//                    P_g = {3g, 3g+1, 3g+2} (g < 3) and {9, 10} (g = 3) of
//                    the eleven-point rule. For every barycentric
//                    direction v the matrix core forms
//                      U[q][v][c] = sum_b dphi_b/dlam_v(x_q) u[b][c]
//                    for all points and the 16 elements at once (a 16x4 by
//                    4x16 product per step, rows = points, columns =
//                    elements), and leaves U of the points P_g in lane group
//                    g. Each lane then evaluates grad u, the pointwise f1
//                    and the weighted pulled-back flux
//                      F[q][v][c] = w_q |det J| g_v . f1_c(x_q)
//                    at its own points, in vector registers.
//  basis phase       (basis-parallel) the matrix core forms
//                      R[b][c] = sum_{q,v} dphi_b/dlam_v(x_q) F[q][v][c]
//                    with the (q, v) pairs of all four lane groups as the
//                    inner dimension: the switch from point-parallel to
//                    basis-parallel work happens inside the product, so no
//                    lane sums another lane's values and nothing passes
//                    through LDS. Lane group g receives the rows b of its
//                    output block and stores them.
//
// The tabulated derivatives are the products' left operands: one register
// per lane and step, loaded once per kernel from a table built at compile
// time from the same basis the lane kernel uses (p3_device.hpp).
//
// Inner-dimension classes. In the quadrature phase lane group g supplies the
// closure values of five basis functions, cls[p][g] for p = 0..4. Class 0
// (vertices 0, 1 and the nodes of edge (0,1)) does not depend on lam_2 or
// lam_3 and class 1 (vertices 2, 3 and the nodes of edge (2,3)) not on lam_0
// or lam_1, so each direction v needs only four of the five classes (four
// steps of the 16x16x4 product instead of five). In the basis phase the
// output rows are the 16 functions outside class 1 (block 0) and class 1
// itself (block 1, four of sixteen rows used), and block 1 receives
// contributions only from the directions v = 2, 3.
//
// Products: 16 (quadrature) + 12 + 6 (basis) per component and 16
// elements. Every element's result is fixed by the instruction sequence, so
// repeated calls are bitwise equal; the summation order differs from the
// lane kernel's, so the two strategies agree to rounding, not bitwise.
#include "fem_internal.hpp"
#include "p3_device.hpp"

namespace femq {
namespace p3m {

constexpr int RULE = FEM_RULE_TET11;
using Basis = P3Basis<3, RULE>;
using QR = RuleP2<3, RULE>;

// closure class p, member of lane group g
__host__ __device__ constexpr int cls(int p, int g) {
    return p == 0 ? (g < 2 ? g : g + 2)        // 0, 1, 4, 5
         : p == 1 ? (g < 2 ? g + 2 : g + 12)   // 2, 3, 14, 15
         : p == 2 ? 6 + g                      // 6..9
         : p == 3 ? 10 + g                     // 10..13
                  : 16 + g;                    // 16..19
}
// the four classes used for direction v (class 1 has no lam_0, lam_1
// derivative, class 0 none in lam_2, lam_3)
__host__ __device__ constexpr int use(int v, int s) { return s == 0 ? (v < 2 ? 0 : 1) : s + 1; }
// point of lane group g, local index p (-1: padding)
__host__ __device__ constexpr int point(int g, int p) { return g < 3 ? 3 * g + p : (p < 2 ? 9 + p : -1); }

// Where row i of a 16x16 result lands: lane group g (lanes 16 g .. 16 g + 15,
// one column each) and accumulator register r. The FP32 product puts rows
// 4g .. 4g + 3 in lane group g; the FP64 product puts rows g, g + 4, g + 8,
// g + 12 there (both checked on the device). The left-operand tables below
// order their rows so that lane group g's register r always receives the
// quantity of (g, r), whichever the type.
template <typename Real> __host__ __device__ constexpr int row_g(int i);
template <typename Real> __host__ __device__ constexpr int row_r(int i);
template <> __host__ __device__ constexpr int row_g<float>(int i) { return i / 4; }
template <> __host__ __device__ constexpr int row_r<float>(int i) { return i % 4; }
template <> __host__ __device__ constexpr int row_g<double>(int i) { return i % 4; }
template <> __host__ __device__ constexpr int row_r<double>(int i) { return i / 4; }

// point of product row i (register p of lane group g holds point (g, p))
template <typename Real>
__host__ __device__ constexpr int row_point(int i) { return row_r<Real>(i) == 3 ? -1 : point(row_g<Real>(i), row_r<Real>(i)); }
// basis function of output row i in block 0 (lane group g holds class
// {0, 2, 3, 4}[g], register r its member r) and block 1 (class 1, in lane
// group 0)
template <typename Real>
__host__ __device__ constexpr int out_row0(int i) {
    return cls(row_g<Real>(i) == 0 ? 0 : row_g<Real>(i) + 1, row_r<Real>(i));
}
template <typename Real>
__host__ __device__ constexpr int out_row1(int i) { return row_g<Real>(i) == 0 ? cls(1, row_r<Real>(i)) : -1; }

constexpr int STEPS_U = 16;   // 4 directions x 4 classes
constexpr int STEPS_R0 = 12;  // 4 directions x 3 local points
constexpr int STEPS_R1 = 6;   // directions 2, 3 only
constexpr int STEPS = STEPS_U + STEPS_R0 + STEPS_R1;

// Left operands: lane l = 16 g + j holds A[i = j][k = g] of every step.
template <typename Real>
struct Tab {
    Real a[STEPS][64];
    constexpr Tab() : a() {
        for (int l = 0; l < 64; ++l) {
            const int g = l / 16, j = l % 16;
            for (int v = 0; v < 4; ++v)
                for (int s = 0; s < 4; ++s) {
                    const int q = row_point<Real>(j);
                    a[v * 4 + s][l] = q < 0 ? Real(0) : Real(Basis::dl(q, cls(use(v, s), g), v));
                }
            for (int s = 0; s < STEPS_R0; ++s) {
                const int q = point(g, s % 3), v = s / 3;
                a[STEPS_U + s][l] = q < 0 ? Real(0) : Real(Basis::dl(q, out_row0<Real>(j), v));
            }
            for (int s = 0; s < STEPS_R1; ++s) {
                const int q = point(g, s % 3), v = 2 + s / 3, b = out_row1<Real>(j);
                a[STEPS_U + STEPS_R0 + s][l] = (q < 0 || b < 0) ? Real(0) : Real(Basis::dl(q, b, v));
            }
        }
    }
};

// Barycentric coordinates and weights of the lane's points (for the P1
// coefficient space and the measure), per lane group.
template <typename Real>
struct PointTab {
    Real lam[4][3][4];
    Real w[4][3];
    constexpr PointTab() : lam(), w() {
        for (int g = 0; g < 4; ++g)
            for (int p = 0; p < 3; ++p) {
                const int q = point(g, p);
                w[g][p] = q < 0 ? Real(0) : Real(QR::w(q));
                for (int v = 0; v < 4; ++v) lam[g][p][v] = q < 0 ? Real(0) : Real(QR::lam(q, v));
            }
    }
};

__device__ const Tab<float> kTabF = Tab<float>();
__device__ const Tab<double> kTabD = Tab<double>();
__device__ const PointTab<float> kPtF = PointTab<float>();
__device__ const PointTab<double> kPtD = PointTab<double>();

template <typename Real> __device__ __forceinline__ const Tab<Real>& tab();
template <> __device__ __forceinline__ const Tab<float>& tab<float>() { return kTabF; }
template <> __device__ __forceinline__ const Tab<double>& tab<double>() { return kTabD; }
template <typename Real> __device__ __forceinline__ const PointTab<Real>& pts();
template <> __device__ __forceinline__ const PointTab<float>& pts<float>() { return kPtF; }
template <> __device__ __forceinline__ const PointTab<double>& pts<double>() { return kPtD; }

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename Real> struct Acc;
template <> struct Acc<float> { typedef f32x4 T; };
template <> struct Acc<double> { typedef f64x4 T; };

// Element data accesses. A wave touches 16 consecutive elements of a row
// per access: 64 bytes in FP32, half a 128-byte cache line whose other half
// a neighbouring wave touches, so FP32 uses ordinary (cached) accesses and
// the other half comes from L2 (streaming accesses measured 1.3-1.9x the
// row bytes fetched from HBM); FP64 rows fill whole lines and stream.
template <typename Real>
__device__ __forceinline__ Real ld(const Real* p) {
    if constexpr (sizeof(Real) == 4) return *p;
    else return __builtin_nontemporal_load(p);
}
template <typename Real>
__device__ __forceinline__ void st(Real v, Real* p) {
    if constexpr (sizeof(Real) == 4) *p = v;
    else __builtin_nontemporal_store(v, p);
}

// D = A B + C for one 16x4 by 4x16 step (lane layout above).
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace p3m

template <int PHYS, typename Real>
__global__ void __launch_bounds__(256)
residual_p3_mfma_kernel(int64_t n, int space, const Real* __restrict__ inv_j, const Real* __restrict__ det_j,
                        const Real* __restrict__ u, const Real* __restrict__ coef, Real* __restrict__ out) {
    using namespace p3m;
    using E = ElemP3<3, PHYS, RULE, FEM_COEF_QUAD>;
    using P = Physics<PHYS>;
    using V4 = typename Acc<Real>::T;
    constexpr int NC = E::NC, NCOEF = E::NCOEF;
    static_assert(!P::HAS_F0 && P::HAS_F1, "the matrix-core strategy covers the f1 physics");

    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    // left operands of every step, and the lane's point data
    Real A[STEPS];
#pragma unroll
    for (int s = 0; s < STEPS; ++s) A[s] = tab<Real>().a[s][lane];
    Real wq[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) wq[p] = pts<Real>().w[g][p];
    // coefficient row of local point p (clamped to a real point for padding,
    // whose weight is zero)
    int qrow[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) qrow[p] = g < 3 ? 3 * g + p : (p < 2 ? 9 + p : 10);
    int urow[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) urow[p] = (p == 0 ? (g < 2 ? g : g + 2) : p == 1 ? (g < 2 ? g + 2 : g + 12)
                                           : p == 2 ? 6 + g : p == 3 ? 10 + g : 16 + g);
    int orow0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) orow0[r] = g == 0 ? r + (r < 2 ? 0 : 2) : (g == 1 ? 6 + r : g == 2 ? 10 + r : 16 + r);

    const int64_t n_sub = (n + 15) >> 4;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t sub = w0; sub < n_sub; sub += waves) {
        const int64_t e = sub * 16 + j;
        const bool valid = e < n;
        const int64_t ec = valid ? e : n - 1;
        // ---- loads: geometry, this lane group's closure classes, the
        // coefficients at this lane's points
        Real ij[9];
#pragma unroll
        for (int f = 0; f < 9; ++f) ij[f] = ld(inv_j + f * n + ec);
        const Real adj = fabs(ld(det_j + ec));
        Real ub[5][NC];
#pragma unroll
        for (int p = 0; p < 5; ++p)
#pragma unroll
            for (int c = 0; c < NC; ++c) ub[p][c] = ld(u + (int64_t)(urow[p] * NC + c) * n + ec);
        Real a[NCOEF][3];
        if (space == FEM_COEF_QUAD) {
#pragma unroll
            for (int m = 0; m < NCOEF; ++m)
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    a[m][p] = ld(coef + (int64_t)(m * E::NQ + qrow[p]) * n + ec);
        } else if (space == FEM_COEF_P1) {
#pragma unroll
            for (int m = 0; m < NCOEF; ++m) {
                Real cv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) cv[v] = ld(coef + (int64_t)(m * 4 + v) * n + ec);
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const Real* lam = pts<Real>().lam[g][p];
                    Real t = lam[0] * cv[0];
#pragma unroll
                    for (int v = 1; v < 4; ++v) t = fmadd(lam[v], cv[v], t);
                    a[m][p] = t;
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < NCOEF; ++m) {
                const Real cc = ld(coef + (int64_t)m * n + ec);
#pragma unroll
                for (int p = 0; p < 3; ++p) a[m][p] = cc;
            }
        }

        Real gv[4][3];   // gradients of the barycentric coordinates
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Real s = ij[i];
            gv[1][i] = ij[i];
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                gv[k + 1][i] = ij[k * 3 + i];
                s += ij[k * 3 + i];
            }
            gv[0][i] = -s;
        }

        // ---- quadrature phase, one component at a time: the matrix core
        // gives lane group g the derivatives of u_c along every lam_v at
        // its points P_g; the lane turns them into grad u_c there
        Real gq[3][NC][3];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            V4 U[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                V4 acc = {Real(0), Real(0), Real(0), Real(0)};
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mma(A[v * 4 + s], ub[use(v, s)][c], acc);
                U[v] = acc;
            }
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    Real t = U[0][p] * gv[0][i];
#pragma unroll
                    for (int v = 1; v < 4; ++v) t = fmadd(U[v][p], gv[v][i], t);
                    gq[p][c][i] = t;
                }
        }

        // ---- pointwise physics at this lane's points, weighted:
        // f1 is overwritten into gq (w_q |det J| f1)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            Real am[NCOEF];
#pragma unroll
            for (int m = 0; m < NCOEF; ++m) am[m] = a[m][p];
            Real uq[NC], f0[NC], f1[NC][3];
            P::template point<3, Real>(uq, gq[p], am, f0, f1);
            const Real sw = wq[p] * adj;
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) gq[p][c][i] = sw * f1[c][i];
        }

        // ---- basis phase, one component at a time: the pulled-back flux
        // F[q][v] = g_v . (w_q |J| f1_c) at this lane's points is the right
        // operand; the matrix core sums over the points of all four lane
        // groups and hands lane group g its output rows
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Real F[3][4];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    Real t = gv[v][0] * gq[p][c][0];
#pragma unroll
                    for (int i = 1; i < 3; ++i) t = fmadd(gv[v][i], gq[p][c][i], t);
                    F[p][v] = t;
                }
            V4 r0 = {Real(0), Real(0), Real(0), Real(0)};
            V4 r1 = {Real(0), Real(0), Real(0), Real(0)};
#pragma unroll
            for (int s = 0; s < STEPS_R0; ++s) r0 = mma(A[STEPS_U + s], F[s % 3][s / 3], r0);
#pragma unroll
            for (int s = 0; s < STEPS_R1; ++s) r1 = mma(A[STEPS_U + STEPS_R0 + s], F[s % 3][2 + s / 3], r1);
            if (valid) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    st(r0[r], out + (int64_t)(orow0[r] * NC + c) * n + e);
                if (g == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        st(r1[r], out + (int64_t)(cls(1, r) * NC + c) * n + e);
                }
            }
        }
    }
}

hipError_t launch_residual_p3_mfma(int phys, int space, int dtype, const ResidualArgs& a, const Launch& l) {
#define FEMQ_LAUNCH(PH, T)                                                                                     \
    hipLaunchKernelGGL((residual_p3_mfma_kernel<PH, T>), dim3(l.grid), dim3(l.block), 0, l.stream, a.n, space, \
                       static_cast<const T*>(a.inv_j), static_cast<const T*>(a.det_j), static_cast<const T*>(a.u), \
                       static_cast<const T*>(a.coef), static_cast<T*>(a.out))
    if (phys == FEM_LAPLACE && dtype == FEM_F32) FEMQ_LAUNCH(FEM_LAPLACE, float);
    else if (phys == FEM_LAPLACE && dtype == FEM_F64) FEMQ_LAUNCH(FEM_LAPLACE, double);
    else if (phys == FEM_ELASTICITY && dtype == FEM_F32) FEMQ_LAUNCH(FEM_ELASTICITY, float);
    else if (phys == FEM_ELASTICITY && dtype == FEM_F64) FEMQ_LAUNCH(FEM_ELASTICITY, double);
    else return hipErrorInvalidValue;
#undef FEMQ_LAUNCH
    return hipGetLastError();
}

}  // namespace femq
