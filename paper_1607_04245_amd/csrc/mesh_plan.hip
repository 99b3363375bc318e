// mesh_plan.hip -- a per-mesh plan of the distinct vertices of every
// 64-element tile, and the from-mesh residual kernels that use it.
//
// The fused from-mesh kernels (mesh_kernel.hpp) let every lane gather the
// vertices of its own element: d+1 vertex records per element, while the
// elements of a 64-element tile of a conforming mesh share most of their
// vertices (47 distinct vertices for 256 references on a tetrahedral grid).
// The per-lane gathers, not the bytes, bound those kernels. A plan, built
// once per mesh from the connectivity, lists each tile's distinct vertices
// (ascending) and, per element, the position of each of its vertices in
// that list (one byte each, packed in 32 bits, in place of the 4(d+1)-byte
// connectivity row). The planned kernel gives each wave one tile: the lanes
// load the tile's distinct vertex records once (coordinates; in the gather
// form also u and a P1 coefficient) into LDS, then every lane reads its
// element's vertices from LDS and runs the fused kernel's element arithmetic
// on them, so the element vectors are bitwise those of
// fem_integrate_residual_mesh / fem_integrate_residual_gather.
//
// The plan is built on the host (the connectivity is copied back once); it
// validates every vertex index, so the planned kernels need no index checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mesh_kernel.hpp"

struct fem_mesh_plan {
    int dim = 0;
    int device = 0;
    int max_tile = 0;                // distinct vertices of the fullest tile (<= 64 (dim+1))
    int64_t n_elem = 0;
    int64_t n_vert = 0;
    int64_t n_tiles = 0;
    int64_t* tile_off = nullptr;     // [n_tiles + 1]: tile t's vertices are tile_verts[tile_off[t] ..)
    int32_t* tile_verts = nullptr;   // [tile_off[n_tiles]], ascending within a tile
    uint32_t* lidx = nullptr;        // [n_elem]: byte b = position of the element's vertex b in its tile's list
};

namespace femq {

constexpr int kPlanTile = 64;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave (the whole workgroup) per TPW consecutive tiles, whose loads are
// all issued before the first element is finished (two in the gather form on
// triangles, one otherwise). LDS
// holds, per tile, maxc x DIM coordinates (FP64), then, after all tiles'
// coordinates, maxc x (NU + NK) values of u and of a P1 coefficient (gather
// form).
template <int DIM, int PHYS, int RULE, typename Real, bool GATHER, bool STORE_GEOM, int TPW>
__global__ void __launch_bounds__(64)
residual_planned_kernel(int64_t n, int64_t n_tiles, const int64_t* __restrict__ tile_off,
                        const int32_t* __restrict__ tile_verts, const uint32_t* __restrict__ lidx,
                        const double* __restrict__ X, const Real* __restrict__ u, const Real* __restrict__ coef,
                        Real* __restrict__ out, Real* __restrict__ inv_j, Real* __restrict__ det_j,
                        int32_t* __restrict__ counts, int maxc) {
    using E = Elem<DIM, PHYS, RULE>;
    constexpr bool CV = coef_per_vertex<DIM, PHYS, RULE, GATHER>();
    constexpr int NU = GATHER ? E::NC : 0, NK = CV ? E::NCOEF : 0, NR = NU + NK;
    extern __shared__ double plan_lds[];
    double* xs = plan_lds;
    Real* vs = reinterpret_cast<Real*>(plan_lds + (int64_t)TPW * maxc * DIM);
    const int lane = threadIdx.x;
    int ndeg = 0, npoor = 0;
    for (int64_t t0 = (int64_t)blockIdx.x * TPW; t0 < n_tiles; t0 += (int64_t)gridDim.x * TPW) {
        int64_t off[TPW], e[TPW];
        int cnt[TPW];
        uint32_t li[TPW];
        Real uu[TPW][E::NBT], cf[TPW][E::NCQ];
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            // a tile past the end is skipped: no records, masked stores
            const bool live = t0 + k < n_tiles;
            const int64_t t = live ? t0 + k : n_tiles - 1;
            off[k] = tile_off[t];
            cnt[k] = live ? (int)(tile_off[t + 1] - off[k]) : 0;
            // per-element streams, independent of the vertex records
            e[k] = (t0 + k) * kPlanTile + lane;
            const int64_t ec = e[k] < n ? e[k] : n - 1;
            li[k] = __builtin_nontemporal_load(lidx + ec);
            if constexpr (!GATHER) {
#pragma unroll
                for (int f = 0; f < E::NBT; ++f) uu[k][f] = __builtin_nontemporal_load(u + f * n + ec);
            }
            if constexpr (!CV) {
#pragma unroll
                for (int f = 0; f < E::NCQ; ++f) cf[k][f] = __builtin_nontemporal_load(coef + f * n + ec);
            }
        }
        // the tiles' distinct vertex records, once each (a version that
        // issued all of a lane's record loads before its first LDS store
        // measured slower on tetrahedra and barely faster on triangles)
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            double* xk = xs + (int64_t)k * maxc * DIM;
            Real* vk = vs + (int64_t)k * maxc * NR;
            for (int j = lane; j < cnt[k]; j += kPlanTile) {
                const int64_t v = tile_verts[off[k] + j];
#pragma unroll
                for (int i = 0; i < DIM; ++i) xk[j * DIM + i] = X[v * DIM + i];
                if constexpr (GATHER) {
#pragma unroll
                    for (int c = 0; c < E::NC; ++c) vk[j * NR + c] = u[v * E::NC + c];
                }
                if constexpr (CV) {
#pragma unroll
                    for (int m = 0; m < E::NCOEF; ++m) vk[j * NR + NU + m] = coef[v * E::NCOEF + m];
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            const double* xk = xs + (int64_t)k * maxc * DIM;
            const Real* vk = vs + (int64_t)k * maxc * NR;
            double x[DIM + 1][DIM];
#pragma unroll
            for (int b = 0; b <= DIM; ++b) {
                const int l = (int)((li[k] >> (8 * b)) & 255u);
#pragma unroll
                for (int i = 0; i < DIM; ++i) x[b][i] = xk[l * DIM + i];
                if constexpr (GATHER) {
#pragma unroll
                    for (int c = 0; c < E::NC; ++c) uu[k][b * E::NC + c] = vk[l * NR + c];
                }
                if constexpr (CV) {
#pragma unroll
                    for (int m = 0; m < E::NCOEF; ++m) cf[k][m * E::NB + b] = vk[l * NR + NU + m];
                }
            }
            mesh_element_finish<DIM, PHYS, RULE, Real, STORE_GEOM>(e[k] < n, e[k], n, true, x, uu[k], cf[k], out,
                                                                   inv_j, det_j, ndeg, npoor);
        }
        wave_sync();  // every lane has read the tiles before the next ones are staged
    }
    add_counts(counts, ndeg, npoor);
}

// The geometry alone through the plan: coordinates staged as above, then
// the epilogue of fem_geometry, so the outputs are bitwise its outputs.
template <int DIM, typename Out>
__global__ void __launch_bounds__(64)
geometry_planned_kernel(int64_t n, int64_t n_tiles, const int64_t* __restrict__ tile_off,
                        const int32_t* __restrict__ tile_verts, const uint32_t* __restrict__ lidx,
                        const double* __restrict__ X, Out* __restrict__ inv_j, Out* __restrict__ det_j,
                        int32_t* __restrict__ counts) {
    extern __shared__ double plan_lds[];
    const int lane = threadIdx.x;
    int ndeg = 0, npoor = 0;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t off = tile_off[t];
        const int cnt = (int)(tile_off[t + 1] - off);
        const int64_t e = t * kPlanTile + lane, ec = e < n ? e : n - 1;
        const uint32_t li = __builtin_nontemporal_load(lidx + ec);
        for (int j = lane; j < cnt; j += kPlanTile) {
            const int64_t v = tile_verts[off + j];
#pragma unroll
            for (int i = 0; i < DIM; ++i) plan_lds[j * DIM + i] = X[v * DIM + i];
        }
        wave_sync();
        double x[DIM + 1][DIM];
#pragma unroll
        for (int b = 0; b <= DIM; ++b) {
            const int l = (int)((li >> (8 * b)) & 255u);
#pragma unroll
            for (int i = 0; i < DIM; ++i) x[b][i] = plan_lds[l * DIM + i];
        }
        geometry_finish<DIM, Out>(e < n, e, n, true, x, inv_j, det_j, ndeg, npoor);
        wave_sync();
    }
    add_counts(counts, ndeg, npoor);
}

struct PlannedArgs {
    const fem_mesh_plan* p;
    const double* coords;
    const void* u;
    const void* coef;
    void* out;
    void* inv_j;
    void* det_j;
    int32_t* counts;
    int dtype;
    hipStream_t stream;
};

template <int DIM, int PHYS, int RULE, typename Real, bool GATHER>
static hipError_t launch_planned_t(const PlannedArgs& a) {
    using E = Elem<DIM, PHYS, RULE>;
    constexpr bool CV = coef_per_vertex<DIM, PHYS, RULE, GATHER>();
    constexpr int NR = (GATHER ? E::NC : 0) + (CV ? E::NCOEF : 0);
    // measured: two tiles per wave pay in the triangle gather form only
    constexpr int TPW = (DIM == 2 && GATHER) ? 2 : 1;
    const int maxc = std::max(a.p->max_tile, 1);
    const size_t lds = (size_t)TPW * maxc * (DIM * sizeof(double) + NR * sizeof(Real));
    const int64_t grid =
        std::min<int64_t>(std::max<int64_t>((a.p->n_tiles + TPW - 1) / TPW, 1), (int64_t)1 << 30);
    if (a.inv_j != nullptr)
        hipLaunchKernelGGL((residual_planned_kernel<DIM, PHYS, RULE, Real, GATHER, true, TPW>), dim3((unsigned)grid),
                           dim3(64), lds, a.stream, a.p->n_elem, a.p->n_tiles, a.p->tile_off, a.p->tile_verts, a.p->lidx,
                           a.coords, static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef),
                           static_cast<Real*>(a.out), static_cast<Real*>(a.inv_j), static_cast<Real*>(a.det_j),
                           a.counts, maxc);
    else
        hipLaunchKernelGGL((residual_planned_kernel<DIM, PHYS, RULE, Real, GATHER, false, TPW>), dim3((unsigned)grid),
                           dim3(64), lds, a.stream, a.p->n_elem, a.p->n_tiles, a.p->tile_off, a.p->tile_verts, a.p->lidx,
                           a.coords, static_cast<const Real*>(a.u), static_cast<const Real*>(a.coef),
                           static_cast<Real*>(a.out), nullptr, nullptr, a.counts, maxc);
    return hipGetLastError();
}

template <bool GATHER>
struct PlannedDispatch {
    const PlannedArgs& a;
    template <int D, int P, int S>
    hipError_t operator()() const {
        return a.dtype == FEM_F32 ? launch_planned_t<D, P, S, float, GATHER>(a)
                                  : launch_planned_t<D, P, S, double, GATHER>(a);
    }
};

static void mesh_plan_free(fem_mesh_plan* p) {
    if (!p) return;
    if (p->tile_off) (void)hipFree(p->tile_off);
    if (p->tile_verts) (void)hipFree(p->tile_verts);
    if (p->lidx) (void)hipFree(p->lidx);
    delete p;
}

static fem_status planned_common(const char* fn, const fem_mesh_plan* plan, int physics, int rule, int coef_space,
                                 int dtype, const double* coords, const void* u, const void* coef, void* out,
                                 const void* inv_j, const void* det_j) {
    if (!plan) { set_error("%s: NULL plan", fn); return FEM_ERR_INVALID_ARG; }
    const int dim = plan->dim;
    if (physics != FEM_LAPLACE && physics != FEM_ELASTICITY && physics != FEM_MASS) {
        set_error("%s: unknown physics %d", fn, physics);
        return FEM_ERR_UNSUPPORTED;
    }
    const bool rule_ok = rule == FEM_RULE_CENTROID || (dim == 2 ? rule == FEM_RULE_TRI3 : rule == FEM_RULE_TET4);
    if (!rule_ok) { set_error("%s: rule %d is not defined in %dD", fn, rule, dim); return FEM_ERR_UNSUPPORTED; }
    if (coef_space != FEM_COEF_QUAD && coef_space != FEM_COEF_P1 && coef_space != FEM_COEF_P0) {
        set_error("%s: unknown coefficient space %d", fn, coef_space);
        return FEM_ERR_UNSUPPORTED;
    }
    if (dtype != FEM_F32 && dtype != FEM_F64) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    if (plan->n_elem == 0) return FEM_OK;
    if (!coords || !u || !coef || !out || (!inv_j) != (!det_j)) {
        set_error("%s: NULL array (inv_j and det_j must both be set or both NULL)", fn);
        return FEM_ERR_INVALID_ARG;
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev != plan->device) {
        set_error("%s: the plan was built on device %d, current device is %d", fn, plan->device, dev);
        return FEM_ERR_INVALID_ARG;
    }
    return FEM_OK;
}

}  // namespace femq

using namespace femq;

extern "C" {

fem_status fem_mesh_plan_create(int dim, int64_t n_elem, int64_t n_vert, const int32_t* conn, void* stream,
                                fem_mesh_plan** out) {
    if (!out) { set_error("fem_mesh_plan_create: out is NULL"); return FEM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { set_error("fem_mesh_plan_create: dim must be 2 or 3 (got %d)", dim); return FEM_ERR_UNSUPPORTED; }
    if (n_elem < 0 || n_vert < 0) { set_error("fem_mesh_plan_create: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem > 0 && (n_vert == 0 || !conn)) {
        set_error("fem_mesh_plan_create: elements without vertices or NULL connectivity");
        return FEM_ERR_INVALID_ARG;
    }
    const int nb = dim + 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> hc;
    try {
        hc.resize((size_t)n_elem * nb);
    } catch (...) {
        set_error("fem_mesh_plan_create: out of host memory");
        return FEM_ERR_INVALID_ARG;
    }
    hipError_t e = hipSuccess;
    if (n_elem > 0) {
        e = hipMemcpyAsync(hc.data(), conn, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "fem_mesh_plan_create: connectivity copy");
    }
    const int64_t n_tiles = (n_elem + kPlanTile - 1) / kPlanTile;
    std::vector<int64_t> off((size_t)n_tiles + 1, 0);
    std::vector<int32_t> verts;
    std::vector<uint32_t> lidx((size_t)n_elem, 0u);
    int max_tile = 0;
    int64_t bad = 0;
    std::vector<int32_t> ids;
    ids.reserve(kPlanTile * nb);
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int64_t e0 = t * kPlanTile, e1 = std::min<int64_t>(e0 + kPlanTile, n_elem);
        ids.assign(hc.begin() + e0 * nb, hc.begin() + e1 * nb);
        for (int32_t v : ids) bad += (v < 0) | ((int64_t)v >= n_vert);
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        off[(size_t)t] = (int64_t)verts.size();
        verts.insert(verts.end(), ids.begin(), ids.end());
        max_tile = std::max(max_tile, (int)ids.size());
        for (int64_t el = e0; el < e1; ++el) {
            uint32_t packed = 0;
            for (int b = 0; b < nb; ++b) {
                const int32_t v = hc[(size_t)(el * nb + b)];
                const uint32_t pos = (uint32_t)(std::lower_bound(ids.begin(), ids.end(), v) - ids.begin());
                packed |= pos << (8 * b);
            }
            lidx[(size_t)el] = packed;
        }
    }
    off[(size_t)n_tiles] = (int64_t)verts.size();
    if (bad) {
        set_error("fem_mesh_plan_create: %lld vertex indices outside [0, %lld)", (long long)bad, (long long)n_vert);
        return FEM_ERR_INVALID_ARG;
    }
    fem_mesh_plan* p = new (std::nothrow) fem_mesh_plan();
    if (!p) { set_error("fem_mesh_plan_create: out of host memory"); return FEM_ERR_INVALID_ARG; }
    p->dim = dim;
    p->n_elem = n_elem;
    p->n_vert = n_vert;
    p->n_tiles = n_tiles;
    p->max_tile = max_tile;
    e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->tile_off, off.size() * sizeof(int64_t));
    if (e == hipSuccess && !verts.empty()) e = hipMalloc(&p->tile_verts, verts.size() * sizeof(int32_t));
    if (e == hipSuccess && n_elem > 0) e = hipMalloc(&p->lidx, lidx.size() * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->tile_off, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !verts.empty())
        e = hipMemcpyAsync(p->tile_verts, verts.data(), verts.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_elem > 0)
        e = hipMemcpyAsync(p->lidx, lidx.data(), lidx.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vectors die here
    if (e != hipSuccess) { mesh_plan_free(p); return hip_fail(e, "fem_mesh_plan_create: upload"); }
    *out = p;
    return FEM_OK;
}

fem_status fem_mesh_plan_info(const fem_mesh_plan* plan, int* dim, int64_t* n_elem, int64_t* n_vert,
                              int* max_tile_vertices, int64_t* tile_vertices) {
    if (!plan) { set_error("fem_mesh_plan_info: NULL plan"); return FEM_ERR_INVALID_ARG; }
    if (dim) *dim = plan->dim;
    if (n_elem) *n_elem = plan->n_elem;
    if (n_vert) *n_vert = plan->n_vert;
    if (max_tile_vertices) *max_tile_vertices = plan->max_tile;
    if (tile_vertices) {
        int64_t total = 0;
        if (plan->n_tiles > 0) {
            hipError_t e = hipMemcpy(&total, plan->tile_off + plan->n_tiles, sizeof(int64_t), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "fem_mesh_plan_info");
        }
        *tile_vertices = total;
    }
    return FEM_OK;
}

void fem_mesh_plan_destroy(fem_mesh_plan* plan) { mesh_plan_free(plan); }

fem_status fem_geometry_planned(const fem_mesh_plan* plan, const double* coords, int out_dtype, void* inv_j,
                               void* det_j, int32_t* counts, void* stream) {
    if (!plan) { set_error("fem_geometry_planned: NULL plan"); return FEM_ERR_INVALID_ARG; }
    if (out_dtype != FEM_F32 && out_dtype != FEM_F64) {
        set_error("fem_geometry_planned: unknown dtype %d", out_dtype);
        return FEM_ERR_UNSUPPORTED;
    }
    if (plan->n_elem == 0) return FEM_OK;
    if (!coords || !inv_j || !det_j) { set_error("fem_geometry_planned: NULL array"); return FEM_ERR_INVALID_ARG; }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev != plan->device) {
        set_error("fem_geometry_planned: the plan was built on device %d, current device is %d", plan->device, dev);
        return FEM_ERR_INVALID_ARG;
    }
    const int maxc = std::max(plan->max_tile, 1);
    const size_t lds = (size_t)maxc * plan->dim * sizeof(double);
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(plan->n_tiles, 1), (int64_t)1 << 30);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto go = [&](auto dim_c, auto out_c) {
        constexpr int D = decltype(dim_c)::value;
        using Out = typename decltype(out_c)::type;
        hipLaunchKernelGGL((geometry_planned_kernel<D, Out>), dim3(grid), dim3(64), lds, s, plan->n_elem,
                           plan->n_tiles, plan->tile_off, plan->tile_verts, plan->lidx, coords,
                           static_cast<Out*>(inv_j), static_cast<Out*>(det_j), counts);
    };
    struct F32 { using type = float; };
    struct F64 { using type = double; };
    if (plan->dim == 2) {
        if (out_dtype == FEM_F32) go(std::integral_constant<int, 2>(), F32{});
        else go(std::integral_constant<int, 2>(), F64{});
    } else {
        if (out_dtype == FEM_F32) go(std::integral_constant<int, 3>(), F32{});
        else go(std::integral_constant<int, 3>(), F64{});
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_geometry_planned launch");
}

fem_status fem_integrate_residual_planned(const fem_mesh_plan* plan, int physics, int rule, int coef_space, int dtype,
                                          const double* coords, const void* u, const void* coef, void* elem_vec,
                                          void* inv_j, void* det_j, int32_t* counts, void* stream) {
    fem_status st = planned_common("fem_integrate_residual_planned", plan, physics, rule, coef_space, dtype, coords, u,
                                   coef, elem_vec, inv_j, det_j);
    if (st || plan->n_elem == 0) return st;
    const PlannedArgs a{plan, coords, u, coef, elem_vec, inv_j, det_j, counts, dtype, static_cast<hipStream_t>(stream)};
    const PlannedDispatch<false> f{a};
    hipError_t e = dispatch_element(plan->dim, physics, rule, coef_space, f, hipErrorInvalidValue);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_planned launch");
}

fem_status fem_integrate_residual_gather_planned(const fem_mesh_plan* plan, int physics, int rule, int coef_space,
                                                 int dtype, const double* coords, const void* u_vertex,
                                                 const void* coef, void* elem_vec, void* inv_j, void* det_j,
                                                 int32_t* counts, void* stream) {
    fem_status st = planned_common("fem_integrate_residual_gather_planned", plan, physics, rule, coef_space, dtype,
                                   coords, u_vertex, coef, elem_vec, inv_j, det_j);
    if (st || plan->n_elem == 0) return st;
    const PlannedArgs a{plan, coords, u_vertex, coef, elem_vec, inv_j, det_j, counts, dtype,
                        static_cast<hipStream_t>(stream)};
    const PlannedDispatch<true> f{a};
    hipError_t e = dispatch_element(plan->dim, physics, rule, coef_space, f, hipErrorInvalidValue);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_gather_planned launch");
}

}  // extern "C"
