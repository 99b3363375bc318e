// assembly.hip -- the global residual from element vectors, and its adjoint.
//
// Section 2 writes the global residual as the sum over elements of each
// element vector mapped back through the element restriction (the transpose
// of the closure). Here that sum is a gather, not a scatter: a plan built
// once per mesh holds, for every vertex, the list of (element, local vertex)
// slots that touch it (the transpose of the connectivity, in compressed-row
// form), sorted by element. The assembly kernel gives each vertex one lane
// that adds its slots' entries in that order, starting from zero, so the
// result is deterministic (no atomics) and is exactly the element-by-element
// sum in increasing element order, evaluated in the working precision.
//
// The plan is built on the device: a count of slots per vertex with integer
// atomics (which also finds indices outside [0, n_vert)), an exclusive scan
// for the row offsets, and a stable radix sort of the slot numbers keyed by
// vertex, which leaves every row in increasing slot, hence element, order.
// The rows are then stored sliced: for each group of 64 consecutive vertices
// (one wave), slot j of all 64 rows is contiguous, and every row of the group
// is padded with an empty marker to the group's longest row. A wave's j-th
// slot load is then one contiguous 256-byte access instead of 64 accesses
// one row apart; each vertex still sees its own slots in element order.
//
// The restriction (closure) kernel is the adjoint: one lane per element
// copies the vertex values of its d+1 vertices into the SoA closure rows.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <new>

#include "fem_device.hpp"
#include "fem_internal.hpp"

struct fem_assembly_plan {
    int dim = 0;
    int device = 0;
    int64_t n_elem = 0;
    int64_t n_vert = 0;
    int64_t n_groups = 0;          // ceil(n_vert / 64)
    int64_t* grp_off = nullptr;    // [n_groups + 1], first entry of each group in `sell`
    int32_t* grp_width = nullptr;  // [n_groups], slots per row in the group (its longest row)
    uint32_t* sell = nullptr;      // [grp_off[n_groups]]: group g, slot j, lane l at grp_off[g] + 64 j + l;
                                   // slot = e * (dim + 1) + b, or kNoSlot past the row's end
};

namespace femq {

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// Slots per vertex, bad indices, and the identity slot numbering.
__global__ void __launch_bounds__(256)
assembly_count_kernel(int64_t m, int64_t n_vert, const int32_t* __restrict__ conn, int32_t* __restrict__ count,
                      uint32_t* __restrict__ ids, int32_t* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int nbad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int32_t v = conn[i];
        ids[i] = (uint32_t)i;
        if (v >= 0 && (int64_t)v < n_vert)
            atomicAdd(count + v, 1);
        else
            ++nbad;
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Group widths: the longest row among each group's 64 vertices (vertices
// past n_vert count as empty rows), and the padded size of the group.
__global__ void __launch_bounds__(256)
assembly_width_kernel(int64_t n_groups, int64_t n_vert, const int32_t* __restrict__ row_ptr,
                      int32_t* __restrict__ width, int64_t* __restrict__ size) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups; g += stride) {
        const int64_t v0 = g * 64, v1 = v0 + 64 < n_vert ? v0 + 64 : n_vert;
        int32_t w = 0;
        for (int64_t v = v0; v < v1; ++v) w = max(w, row_ptr[v + 1] - row_ptr[v]);
        width[g] = w;
        size[g] = (int64_t)w * 64;
    }
}

// Sliced storage: entry (g, j, l) = slot j of vertex 64 g + l, or kNoSlot.
__global__ void __launch_bounds__(256)
assembly_slice_kernel(int64_t n_groups, int64_t n_vert, const int32_t* __restrict__ row_ptr,
                      const uint32_t* __restrict__ slots, const int32_t* __restrict__ width,
                      const int64_t* __restrict__ off, uint32_t* __restrict__ sell) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_groups * 64; i += stride) {
        const int64_t g = i / 64, v = i;
        const int l = (int)(i % 64);
        const int32_t s0 = v < n_vert ? row_ptr[v] : 0, len = v < n_vert ? row_ptr[v + 1] - s0 : 0;
        const int32_t w = width[g];
        uint32_t* dst = sell + off[g] + l;
        for (int32_t j = 0; j < w; ++j) dst[(int64_t)j * 64] = j < len ? slots[s0 + j] : kNoSlot;
    }
}

// One wave per group of 64 vertices, one lane per vertex: vertex_vec[v][c] =
// sum over the vertex's slots, in slot order, of elem_vec[b * NC + c][e]. The
// rows are walked in chunks of CH slots whose loads are all issued before the
// first add (empty entries read a valid slot and their adds are skipped), so
// a lane waits about once per chunk instead of once per slot; the adds stay
// in slot order.
template <int NB, int NC, typename Real>
__global__ void __launch_bounds__(256)
assemble_kernel(int64_t n_vert, int64_t n_elem, int64_t n_groups, const int64_t* __restrict__ grp_off,
                const int32_t* __restrict__ grp_width, const uint32_t* __restrict__ sell,
                const Real* __restrict__ R, Real* __restrict__ out) {
    // chunk of slots in flight per lane: vertices of tetrahedral meshes lie in
    // about 24 elements, of triangular meshes in about 6
    constexpr int CH = NB == 4 ? 16 : 8;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    for (int64_t g = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * wpb + (threadIdx.x >> 6))); g < n_groups;
         g += n_waves) {
        Real acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = Real(0);
        const uint32_t* row = sell + grp_off[g] + lane;
        const int32_t w = grp_width[g];
        for (int32_t s = 0; s < w; s += CH) {
            uint32_t sl[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) sl[j] = s + j < w ? row[(int64_t)(s + j) * 64] : kNoSlot;
            Real r[CH][NC];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const uint32_t sj = sl[j] != kNoSlot ? sl[j] : 0u;
                const uint32_t e = sj / NB, b = sj - e * NB;
#pragma unroll
                for (int c = 0; c < NC; ++c) r[j][c] = R[(int64_t)(b * NC + c) * n_elem + e];
            }
#pragma unroll
            for (int j = 0; j < CH; ++j)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] = sl[j] != kNoSlot ? acc[c] + r[j][c] : acc[c];
        }
        const int64_t v = g * 64 + lane;
        if (v < n_vert) {
#pragma unroll
            for (int c = 0; c < NC; ++c) out[v * NC + c] = acc[c];
        }
    }
}

// One lane per element: elem_vec[b * NC + c][e] = vertex_vec[conn[e][b]][c];
// an index outside [0, n_vert) gives NaN entries and reads nothing outside.
template <int NB, int NC, typename Real>
__global__ void __launch_bounds__(256)
restrict_kernel(int64_t n_elem, int64_t n_vert, const int32_t* __restrict__ conn, const Real* __restrict__ vert,
                Real* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t hi = vertex_hi(n_vert);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int32_t v = conn[e * NB + b];
            const bool ok = (v >= 0) & ((int64_t)v < n_vert);
            const int64_t vi = (int64_t)min(max(v, 0), hi);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const Real x = vert[vi * NC + c];
                out[(int64_t)(b * NC + c) * n_elem + e] = ok ? x : Real(__builtin_nan(""));
            }
        }
    }
}

static int grid_for(int64_t items) {
    const int64_t cap = (int64_t)std::max(device_cus(), 1) * 32;
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, cap));
}

template <int NB, typename Real>
static hipError_t launch_assemble_nc(int nc, const fem_assembly_plan* p, const void* R, void* out, hipStream_t s) {
    const dim3 g(grid_for(p->n_groups * 64)), b(256);
    const Real* r = static_cast<const Real*>(R);
    Real* o = static_cast<Real*>(out);
    switch (nc) {
    case 1: hipLaunchKernelGGL((assemble_kernel<NB, 1, Real>), g, b, 0, s, p->n_vert, p->n_elem, p->n_groups, p->grp_off, p->grp_width, p->sell, r, o); break;
    case 2: hipLaunchKernelGGL((assemble_kernel<NB, 2, Real>), g, b, 0, s, p->n_vert, p->n_elem, p->n_groups, p->grp_off, p->grp_width, p->sell, r, o); break;
    case 3: hipLaunchKernelGGL((assemble_kernel<NB, 3, Real>), g, b, 0, s, p->n_vert, p->n_elem, p->n_groups, p->grp_off, p->grp_width, p->sell, r, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NB, typename Real>
static hipError_t launch_restrict_nc(int nc, int64_t n_elem, int64_t n_vert, const int32_t* conn, const void* vert,
                                     void* out, hipStream_t s) {
    const dim3 g(grid_for(n_elem)), b(256);
    const Real* v = static_cast<const Real*>(vert);
    Real* o = static_cast<Real*>(out);
    switch (nc) {
    case 1: hipLaunchKernelGGL((restrict_kernel<NB, 1, Real>), g, b, 0, s, n_elem, n_vert, conn, v, o); break;
    case 2: hipLaunchKernelGGL((restrict_kernel<NB, 2, Real>), g, b, 0, s, n_elem, n_vert, conn, v, o); break;
    case 3: hipLaunchKernelGGL((restrict_kernel<NB, 3, Real>), g, b, 0, s, n_elem, n_vert, conn, v, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static void plan_free(fem_assembly_plan* p) {
    if (!p) return;
    if (p->grp_off) (void)hipFree(p->grp_off);
    if (p->grp_width) (void)hipFree(p->grp_width);
    if (p->sell) (void)hipFree(p->sell);
    delete p;
}

}  // namespace femq

using namespace femq;

extern "C" {

fem_status fem_assembly_plan_create(int dim, int64_t n_elem, int64_t n_vert, const int32_t* conn, void* stream,
                                    fem_assembly_plan** out) {
    if (!out) { set_error("fem_assembly_plan_create: out is NULL"); return FEM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { set_error("fem_assembly_plan_create: dim must be 2 or 3 (got %d)", dim); return FEM_ERR_UNSUPPORTED; }
    if (n_elem < 0 || n_vert < 0) { set_error("fem_assembly_plan_create: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem > 0 && (n_vert == 0 || !conn)) {
        set_error("fem_assembly_plan_create: elements without vertices or NULL connectivity");
        return FEM_ERR_INVALID_ARG;
    }
    const int64_t m = n_elem * (dim + 1);
    if (m > (int64_t)INT32_MAX || n_vert >= (int64_t)INT32_MAX) {
        set_error("fem_assembly_plan_create: n_elem * (dim + 1) and n_vert must stay below 2^31");
        return FEM_ERR_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    fem_assembly_plan* p = new (std::nothrow) fem_assembly_plan();
    if (!p) { set_error("fem_assembly_plan_create: out of host memory"); return FEM_ERR_INVALID_ARG; }
    p->dim = dim;
    p->n_elem = n_elem;
    p->n_vert = n_vert;
    p->n_groups = (n_vert + 63) / 64;
    const int64_t ng = p->n_groups;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->grp_off, (size_t)(ng + 1) * sizeof(int64_t));
    if (e == hipSuccess && ng > 0) e = hipMalloc(&p->grp_width, (size_t)ng * sizeof(int32_t));
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "fem_assembly_plan_create: hipMalloc"); }
    if (m == 0) {  // no slots: every group has width 0
        e = hipMemsetAsync(p->grp_off, 0, (size_t)(ng + 1) * sizeof(int64_t), s);
        if (e == hipSuccess && ng > 0) e = hipMemsetAsync(p->grp_width, 0, (size_t)ng * sizeof(int32_t), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { plan_free(p); return hip_fail(e, "fem_assembly_plan_create"); }
        *out = p;
        return FEM_OK;
    }

    // scratch: counts (+ bad counter), compressed rows, identity slots, sorted
    // keys and slots, group sizes, cub temp
    int32_t* count = nullptr;
    int32_t* row_ptr = nullptr;
    uint32_t* ids = nullptr;
    uint32_t* keys_out = nullptr;
    uint32_t* slots = nullptr;
    int64_t* gsize = nullptr;
    void* temp = nullptr;
    size_t scan_bytes = 0, sort_bytes = 0, gscan_bytes = 0;
    int end_bit = 1;
    while (end_bit < 32 && ((int64_t)1 << end_bit) < n_vert) ++end_bit;
    const uint32_t* keys_in = reinterpret_cast<const uint32_t*>(conn);  // valid indices are non-negative
    auto cleanup = [&]() {
        for (void* q : {(void*)count, (void*)row_ptr, (void*)ids, (void*)keys_out, (void*)slots, (void*)gsize, temp})
            if (q) (void)hipFree(q);
    };
    e = hipMalloc(&count, (size_t)(n_vert + 2) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&row_ptr, (size_t)(n_vert + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&ids, (size_t)m * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&keys_out, (size_t)m * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&slots, (size_t)m * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&gsize, (size_t)(ng + 1) * sizeof(int64_t));
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, count, row_ptr, (int)(n_vert + 1), s);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, keys_in, keys_out, ids, slots, (int)m, 0, end_bit, s);
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, gscan_bytes, gsize, p->grp_off, (int)(ng + 1), s);
    if (e == hipSuccess) e = hipMalloc(&temp, std::max(std::max(scan_bytes, sort_bytes), gscan_bytes) + 16);
    if (e == hipSuccess) e = hipMemsetAsync(count, 0, (size_t)(n_vert + 2) * sizeof(int32_t), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(assembly_count_kernel, dim3(grid_for(m)), dim3(256), 0, s, m, n_vert, conn, count, ids,
                           count + n_vert + 1);
        e = hipGetLastError();
    }
    int32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, count + n_vert + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); plan_free(p); return hip_fail(e, "fem_assembly_plan_create: count"); }
    if (bad) {
        cleanup();
        plan_free(p);
        set_error("fem_assembly_plan_create: %d vertex indices outside [0, %lld)", bad, (long long)n_vert);
        return FEM_ERR_INVALID_ARG;
    }
    // count[n_vert] is zero, so row_ptr[n_vert] = m
    e = hipcub::DeviceScan::ExclusiveSum(temp, scan_bytes, count, row_ptr, (int)(n_vert + 1), s);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(temp, sort_bytes, keys_in, keys_out, ids, slots, (int)m, 0, end_bit, s);
    // group widths and offsets (gsize[ng] = 0, so grp_off[ng] is the total)
    if (e == hipSuccess) e = hipMemsetAsync(gsize + ng, 0, sizeof(int64_t), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(assembly_width_kernel, dim3(grid_for(ng)), dim3(256), 0, s, ng, n_vert, row_ptr,
                           p->grp_width, gsize);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(temp, gscan_bytes, gsize, p->grp_off, (int)(ng + 1), s);
    int64_t total = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&total, p->grp_off + ng, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMalloc(&p->sell, (size_t)std::max<int64_t>(total, 1) * sizeof(uint32_t));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(assembly_slice_kernel, dim3(grid_for(ng * 64)), dim3(256), 0, s, ng, n_vert, row_ptr, slots,
                           p->grp_width, p->grp_off, p->sell);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "fem_assembly_plan_create: index build"); }
    *out = p;
    return FEM_OK;
}

fem_status fem_assemble(const fem_assembly_plan* plan, int n_comp, int dtype, const void* elem_vec, void* vertex_vec,
                        void* stream) {
    if (!plan) { set_error("fem_assemble: NULL plan"); return FEM_ERR_INVALID_ARG; }
    if (n_comp < 1 || n_comp > 3) { set_error("fem_assemble: n_comp must be 1, 2 or 3 (got %d)", n_comp); return FEM_ERR_UNSUPPORTED; }
    if (dtype != FEM_F32 && dtype != FEM_F64) { set_error("fem_assemble: unknown dtype %d", dtype); return FEM_ERR_UNSUPPORTED; }
    if (plan->n_vert == 0) return FEM_OK;
    if (!vertex_vec || (plan->n_elem > 0 && !elem_vec)) { set_error("fem_assemble: NULL array"); return FEM_ERR_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (plan->dim == 2)
        e = dtype == FEM_F32 ? launch_assemble_nc<3, float>(n_comp, plan, elem_vec, vertex_vec, s)
                             : launch_assemble_nc<3, double>(n_comp, plan, elem_vec, vertex_vec, s);
    else
        e = dtype == FEM_F32 ? launch_assemble_nc<4, float>(n_comp, plan, elem_vec, vertex_vec, s)
                             : launch_assemble_nc<4, double>(n_comp, plan, elem_vec, vertex_vec, s);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_assemble launch");
}

fem_status fem_assembly_plan_info(const fem_assembly_plan* plan, int* dim, int64_t* n_elem, int64_t* n_vert) {
    if (!plan) { set_error("fem_assembly_plan_info: NULL plan"); return FEM_ERR_INVALID_ARG; }
    if (dim) *dim = plan->dim;
    if (n_elem) *n_elem = plan->n_elem;
    if (n_vert) *n_vert = plan->n_vert;
    return FEM_OK;
}

void fem_assembly_plan_destroy(fem_assembly_plan* plan) { plan_free(plan); }

fem_status fem_restrict(int dim, int n_comp, int dtype, int64_t n_elem, int64_t n_vert, const int32_t* conn,
                        const void* vertex_vec, void* elem_vec, void* stream) {
    if (dim != 2 && dim != 3) { set_error("fem_restrict: dim must be 2 or 3 (got %d)", dim); return FEM_ERR_UNSUPPORTED; }
    if (n_comp < 1 || n_comp > 3) { set_error("fem_restrict: n_comp must be 1, 2 or 3 (got %d)", n_comp); return FEM_ERR_UNSUPPORTED; }
    if (dtype != FEM_F32 && dtype != FEM_F64) { set_error("fem_restrict: unknown dtype %d", dtype); return FEM_ERR_UNSUPPORTED; }
    if (n_elem < 0 || n_vert < 0) { set_error("fem_restrict: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (n_vert == 0) { set_error("fem_restrict: elements without vertices"); return FEM_ERR_INVALID_ARG; }
    if (!conn || !vertex_vec || !elem_vec) { set_error("fem_restrict: NULL array"); return FEM_ERR_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (dim == 2)
        e = dtype == FEM_F32 ? launch_restrict_nc<3, float>(n_comp, n_elem, n_vert, conn, vertex_vec, elem_vec, s)
                             : launch_restrict_nc<3, double>(n_comp, n_elem, n_vert, conn, vertex_vec, elem_vec, s);
    else
        e = dtype == FEM_F32 ? launch_restrict_nc<4, float>(n_comp, n_elem, n_vert, conn, vertex_vec, elem_vec, s)
                             : launch_restrict_nc<4, double>(n_comp, n_elem, n_vert, conn, vertex_vec, elem_vec, s);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_restrict launch");
}

}  // extern "C"
