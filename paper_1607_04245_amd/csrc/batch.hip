// batch.hip -- many meshes of mixed dimension and physics integrated by one
// persistent launch, optionally recorded into a HIP graph.
//
// The plan concatenates the meshes' element ranges into one list of tiles
// (one tile = one workgroup's worth of elements, one element per lane) and
// stores, per tile, the index of its mesh. Each persistent workgroup takes a
// fixed contiguous run of tiles, so there is no work counter to reset between
// launches and the assignment is the same on every replay. The workgroup
// reads the descriptor of its first tile's mesh (wave-uniform loads), keeps
// it while its tiles stay in that mesh, and branches, uniformly, into the
// element code of the mesh's (dim, physics, rule, coefficient space). Each element runs exactly the arithmetic of the
// single-mesh lane kernel, so batched and single-mesh results are bitwise
// equal. This plays the role of the paper's assignment of cell chunks to
// thread blocks (Section 3), across meshes instead of within one.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

constexpr int type_code(int dim, int phys, int rule, int space) { return dim * 64 + space * 16 + phys * 4 + rule; }

template <int DIM, int PHYS, int RULE, typename Real>
__device__ __forceinline__ void batch_element(const BatchMesh& M, int64_t e) {
    using E = Elem<DIM, PHYS, RULE>;
    const int64_t n = M.n_elem;
    const Real* __restrict__ ijp = static_cast<const Real*>(M.inv_j);
    const Real* __restrict__ djp = static_cast<const Real*>(M.det_j);
    const Real* __restrict__ up = static_cast<const Real*>(M.u);
    const Real* __restrict__ cfp = static_cast<const Real*>(M.coef);
    Real* __restrict__ outp = static_cast<Real*>(M.out);
    Real ij[E::NG], uu[E::NBT], cf[E::NCQ], r[E::NBT];
#pragma unroll
    for (int f = 0; f < E::NG; ++f) ij[f] = __builtin_nontemporal_load(ijp + f * n + e);
    const Real dj = __builtin_nontemporal_load(djp + e);
#pragma unroll
    for (int f = 0; f < E::NBT; ++f) uu[f] = __builtin_nontemporal_load(up + f * n + e);
#pragma unroll
    for (int f = 0; f < E::NCQ; ++f) cf[f] = __builtin_nontemporal_load(cfp + f * n + e);
    element_residual<DIM, PHYS, RULE, Real>(ij, dj, uu, cf, r);
#pragma unroll
    for (int f = 0; f < E::NBT; ++f) __builtin_nontemporal_store(r[f], outp + f * n + e);
}

template <typename Real>
__device__ __forceinline__ void batch_tile(const BatchMesh& M, int64_t t) {
    const int64_t e = (t - M.tile_begin) * blockDim.x + threadIdx.x;
    if (e >= M.n_elem) return;
    switch (M.type) {
#define FEMQ_CASE_S(D, P, RU, SP) \
    case type_code(D, P, RU, SP): batch_element<D, P, scheme(RU, SP), Real>(M, e); break;
#define FEMQ_CASE(D, P, RU)                \
    FEMQ_CASE_S(D, P, RU, FEM_COEF_QUAD)   \
    FEMQ_CASE_S(D, P, RU, FEM_COEF_P1)     \
    FEMQ_CASE_S(D, P, RU, FEM_COEF_P0)
        FEMQ_CASE(2, FEM_LAPLACE, FEM_RULE_TRI3)
        FEMQ_CASE(3, FEM_LAPLACE, FEM_RULE_TET4)
        FEMQ_CASE(2, FEM_ELASTICITY, FEM_RULE_TRI3)
        FEMQ_CASE(3, FEM_ELASTICITY, FEM_RULE_TET4)
        FEMQ_CASE(2, FEM_MASS, FEM_RULE_TRI3)
        FEMQ_CASE(3, FEM_MASS, FEM_RULE_TET4)
        FEMQ_CASE(2, FEM_LAPLACE, FEM_RULE_CENTROID)
        FEMQ_CASE(3, FEM_LAPLACE, FEM_RULE_CENTROID)
        FEMQ_CASE(2, FEM_ELASTICITY, FEM_RULE_CENTROID)
        FEMQ_CASE(3, FEM_ELASTICITY, FEM_RULE_CENTROID)
        FEMQ_CASE(2, FEM_MASS, FEM_RULE_CENTROID)
        FEMQ_CASE(3, FEM_MASS, FEM_RULE_CENTROID)
#undef FEMQ_CASE
#undef FEMQ_CASE_S
    default: break;
    }
}

// Each workgroup owns a contiguous run of tiles, which mostly lies in one
// mesh: the descriptor is read once and kept until the run crosses into the
// next mesh (tiles of a mesh are consecutive). The mesh of the first tile
// comes from the per-tile table, or, without one, from a binary search over
// the descriptors' tile ranges (every mesh in the table is non-empty, so the
// tile_begin values strictly increase).
template <typename Real>
__global__ void __launch_bounds__(512)
batch_kernel(const BatchMesh* __restrict__ meshes, int n_mesh, const int32_t* __restrict__ tile_mesh,
             int64_t n_tiles) {
    const int64_t t_begin = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t_end = ((int64_t)blockIdx.x + 1) * n_tiles / gridDim.x;
    if (t_begin >= t_end) return;
    int m;
    if (tile_mesh) {
        m = tile_mesh[t_begin];
    } else {
        int lo = 0, hi = n_mesh - 1;   // last mesh with tile_begin <= t_begin
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (meshes[mid].tile_begin <= t_begin) lo = mid; else hi = mid - 1;
        }
        m = lo;
    }
    BatchMesh M = meshes[m];
    for (int64_t t = t_begin; t < t_end; ++t) {
        while (t >= M.tile_end) M = meshes[++m];
        batch_tile<Real>(M, t);
    }
}

hipError_t launch_batch(int dtype, const BatchMesh* d_meshes, int n_mesh, const int32_t* d_tile_mesh,
                        int64_t n_tiles, int tile_elems, const Launch& l) {
    if (tile_elems != l.block || n_mesh < 1) return hipErrorInvalidValue;
    if (dtype == FEM_F32)
        hipLaunchKernelGGL(batch_kernel<float>, dim3(l.grid), dim3(l.block), 0, l.stream, d_meshes, n_mesh,
                           d_tile_mesh, n_tiles);
    else
        hipLaunchKernelGGL(batch_kernel<double>, dim3(l.grid), dim3(l.block), 0, l.stream, d_meshes, n_mesh,
                           d_tile_mesh, n_tiles);
    return hipGetLastError();
}

}  // namespace femq

using namespace femq;

struct fem_batch_plan {
    int device = -1;
    int dtype = FEM_F32;
    int n_mesh = 0;              // non-empty meshes in the device table
    int64_t n_tiles = 0;
    int64_t n_elem_total = 0;
    int waves_per_block = 8;   // measured on MI355X: one 512-element tile per
    int blocks_per_cu = 0;     // workgroup beats persistent grids
    BatchMesh* d_meshes = nullptr;
    int32_t* d_tile_mesh = nullptr;   // mesh index of every tile
    int64_t tile_mesh_cap = 0;        // elements allocated in d_tile_mesh
    std::vector<BatchMesh> h_meshes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Launch shape of the persistent kernel: one workgroup per tile, or
// blocks_per_cu workgroups per compute unit, each taking a contiguous run.
static Launch batch_shape(int64_t n_tiles, int waves_per_block, int blocks_per_cu, hipStream_t s) {
    Launch l;
    l.block = 64 * waves_per_block;
    l.vec = 1;
    l.stream = s;
    int cus = device_cus();
    int64_t grid = (int64_t)blocks_per_cu * (cus > 0 ? cus : 256);
    if (blocks_per_cu == 0 || grid > n_tiles) grid = n_tiles;
    if (grid > (1 << 22)) grid = 1 << 22;
    l.grid = (int)grid;
    return l;
}

static bool valid_batch_shape(int waves_per_block, int blocks_per_cu) {
    return (waves_per_block == 1 || waves_per_block == 2 || waves_per_block == 4 || waves_per_block == 8) &&
           blocks_per_cu >= 0 && blocks_per_cu <= 64;
}

// Global tile ranges of the meshes (consecutive, in table order); returns
// the number of tiles.
static int64_t assign_tiles(BatchMesh* m, int n, int tile) {
    int64_t t = 0;
    for (int i = 0; i < n; ++i) {
        m[i].tile_begin = t;
        t += (m[i].n_elem + tile - 1) / tile;
        m[i].tile_end = t;
    }
    return t;
}

// Device descriptor of one caller mesh (tile range left to assign_tiles).
static void make_descriptor(const fem_mesh_desc& d, BatchMesh& m) {
    std::memset(&m, 0, sizeof m);
    m.type = type_code(d.dim, d.physics, d.rule, d.coef_space);
    m.n_elem = d.n_elem;
    m.inv_j = d.inv_j;
    m.det_j = d.det_j;
    m.u = d.u;
    m.coef = d.coef;
    m.out = d.elem_vec;
}

// Checks the caller's mesh list and, when out is not NULL, writes the
// device descriptor of every non-empty mesh to out (room for n_mesh);
// *n_out = their number, *total_out = their elements.
static fem_status fill_descriptors(const char* fn, const fem_mesh_desc* meshes, int n_mesh, BatchMesh* out,
                                   int* n_out, int64_t* total_out) {
    int k = 0;
    int64_t total = 0;
    for (int i = 0; i < n_mesh; ++i) {
        const fem_mesh_desc& d = meshes[i];
        const bool dim_ok = d.dim == 2 || d.dim == 3;
        const bool phys_ok = d.physics == FEM_LAPLACE || d.physics == FEM_ELASTICITY || d.physics == FEM_MASS;
        const bool rule_ok = d.rule == FEM_RULE_CENTROID || (d.dim == 2 && d.rule == FEM_RULE_TRI3) ||
                             (d.dim == 3 && d.rule == FEM_RULE_TET4);
        const bool space_ok = d.coef_space == FEM_COEF_QUAD || d.coef_space == FEM_COEF_P1 ||
                              d.coef_space == FEM_COEF_P0;
        if (!dim_ok || !phys_ok || !rule_ok || !space_ok) {
            set_error("%s: mesh %d has an unsupported (dim, physics, rule, coef_space)", fn, i);
            return FEM_ERR_UNSUPPORTED;
        }
        if (d.n_elem < 0) { set_error("%s: mesh %d has negative n_elem", fn, i); return FEM_ERR_INVALID_ARG; }
        if (d.n_elem == 0) continue;
        if (!d.inv_j || !d.det_j || !d.u || !d.coef || !d.elem_vec) {
            set_error("%s: mesh %d has a NULL array", fn, i);
            return FEM_ERR_INVALID_ARG;
        }
        if (out) make_descriptor(d, out[k]);
        ++k;
        total += d.n_elem;
    }
    *n_out = k;
    *total_out = total;
    return FEM_OK;
}

static fem_status plan_launch(fem_batch_plan* p, hipStream_t s) {
    if (p->n_tiles == 0) return FEM_OK;
    const Launch l = batch_shape(p->n_tiles, p->waves_per_block, p->blocks_per_cu, s);
    hipError_t e = launch_batch(p->dtype, p->d_meshes, p->n_mesh, p->d_tile_mesh, p->n_tiles, l.block, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_batch launch");
}

static fem_status plan_build_table(fem_batch_plan* p) {
    const int tile = 64 * p->waves_per_block;
    const int64_t t = assign_tiles(p->h_meshes.data(), (int)p->h_meshes.size(), tile);
    p->n_tiles = t;
    if (p->h_meshes.empty()) return FEM_OK;
    hipError_t e = hipMemcpy(p->d_meshes, p->h_meshes.data(), p->h_meshes.size() * sizeof(BatchMesh),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "fem_batch descriptor upload");
    std::vector<int32_t> tm((size_t)t);
    for (size_t m = 0; m < p->h_meshes.size(); ++m) {
        const int64_t b = p->h_meshes[m].tile_begin;
        const int64_t end = m + 1 < p->h_meshes.size() ? p->h_meshes[m + 1].tile_begin : t;
        for (int64_t k = b; k < end; ++k) tm[(size_t)k] = (int32_t)m;
    }
    if (t > p->tile_mesh_cap) {
        if (p->d_tile_mesh) (void)hipFree(p->d_tile_mesh);
        p->d_tile_mesh = nullptr;
        p->tile_mesh_cap = 0;
        e = hipMalloc(&p->d_tile_mesh, (size_t)t * sizeof(int32_t));
        if (e != hipSuccess) return hip_fail(e, "fem_batch tile table");
        p->tile_mesh_cap = t;
    }
    e = hipMemcpy(p->d_tile_mesh, tm.data(), (size_t)t * sizeof(int32_t), hipMemcpyHostToDevice);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_batch tile table upload");
}

// ------------------------------------------------- no-allocation launch --
//
// The descriptor table of fem_batch_run_noalloc lives in this file-scope
// device array, one copy per GPU, for the life of the process. Host code
// never passes the array's name to a kernel or a copy: on the host that name
// stands for a host-side shadow, not a device address. The device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) and used everywhere instead.
static __device__ __align__(256) BatchMesh scratch[FEM_BATCH_NOALLOC_MAX_MESHES];

// Descriptors travel to the device array as kernel arguments (a chunk per
// launch, copied by the runtime when the launch is enqueued), so no host
// buffer has to outlive the call and nothing is copied from pageable memory.
constexpr int kDescChunk = 32;   // 32 x 72 bytes of kernel arguments
struct DescChunk {
    BatchMesh m[kDescChunk];
};

__global__ void __launch_bounds__(kDescChunk) store_descriptors_kernel(BatchMesh* table, DescChunk chunk, int k) {
    const int i = threadIdx.x;
    if (i < k) table[i] = chunk.m[i];
}

static std::mutex g_scratch_mu;
static BatchMesh* g_scratch_ptr[64] = {};

// Device address of the current device's descriptor array (NULL on failure,
// with the error set).
static BatchMesh* scratch_table(const char* fn) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { hip_fail(e, fn); return nullptr; }
    if (dev < 0 || dev >= 64) { set_error("%s: device %d out of range", fn, dev); return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        BatchMesh* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, fn);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

static void plan_drop_graph(fem_batch_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

extern "C" {

fem_status fem_batch_plan_create(const fem_mesh_desc* meshes, int n_mesh, int dtype, fem_batch_plan** out) {
    if (!out) { set_error("fem_batch_plan_create: out is NULL"); return FEM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (n_mesh < 0 || (n_mesh > 0 && !meshes)) { set_error("fem_batch_plan_create: bad mesh list"); return FEM_ERR_INVALID_ARG; }
    if (dtype != FEM_F32 && dtype != FEM_F64) { set_error("fem_batch_plan_create: unknown dtype %d", dtype); return FEM_ERR_UNSUPPORTED; }
    std::vector<BatchMesh> hm((size_t)n_mesh);
    int n_used = 0;
    int64_t total = 0;
    fem_status vst = fill_descriptors("fem_batch_plan_create", meshes, n_mesh, hm.data(), &n_used, &total);
    if (vst) return vst;
    hm.resize((size_t)n_used);
    fem_batch_plan* p = new (std::nothrow) fem_batch_plan();
    if (!p) { set_error("fem_batch_plan_create: out of host memory"); return FEM_ERR_INVALID_ARG; }
    p->dtype = dtype;
    p->h_meshes = std::move(hm);
    p->n_mesh = (int)p->h_meshes.size();
    p->n_elem_total = total;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return hip_fail(e, "fem_batch_plan_create"); }
    if (p->n_mesh > 0) {
        e = hipMalloc(&p->d_meshes, p->h_meshes.size() * sizeof(BatchMesh));
        if (e != hipSuccess) { delete p; return hip_fail(e, "fem_batch_plan_create: hipMalloc"); }
    }
    fem_status st = plan_build_table(p);
    if (st) { fem_batch_plan_destroy(p); return st; }
    *out = p;
    return FEM_OK;
}

fem_status fem_batch_plan_set_launch(fem_batch_plan* plan, int waves_per_block, int blocks_per_cu) {
    if (!plan) { set_error("fem_batch_plan_set_launch: NULL plan"); return FEM_ERR_INVALID_ARG; }
    if (!valid_batch_shape(waves_per_block, blocks_per_cu)) {
        set_error("fem_batch_plan_set_launch: invalid launch shape");
        return FEM_ERR_INVALID_ARG;
    }
    hipError_t e = hipDeviceSynchronize();  // no launch of this plan may still read the table
    if (e != hipSuccess) return hip_fail(e, "fem_batch_plan_set_launch");
    plan->waves_per_block = waves_per_block;
    plan->blocks_per_cu = blocks_per_cu;
    plan_drop_graph(plan);  // a recorded graph would still use the old shape
    return plan_build_table(plan);
}

fem_status fem_batch_plan_autotune(fem_batch_plan* plan, void* stream, int* waves_out, int* bpc_out) {
    if (!plan) { set_error("fem_batch_plan_autotune: NULL plan"); return FEM_ERR_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return hip_fail(e, "fem_batch_plan_autotune: events");
    }
    int best_w = plan->waves_per_block, best_b = plan->blocks_per_cu;
    float best_ms = 1e30f;
    fem_status st = FEM_OK;
    const int reps = 5;
    for (int w : {1, 2, 4, 8}) {
        for (int b : {0, 2, 4, 8, 16}) {
            st = fem_batch_plan_set_launch(plan, w, b);
            for (int r = 0; r < 2 && !st; ++r) st = plan_launch(plan, s);  // warm-up
            if (!st) e = hipEventRecord(t0, s);
            for (int r = 0; r < reps && !st && e == hipSuccess; ++r) st = plan_launch(plan, s);
            if (!st && e == hipSuccess) e = hipEventRecord(t1, s);
            if (!st && e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (!st && e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (st || e != hipSuccess) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_w = w;
                best_b = b;
            }
        }
        if (st || e != hipSuccess) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "fem_batch_plan_autotune: timing");
    if (st) return st;
    st = fem_batch_plan_set_launch(plan, best_w, best_b);
    if (st) return st;
    if (waves_out) *waves_out = best_w;
    if (bpc_out) *bpc_out = best_b;
    return FEM_OK;
}

fem_status fem_batch_run(fem_batch_plan* plan, void* stream) {
    if (!plan) { set_error("fem_batch_run: NULL plan"); return FEM_ERR_INVALID_ARG; }
    return plan_launch(plan, static_cast<hipStream_t>(stream));
}

fem_status fem_batch_run_noalloc(const fem_mesh_desc* meshes, int n_mesh, int dtype, int waves_per_block,
                                 int blocks_per_cu, void* stream) {
    static const char* fn = "fem_batch_run_noalloc";
    if (n_mesh < 0 || (n_mesh > 0 && !meshes)) { set_error("%s: bad mesh list", fn); return FEM_ERR_INVALID_ARG; }
    if (n_mesh > FEM_BATCH_NOALLOC_MAX_MESHES) {
        set_error("%s: %d meshes exceed the limit of %d (use a plan)", fn, n_mesh, FEM_BATCH_NOALLOC_MAX_MESHES);
        return FEM_ERR_INVALID_ARG;
    }
    if (dtype != FEM_F32 && dtype != FEM_F64) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    if (!valid_batch_shape(waves_per_block, blocks_per_cu)) { set_error("%s: invalid launch shape", fn); return FEM_ERR_INVALID_ARG; }
    // every mesh is checked before the first HIP call
    int n_used = 0;
    int64_t total = 0;
    fem_status st = fill_descriptors(fn, meshes, n_mesh, nullptr, &n_used, &total);
    if (st) return st;
    if (n_used == 0) return FEM_OK;
    BatchMesh* table = scratch_table(fn);
    if (!table) return FEM_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the table goes up in stream-ordered launches of kDescChunk descriptors
    DescChunk chunk;
    const int tile = 64 * waves_per_block;
    int k = 0, sent = 0;
    int64_t n_tiles = 0;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_mesh && e == hipSuccess; ++i) {
        if (meshes[i].n_elem == 0) continue;
        BatchMesh& m = chunk.m[k++];
        make_descriptor(meshes[i], m);
        m.tile_begin = n_tiles;
        n_tiles += (m.n_elem + tile - 1) / tile;
        m.tile_end = n_tiles;
        if (k == kDescChunk || sent + k == n_used) {
            hipLaunchKernelGGL(store_descriptors_kernel, dim3(1), dim3(kDescChunk), 0, s, table + sent, chunk, k);
            e = hipGetLastError();
            sent += k;
            k = 0;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "fem_batch_run_noalloc: descriptor upload");
    const Launch l = batch_shape(n_tiles, waves_per_block, blocks_per_cu, s);
    e = launch_batch(dtype, table, n_used, nullptr, n_tiles, l.block, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_batch_run_noalloc launch");
}

fem_status fem_batch_capture(fem_batch_plan* plan, void* stream) {
    if (!plan) { set_error("fem_batch_capture: NULL plan"); return FEM_ERR_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s == nullptr) { set_error("fem_batch_capture: capture needs a non-default stream"); return FEM_ERR_INVALID_ARG; }
    plan_drop_graph(plan);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "fem_batch_capture: begin");
    fem_status st = plan_launch(plan, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(e, "fem_batch_capture: end");
    plan->graph = g;
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { plan_drop_graph(plan); return hip_fail(e, "fem_batch_capture: instantiate"); }
    return FEM_OK;
}

fem_status fem_batch_replay(fem_batch_plan* plan, void* stream) {
    if (!plan || !plan->exec) { set_error("fem_batch_replay: plan not captured"); return FEM_ERR_INVALID_ARG; }
    hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_batch_replay");
}

void fem_batch_plan_destroy(fem_batch_plan* plan) {
    if (!plan) return;
    plan_drop_graph(plan);
    if (plan->d_meshes) (void)hipFree(plan->d_meshes);
    if (plan->d_tile_mesh) (void)hipFree(plan->d_tile_mesh);
    delete plan;
}

}  // extern "C"
