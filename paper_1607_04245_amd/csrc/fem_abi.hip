// fem_abi.hip -- the extern "C" entry points of libfemq (include/fem.h):
// argument validation, launch configuration, dispatch to the kernels.
//
// Validation happens before any HIP call, so invalid arguments are reported
// without touching a device. The hot-path calls never allocate, free or
// synchronize.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "fem.h"
#include "fem_internal.hpp"

namespace femq {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
}

fem_status hip_fail(hipError_t e, const char* what) {
    set_error("%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return FEM_ERR_HIP;
}

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) cache[dev] = cus;
    }
    return cache[dev];
}

// ------------------------------------------------------------- validation --

static bool valid_dim(int dim) { return dim == 2 || dim == 3; }
static bool valid_dtype(int dt) { return dt == FEM_F32 || dt == FEM_F64; }
static bool valid_phys(int p) { return p == FEM_LAPLACE || p == FEM_ELASTICITY || p == FEM_MASS; }
static bool valid_rule(int dim, int rule) {
    return rule == FEM_RULE_CENTROID || (dim == 2 && rule == FEM_RULE_TRI3) || (dim == 3 && rule == FEM_RULE_TET4);
}

static bool valid_space(int sp) { return sp == FEM_COEF_QUAD || sp == FEM_COEF_P1 || sp == FEM_COEF_P0; }

static fem_status check_space(const char* fn, int space) {
    if (!valid_space(space)) { set_error("%s: unknown coefficient space %d", fn, space); return FEM_ERR_UNSUPPORTED; }
    return FEM_OK;
}

// Rules of the second-order entry points: the degree-2 and degree-4 rules.
static bool valid_rule_p2(int dim, int rule) {
    return dim == 2 ? (rule == FEM_RULE_TRI3 || rule == FEM_RULE_TRI6) : (rule == FEM_RULE_TET4 || rule == FEM_RULE_TET11);
}

static fem_status check_combo_p2(const char* fn, int dim, int phys, int rule, int dtype) {
    if (!valid_dim(dim)) { set_error("%s: dim must be 2 or 3 (got %d)", fn, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_phys(phys)) { set_error("%s: unknown physics %d", fn, phys); return FEM_ERR_UNSUPPORTED; }
    if (!valid_rule_p2(dim, rule)) { set_error("%s: rule %d is not available for P2 in %dD", fn, rule, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_dtype(dtype)) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    return FEM_OK;
}

// P3 elements take the degree-4 rule of their dimension, which integrates
// a stiffness entry with a constant coefficient exactly.
static fem_status check_combo_p3(const char* fn, int dim, int phys, int rule, int dtype) {
    if (!valid_dim(dim)) { set_error("%s: dim must be 2 or 3 (got %d)", fn, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_phys(phys)) { set_error("%s: unknown physics %d", fn, phys); return FEM_ERR_UNSUPPORTED; }
    if (rule != (dim == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11)) {
        set_error("%s: P3 in %dD takes rule %d only (got %d)", fn, dim, dim == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11, rule);
        return FEM_ERR_UNSUPPORTED;
    }
    if (!valid_dtype(dtype)) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    return FEM_OK;
}

// Rules of the element-matrix entry point for each order.
static bool valid_rule_jac(int dim, int order, int rule) {
    const int low = dim == 2 ? FEM_RULE_TRI3 : FEM_RULE_TET4, high = dim == 2 ? FEM_RULE_TRI6 : FEM_RULE_TET11;
    if (order == 3) return rule == high;
    return rule == low || (order == 1 && rule == FEM_RULE_CENTROID) || (order == 2 && rule == high);
}

static fem_status check_combo_jac(const char* fn, int dim, int phys, int order, int rule, int dtype) {
    if (!valid_dim(dim)) { set_error("%s: dim must be 2 or 3 (got %d)", fn, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_phys(phys)) { set_error("%s: unknown physics %d", fn, phys); return FEM_ERR_UNSUPPORTED; }
    if (order < 1 || order > 3) { set_error("%s: order must be 1, 2 or 3 (got %d)", fn, order); return FEM_ERR_UNSUPPORTED; }
    if (!valid_rule_jac(dim, order, rule)) {
        set_error("%s: rule %d is not available for order %d in %dD", fn, rule, order, dim);
        return FEM_ERR_UNSUPPORTED;
    }
    if (!valid_dtype(dtype)) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    return FEM_OK;
}

static fem_status check_combo(const char* fn, int dim, int phys, int rule, int dtype) {
    if (!valid_dim(dim)) { set_error("%s: dim must be 2 or 3 (got %d)", fn, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_phys(phys)) { set_error("%s: unknown physics %d", fn, phys); return FEM_ERR_UNSUPPORTED; }
    if (!valid_rule(dim, rule)) { set_error("%s: rule %d is not defined in %dD", fn, rule, dim); return FEM_ERR_UNSUPPORTED; }
    if (!valid_dtype(dtype)) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
    return FEM_OK;
}

// ---------------------------------------------------------------- tuning --

typedef std::tuple<int, int, int, int, int> TuneKey;
static std::mutex g_tune_mu;
static std::map<TuneKey, fem_tuning> g_tune;

static bool valid_op(int op) {
    return op == FEM_OP_RESIDUAL || op == FEM_OP_RESIDUAL_MESH || op == FEM_OP_GEOMETRY || op == FEM_OP_BACKWARD ||
           op == FEM_OP_RESIDUAL_GATHER || op == FEM_OP_RESIDUAL_P2 || op == FEM_OP_BACKWARD_P2 ||
           op == FEM_OP_JACOBIAN || op == FEM_OP_JACOBIAN_P2 || op == FEM_OP_RESIDUAL_P3 || op == FEM_OP_BACKWARD_P3 ||
           op == FEM_OP_JACOBIAN_P3;
}

// Ops whose kernels take one element per lane and at most four waves per
// workgroup (register-heavy elements).
static bool one_per_lane_op(int op) {
    return op == FEM_OP_RESIDUAL_P2 || op == FEM_OP_BACKWARD_P2 || op == FEM_OP_JACOBIAN || op == FEM_OP_JACOBIAN_P2 ||
           op == FEM_OP_RESIDUAL_P3 || op == FEM_OP_BACKWARD_P3 || op == FEM_OP_JACOBIAN_P3;
}

// The geometry does not depend on physics or rule: one key per (dim, dtype).
static TuneKey tune_key(int op, int dim, int phys, int rule, int dtype) {
    if (op == FEM_OP_GEOMETRY) phys = rule = 0;
    return TuneKey(op, dim, phys, rule, dtype);
}

// Built-in launch configurations: the winners of the autotuner's sweep on
// one MI355X for the benchmark workloads (one element per lane was within a
// few percent of the best everywhere; wider accesses raise register pressure
// without adding bandwidth); other combinations use the robust middle choice.
static fem_tuning default_tuning(int op, int dim, int phys, int rule, int dtype) {
    fem_tuning t{FEM_STRATEGY_LANE, 1, 2, 0};
    const bool f32 = dtype == FEM_F32;
    if (op == FEM_OP_GEOMETRY) return fem_tuning{FEM_STRATEGY_LANE, 4, 4, 0};
    if (op == FEM_OP_JACOBIAN || op == FEM_OP_JACOBIAN_P2) {  // store-bound: more waves for the large matrices
        if (phys == FEM_ELASTICITY) return fem_tuning{FEM_STRATEGY_LANE, 1, 4, 16};
        return op == FEM_OP_JACOBIAN_P2 ? fem_tuning{FEM_STRATEGY_LANE, 1, 4, 0} : fem_tuning{FEM_STRATEGY_LANE, 1, 2, 0};
    }
    // P3: the 3D elements hold 20-60 closure and output words per lane, and
    // single-wave workgroups measured fastest there; 2D streams better with
    // four. (The component split of 3D elasticity measured 5-10 % slower than
    // the lane kernel with both timed on a warmed-up GPU.)
    if (op == FEM_OP_RESIDUAL_P3 || op == FEM_OP_BACKWARD_P3) return fem_tuning{FEM_STRATEGY_LANE, 1, dim == 3 ? 1 : 4, 0};
    if (op == FEM_OP_JACOBIAN_P3) return fem_tuning{FEM_STRATEGY_LANE, 1, 4, 0};
    if (one_per_lane_op(op)) return fem_tuning{FEM_STRATEGY_LANE, 1, 2, 0};
    if (op == FEM_OP_RESIDUAL_GATHER) return fem_tuning{FEM_STRATEGY_LANE, 2, 1, 0};
    if (op == FEM_OP_RESIDUAL_MESH) {
        if (phys == FEM_LAPLACE && f32) return fem_tuning{FEM_STRATEGY_LANE, 1, 1, 8};
        if (phys == FEM_ELASTICITY && f32) return fem_tuning{FEM_STRATEGY_LANE, 2, 2, 0};
        return fem_tuning{FEM_STRATEGY_LANE, 2, 1, 0};
    }
    const bool deg2 = rule != FEM_RULE_CENTROID;
    if (deg2 && phys == FEM_LAPLACE && dim == 3) t = f32 ? fem_tuning{0, 1, 2, 16} : fem_tuning{0, 1, 1, 0};
    if (deg2 && phys == FEM_ELASTICITY && dim == 2) t = f32 ? fem_tuning{0, 1, 4, 4} : fem_tuning{0, 1, 4, 0};
    if (deg2 && phys == FEM_ELASTICITY && dim == 3) t = f32 ? fem_tuning{0, 1, 4, 2} : fem_tuning{0, 1, 1, 2};
    return t;
}

// The matrix-core transposition exists for P3 tetrahedra with an f1 physics.
static bool mfma_available(int op, int dim, int phys) {
    return op == FEM_OP_RESIDUAL_P3 && dim == 3 && (phys == FEM_LAPLACE || phys == FEM_ELASTICITY);
}

// The component-parallel kernel exists for P3 tetrahedra with elasticity.
static bool component_available(int op, int dim, int phys) {
    return op == FEM_OP_RESIDUAL_P3 && dim == 3 && phys == FEM_ELASTICITY;
}

static bool valid_tuning(int op, const fem_tuning& t) {
    const bool strategy_ok = t.strategy == FEM_STRATEGY_LANE ||
                             ((t.strategy == FEM_STRATEGY_TRANSPOSE || t.strategy == FEM_STRATEGY_SHUFFLE) &&
                              op == FEM_OP_RESIDUAL) ||
                             ((t.strategy == FEM_STRATEGY_MFMA || t.strategy == FEM_STRATEGY_COMPONENT) &&
                              op == FEM_OP_RESIDUAL_P3) ||
                             (t.strategy == FEM_STRATEGY_DEDUP && op == FEM_OP_RESIDUAL_MESH && t.vec == 1);
    const bool one = one_per_lane_op(op);
    const bool vec_ok = one ? t.vec == 1 : (t.vec == 1 || t.vec == 2 || t.vec == 4);
    const bool waves_ok = t.waves_per_block == 1 || t.waves_per_block == 2 || t.waves_per_block == 4 ||
                          (t.waves_per_block == 8 && !one);
    return strategy_ok && vec_ok && waves_ok &&
           t.blocks_per_cu >= 0 && t.blocks_per_cu <= 64;
}

// The tuning cache named by the FEM_TUNE_CACHE environment variable is loaded
// once, before the first lookup or change of a tuning, so that explicit
// settings made afterwards take precedence. A missing file, or one without
// entries for this device, leaves the defaults (and the caller's error
// message) untouched. Lookups from other threads while the file is being
// read see the defaults.
static std::atomic<int> g_env_cache{0};   // 0 not loaded, 1 loading, 2 done

static void load_env_cache() {
    if (g_env_cache.load(std::memory_order_acquire) == 2) return;
    int expected = 0;
    if (!g_env_cache.compare_exchange_strong(expected, 1)) return;   // loaded or being loaded
    const char* path = std::getenv("FEM_TUNE_CACHE");
    if (path && *path) {
        const std::string saved = g_error;
        (void)fem_load_tuning(path);   // its fem_set_tuning calls return here at once
        g_error = saved;
    }
    g_env_cache.store(2, std::memory_order_release);
}

fem_tuning get_tuning(int op, int dim, int phys, int rule, int dtype) {
    load_env_cache();
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tune_key(op, dim, phys, rule, dtype));
    return it != g_tune.end() ? it->second : default_tuning(op, dim, phys, rule, dtype);
}

void put_tuning(int op, int dim, int phys, int rule, int dtype, const fem_tuning& t) {
    load_env_cache();
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[tune_key(op, dim, phys, rule, dtype)] = t;
}

// Largest vector width <= want such that every row of every array starts on
// a vec-word boundary.
static int usable_vec(int want, int64_t n, size_t word, const void* const* ptrs, int nptr) {
    for (int v = want; v > 1; v >>= 1) {
        if (n % v) continue;
        bool ok = true;
        for (int i = 0; i < nptr; ++i)
            if (ptrs[i] && (reinterpret_cast<uintptr_t>(ptrs[i]) % (v * word))) ok = false;
        if (ok) return v;
    }
    return 1;
}

static Launch make_launch(const fem_tuning& t, int64_t work_items, int vec, hipStream_t s) {
    Launch l;
    l.vec = vec;
    l.block = 64 * t.waves_per_block;
    l.stream = s;
    int64_t need = (work_items + l.block - 1) / l.block;
    if (need < 1) need = 1;
    if (t.blocks_per_cu > 0) {
        int cus = device_cus();
        int64_t cap = (int64_t)t.blocks_per_cu * (cus > 0 ? cus : 256);
        if (need > cap) need = cap;
    }
    if (need > (1 << 22)) need = 1 << 22;  // the grid-stride loop covers the rest
    l.grid = (int)need;
    return l;
}

// Kernels that give each wave tiles of 64*ept elements.
static Launch make_tile_launch(const fem_tuning& t, int64_t n, hipStream_t s) {
    const int64_t tiles = (n + 64 * t.vec - 1) / (64 * t.vec);
    Launch l = make_launch(t, tiles * 64, t.vec, s);
    return l;
}

static fem_status check_tuning_args(const char* fn, int op, int dim, int physics, int rule, int dtype) {
    if (!valid_op(op)) { set_error("%s: unknown op %d", fn, op); return FEM_ERR_UNSUPPORTED; }
    if (op == FEM_OP_GEOMETRY) {
        if (!valid_dim(dim)) { set_error("%s: dim must be 2 or 3 (got %d)", fn, dim); return FEM_ERR_UNSUPPORTED; }
        if (!valid_dtype(dtype)) { set_error("%s: unknown dtype %d", fn, dtype); return FEM_ERR_UNSUPPORTED; }
        return FEM_OK;
    }
    if (op == FEM_OP_RESIDUAL_P2 || op == FEM_OP_BACKWARD_P2) return check_combo_p2(fn, dim, physics, rule, dtype);
    if (op == FEM_OP_RESIDUAL_P3 || op == FEM_OP_BACKWARD_P3) return check_combo_p3(fn, dim, physics, rule, dtype);
    if (op == FEM_OP_JACOBIAN || op == FEM_OP_JACOBIAN_P2)
        return check_combo_jac(fn, dim, physics, op == FEM_OP_JACOBIAN ? 1 : 2, rule, dtype);
    if (op == FEM_OP_JACOBIAN_P3) return check_combo_jac(fn, dim, physics, 3, rule, dtype);
    return check_combo(fn, dim, physics, rule, dtype);
}

}  // namespace femq

using namespace femq;

extern "C" {

const char* fem_last_error(void) { return g_error.c_str(); }

fem_status fem_get_tuning(int op, int dim, int physics, int rule, int dtype, fem_tuning* out) {
    fem_status st = check_tuning_args("fem_get_tuning", op, dim, physics, rule, dtype);
    if (st) return st;
    if (!out) { set_error("fem_get_tuning: out is NULL"); return FEM_ERR_INVALID_ARG; }
    *out = get_tuning(op, dim, physics, rule, dtype);
    return FEM_OK;
}

fem_status fem_set_tuning(int op, int dim, int physics, int rule, int dtype, const fem_tuning* t) {
    fem_status st = check_tuning_args("fem_set_tuning", op, dim, physics, rule, dtype);
    if (st) return st;
    if (!t || !valid_tuning(op, *t)) { set_error("fem_set_tuning: invalid tuning for op %d", op); return FEM_ERR_INVALID_ARG; }
    if (t->strategy == FEM_STRATEGY_SHUFFLE && physics == FEM_ELASTICITY) {
        set_error("fem_set_tuning: the quad-permutation strategy covers scalar fields (Laplacian, mass)");
        return FEM_ERR_UNSUPPORTED;
    }
    if (t->strategy == FEM_STRATEGY_DEDUP && t->waves_per_block != 2 && t->waves_per_block != 4) {
        set_error("fem_set_tuning: the deduplicating strategy runs two or four waves per workgroup");
        return FEM_ERR_UNSUPPORTED;
    }
    if (t->strategy == FEM_STRATEGY_MFMA && !mfma_available(op, dim, physics)) {
        set_error("fem_set_tuning: the matrix-core strategy covers P3 tetrahedra with the Laplacian or elasticity");
        return FEM_ERR_UNSUPPORTED;
    }
    if (t->strategy == FEM_STRATEGY_COMPONENT && !component_available(op, dim, physics)) {
        set_error("fem_set_tuning: the component-parallel strategy covers P3 tetrahedra with elasticity");
        return FEM_ERR_UNSUPPORTED;
    }
    if (t->strategy == FEM_STRATEGY_COMPONENT && t->waves_per_block > comp_max_groups(dtype)) {
        set_error("fem_set_tuning: the component-parallel strategy runs at most %d three-wave group(s) per workgroup "
                  "for this dtype", comp_max_groups(dtype));
        return FEM_ERR_UNSUPPORTED;
    }
    put_tuning(op, dim, physics, rule, dtype, *t);
    return FEM_OK;
}

fem_status fem_geometry(int dim, int64_t n_elem, int64_t n_vert, const double* coords, const int32_t* conn,
                        int out_dtype, void* inv_j, void* det_j, int32_t* counts, void* stream) {
    if (!valid_dim(dim)) { set_error("fem_geometry: dim must be 2 or 3 (got %d)", dim); return FEM_ERR_INVALID_ARG; }
    if (!valid_dtype(out_dtype)) { set_error("fem_geometry: unknown dtype %d", out_dtype); return FEM_ERR_UNSUPPORTED; }
    if (n_elem < 0 || n_vert < 0) { set_error("fem_geometry: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (n_vert == 0) { set_error("fem_geometry: elements without vertices"); return FEM_ERR_INVALID_ARG; }
    if (!coords || !conn || !inv_j || !det_j) { set_error("fem_geometry: NULL array"); return FEM_ERR_INVALID_ARG; }
    const fem_tuning t = get_tuning(FEM_OP_GEOMETRY, dim, 0, 0, out_dtype);
    Launch l = make_tile_launch(t, n_elem, static_cast<hipStream_t>(stream));
    hipError_t e = launch_geometry(dim, out_dtype, n_elem, n_vert, coords, conn, inv_j, det_j, counts, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_geometry launch");
}

fem_status fem_integrate_residual(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                  const void* inv_j, const void* det_j, const void* u, const void* coef, void* elem_vec,
                                  void* stream) {
    fem_status st = check_combo("fem_integrate_residual", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (!inv_j || !det_j || !u || !coef || !elem_vec) {
        set_error("fem_integrate_residual: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    fem_tuning t = get_tuning(FEM_OP_RESIDUAL, dim, physics, rule, dtype);
    ResidualArgs a{n_elem, inv_j, det_j, u, coef, elem_vec};
    const size_t word = dtype == FEM_F32 ? 4 : 8;
    hipError_t e;
    if (t.strategy == FEM_STRATEGY_TRANSPOSE) {
        int threads = transpose_block_threads(dim, physics, rule, coef_space, dtype, t.waves_per_block);
        if (threads == 0) { set_error("fem_integrate_residual: transpose strategy unavailable"); return FEM_ERR_UNSUPPORTED; }
        Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
        l.block = threads;
        e = launch_residual_transpose(dim, physics, rule, coef_space, dtype, a, l);
    } else if (t.strategy == FEM_STRATEGY_SHUFFLE) {
        if (physics == FEM_ELASTICITY) {
            set_error("fem_integrate_residual: the quad-permutation strategy covers scalar fields");
            return FEM_ERR_UNSUPPORTED;
        }
        Launch l = make_launch(t, (n_elem + 15) / 16 * 64, 1, static_cast<hipStream_t>(stream));
        e = launch_residual_shuffle(dim, physics, rule, coef_space, dtype, a, l);
    } else {
        const void* ptrs[5] = {inv_j, det_j, u, coef, elem_vec};
        int vec = usable_vec(t.vec, n_elem, word, ptrs, 5);
        Launch l = make_launch(t, n_elem / vec, vec, static_cast<hipStream_t>(stream));
        e = launch_residual_lane(dim, physics, rule, coef_space, dtype, a, l);
    }
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual launch");
}

fem_status fem_integrate_residual_mesh(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                       int64_t n_vert,
                                       const double* coords, const int32_t* conn, const void* u, const void* coef,
                                       void* elem_vec, void* inv_j, void* det_j, int32_t* counts, void* stream) {
    fem_status st = check_combo("fem_integrate_residual_mesh", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_mesh", coef_space);
    if (st) return st;
    if (n_elem < 0 || n_vert < 0) { set_error("fem_integrate_residual_mesh: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (n_vert == 0) { set_error("fem_integrate_residual_mesh: elements without vertices"); return FEM_ERR_INVALID_ARG; }
    if (!coords || !conn || !u || !coef || !elem_vec || (!inv_j) != (!det_j)) {
        set_error("fem_integrate_residual_mesh: NULL array (inv_j and det_j must both be set or both NULL)");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_RESIDUAL_MESH, dim, physics, rule, dtype);
    MeshArgs a{n_elem, n_vert, coords, conn, u, coef, elem_vec, inv_j, det_j, counts};
    Launch l = make_tile_launch(t, n_elem, static_cast<hipStream_t>(stream));
    hipError_t e = t.strategy == FEM_STRATEGY_DEDUP ? launch_residual_dedup(dim, physics, rule, coef_space, dtype, a, l)
                                                    : launch_residual_mesh(dim, physics, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_mesh launch");
}

fem_status fem_integrate_residual_gather(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                         int64_t n_vert, const double* coords, const int32_t* conn,
                                         const void* u_vertex, const void* coef, void* elem_vec, void* inv_j,
                                         void* det_j, int32_t* counts, void* stream) {
    fem_status st = check_combo("fem_integrate_residual_gather", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_gather", coef_space);
    if (st) return st;
    if (n_elem < 0 || n_vert < 0) { set_error("fem_integrate_residual_gather: negative size"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (n_vert == 0) { set_error("fem_integrate_residual_gather: elements without vertices"); return FEM_ERR_INVALID_ARG; }
    if (!coords || !conn || !u_vertex || !coef || !elem_vec || (!inv_j) != (!det_j)) {
        set_error("fem_integrate_residual_gather: NULL array (inv_j and det_j must both be set or both NULL)");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_RESIDUAL_GATHER, dim, physics, rule, dtype);
    MeshArgs a{n_elem, n_vert, coords, conn, u_vertex, coef, elem_vec, inv_j, det_j, counts};
    Launch l = make_tile_launch(t, n_elem, static_cast<hipStream_t>(stream));
    hipError_t e = launch_residual_gather(dim, physics, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_gather launch");
}

fem_status fem_integrate_residual_backward(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                           const void* inv_j, const void* det_j, const void* u, const void* coef,
                                           const void* w, void* du, void* dcoef, void* stream) {
    fem_status st = check_combo("fem_integrate_residual_backward", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_backward", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual_backward: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0 || (!du && !dcoef)) return FEM_OK;
    if (!inv_j || !det_j || !w || (du && !coef) || (dcoef && !u)) {
        set_error("fem_integrate_residual_backward: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    fem_tuning t = get_tuning(FEM_OP_BACKWARD, dim, physics, rule, dtype);
    const size_t word = dtype == FEM_F32 ? 4 : 8;
    const void* ptrs[7] = {inv_j, det_j, w, du ? coef : nullptr, du, dcoef ? u : nullptr, dcoef};
    int vec = usable_vec(t.vec, n_elem, word, ptrs, 7);
    BackwardArgs a{n_elem, inv_j, det_j, u, coef, w, du, dcoef};
    Launch l = make_launch(t, n_elem / vec, vec, static_cast<hipStream_t>(stream));
    hipError_t e = launch_backward_lane(dim, physics, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_backward launch");
}

fem_status fem_integrate_residual_p2(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                     const void* inv_j, const void* det_j, const void* u, const void* coef,
                                     void* elem_vec, void* stream) {
    fem_status st = check_combo_p2("fem_integrate_residual_p2", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_p2", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual_p2: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (!inv_j || !det_j || !u || !coef || !elem_vec) {
        set_error("fem_integrate_residual_p2: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_RESIDUAL_P2, dim, physics, rule, dtype);
    ResidualArgs a{n_elem, inv_j, det_j, u, coef, elem_vec};
    Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
    hipError_t e = launch_residual_p2(dim, physics, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_p2 launch");
}

fem_status fem_integrate_residual_p3(int dim, int physics, int rule, int coef_space, int dtype, int64_t n_elem,
                                     const void* inv_j, const void* det_j, const void* u, const void* coef,
                                     void* elem_vec, void* stream) {
    fem_status st = check_combo_p3("fem_integrate_residual_p3", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_p3", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual_p3: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (!inv_j || !det_j || !u || !coef || !elem_vec) {
        set_error("fem_integrate_residual_p3: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_RESIDUAL_P3, dim, physics, rule, dtype);
    ResidualArgs a{n_elem, inv_j, det_j, u, coef, elem_vec};
    hipError_t e;
    if (t.strategy == FEM_STRATEGY_MFMA && mfma_available(FEM_OP_RESIDUAL_P3, dim, physics)) {
        // one wave per 16 elements
        Launch l = make_launch(t, (n_elem + 15) / 16 * 64, 1, static_cast<hipStream_t>(stream));
        e = launch_residual_p3_mfma(physics, coef_space, dtype, a, l);
    } else if (t.strategy == FEM_STRATEGY_COMPONENT && component_available(FEM_OP_RESIDUAL_P3, dim, physics)) {
        // three waves per 64-element tile; waves_per_block counts the
        // three-wave groups of a workgroup
        fem_tuning tg = t;
        tg.waves_per_block = 3 * t.waves_per_block;
        Launch l = make_launch(tg, (n_elem + 63) / 64 * 192, 1, static_cast<hipStream_t>(stream));
        e = launch_residual_p3_comp(coef_space, dtype, a, l);
    } else {
        Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
        e = launch_residual_p3(dim, physics, coef_space, dtype, a, l);
    }
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_p3 launch");
}

fem_status fem_integrate_residual_p2_backward(int dim, int physics, int rule, int coef_space, int dtype,
                                              int64_t n_elem, const void* inv_j, const void* det_j, const void* u,
                                              const void* coef, const void* w, void* du, void* dcoef, void* stream) {
    fem_status st = check_combo_p2("fem_integrate_residual_p2_backward", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_p2_backward", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual_p2_backward: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0 || (!du && !dcoef)) return FEM_OK;
    if (!inv_j || !det_j || !w || (du && !coef) || (dcoef && !u)) {
        set_error("fem_integrate_residual_p2_backward: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_BACKWARD_P2, dim, physics, rule, dtype);
    BackwardArgs a{n_elem, inv_j, det_j, u, coef, w, du, dcoef};
    Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
    hipError_t e = launch_backward_p2(dim, physics, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_p2_backward launch");
}

fem_status fem_integrate_residual_p3_backward(int dim, int physics, int rule, int coef_space, int dtype,
                                              int64_t n_elem, const void* inv_j, const void* det_j, const void* u,
                                              const void* coef, const void* w, void* du, void* dcoef, void* stream) {
    fem_status st = check_combo_p3("fem_integrate_residual_p3_backward", dim, physics, rule, dtype);
    if (!st) st = check_space("fem_integrate_residual_p3_backward", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_residual_p3_backward: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0 || (!du && !dcoef)) return FEM_OK;
    if (!inv_j || !det_j || !w || (du && !coef) || (dcoef && !u)) {
        set_error("fem_integrate_residual_p3_backward: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    const fem_tuning t = get_tuning(FEM_OP_BACKWARD_P3, dim, physics, rule, dtype);
    BackwardArgs a{n_elem, inv_j, det_j, u, coef, w, du, dcoef};
    Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
    hipError_t e = launch_backward_p3(dim, physics, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_residual_p3_backward launch");
}

fem_status fem_integrate_jacobian(int dim, int physics, int rule, int coef_space, int order, int dtype,
                                  int64_t n_elem, const void* inv_j, const void* det_j, const void* coef,
                                  void* elem_mat, void* stream) {
    fem_status st = check_combo_jac("fem_integrate_jacobian", dim, physics, order, rule, dtype);
    if (!st) st = check_space("fem_integrate_jacobian", coef_space);
    if (st) return st;
    if (n_elem < 0) { set_error("fem_integrate_jacobian: negative n_elem"); return FEM_ERR_INVALID_ARG; }
    if (n_elem == 0) return FEM_OK;
    if (!inv_j || !det_j || !coef || !elem_mat) {
        set_error("fem_integrate_jacobian: NULL array");
        return FEM_ERR_INVALID_ARG;
    }
    const int op = order == 1 ? FEM_OP_JACOBIAN : order == 2 ? FEM_OP_JACOBIAN_P2 : FEM_OP_JACOBIAN_P3;
    const fem_tuning t = get_tuning(op, dim, physics, rule, dtype);
    JacobianArgs a{n_elem, inv_j, det_j, coef, elem_mat};
    Launch l = make_launch(t, n_elem, 1, static_cast<hipStream_t>(stream));
    hipError_t e = order == 3 ? launch_jacobian_p3(dim, physics, coef_space, dtype, a, l)
                              : launch_jacobian(dim, physics, order, rule, coef_space, dtype, a, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_integrate_jacobian launch");
}

fem_status fem_stream_copy(const void* src, void* dst, int64_t n_bytes, void* stream) {
    if (n_bytes < 0 || (n_bytes % 16) || (reinterpret_cast<uintptr_t>(src) % 16) ||
        (reinterpret_cast<uintptr_t>(dst) % 16)) {
        set_error("fem_stream_copy: sizes and pointers must be multiples of 16 bytes");
        return FEM_ERR_INVALID_ARG;
    }
    if (n_bytes == 0) return FEM_OK;
    if (!src || !dst) { set_error("fem_stream_copy: NULL pointer"); return FEM_ERR_INVALID_ARG; }
    fem_tuning t{FEM_STRATEGY_LANE, 1, 4, 0};
    Launch l = make_launch(t, n_bytes / 16, 1, static_cast<hipStream_t>(stream));
    hipError_t e = launch_stream_copy(src, dst, n_bytes, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_stream_copy launch");
}

fem_status fem_stream_rows(int dtype, int64_t n, int n_in, int n_out, const void* src, void* dst, void* stream) {
    if (!valid_dtype(dtype)) { set_error("fem_stream_rows: unknown dtype %d", dtype); return FEM_ERR_UNSUPPORTED; }
    if (n < 0 || n_in < 1 || n_in > FEM_STREAM_ROWS_MAX || n_out < 1 || n_out > FEM_STREAM_ROWS_MAX) {
        set_error("fem_stream_rows: n must be >= 0 and the row counts in 1..%d", FEM_STREAM_ROWS_MAX);
        return FEM_ERR_INVALID_ARG;
    }
    if (n == 0) return FEM_OK;
    if (!src || !dst) { set_error("fem_stream_rows: NULL pointer"); return FEM_ERR_INVALID_ARG; }
    fem_tuning t{FEM_STRATEGY_LANE, 1, 4, 0};
    Launch l = make_launch(t, n, 1, static_cast<hipStream_t>(stream));
    hipError_t e = launch_stream_rows(dtype, n, n_in, n_out, src, dst, l);
    return e == hipSuccess ? FEM_OK : hip_fail(e, "fem_stream_rows launch");
}

}  // extern "C"
