// tune.hip -- the autotuner and its JSON cache.
//
// The paper sweeps blocks per batch and batches per chunk and finds only a
// mild dependence (Section 6, Table 2); its analog here is a sweep over the
// kernel strategy (lane-per-element or thread transposition), the elements
// per lane of the coalesced accesses, the waves per workgroup and the
// persistent grid size. Every candidate runs on synthetic device data that
// rotates through enough copies to defeat the last-level cache, and is timed
// with HIP events; the fastest becomes the configuration of this process and
// is merged into an optional JSON cache keyed by GPU architecture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fem_device.hpp"
#include "fem_internal.hpp"

namespace femq {

// Deterministic pseudo-random fill (SplitMix64 finalizer on the index).
template <typename Real>
__global__ void __launch_bounds__(256)
fill_kernel(Real* __restrict__ p, int64_t n, uint64_t seed, double lo, double hi) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double x = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        p[i] = static_cast<Real>(lo + (hi - lo) * x);
    }
}

static hipError_t fill(int dtype, void* p, int64_t n, uint64_t seed, double lo, double hi) {
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (dtype == FEM_F32)
        hipLaunchKernelGGL(fill_kernel<float>, dim3(grid), dim3(256), 0, nullptr, static_cast<float*>(p), n, seed, lo, hi);
    else
        hipLaunchKernelGGL(fill_kernel<double>, dim3(grid), dim3(256), 0, nullptr, static_cast<double*>(p), n, seed, lo, hi);
    return hipGetLastError();
}

// Structured probe mesh: n_c^dim cells of the unit square/cube, two
// triangles or six Kuhn tetrahedra per cell, vertex (i, j[, k]) at
// (i, j[, k]) / n_c. Only used to time the mesh operations.
template <int DIM>
__global__ void __launch_bounds__(256)
probe_mesh_kernel(int64_t n_elem, int nc, int32_t* __restrict__ conn, double* __restrict__ X, int64_t n_vert) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t m = nc + 1;
    const double h = 1.0 / nc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vert; i += stride) {
        int64_t r = i;
        for (int d = DIM - 1; d >= 0; --d) {
            X[i * DIM + d] = h * (double)(r % m);
            r /= m;
        }
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        if constexpr (DIM == 2) {
            const int64_t cell = e / 2, ci = cell / nc, cj = cell % nc;
            const int32_t v00 = (int32_t)(ci * m + cj), v10 = (int32_t)((ci + 1) * m + cj);
            const int32_t v01 = v00 + 1, v11 = v10 + 1;
            int32_t* c = conn + e * 3;
            c[0] = v00;
            c[1] = (e & 1) ? v11 : v10;
            c[2] = (e & 1) ? v01 : v11;
        } else {
            const int64_t cell = e / 6, t = e % 6;
            const int64_t ci = cell / ((int64_t)nc * nc), cj = (cell / nc) % nc, ck = cell % nc;
            const int p0 = (int)(t / 2), p1 = (p0 + 1 + (int)(t & 1)) % 3;  // two distinct axes
            int off0[3] = {0, 0, 0}, off1[3] = {0, 0, 0};
            off0[p0] = 1;
            off1[p0] = 1;
            off1[p1] = 1;
            auto vid = [&](int a, int b, int c) { return (int32_t)(((ci + a) * m + (cj + b)) * m + (ck + c)); };
            int32_t* c = conn + e * 4;
            c[0] = vid(0, 0, 0);
            c[1] = vid(off0[0], off0[1], off0[2]);
            c[2] = vid(off1[0], off1[1], off1[2]);
            c[3] = vid(1, 1, 1);
        }
    }
}

static std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// ------------------------------------------------------------ JSON cache --
// Format written here:
// {"version": 1, "entries": [
//   {"arch": "gfx950", "op": 0, "dim": 3, "physics": 0, "rule": 1, "dtype": 0,
//    "strategy": 0, "vec": 4, "waves_per_block": 4, "blocks_per_cu": 0, "us": 12.5},
//   ...]}

struct CacheEntry {
    std::string arch;
    int op = 0, dim = 0, physics = 0, rule = 0, dtype = 0;
    fem_tuning t{0, 1, 4, 0};
    double us = 0.0;
};

static bool read_file(const char* path, std::string& out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, k);
    std::fclose(f);
    return true;
}

// A JSON number as an int: values that are not finite or lie outside
// +-1e9 become -1 (which no field accepts) instead of an undefined
// conversion.
static int as_int(double x) { return (std::isfinite(x) && x > -1e9 && x < 1e9) ? (int)x : -1; }

// Parses the objects inside the "entries" array. Unknown keys are ignored;
// malformed input yields no entries rather than an error.
static std::vector<CacheEntry> parse_cache(const std::string& s) {
    std::vector<CacheEntry> out;
    size_t pos = s.find("\"entries\"");
    if (pos == std::string::npos) return out;
    pos = s.find('[', pos);
    if (pos == std::string::npos) return out;
    while (true) {
        size_t open = s.find('{', pos), close_arr = s.find(']', pos);
        if (open == std::string::npos || (close_arr != std::string::npos && close_arr < open)) break;
        size_t close = s.find('}', open);
        if (close == std::string::npos) break;
        std::string obj = s.substr(open + 1, close - open - 1);
        CacheEntry e;
        bool have_arch = false;
        size_t p = 0;
        while (true) {
            size_t k0 = obj.find('"', p);
            if (k0 == std::string::npos) break;
            size_t k1 = obj.find('"', k0 + 1);
            if (k1 == std::string::npos) break;
            std::string key = obj.substr(k0 + 1, k1 - k0 - 1);
            size_t colon = obj.find(':', k1);
            if (colon == std::string::npos) break;
            size_t v = colon + 1;
            while (v < obj.size() && std::isspace((unsigned char)obj[v])) ++v;
            if (v < obj.size() && obj[v] == '"') {
                size_t v1 = obj.find('"', v + 1);
                if (v1 == std::string::npos) break;
                if (key == "arch") { e.arch = obj.substr(v + 1, v1 - v - 1); have_arch = true; }
                p = v1 + 1;
            } else {
                char* end = nullptr;
                double x = std::strtod(obj.c_str() + v, &end);
                size_t used = end ? (size_t)(end - obj.c_str()) : v;
                if (key == "op") e.op = as_int(x);
                else if (key == "dim") e.dim = as_int(x);
                else if (key == "physics") e.physics = as_int(x);
                else if (key == "rule") e.rule = as_int(x);
                else if (key == "dtype") e.dtype = as_int(x);
                else if (key == "strategy") e.t.strategy = as_int(x);
                else if (key == "vec") e.t.vec = as_int(x);
                else if (key == "waves_per_block") e.t.waves_per_block = as_int(x);
                else if (key == "blocks_per_cu") e.t.blocks_per_cu = as_int(x);
                else if (key == "us") e.us = x;
                p = used > v ? used : v + 1;
            }
        }
        if (have_arch) out.push_back(e);
        pos = close + 1;
    }
    return out;
}

static bool write_cache(const char* path, const std::vector<CacheEntry>& es) {
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"version\": 1, \"entries\": [\n");
    for (size_t i = 0; i < es.size(); ++i) {
        const CacheEntry& e = es[i];
        std::fprintf(f,
                     "  {\"arch\": \"%s\", \"op\": %d, \"dim\": %d, \"physics\": %d, \"rule\": %d, \"dtype\": %d, "
                     "\"strategy\": %d, \"vec\": %d, \"waves_per_block\": %d, \"blocks_per_cu\": %d, "
                     "\"us\": %.3f}%s\n",
                     e.arch.c_str(), e.op, e.dim, e.physics, e.rule, e.dtype, e.t.strategy, e.t.vec,
                     e.t.waves_per_block, e.t.blocks_per_cu, e.us, i + 1 < es.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace femq

using namespace femq;

extern "C" {

fem_status fem_load_tuning(const char* cache_path) {
    if (!cache_path) { set_error("fem_load_tuning: NULL path"); return FEM_ERR_INVALID_ARG; }
    std::string text;
    if (!read_file(cache_path, text)) { set_error("fem_load_tuning: cannot read %s", cache_path); return FEM_ERR_NO_TUNING; }
    const std::string arch = device_arch();
    int used = 0;
    for (const CacheEntry& e : parse_cache(text)) {
        if (e.arch != arch) continue;
        fem_tuning t = e.t;
        if (fem_set_tuning(e.op, e.dim, e.physics, e.rule, e.dtype, &t) == FEM_OK) ++used;
    }
    if (!used) { set_error("fem_load_tuning: no valid entry for %s in %s", arch.c_str(), cache_path); return FEM_ERR_NO_TUNING; }
    return FEM_OK;
}

fem_status fem_autotune(int op, int dim, int physics, int rule, int dtype, int64_t n_probe, const char* cache_path) {
    fem_tuning current;
    fem_status st = fem_get_tuning(op, dim, physics, rule, dtype, &current);
    if (st) return st;
    if (op == FEM_OP_GEOMETRY) physics = FEM_LAPLACE, rule = FEM_RULE_CENTROID;
    if (n_probe < 4096 || n_probe > (int64_t)1 << 28) {
        set_error("fem_autotune: n_elem_probe must be in [4096, 2^28]");
        return FEM_ERR_INVALID_ARG;
    }
    const bool jac = op == FEM_OP_JACOBIAN || op == FEM_OP_JACOBIAN_P2 || op == FEM_OP_JACOBIAN_P3;
    const bool p2 = op == FEM_OP_RESIDUAL_P2 || op == FEM_OP_BACKWARD_P2 || op == FEM_OP_JACOBIAN_P2;
    const bool p3 = op == FEM_OP_RESIDUAL_P3 || op == FEM_OP_BACKWARD_P3 || op == FEM_OP_JACOBIAN_P3;
    const bool one = p2 || p3 || jac;  // one element per lane
    const int nc = physics == FEM_ELASTICITY ? dim : 1;
    const int nbt = (p3 ? (dim + 1) * (dim + 2) * (dim + 3) / 6 : p2 ? (dim + 1) * (dim + 2) / 2 : dim + 1) * nc;
    const int out_rows = jac ? nbt * nbt : nbt;
    const int nq = rule == FEM_RULE_CENTROID ? 1 : rule == FEM_RULE_TRI6 ? 6 : rule == FEM_RULE_TET11 ? 11 : dim + 1;
    const int ncq = (physics == FEM_ELASTICITY ? 2 : 1) * nq;
    const size_t word = dtype == FEM_F32 ? 4 : 8;
    const int64_t n = n_probe;
    const bool mesh_op = op == FEM_OP_GEOMETRY || op == FEM_OP_RESIDUAL_MESH || op == FEM_OP_RESIDUAL_GATHER;
    // probe mesh
    const int per = dim == 2 ? 2 : 6;
    int grid_n = 1;
    while ((int64_t)per * (dim == 2 ? (int64_t)grid_n * grid_n : (int64_t)grid_n * grid_n * grid_n) < n) ++grid_n;
    const int64_t n_vert = dim == 2 ? (int64_t)(grid_n + 1) * (grid_n + 1) : (int64_t)(grid_n + 1) * (grid_n + 1) * (grid_n + 1);

    if (n_vert * nc > (int64_t)nbt * n) {  // the gather probe reads vertex values from the closure buffer
        set_error("fem_autotune: probe mesh too coarse");
        return FEM_ERR_INVALID_ARG;
    }
    // one copy: geometry, u, coef, w, outputs, and for mesh ops the mesh
    struct Copy { void *ij, *dj, *u, *cf, *w, *out, *du, *dc; double* X; int32_t* conn; };
    const size_t rows_words = (size_t)n * (dim * dim + 1 + 3 * nbt + out_rows + 2 * ncq);
    const size_t bytes_per_copy = rows_words * word + (mesh_op ? (size_t)n * 4 * (dim + 1) + (size_t)n_vert * 8 * dim : 0);
    const int copies = (int)std::min<size_t>(8, std::max<size_t>(2, (size_t)(768u << 20) / bytes_per_copy + 1));
    std::vector<void*> bufs;
    auto cleanup = [&]() { for (void* b : bufs) (void)hipFree(b); };
    auto alloc = [&](void** p, size_t bytes) {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) bufs.push_back(*p);
        return e;
    };
    std::vector<Copy> cs(copies);
    hipError_t e = hipSuccess;
    for (int c = 0; c < copies && e == hipSuccess; ++c) {
        Copy& cp = cs[c];
        cp = Copy{};
        if ((e = alloc(&cp.ij, (size_t)dim * dim * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.dj, (size_t)n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.u, (size_t)nbt * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.cf, (size_t)ncq * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.w, (size_t)nbt * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.out, (size_t)out_rows * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.du, (size_t)nbt * n * word)) != hipSuccess) break;
        if ((e = alloc(&cp.dc, (size_t)ncq * n * word)) != hipSuccess) break;
        // well-conditioned synthetic geometry, values in the benchmark ranges
        e = fill(dtype, cp.ij, (int64_t)dim * dim * n, 11 + c, -1.5, 1.5);
        if (e == hipSuccess) e = fill(dtype, cp.dj, n, 23 + c, 0.5, 2.0);
        if (e == hipSuccess) e = fill(dtype, cp.u, (int64_t)nbt * n, 37 + c, -1.0, 1.0);
        if (e == hipSuccess) e = fill(dtype, cp.cf, (int64_t)ncq * n, 41 + c, 0.5, 2.0);
        if (e == hipSuccess) e = fill(dtype, cp.w, (int64_t)nbt * n, 53 + c, -1.0, 1.0);
        if (e == hipSuccess && mesh_op) {
            void* px = nullptr;
            void* pc = nullptr;
            if ((e = alloc(&px, (size_t)n_vert * dim * 8)) != hipSuccess) break;
            if ((e = alloc(&pc, (size_t)n * (dim + 1) * 4)) != hipSuccess) break;
            cp.X = static_cast<double*>(px);
            cp.conn = static_cast<int32_t*>(pc);
            const int grid = (int)std::min<int64_t>((std::max(n, n_vert) + 255) / 256, 65536);
            if (dim == 2)
                hipLaunchKernelGGL(probe_mesh_kernel<2>, dim3(grid), dim3(256), 0, nullptr, n, grid_n, cp.conn, cp.X, n_vert);
            else
                hipLaunchKernelGGL(probe_mesh_kernel<3>, dim3(grid), dim3(256), 0, nullptr, n, grid_n, cp.conn, cp.X, n_vert);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "fem_autotune: probe buffers"); }

    auto run = [&](const Copy& c) -> fem_status {
        switch (op) {
        case FEM_OP_RESIDUAL_P2:
            return fem_integrate_residual_p2(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf, c.out,
                                             nullptr);
        case FEM_OP_RESIDUAL_P3:
            return fem_integrate_residual_p3(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf, c.out,
                                             nullptr);
        case FEM_OP_BACKWARD_P3:
            return fem_integrate_residual_p3_backward(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf,
                                                      c.w, c.du, c.dc, nullptr);
        case FEM_OP_BACKWARD_P2:
            return fem_integrate_residual_p2_backward(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf,
                                                      c.w, c.du, c.dc, nullptr);
        case FEM_OP_JACOBIAN:
        case FEM_OP_JACOBIAN_P2:
        case FEM_OP_JACOBIAN_P3:
            return fem_integrate_jacobian(dim, physics, rule, FEM_COEF_QUAD,
                                          op == FEM_OP_JACOBIAN ? 1 : op == FEM_OP_JACOBIAN_P2 ? 2 : 3, dtype, n, c.ij,
                                          c.dj, c.cf, c.out, nullptr);
        case FEM_OP_RESIDUAL:
            return fem_integrate_residual(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf, c.out, nullptr);
        case FEM_OP_BACKWARD:
            return fem_integrate_residual_backward(dim, physics, rule, FEM_COEF_QUAD, dtype, n, c.ij, c.dj, c.u, c.cf, c.w, c.du,
                                                   c.dc, nullptr);
        case FEM_OP_GEOMETRY:
            return fem_geometry(dim, n, n_vert, c.X, c.conn, dtype, c.ij, c.dj, nullptr, nullptr);
        case FEM_OP_RESIDUAL_GATHER:  // the closure buffer holds at least n_vert * N_comp vertex values
            return fem_integrate_residual_gather(dim, physics, rule, FEM_COEF_QUAD, dtype, n, n_vert, c.X, c.conn, c.u,
                                                 c.cf, c.out, nullptr, nullptr, nullptr, nullptr);
        default:
            return fem_integrate_residual_mesh(dim, physics, rule, FEM_COEF_QUAD, dtype, n, n_vert, c.X, c.conn, c.u, c.cf, c.out,
                                               nullptr, nullptr, nullptr, nullptr);
        }
    };

    std::vector<fem_tuning> cands;
    const std::vector<int> vecs = one ? std::vector<int>{1} : std::vector<int>{1, 2, 4};
    for (int v : vecs)
        for (int w : {1, 2, 4, 8})
            for (int b : {0, 2, 4, 8, 16}) cands.push_back(fem_tuning{FEM_STRATEGY_LANE, v, w, b});
    if (op == FEM_OP_RESIDUAL)
        for (int w : {1, 2, 4, 8})
            for (int b : {0, 4, 8}) cands.push_back(fem_tuning{FEM_STRATEGY_TRANSPOSE, 1, w, b});
    if (op == FEM_OP_RESIDUAL && physics != FEM_ELASTICITY)
        for (int w : {1, 2, 4, 8})
            for (int b : {0, 4, 8}) cands.push_back(fem_tuning{FEM_STRATEGY_SHUFFLE, 1, w, b});
    if (op == FEM_OP_RESIDUAL_MESH)
        for (int w : {2, 4})
            for (int b : {0, 2, 4, 8}) cands.push_back(fem_tuning{FEM_STRATEGY_DEDUP, 1, w, b});
    if (op == FEM_OP_RESIDUAL_P3 && dim == 3 && physics != FEM_MASS)
        for (int w : {1, 2, 4})
            for (int b : {0, 2, 4, 8}) cands.push_back(fem_tuning{FEM_STRATEGY_MFMA, 1, w, b});
    if (op == FEM_OP_RESIDUAL_P3 && dim == 3 && physics == FEM_ELASTICITY)
        for (int w = 1; w <= comp_max_groups(dtype); ++w)   // three-wave groups per workgroup
            for (int b : {0, 2, 4, 8}) cands.push_back(fem_tuning{FEM_STRATEGY_COMPONENT, 1, w, b});

    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    const int reps = 12;
    fem_tuning best = current;
    float best_ms = 1e30f;
    for (const fem_tuning& t : cands) {
        if (fem_set_tuning(op, dim, physics, rule, dtype, &t) != FEM_OK) continue;
        bool ok = true;
        for (int r = 0; r < 2 && ok; ++r) ok = run(cs[r % copies]) == FEM_OK;
        if (!ok) continue;  // not available for this combination (e.g. LDS too large)
        (void)hipEventRecord(t0, nullptr);
        for (int r = 0; r < reps; ++r) (void)run(cs[r % copies]);
        (void)hipEventRecord(t1, nullptr);
        if (hipEventSynchronize(t1) != hipSuccess) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        ms /= reps;
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    hipError_t sync = hipDeviceSynchronize();
    cleanup();
    fem_set_tuning(op, dim, physics, rule, dtype, &best);
    if (sync != hipSuccess) return hip_fail(sync, "fem_autotune");
    if (best_ms >= 1e29f) { set_error("fem_autotune: no candidate ran"); return FEM_ERR_HIP; }

    if (cache_path) {
        std::string text;
        std::vector<CacheEntry> es;
        if (read_file(cache_path, text)) es = parse_cache(text);
        CacheEntry ne;
        ne.arch = device_arch();
        ne.op = op; ne.dim = dim; ne.physics = physics; ne.rule = rule; ne.dtype = dtype;
        ne.t = best;
        ne.us = best_ms * 1e3;
        bool replaced = false;
        for (CacheEntry& x : es)
            if (x.arch == ne.arch && x.op == op && x.dim == dim && x.physics == physics && x.rule == rule &&
                x.dtype == dtype) {
                x = ne;
                replaced = true;
            }
        if (!replaced) es.push_back(ne);
        if (!write_cache(cache_path, es)) { set_error("fem_autotune: cannot write %s", cache_path); return FEM_ERR_INVALID_ARG; }
    }
    return FEM_OK;
}

}  // extern "C"
