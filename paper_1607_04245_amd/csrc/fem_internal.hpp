// fem_internal.hpp -- host-side interfaces between the C ABI layer and the
// kernel translation units of libfemq.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fem.h"

namespace femq {

struct ResidualArgs {
    int64_t n;
    const void* inv_j;
    const void* det_j;
    const void* u;
    const void* coef;
    void* out;
};

struct BackwardArgs {
    int64_t n;
    const void* inv_j;
    const void* det_j;
    const void* u;
    const void* coef;
    const void* w;
    void* du;
    void* dcoef;
};

struct JacobianArgs {
    int64_t n;
    const void* inv_j;
    const void* det_j;
    const void* coef;
    void* out;
};

struct MeshArgs {
    int64_t n;
    int64_t n_vert;
    const double* coords;
    const int32_t* conn;
    const void* u;
    const void* coef;
    void* out;
    void* inv_j;      // optional geometry outputs (both or neither)
    void* det_j;
    int32_t* counts;  // optional
};

struct Launch {
    int grid;      // workgroups
    int block;     // threads per workgroup (multiple of 64)
    int vec;       // elements per lane in load/store phases
    hipStream_t stream;
};

// Each returns hipErrorInvalidValue when the combination has no kernel;
// `space` is the coefficient space (fem_coef_space).
hipError_t launch_residual_lane(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                const Launch& l);
hipError_t launch_residual_transpose(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                     const Launch& l);
// The transposition through quad permutations (scalar fields; four lanes per
// element, a wave takes 16 elements at a time).
hipError_t launch_residual_shuffle(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                                   const Launch& l);
hipError_t launch_residual_mesh(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                const Launch& l);
// The fused from-mesh kernel with per-wave run-time vertex deduplication in
// LDS (residual_dedup.hip); one element per lane, block = 64 x waves (2 or 4).
hipError_t launch_residual_dedup(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                 const Launch& l);
// u and a P1 coefficient per vertex (MeshArgs.u, MeshArgs.coef), gathered.
hipError_t launch_residual_gather(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                  const Launch& l);
// Third-order elements (residual_p3.hip), degree-4 rules (TRI6, TET11).
hipError_t launch_residual_p3(int dim, int phys, int space, int dtype, const ResidualArgs& a, const Launch& l);
// P3 tetrahedra, Laplacian or elasticity, with the transposition on the
// matrix cores (residual_p3_mfma.hip); four lanes per element, a wave takes
// 16 elements at a time.
hipError_t launch_residual_p3_mfma(int phys, int space, int dtype, const ResidualArgs& a, const Launch& l);
// P3 tetrahedral elasticity with one wave per displacement component
// (residual_p3_comp.hip): three waves per 64-element tile, up to
// comp_max_groups(dtype) such groups per workgroup (l.block 192 or 384).
hipError_t launch_residual_p3_comp(int space, int dtype, const ResidualArgs& a, const Launch& l);
int comp_max_groups(int dtype);
size_t p3_comp_shared_bytes(int dtype, int groups);   // dynamic LDS of a workgroup
hipError_t launch_backward_p3(int dim, int phys, int space, int dtype, const BackwardArgs& a, const Launch& l);
hipError_t launch_jacobian_p3(int dim, int phys, int space, int dtype, const JacobianArgs& a, const Launch& l);
// Second-order elements (residual_p2.hip); rules TRI3/TRI6 (2D), TET4/TET11 (3D).
hipError_t launch_residual_p2(int dim, int phys, int rule, int space, int dtype, const ResidualArgs& a,
                              const Launch& l);
hipError_t launch_backward_p2(int dim, int phys, int rule, int space, int dtype, const BackwardArgs& a,
                              const Launch& l);
// Element matrices: order 1 or 2 (jacobian.hip), order 3 (residual_p3.hip).
hipError_t launch_jacobian(int dim, int phys, int order, int rule, int space, int dtype, const JacobianArgs& a,
                           const Launch& l);
hipError_t launch_backward_lane(int dim, int phys, int rule, int space, int dtype, const BackwardArgs& a,
                                const Launch& l);
hipError_t launch_geometry(int dim, int dtype, int64_t n_elem, int64_t n_vert, const double* coords,
                           const int32_t* conn, void* inv_j, void* det_j, int32_t* counts,
                           const Launch& l);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t n_bytes, const Launch& l);
// The structure-of-arrays streaming yardstick (stream_rows.hip).
hipError_t launch_stream_rows(int dtype, int64_t n, int n_in, int n_out, const void* src, void* dst,
                              const Launch& l);

// Batched persistent kernel (batch.hip).
struct BatchMesh {              // device-side descriptor, one per mesh
    int32_t type;               // dim*64 + coef_space*16 + physics*4 + rule
    int32_t pad;
    int64_t n_elem;
    int64_t tile_begin;         // first global tile of this mesh
    int64_t tile_end;           // one past its last tile
    const void* inv_j;
    const void* det_j;
    const void* u;
    const void* coef;
    void* out;
};

// d_tile_mesh may be NULL: each workgroup then finds its first mesh by a
// binary search over the n_mesh descriptors' tile ranges.
hipError_t launch_batch(int dtype, const BatchMesh* d_meshes, int n_mesh, const int32_t* d_tile_mesh,
                        int64_t n_tiles, int tile_elems, const Launch& l);

// Threads the transpose kernel needs per workgroup for a given tuning, or 0 if
// the combination is not supported by that strategy.
int transpose_block_threads(int dim, int phys, int rule, int space, int dtype, int waves_per_block);

}  // namespace femq

namespace femq {

// Thread-local error message behind fem_last_error().
void set_error(const char* fmt, ...);
fem_status hip_fail(hipError_t e, const char* what);

// Compute units of the current device (cached per device); 0 if unknown.
int device_cus();

// Launch configuration table (fem_abi.hip), keyed by operation.
fem_tuning get_tuning(int op, int dim, int phys, int rule, int dtype);
void put_tuning(int op, int dim, int phys, int rule, int dtype, const fem_tuning& t);

}  // namespace femq
