/*
 * fem.h -- C ABI of libfemq: P1 finite-element residual integration on
 * AMD MI355X (gfx950).
 *
 * The library evaluates, for every element e of a simplex mesh, the element
 * residual vector of the paper's Eq. (2) (Section 2, "Formulation"), before
 * assembly:
 *
 *     R_e = B^T W f0(u^q, grad u^q) + sum_k D_k^T W f1^k(u^q, grad u^q),
 *
 * with u^q and grad u^q evaluated at quadrature points from tabulated P1
 * basis values and W the quadrature weights times |det J|. The kernel inputs
 * follow the paper's integration routine (Appendix): per-element geometry
 * (inverse Jacobian and determinant), the element closure of u, and per
 * element outputs. Auxiliary coefficients live on quadrature points
 * (Section 4, "Variable Coefficients").
 *
 * Conventions shared by every call:
 *  - All array arguments are DEVICE pointers owned by the caller. The library
 *    never allocates, frees or synchronizes on them (plans below own their
 *    own descriptor memory).
 *  - Layouts are structure of arrays over elements, n = n_elem:
 *      inv_j   [dim*dim][n]  row k*dim+i holds d xi_k / d x_i (J^{-1}, row-major)
 *      det_j   [n]           det J, signed; the measure factor is |det J|
 *      u, w, elem_vec, du    [N_b*N_comp][n], row b*N_comp + c
 *      coef, dcoef           [N_coef][N_w][n]
 *    with N_b = dim+1, N_comp = 1 (Laplacian, mass) or dim (elasticity),
 *    N_coef = 1 (kappa) or 2 (lambda, mu), N_q from the rule, and N_w the
 *    words of one coefficient field per element in its space (below).
 *  - Coefficient spaces (paper Section 4, "Variable Coefficients": an
 *    auxiliary field may live on quadrature points, in the space of u, or be
 *    constant per cell):
 *      FEM_COEF_QUAD  values at the quadrature points, N_w = N_q
 *      FEM_COEF_P1    nodal values of a P1 field, element closure in vertex
 *                     order, N_w = N_b; evaluated at point q as
 *                     sum_b phi_b(xi_q) a_b
 *      FEM_COEF_P0    one value per element, N_w = 1
 *    Real arrays are float (FEM_F32) or double (FEM_F64) as selected.
 *  - Reference element: unit simplex, phi_0 = 1 - sum xi, phi_k = xi_k.
 *    Rules: FEM_RULE_TRI3 (dim 2; barycentric (2/3,1/6,1/6), point q has 2/3
 *    at vertex q; weights 1/6), FEM_RULE_TET4 (dim 3; (a,b,b,b) with
 *    a = (5+3 sqrt 5)/20, point q has a at vertex q; weights 1/24),
 *    FEM_RULE_CENTROID (one point, weight 1/dim!; the paper's N_q = 1 model).
 *  - Inputs are read-only; outputs are fully overwritten (no accumulation),
 *    except the counters of fem_geometry, which are added to.
 *  - `stream` is a hipStream_t (NULL = the default stream). Calls are
 *    asynchronous on that stream.
 *  - Arguments are validated before any HIP call: bad values give
 *    FEM_ERR_INVALID_ARG or FEM_ERR_UNSUPPORTED with a message in
 *    fem_last_error(). A failed launch gives FEM_ERR_HIP. n_elem == 0 returns
 *    FEM_OK without launching. No C++ exception crosses this interface.
 *  - Results do not depend on the launch configuration: each element's
 *    arithmetic is fixed, so repeated calls are bitwise identical.
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fem_status;

#define FEM_OK 0
#define FEM_ERR_INVALID_ARG (-1)
#define FEM_ERR_UNSUPPORTED (-2)
#define FEM_ERR_DEGENERATE (-3)
#define FEM_ERR_HIP (-4)
#define FEM_ERR_NO_TUNING (-5)

enum fem_dtype { FEM_F32 = 0, FEM_F64 = 1 };

/* Pointwise physics (paper Section 2 and Section 6):
 *  FEM_LAPLACE     f0 = 0, f1 = kappa grad u                     (N_comp 1, N_coef 1)
 *  FEM_ELASTICITY  f0 = 0, f1 = lambda tr(eps) I + 2 mu eps,
 *                  eps = (grad u + grad u^T)/2; the paper's Lame
 *                  function is lambda = 0, mu = 1/2             (N_comp dim, N_coef 2)
 *  FEM_MASS        f0 = kappa u, f1 = 0 (exercises the B^T W f0 term)
 *                                                                (N_comp 1, N_coef 1) */
enum fem_physics { FEM_LAPLACE = 0, FEM_ELASTICITY = 1, FEM_MASS = 2 };

enum fem_rule {
    FEM_RULE_TRI3 = 0, FEM_RULE_TET4 = 1, FEM_RULE_CENTROID = 2,
    /* degree-4 rules, second-order elements only (see fem_integrate_residual_p2) */
    FEM_RULE_TRI6 = 3, FEM_RULE_TET11 = 4
};

enum fem_coef_space { FEM_COEF_QUAD = 0, FEM_COEF_P1 = 1, FEM_COEF_P0 = 2 };

/* Kernel strategies (see fem_tuning).
 *  FEM_STRATEGY_LANE       each lane owns whole elements; the quadrature and
 *                          basis phases run in registers.
 *  FEM_STRATEGY_TRANSPOSE  the paper's thread transposition (Section 3):
 *                          lanes work per (element, quadrature point) in the
 *                          quadrature phase, write weighted, pulled-back
 *                          f0/f1 to LDS, and
 *                          switch to one lane per (element, basis function)
 *                          for the basis phase, with no cross-lane reduction
 *                          (P1 only; for vector fields on four-point rules
 *                          the four point lanes of an element share their
 *                          terms by quad permutations instead, form the sums
 *                          over the points in point order, and lane b stores
 *                          basis function b's).
 *  FEM_STRATEGY_MFMA       the same transposition for P3 tetrahedra (Laplacian,
 *                          elasticity; FEM_OP_RESIDUAL_P3 only) with the two
 *                          tabulation contractions on the matrix cores: four
 *                          lanes share an element, each evaluates the
 *                          pointwise physics at its own quadrature points,
 *                          and the products switch between the point- and
 *                          basis-parallel layouts. Agrees with the lane
 *                          kernel to rounding (another summation order).
 *  FEM_STRATEGY_SHUFFLE    the transposition of FEM_STRATEGY_TRANSPOSE for
 *                          scalar fields (Laplacian, mass; FEM_OP_RESIDUAL
 *                          only) with cross-lane permutations instead of LDS:
 *                          four lanes share an element, lane r being point r
 *                          and then basis function r. */
enum fem_strategy { FEM_STRATEGY_LANE = 0, FEM_STRATEGY_TRANSPOSE = 1, FEM_STRATEGY_MFMA = 2,
                    FEM_STRATEGY_SHUFFLE = 3, FEM_STRATEGY_DEDUP = 4, FEM_STRATEGY_COMPONENT = 5 };

/*  FEM_STRATEGY_DEDUP      (FEM_OP_RESIDUAL_MESH only; vec 1, two or four
 *                          waves per workgroup) each wave
 *                          deduplicates its 64-element tile's vertex indices
 *                          in an LDS hash table and gathers every distinct
 *                          vertex record once, then reads the elements'
 *                          vertices from LDS; bitwise equal to the lane
 *                          strategy.
 *  FEM_STRATEGY_COMPONENT  (FEM_OP_RESIDUAL_P3 with 3D elasticity only; vec
 *                          1) three waves per 64-element tile, wave c holding
 *                          displacement component c of every element: its
 *                          closure words, its gradient at each point and its
 *                          output sums. The stress row of a point takes the
 *                          trace and the paired off-diagonal gradient entries
 *                          from the two other waves through LDS (Section 3's
 *                          transposition, split by component).
 *                          waves_per_block counts three-wave groups (1 or 2
 *                          in FP32, 1 in FP64; FEM_ERR_UNSUPPORTED beyond).
 *                          Agrees with the lane kernel to rounding (another
 *                          summation order). */

/* Operations; each has its own launch configuration (see fem_tuning). */
enum fem_op {
    FEM_OP_RESIDUAL = 0,       /* fem_integrate_residual */
    FEM_OP_RESIDUAL_MESH = 1,  /* fem_integrate_residual_mesh */
    FEM_OP_GEOMETRY = 2,       /* fem_geometry (physics and rule ignored) */
    FEM_OP_BACKWARD = 3,       /* fem_integrate_residual_backward */
    FEM_OP_RESIDUAL_GATHER = 4, /* fem_integrate_residual_gather */
    FEM_OP_RESIDUAL_P2 = 5,     /* fem_integrate_residual_p2 */
    FEM_OP_BACKWARD_P2 = 6,     /* fem_integrate_residual_p2_backward */
    FEM_OP_JACOBIAN = 7,        /* fem_integrate_jacobian, order 1 */
    FEM_OP_JACOBIAN_P2 = 8,     /* fem_integrate_jacobian, order 2 */
    FEM_OP_RESIDUAL_P3 = 9,     /* fem_integrate_residual_p3 */
    FEM_OP_BACKWARD_P3 = 10,    /* fem_integrate_residual_p3_backward */
    FEM_OP_JACOBIAN_P3 = 11     /* fem_integrate_jacobian, order 3 */
};

/* ------------------------------------------------------------------ */
/* Geometry (paper Section 3: the kernel reads precomputed Jacobian    */
/* inverses and determinants; this call produces them).                */
/* ------------------------------------------------------------------ */

/* For each element, gather its dim+1 vertices, form J[i][k] = (x_k - x_0)_i,
 * and write det J and J^{-1}. Arithmetic is FP64 for both output types; for
 * FEM_F32 the results are rounded once at the store.
 *   coords [n_vert][dim] double, conn [n_elem][dim+1] int32 (0-based).
 *   counts, if not NULL, points to 2 int32 on the device that are ADDED to:
 *     counts[0] += elements with det J == 0, non-finite, or a vertex index
 *                  outside [0, n_vert) (these get NaN geometry, and no
 *                  out-of-range coordinate is read);
 *     counts[1] += poorly shaped elements, |det J| < 1e-3 prod_k |J[:,k]|
 *                  (evaluated as det^2 < 1e-6 prod_k |J[:,k]|^2).
 * Errors: FEM_ERR_INVALID_ARG (dim not 2/3, negative sizes, NULL arrays with
 * n_elem > 0, n_vert == 0 with n_elem > 0), FEM_ERR_UNSUPPORTED (dtype),
 * FEM_ERR_HIP. */
fem_status fem_geometry(int dim, int64_t n_elem, int64_t n_vert, const double* coords,
                        const int32_t* conn, int out_dtype, void* inv_j, void* det_j,
                        int32_t* counts, void* stream);

/* ------------------------------------------------------------------ */
/* Residual (paper Eq. (2); Section 3 quadrature and basis phases).    */
/* ------------------------------------------------------------------ */

/* elem_vec = per-element residual R_e as defined at the top of this file.
 * Errors: FEM_ERR_INVALID_ARG (negative n_elem, NULL arrays with
 * n_elem > 0), FEM_ERR_UNSUPPORTED (dim/physics/rule/coef_space/dtype
 * combination), FEM_ERR_HIP. */
fem_status fem_integrate_residual(int dim, int physics, int rule, int coef_space, int dtype,
                                  int64_t n_elem, const void* inv_j, const void* det_j,
                                  const void* u, const void* coef, void* elem_vec, void* stream);

/* Residual straight from the mesh: geometry and integration fused in one
 * pass over the elements, with no round trip of J^{-1} and det J through
 * memory. The geometry is computed exactly as fem_geometry computes it (FP64,
 * rounded once to `dtype`) and the integration is that of
 * fem_integrate_residual, so elem_vec is bitwise equal to calling the two in
 * turn. inv_j and det_j are optional outputs (both NULL, or both set: then
 * they receive what fem_geometry would write); counts as in fem_geometry
 * (may be NULL). Layouts as above; coords [n_vert][dim] double, conn
 * [n_elem][dim+1] int32.
 * Errors: as fem_integrate_residual and fem_geometry. */
fem_status fem_integrate_residual_mesh(int dim, int physics, int rule, int coef_space, int dtype,
                                       int64_t n_elem, int64_t n_vert, const double* coords,
                                       const int32_t* conn, const void* u, const void* coef,
                                       void* elem_vec, void* inv_j, void* det_j, int32_t* counts,
                                       void* stream);

/* Residual from the mesh with u given per vertex: the element restriction
 * (the closure u_e = E_e u of Section 2, gathered through the connectivity)
 * is applied inside the kernel instead of being read as [N_bt][n] rows, so
 * u costs N_comp words per vertex instead of N_bt words per element.
 *   u_vertex [n_vert][N_comp]  dtype, component c of vertex v at v*N_comp + c
 *   coef     FEM_COEF_P1: [n_vert][N_coef] vertex values (coefficient m of
 *            vertex v at v*N_coef + m), gathered the same way (the paper's
 *            auxiliary field in the space of u, Section 4);
 *            FEM_COEF_QUAD, FEM_COEF_P0: per element as for
 *            fem_integrate_residual.
 * Everything else (geometry outputs, counts, layouts, bitwise agreement
 * with the two-call path) as fem_integrate_residual_mesh: elem_vec is
 * bitwise equal to fem_integrate_residual_mesh called with the gathered
 * closure (and, for P1, the gathered coefficient closure). Vertex indices
 * outside [0, n_vert) make the element degenerate (counted; its geometry
 * and vector are NaN); nothing outside the arrays is read.
 * Errors: as fem_integrate_residual_mesh. */
fem_status fem_integrate_residual_gather(int dim, int physics, int rule, int coef_space, int dtype,
                                         int64_t n_elem, int64_t n_vert, const double* coords,
                                         const int32_t* conn, const void* u_vertex, const void* coef,
                                         void* elem_vec, void* inv_j, void* det_j, int32_t* counts,
                                         void* stream);

/* Adjoint of L = sum_e w_e . R_e (not in the paper; the gradient of the
 * residual for automatic differentiation):
 *   du    = dL/du     [N_bt][n]           (may be NULL: not computed)
 *   dcoef = dL/dcoef  [N_coef][N_w][n]    (may be NULL: not computed), in the
 *                                         coefficient's own space
 * All three physics are symmetric bilinear forms in (u, test function), so
 * du_e = R_e evaluated with u replaced by w_e; dcoef at point q is the
 * weighted pointwise derivative, e.g. w_q |det J| grad u . grad w for the
 * Laplacian (for P1 and P0 coefficients, summed back onto the nodal or cell
 * value by the chain rule). u is not read when dcoef is NULL.
 * Errors as fem_integrate_residual. */
fem_status fem_integrate_residual_backward(int dim, int physics, int rule, int coef_space,
                                           int dtype, int64_t n_elem, const void* inv_j,
                                           const void* det_j, const void* u, const void* coef,
                                           const void* w, void* du, void* dcoef, void* stream);

/* ------------------------------------------------------------------ */
/* Second-order (P2) Lagrange elements on affine simplices: the same    */
/* quadrature discretization of Eq. (2) with the P2 basis.              */
/* ------------------------------------------------------------------ */

/* Element residuals of P2 elements from precomputed affine geometry
 * (fem_geometry of the vertices). N_b = (dim+1)(dim+2)/2 nodes per element,
 * in the order vertices 0..dim, then the edges (i, j), i < j, in
 * lexicographic order; basis lam_v (2 lam_v - 1) at vertices and
 * 4 lam_i lam_j on edges (lam the barycentric coordinates of the unit
 * simplex). u and elem_vec are [N_b*N_comp][n] (row b*N_comp + c); a P1
 * coefficient has N_w = dim+1 vertex values and is evaluated with the P1
 * basis. Rules: FEM_RULE_TRI3 / FEM_RULE_TET4 (degree 2: exact for the
 * stiffness of constant coefficients) and the degree-4 rules
 * FEM_RULE_TRI6 (six points, two orbits: barycentric a at vertex q for
 * point q and q+3, a = 0.108103018168070227 and 0.816847572980458513,
 * weights 0.223381589678011466/2 and 0.109951743655321867/2) and
 * FEM_RULE_TET11 (the centroid, weight -148/1875; (11/14, 1/14, 1/14,
 * 1/14) per vertex, weight 343/7500; (a, a, b, b) per edge with
 * a = (1 + sqrt(5/14))/4, b = (1 - sqrt(5/14))/4, weight 56/375; all
 * weights times 1/6), which integrate the P2 mass matrix exactly.
 * Errors as fem_integrate_residual (FEM_ERR_UNSUPPORTED for other rules). */
fem_status fem_integrate_residual_p2(int dim, int physics, int rule, int coef_space, int dtype,
                                     int64_t n_elem, const void* inv_j, const void* det_j,
                                     const void* u, const void* coef, void* elem_vec, void* stream);
/* Element residuals for third-order (P3) Lagrange elements: the bracket
 * of Eq. (2) with the P3 basis tabulated at the points (Section 3 takes
 * any basis; the paper evaluates P1). Node order: vertices 0..d; per edge
 * (i, j), i < j, lexicographic, the node at (2/3, 1/3) of (i, j) then the
 * one at (1/3, 2/3); per face (i, j, k), lexicographic, its centroid
 * (N_b = 10 in 2D, 20 in 3D). rule must be FEM_RULE_TRI6 (2D) or
 * FEM_RULE_TET11 (3D), the degree-4 rules. Layouts as
 * fem_integrate_residual_p2: inv_j [d*d][n_elem], det_j [n_elem], u
 * [N_b*N_comp][n_elem] (row b*N_comp + c), coef [N_coef*N_w][n_elem],
 * elem_vec [N_b*N_comp][n_elem], all device arrays of dtype. Errors: an
 * unsupported dim, physics, rule, space or dtype -> FEM_ERR_UNSUPPORTED;
 * negative n_elem or a NULL array -> FEM_ERR_INVALID_ARG. Asynchronous. */
fem_status fem_integrate_residual_p3(int dim, int physics, int rule, int coef_space, int dtype,
                                     int64_t n_elem, const void* inv_j, const void* det_j,
                                     const void* u, const void* coef, void* elem_vec, void* stream);
/* Adjoint of L = sum_e w_e . R_e for P3 elements; arguments, NULL rules
 * and meaning as fem_integrate_residual_backward with the P3 layouts of
 * fem_integrate_residual_p3 (du = R(w), the forms being symmetric; dcoef in
 * the coefficient's space). */
fem_status fem_integrate_residual_p3_backward(int dim, int physics, int rule, int coef_space, int dtype,
                                              int64_t n_elem, const void* inv_j, const void* det_j,
                                              const void* u, const void* coef, const void* w, void* du,
                                              void* dcoef, void* stream);
/* Adjoint of L = sum_e w_e . R_e for P2 elements; arguments and meaning as
 * fem_integrate_residual_backward with the P2 layouts above. */
fem_status fem_integrate_residual_p2_backward(int dim, int physics, int rule, int coef_space, int dtype,
                                              int64_t n_elem, const void* inv_j, const void* det_j,
                                              const void* u, const void* coef, const void* w, void* du,
                                              void* dcoef, void* stream);

/* ------------------------------------------------------------------ */
/* Mesh plans: the fused from-mesh residual for meshes that are         */
/* integrated many times (not in the paper; the paper's kernel reads    */
/* precomputed geometry).                                               */
/* ------------------------------------------------------------------ */

/* A plan lists, for every tile of 64 consecutive elements, the tile's
 * distinct vertices, and for every element the position of each of its
 * vertices in that list (replacing the connectivity row). The planned
 * entry points load each distinct vertex record of a tile once into LDS
 * instead of once per element that uses it, and otherwise compute exactly
 * what fem_integrate_residual_mesh / fem_integrate_residual_gather compute:
 * the element vectors are bitwise equal to theirs.
 *   conn [n_elem][dim+1] int32 device array; it is copied to the host once
 *   (the plan is built there and uploaded) and not referenced afterwards.
 * Every vertex index must lie in [0, n_vert) (else FEM_ERR_INVALID_ARG). The
 * plan holds about 4 + 4 N_tile_vertices / 64 bytes per element of device
 * memory and is bound to the device current at creation. Synchronizes
 * `stream`. The plan pays where vertex gathers bound the kernel
 * (tetrahedra); on triangle meshes the unplanned entry points measured
 * faster. */
typedef struct fem_mesh_plan fem_mesh_plan;
fem_status fem_mesh_plan_create(int dim, int64_t n_elem, int64_t n_vert, const int32_t* conn, void* stream,
                                fem_mesh_plan** out);
/* Sizes of a plan; max_tile_vertices is the largest number of distinct
 * vertices of one tile, tile_vertices their total over all tiles. Any
 * pointer may be NULL. */
fem_status fem_mesh_plan_info(const fem_mesh_plan* plan, int* dim, int64_t* n_elem, int64_t* n_vert,
                              int* max_tile_vertices, int64_t* tile_vertices);
void fem_mesh_plan_destroy(fem_mesh_plan* plan);
/* fem_geometry through a plan (the affine element geometry of Section 3:
 * J^{-1} and |det J| per element): coords [n_vert][dim] FP64 device array;
 * out_dtype FEM_F32 or FEM_F64; inv_j [dim*dim][n_elem], det_j [n_elem] and
 * counts (may be NULL) as fem_geometry, whose outputs these are bit for bit.
 * Errors: NULL plan or array, a device other than the plan's ->
 * FEM_ERR_INVALID_ARG; another dtype -> FEM_ERR_UNSUPPORTED. An empty plan
 * returns FEM_OK at once. Asynchronous on `stream`. */
fem_status fem_geometry_planned(const fem_mesh_plan* plan, const double* coords, int out_dtype, void* inv_j,
                               void* det_j, int32_t* counts, void* stream);
/* fem_integrate_residual_mesh through a plan: coords [n_vert][dim] FP64, u
 * and coef per element as there, elem_vec [N_bt][n_elem]; inv_j/det_j
 * (both or neither) and counts as there (may be NULL). */
fem_status fem_integrate_residual_planned(const fem_mesh_plan* plan, int physics, int rule, int coef_space,
                                          int dtype, const double* coords, const void* u, const void* coef,
                                          void* elem_vec, void* inv_j, void* det_j, int32_t* counts, void* stream);
/* fem_integrate_residual_gather through a plan: u_vertex [n_vert][N_comp],
 * a P1 coefficient per vertex, point and cell coefficients per element. */
fem_status fem_integrate_residual_gather_planned(const fem_mesh_plan* plan, int physics, int rule, int coef_space,
                                                 int dtype, const double* coords, const void* u_vertex,
                                                 const void* coef, void* elem_vec, void* inv_j, void* det_j,
                                                 int32_t* counts, void* stream);

/* ------------------------------------------------------------------ */
/* Element matrices: the Jacobian of the element residual with respect */
/* to the closure (Eq. (2) of Section 2 differentiated in u).          */
/* ------------------------------------------------------------------ */

/* K_e = dR_e / du_e for P1 (order 1), P2 (order 2) or P3 (order 3) elements from
 * precomputed affine geometry: per quadrature point, the derivatives of the
 * pointwise functions, g0 = d f0 / d u and g3 = d f1 / d grad u, between the
 * basis values and physical gradients,
 *   K[(b,c)][(b',c')] = sum_q w_q |det J| ( phi_b g0[c][c'] phi_b'
 *                       + sum_{i,j} G_b,i g3[c][i][c'][j] G_b',j ),
 * Laplacian g3 = kappa delta_ij; elasticity g3 = lambda delta_ci delta_c'j
 * + mu (delta_cc' delta_ij + delta_cj delta_ic'); mass g0 = kappa. The three
 * forms are linear in u, so K_e u_e = R_e(u_e): the matrix is what the
 * residual entry points apply without forming it.
 *   inv_j [dim*dim][n], det_j [n], coef [N_coef][N_w][n] as for the
 *   residual of the same order; elem_mat [N_bt*N_bt][n], N_bt = N_b*N_comp,
 *   row r*N_bt + s for test function r = b*N_comp + c and trial function
 *   s = b'*N_comp + c' (node order as fem_integrate_residual_p2 for P2).
 * The matrices are symmetric and written so exactly (each entry below the
 * diagonal is a copy of its mirror). Rules: order 1 takes FEM_RULE_TRI3 /
 * FEM_RULE_TET4 or FEM_RULE_CENTROID; order 2 takes the degree-2 rule or
 * FEM_RULE_TRI6 / FEM_RULE_TET11; order 3 takes FEM_RULE_TRI6 /
 * FEM_RULE_TET11 (node order as fem_integrate_residual_p3; its columns are
 * the residuals of unit closures). Arrays are device memory owned by the
 * caller; elem_mat may not overlap the inputs. Errors as
 * fem_integrate_residual (FEM_ERR_UNSUPPORTED for another order or rule). */
fem_status fem_integrate_jacobian(int dim, int physics, int rule, int coef_space, int order, int dtype,
                                  int64_t n_elem, const void* inv_j, const void* det_j, const void* coef,
                                  void* elem_mat, void* stream);

/* ------------------------------------------------------------------ */
/* Batched persistent launch over many meshes (not in the paper; its   */
/* nearest analog is the assignment of cell chunks to thread blocks,   */
/* Section 3).                                                          */
/* ------------------------------------------------------------------ */

typedef struct fem_mesh_desc {
    int dim, physics, rule, coef_space;
    int64_t n_elem;
    const void* inv_j;
    const void* det_j;
    const void* u;
    const void* coef;
    void* elem_vec;
} fem_mesh_desc;

typedef struct fem_batch_plan fem_batch_plan;

/* Copies the descriptors (the arrays they point to stay owned by the
 * caller and must outlive the plan) into device memory owned by the plan,
 * and builds the tile list. All meshes share one dtype. The plan is bound to
 * the device current at creation. */
fem_status fem_batch_plan_create(const fem_mesh_desc* meshes, int n_mesh, int dtype,
                                 fem_batch_plan** out);
/* Launch shape of the persistent kernel: waves per workgroup (1, 2, 4, 8;
 * one element per lane, so a tile is 64*waves_per_block elements) and
 * workgroups per compute unit (0 = one workgroup per tile). Defaults 8 and 0.
 * Drops a recorded graph (capture again). Synchronizes the device. */
fem_status fem_batch_plan_set_launch(fem_batch_plan* plan, int waves_per_block, int blocks_per_cu);
/* Sweep the launch shapes above (waves per workgroup 1, 2, 4, 8; workgroups
 * per compute unit 0, 2, 4, 8, 16) on the plan's own meshes, timing a few
 * launches of each with HIP events on `stream`, and keep the fastest (as
 * fem_batch_plan_set_launch would; a recorded graph is dropped). The runs
 * write every mesh's element vectors. The chosen shape is returned through
 * the two pointers (either may be NULL). Synchronizes the device. */
fem_status fem_batch_plan_autotune(fem_batch_plan* plan, void* stream, int* waves_per_block, int* blocks_per_cu);
/* One persistent launch covering every mesh, on `stream`. */
fem_status fem_batch_run(fem_batch_plan* plan, void* stream);
/* Record the persistent launch into a HIP graph (captured on `stream`, which
 * must not be capturing already) and instantiate it. */
fem_status fem_batch_capture(fem_batch_plan* plan, void* stream);
/* Launch the instantiated graph on `stream`; FEM_ERR_INVALID_ARG if not
 * captured. */
fem_status fem_batch_replay(fem_batch_plan* plan, void* stream);
/* Frees the plan's device memory and graph. Safe on NULL. */
void fem_batch_plan_destroy(fem_batch_plan* plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * persistent launch as fem_batch_run, with bitwise-equal element vectors,
 * without a plan. The descriptor table goes to a fixed device array inside
 * the library (one per GPU, FEM_BATCH_NOALLOC_MAX_MESHES entries, about
 * 72 KB, held until the process ends), written on `stream` by small kernels
 * that receive the descriptors as kernel arguments (32 per launch), and each
 * workgroup finds its mesh by a binary search over that table, so the call
 * allocates nothing, copies nothing from host memory and needs no tile
 * table. Meshes, dtype
 * and arrays as fem_batch_plan_create; launch shape as
 * fem_batch_plan_set_launch (waves per workgroup 1, 2, 4, 8; workgroups per
 * compute unit 0..64). More than FEM_BATCH_NOALLOC_MAX_MESHES meshes give
 * FEM_ERR_INVALID_ARG. Every call on a GPU shares that GPU's table: calls
 * in order on one stream are safe, calls that overlap (other streams, other
 * host threads) race and may integrate another call's meshes. */
#define FEM_BATCH_NOALLOC_MAX_MESHES 1024
fem_status fem_batch_run_noalloc(const fem_mesh_desc* meshes, int n_mesh, int dtype, int waves_per_block,
                                 int blocks_per_cu, void* stream);

/* ------------------------------------------------------------------ */
/* Launch configuration and autotuning (analog of the paper's sweep of  */
/* blocks per batch and batches per chunk, Section 6, Table 2).         */
/* ------------------------------------------------------------------ */

typedef struct fem_tuning {
    int strategy;        /* enum fem_strategy (each strategy names the operations it serves) */
    int vec;             /* elements per lane: RESIDUAL and BACKWARD read 1, 2 or 4
                          * consecutive elements per vector access; GEOMETRY,
                          * RESIDUAL_MESH and RESIDUAL_GATHER (1, 2, 4) give each lane that
                          * many elements 64 apart, to overlap their dependent vertex
                          * gathers; the P2 and element-matrix ops take 1 */
    int waves_per_block; /* 1, 2, 4 or 8 (wave64; at most 4 for the P2 and
                          * element-matrix ops) */
    int blocks_per_cu;   /* persistent grid = blocks_per_cu * CUs; 0 = one pass, no grid stride */
} fem_tuning;

/* The configuration used for (op, dim, physics, rule, dtype), for every
 * coefficient space: the last one set or tuned in this process, else a
 * built-in default. */
fem_status fem_get_tuning(int op, int dim, int physics, int rule, int dtype, fem_tuning* out);
/* Override the configuration for (op, dim, physics, rule, dtype) in this process. */
fem_status fem_set_tuning(int op, int dim, int physics, int rule, int dtype, const fem_tuning* t);
/* Sweep launch configurations of `op` on synthetic device data of
 * n_elem_probe elements (a structured mesh for the mesh operations;
 * allocated and freed here, on the current device), time each with HIP
 * events (coefficients on quadrature points), keep the fastest for this
 * process, and, if cache_path is not NULL, merge it into that JSON cache
 * file. Synchronizes the device. */
fem_status fem_autotune(int op, int dim, int physics, int rule, int dtype, int64_t n_elem_probe,
                        const char* cache_path);
/* Load tuned configurations from a JSON cache written by fem_autotune.
 * Returns FEM_ERR_NO_TUNING if the file is missing or holds no entry for
 * this device's architecture (defaults stay in force). The library also
 * loads the cache named by the environment variable FEM_TUNE_CACHE, once,
 * before its first tuning lookup or change (explicit settings made later
 * take precedence; a missing or unusable file leaves the defaults). */
fem_status fem_load_tuning(const char* cache_path);

/* ------------------------------------------------------------------ */
/* Assembly (Section 2: the global residual is the sum over elements of  */
/* each element vector mapped back through the element restriction,    */
/* F = sum_e E_e^T R_e) and the restriction itself (the closure).       */
/* ------------------------------------------------------------------ */

/* Vertex field layout: [n_vert][n_comp], component c of vertex v at
 * v*n_comp + c, n_comp in {1, 2, 3}. */
typedef struct fem_assembly_plan fem_assembly_plan;

/* Builds, on the device, the transpose of the connectivity conn
 * [n_elem][dim+1] (device, int32): for every vertex the (element, local
 * vertex) slots that touch it, in increasing element order. The plan owns
 * that index (about 4 (dim+1) n_elem + 4 n_vert bytes) and keeps no pointer
 * to conn. Synchronizes `stream` (the index is validated before returning).
 * Errors: FEM_ERR_INVALID_ARG (negative sizes, NULL, an index outside
 * [0, n_vert)), FEM_ERR_UNSUPPORTED (dim, or n_elem*(dim+1) or n_vert not
 * below 2^31), FEM_ERR_HIP. */
fem_status fem_assembly_plan_create(int dim, int64_t n_elem, int64_t n_vert, const int32_t* conn,
                                    void* stream, fem_assembly_plan** out);
/* vertex_vec[v][c] = sum over the slots (e, b) of v, in increasing e, of
 * elem_vec[b*n_comp + c][e], starting from zero, in `dtype` arithmetic: the
 * same sum in the same order every call (no atomics). elem_vec is
 * [(dim+1)*n_comp][n_elem] as written by the residual entry points.
 * Errors: FEM_ERR_INVALID_ARG (NULL plan or array), FEM_ERR_UNSUPPORTED
 * (n_comp, dtype), FEM_ERR_HIP. */
fem_status fem_assemble(const fem_assembly_plan* plan, int n_comp, int dtype, const void* elem_vec,
                        void* vertex_vec, void* stream);
/* Sizes the plan was built for (any output may be NULL). */
fem_status fem_assembly_plan_info(const fem_assembly_plan* plan, int* dim, int64_t* n_elem,
                                  int64_t* n_vert);
void fem_assembly_plan_destroy(fem_assembly_plan* plan);

/* The element restriction (closure), the adjoint of fem_assemble:
 * elem_vec[b*n_comp + c][e] = vertex_vec[conn[e][b]][c]. An index outside
 * [0, n_vert) gives NaN entries for that element; nothing outside
 * vertex_vec is read. Errors: as fem_assemble, plus FEM_ERR_INVALID_ARG for
 * negative sizes and elements without vertices. */
fem_status fem_restrict(int dim, int n_comp, int dtype, int64_t n_elem, int64_t n_vert, const int32_t* conn,
                        const void* vertex_vec, void* elem_vec, void* stream);

/* ------------------------------------------------------------------ */
/* Measurement helpers                                                  */
/* ------------------------------------------------------------------ */

/* dst[0..n_bytes) = src[0..n_bytes) with a plain streaming copy kernel
 * (16-byte vector loads and stores; n_bytes and both pointers must be
 * multiples of 16). Used to measure the achievable HBM bandwidth and to
 * calibrate hardware byte counters. */
fem_status fem_stream_copy(const void* src, void* dst, int64_t n_bytes, void* stream);

/* The structure-of-arrays streaming yardstick. Reads n_in rows of n words
 * (row r at src + r * n) and writes n_out rows (row w at dst + w * n), one
 * lane per column: dst[w][e] = (sum over r of src[r][e]) + w, the sum taken
 * in row order, words of dtype (FEM_F32 or FEM_F64). An element kernel
 * reads and writes its SoA data as such rows (inverse Jacobian, det J,
 * closure and coefficient rows in; the element-vector rows out), and the
 * rate at which rows stream falls as their number grows; this kernel has
 * the row structure without the arithmetic, so its time is what any kernel
 * with the same rows needs. Both buffers are device memory owned by the
 * caller (n_in * n and n_out * n words). Errors: FEM_ERR_UNSUPPORTED for an
 * unknown dtype; FEM_ERR_INVALID_ARG for negative n, row counts outside
 * 1..FEM_STREAM_ROWS_MAX or NULL buffers (n = 0 does nothing). */
#define FEM_STREAM_ROWS_MAX 256
fem_status fem_stream_rows(int dtype, int64_t n, int n_in, int n_out, const void* src, void* dst, void* stream);

/* Message describing the last error on this thread ("" if none). */
const char* fem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */
