/*
 * c_abi_consumer.c -- a plain C program that uses libfemq through include/fem.h
 * only (device memory from the HIP runtime API, no C++ and no Python), and
 * checks it against the FP64 oracle library (test infrastructure).
 *
 * On a jittered 3D Kuhn grid with a variable coefficient at the quadrature
 * points it checks, in FP64:
 *   - fem_geometry then fem_integrate_residual against fem_oracle_residual
 *     (max |dR| relative to max |R| <= 1e-12);
 *   - fem_integrate_residual_mesh bit for bit against the two calls, and
 *     fem_integrate_residual_planned (through a mesh plan) bit for bit
 *     against fem_integrate_residual_mesh;
 *   - fem_assemble against the element-order sum of the oracle's element
 *     vectors (bit for bit: same values, same order, FP64);
 *   - fem_integrate_jacobian (element matrices) against the oracle's
 *     (max |dK| relative to max |K| <= 1e-12), and K_e u_e against R_e;
 *   - fem_integrate_residual_p3 (third order, eleven-point rule) against
 *     fem_oracle_integrate_p on the oracle's geometry (<= 1e-12 relative);
 *   - the error paths of a few calls (status codes, fem_last_error).
 * Exit status 0 on success; messages on stderr.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fem.h"

/* oracle (liboracle.so) */
int64_t fem_oracle_residual(int dim, int physics, int rule, int space, int64_t n_elem, int64_t n_vert,
                            const double *coords, const int32_t *conn, const double *u, const double *coef,
                            double *elem_vec);
int fem_oracle_assemble(int dim, int n_comp, int64_t n_elem, int64_t n_vert, const int32_t *conn,
                        const double *elem_vec, double *out);
int64_t fem_oracle_geometry(int dim, int64_t n_elem, int64_t n_vert, const double *coords, const int32_t *conn,
                            double *inv_j, double *det_j);
int fem_oracle_jacobian_p(int order, int dim, int physics, int rule, int space, int64_t n_elem, const double *inv_j,
                          const double *det_j, const double *coef, double *elem_mat, int absmode);
int fem_oracle_integrate_p(int order, int dim, int physics, int rule, int space, int64_t n_elem, const double *inv_j,
                           const double *det_j, const double *u, const double *coef, double *elem_vec, int absmode);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform(double lo, double hi) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (hi - lo) * (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK_HIP(x)                                                                  \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "HIP error %d at %s:%d\n", (int)e_, __FILE__, __LINE__);  \
            return 2;                                                                 \
        }                                                                             \
    } while (0)

#define CHECK_FEM(x)                                                                            \
    do {                                                                                        \
        fem_status s_ = (x);                                                                    \
        if (s_ != FEM_OK) {                                                                     \
            fprintf(stderr, "fem error %d (%s) at %s:%d\n", s_, fem_last_error(), __FILE__, __LINE__); \
            return 3;                                                                           \
        }                                                                                       \
    } while (0)

int main(void) {
    const int nc = 6, m = nc + 1;                 /* cells per side, vertices per side */
    const int64_t n_vert = (int64_t)m * m * m, n_elem = 6LL * nc * nc * nc;
    const double h = 1.0 / nc;
    double *X = malloc(sizeof(double) * 3 * n_vert);
    int32_t *conn = malloc(sizeof(int32_t) * 4 * n_elem);
    double *u = malloc(sizeof(double) * 4 * n_elem), *coef = malloc(sizeof(double) * 4 * n_elem);
    double *R_ref = malloc(sizeof(double) * 4 * n_elem), *R = malloc(sizeof(double) * 4 * n_elem);
    double *R_mesh = malloc(sizeof(double) * 4 * n_elem), *R_plan = malloc(sizeof(double) * 4 * n_elem);
    double *F_ref = malloc(sizeof(double) * n_vert), *F = malloc(sizeof(double) * n_vert);
    double *u_vert = malloc(sizeof(double) * n_vert);
    double *K = malloc(sizeof(double) * 16 * n_elem), *K_ref = malloc(sizeof(double) * 16 * n_elem);
    double *ij_ref = malloc(sizeof(double) * 9 * n_elem), *dj_ref = malloc(sizeof(double) * n_elem);
    if (!X || !conn || !u || !coef || !R_ref || !R || !R_mesh || !R_plan || !F_ref || !F || !u_vert || !K || !K_ref ||
        !ij_ref || !dj_ref)
        return 4;

    /* vertices: grid points, interior ones jittered by at most 0.2 h */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < m; ++k) {
                const int64_t v = ((int64_t)i * m + j) * m + k;
                const int idx[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    const int interior = idx[0] > 0 && idx[0] < nc && idx[1] > 0 && idx[1] < nc && idx[2] > 0 &&
                                         idx[2] < nc;
                    X[3 * v + d] = h * idx[d] + (interior ? uniform(-0.2 * h, 0.2 * h) : 0.0);
                }
                u_vert[v] = uniform(-1.0, 1.0);
            }
    /* six Kuhn tetrahedra per cell along v000 -> v111, positively oriented */
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t e = 0;
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j)
            for (int k = 0; k < nc; ++k)
                for (int t = 0; t < 6; ++t, ++e) {
                    int c[3] = {i, j, k};
                    int32_t vv[4];
                    vv[0] = (int32_t)(((int64_t)c[0] * m + c[1]) * m + c[2]);
                    for (int s = 0; s < 3; ++s) {
                        c[perm[t][s]] += 1;
                        vv[s + 1] = (int32_t)(((int64_t)c[0] * m + c[1]) * m + c[2]);
                    }
                    /* odd permutations have negative orientation: swap the last two */
                    const int odd = (t == 1 || t == 2 || t == 5);
                    if (odd) { int32_t tmp = vv[2]; vv[2] = vv[3]; vv[3] = tmp; }
                    for (int b = 0; b < 4; ++b) {
                        conn[4 * e + b] = vv[b];
                        u[(int64_t)b * n_elem + e] = u_vert[vv[b]];
                        coef[(int64_t)b * n_elem + e] = uniform(0.5, 2.0);
                    }
                }

    /* oracle */
    if (fem_oracle_residual(3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, n_elem, n_vert, X, conn, u, coef, R_ref) != 0) {
        fprintf(stderr, "oracle: degenerate elements or bad arguments\n");
        return 5;
    }
    if (fem_oracle_assemble(3, 1, n_elem, n_vert, conn, R_ref, F_ref) != 0) return 5;
    if (fem_oracle_geometry(3, n_elem, n_vert, X, conn, ij_ref, dj_ref) != 0) return 5;
    if (fem_oracle_jacobian_p(1, 3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, n_elem, ij_ref, dj_ref, coef, K_ref,
                              0) != 0)
        return 5;

    /* device buffers */
    double *dX, *du, *dcoef, *dij, *ddj, *dR, *dRm, *dF, *dK, *dRp;
    int32_t *dconn, *dcounts;
    CHECK_HIP(hipMalloc((void**)&dX, sizeof(double) * 3 * n_vert));
    CHECK_HIP(hipMalloc((void**)&dconn, sizeof(int32_t) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&du, sizeof(double) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dcoef, sizeof(double) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dij, sizeof(double) * 9 * n_elem));
    CHECK_HIP(hipMalloc((void**)&ddj, sizeof(double) * n_elem));
    CHECK_HIP(hipMalloc((void**)&dR, sizeof(double) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dRm, sizeof(double) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dF, sizeof(double) * n_vert));
    CHECK_HIP(hipMalloc((void**)&dK, sizeof(double) * 16 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dRp, sizeof(double) * 4 * n_elem));
    CHECK_HIP(hipMalloc((void**)&dcounts, sizeof(int32_t) * 2));
    CHECK_HIP(hipMemcpy(dX, X, sizeof(double) * 3 * n_vert, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dconn, conn, sizeof(int32_t) * 4 * n_elem, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(du, u, sizeof(double) * 4 * n_elem, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dcoef, coef, sizeof(double) * 4 * n_elem, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemset(dcounts, 0, sizeof(int32_t) * 2));

    hipStream_t stream;
    CHECK_HIP(hipStreamCreate(&stream));
    CHECK_FEM(fem_geometry(3, n_elem, n_vert, dX, dconn, FEM_F64, dij, ddj, dcounts, stream));
    CHECK_FEM(fem_integrate_residual(3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, FEM_F64, n_elem, dij, ddj, du,
                                     dcoef, dR, stream));
    CHECK_FEM(fem_integrate_residual_mesh(3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, FEM_F64, n_elem, n_vert, dX,
                                          dconn, du, dcoef, dRm, NULL, NULL, NULL, stream));
    fem_assembly_plan *plan = NULL;
    CHECK_FEM(fem_assembly_plan_create(3, n_elem, n_vert, dconn, stream, &plan));
    CHECK_FEM(fem_assemble(plan, 1, FEM_F64, dR, dF, stream));
    CHECK_FEM(fem_integrate_jacobian(3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, 1, FEM_F64, n_elem, dij, ddj, dcoef,
                                     dK, stream));
    fem_mesh_plan *mplan = NULL;
    CHECK_FEM(fem_mesh_plan_create(3, n_elem, n_vert, dconn, stream, &mplan));
    CHECK_FEM(fem_integrate_residual_planned(mplan, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, FEM_F64, dX, du, dcoef,
                                             dRp, NULL, NULL, NULL, stream));
    CHECK_HIP(hipStreamSynchronize(stream));

    int32_t counts[2];
    CHECK_HIP(hipMemcpy(counts, dcounts, sizeof counts, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(R, dR, sizeof(double) * 4 * n_elem, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(R_mesh, dRm, sizeof(double) * 4 * n_elem, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(F, dF, sizeof(double) * n_vert, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(K, dK, sizeof(double) * 16 * n_elem, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(R_plan, dRp, sizeof(double) * 4 * n_elem, hipMemcpyDeviceToHost));

    int fails = 0;
    if (counts[0] != 0) { fprintf(stderr, "unexpected degenerate elements: %d\n", counts[0]); ++fails; }
    double dmax = 0.0, rmax = 0.0;
    for (int64_t i = 0; i < 4 * n_elem; ++i) {
        dmax = fmax(dmax, fabs(R[i] - R_ref[i]));
        rmax = fmax(rmax, fabs(R_ref[i]));
    }
    if (!(dmax <= 1e-12 * rmax)) { fprintf(stderr, "residual vs oracle: %.3e relative\n", dmax / rmax); ++fails; }
    if (memcmp(R, R_mesh, sizeof(double) * 4 * n_elem) != 0) { fprintf(stderr, "fused != two calls\n"); ++fails; }
    if (memcmp(R_plan, R_mesh, sizeof(double) * 4 * n_elem) != 0) { fprintf(stderr, "planned != fused\n"); ++fails; }
    /* assembly of the GPU element vectors vs the oracle's assembly of the
     * same values: sum the GPU vectors with the oracle's routine */
    if (fem_oracle_assemble(3, 1, n_elem, n_vert, conn, R, F_ref) != 0) return 5;
    if (memcmp(F, F_ref, sizeof(double) * n_vert) != 0) { fprintf(stderr, "assembly differs from element-order sum\n"); ++fails; }
    /* element matrices: against the oracle, and K_e u_e against R_e */
    double kmax = 0.0, kref = 0.0, kumax = 0.0;
    for (int64_t i = 0; i < 16 * n_elem; ++i) {
        kmax = fmax(kmax, fabs(K[i] - K_ref[i]));
        kref = fmax(kref, fabs(K_ref[i]));
    }
    for (int64_t e2 = 0; e2 < n_elem; ++e2)
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int c = 0; c < 4; ++c) s += K[(int64_t)(r * 4 + c) * n_elem + e2] * u[(int64_t)c * n_elem + e2];
            kumax = fmax(kumax, fabs(s - R[(int64_t)r * n_elem + e2]));
        }
    if (!(kmax <= 1e-12 * kref)) { fprintf(stderr, "element matrices vs oracle: %.3e relative\n", kmax / kref); ++fails; }
    if (!(kumax <= 1e-12 * rmax)) { fprintf(stderr, "K u vs R: %.3e relative\n", kumax / rmax); ++fails; }

    /* third order: P3 closure (20 rows) and a coefficient at the 11 points,
     * on the oracle's geometry */
    {
        const int nb3 = 20, nq3 = 11;
        double *u3 = malloc(sizeof(double) * nb3 * n_elem), *c3 = malloc(sizeof(double) * nq3 * n_elem);
        double *R3_ref = malloc(sizeof(double) * nb3 * n_elem), *R3 = malloc(sizeof(double) * nb3 * n_elem);
        if (!u3 || !c3 || !R3_ref || !R3) return 4;
        for (int64_t i = 0; i < nb3 * n_elem; ++i) u3[i] = uniform(-1.0, 1.0);
        for (int64_t i = 0; i < nq3 * n_elem; ++i) c3[i] = uniform(0.5, 2.0);
        if (fem_oracle_integrate_p(3, 3, FEM_LAPLACE, FEM_RULE_TET11, FEM_COEF_QUAD, n_elem, ij_ref, dj_ref, u3, c3,
                                   R3_ref, 0) != 0)
            return 5;
        double *dij3, *ddj3, *du3, *dc3, *dR3;
        CHECK_HIP(hipMalloc((void**)&dij3, sizeof(double) * 9 * n_elem));
        CHECK_HIP(hipMalloc((void**)&ddj3, sizeof(double) * n_elem));
        CHECK_HIP(hipMalloc((void**)&du3, sizeof(double) * nb3 * n_elem));
        CHECK_HIP(hipMalloc((void**)&dc3, sizeof(double) * nq3 * n_elem));
        CHECK_HIP(hipMalloc((void**)&dR3, sizeof(double) * nb3 * n_elem));
        CHECK_HIP(hipMemcpy(dij3, ij_ref, sizeof(double) * 9 * n_elem, hipMemcpyHostToDevice));
        CHECK_HIP(hipMemcpy(ddj3, dj_ref, sizeof(double) * n_elem, hipMemcpyHostToDevice));
        CHECK_HIP(hipMemcpy(du3, u3, sizeof(double) * nb3 * n_elem, hipMemcpyHostToDevice));
        CHECK_HIP(hipMemcpy(dc3, c3, sizeof(double) * nq3 * n_elem, hipMemcpyHostToDevice));
        CHECK_FEM(fem_integrate_residual_p3(3, FEM_LAPLACE, FEM_RULE_TET11, FEM_COEF_QUAD, FEM_F64, n_elem, dij3, ddj3,
                                            du3, dc3, dR3, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        CHECK_HIP(hipMemcpy(R3, dR3, sizeof(double) * nb3 * n_elem, hipMemcpyDeviceToHost));
        double d3 = 0.0, r3 = 0.0;
        for (int64_t i = 0; i < nb3 * n_elem; ++i) {
            d3 = fmax(d3, fabs(R3[i] - R3_ref[i]));
            r3 = fmax(r3, fabs(R3_ref[i]));
        }
        if (!(d3 <= 1e-12 * r3)) { fprintf(stderr, "P3 residual vs oracle: %.3e relative\n", d3 / r3); ++fails; }
        if (fem_integrate_residual_p3(3, FEM_LAPLACE, FEM_RULE_TET4, FEM_COEF_QUAD, FEM_F64, n_elem, dij3, ddj3, du3,
                                      dc3, dR3, stream) != FEM_ERR_UNSUPPORTED) {
            fprintf(stderr, "expected FEM_ERR_UNSUPPORTED for P3 with a degree-2 rule\n");
            ++fails;
        }
        hipFree(dij3); hipFree(ddj3); hipFree(du3); hipFree(dc3); hipFree(dR3);
        free(u3); free(c3); free(R3_ref); free(R3);
    }

    /* error paths */
    if (fem_integrate_residual(3, FEM_LAPLACE, FEM_RULE_TRI3, FEM_COEF_QUAD, FEM_F64, n_elem, dij, ddj, du, dcoef,
                               dR, stream) != FEM_ERR_UNSUPPORTED || strlen(fem_last_error()) == 0) {
        fprintf(stderr, "expected FEM_ERR_UNSUPPORTED for a triangle rule in 3D\n");
        ++fails;
    }
    if (fem_geometry(3, -1, n_vert, dX, dconn, FEM_F64, dij, ddj, NULL, stream) != FEM_ERR_INVALID_ARG) {
        fprintf(stderr, "expected FEM_ERR_INVALID_ARG for a negative size\n");
        ++fails;
    }

    fem_assembly_plan_destroy(plan);
    fem_mesh_plan_destroy(mplan);
    CHECK_HIP(hipStreamDestroy(stream));
    hipFree(dX); hipFree(dconn); hipFree(du); hipFree(dcoef); hipFree(dij); hipFree(ddj);
    hipFree(dR); hipFree(dRm); hipFree(dF); hipFree(dcounts); hipFree(dK); hipFree(dRp);
    free(X); free(conn); free(u); free(coef); free(R_ref); free(R); free(R_mesh); free(F_ref); free(F); free(u_vert);
    free(K); free(K_ref); free(ij_ref); free(dj_ref); free(R_plan);
    if (fails) return 1;
    printf("c_abi_consumer: %lld elements, residual rel. error %.2e, element matrices %.2e, fused and assembly "
           "bitwise: ok\n", (long long)n_elem, dmax / rmax, kmax / kref);
    return 0;
}
