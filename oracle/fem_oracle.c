/*
 * fem_oracle.c -- plain FP64 reference integrator for P1 element residuals.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this file's library. The product path
 * (the HIP library) never calls it, and the two share no code, headers or
 * tables.
 *
 * What it computes (paper, Section 2 "Formulation", Eq. (2), the bracket
 * before assembly): for every element e
 *
 *     R_e = B^T W f0(u^q, grad u^q) + sum_k D_k^T W f1^k(u^q, grad u^q)
 *
 * with u^q and grad u^q evaluated at the quadrature points from tabulated
 * basis values, f0/f1 the pointwise physics, and W the quadrature weights
 * times |det J|. Everything is FP64, in plain loops, in that order: geometry,
 * then per quadrature point (field values, physics, weighting), then the sum
 * back onto the basis functions. No blocking, no fusion, no P1 shortcut:
 * gradients are recomputed from the tabulation at every quadrature point.
 *
 * Readings where the paper is silent (they are the conventions of this
 * project):
 *  - reference element: unit simplex {xi >= 0, sum xi <= 1}, basis
 *    phi_0 = 1 - sum xi, phi_k = xi_k (k = 1..d);
 *  - J[i][k] = (x_k - x_0)_i, the inverse is stored row-major
 *    invJ[k][i] = d xi_k / d x_i, and physical gradients are J^{-T} grad phi;
 *  - the measure factor is |det J|;
 *  - rules: triangle, three points with barycentric (2/3, 1/6, 1/6) and its
 *    permutations (point q has 2/3 at vertex q), weights 1/6; tetrahedron,
 *    four points with barycentric (a, b, b, b), a = (5 + 3 sqrt 5)/20,
 *    b = (5 - sqrt 5)/20 (point q has a at vertex q), weights 1/24;
 *    centroid rule, one point, weight 1/d!; for second-order elements also
 *    degree-4 rules: triangle, six points in two orbits (barycentric a at
 *    one vertex and (1-a)/2 at the others, a = 0.1081030181680702... and
 *    0.8168475729804585..., weights 0.2233815896780115/2 and
 *    0.1099517436553219/2); tetrahedron, eleven points (the centroid with
 *    weight -148/1875, (11/14, 1/14, 1/14, 1/14) with weight 343/7500,
 *    (a, a, b, b) with a = (1 + sqrt(5/14))/4, b = (1 - sqrt(5/14))/4 and
 *    weight 56/375, all times 1/6);
 *  - element order 1 (P1), 2 (P2: vertex functions lam (2 lam - 1), then
 *    edge functions 4 lam_i lam_j, edges (i, j), i < j, lexicographic) or 3
 *    (P3: the Lagrange basis on the nodes of the cubic lattice: vertices,
 *    two nodes per edge, the node nearer i first, then one node per face
 *    (i, j, k), i < j < k, lexicographic); the geometry stays affine, and a
 *    P1 coefficient keeps the d+1 vertex values and the P1 basis whatever
 *    the order of u;
 *  - physics: Laplacian f1 = kappa grad u (Section 2; f0 = 0);
 *    linear elasticity f1 = lambda tr(eps) I + 2 mu eps, eps the symmetric
 *    gradient (the paper's Lame function in Section 6 is lambda = 0,
 *    mu = 1/2); mass/reaction f0 = kappa u, f1 = 0;
 *  - coefficients (Section 4, "Variable Coefficients") live on quadrature
 *    points, or in the P1 space of u (nodal values, evaluated at point q
 *    with the same tabulation as u), or in P0 (one value per cell); they
 *    are evaluated at every quadrature point before the physics.
 *
 * Adjoint: L = sum_e w_e . R_e is linear in u for fixed coefficients and
 * linear in the coefficients for fixed u, so dL/du_j = w . R(u = unit_j) and
 * dL/dcoef_{m,q} = w . R(coef = unit_{m,q}) hold exactly; the oracle computes
 * the adjoint that way, from the forward definition alone.
 *
 * "absmode" evaluates the same sums with |.| applied to every factor; the
 * result bounds every partial sum and is the scale of the rounding-error
 * measure used by the parity tests.
 *
 * Element matrices: K_e = dR_e / du_e, the Jacobian of the bracket of
 * Eq. (2) with respect to the closure. Differentiating the bracket gives, per
 * quadrature point, the derivatives of the pointwise functions sandwiched
 * between the tabulated basis values and physical gradients:
 *
 *   K[(b,c)][(b',c')] = sum_q w_q |det J| ( B_qb g0[c][c'] B_qb'
 *                        + sum_{i,j} G_b,i(q) g3[c][i][c'][j] G_b',j(q) )
 *
 * with g0 = d f0 / d u and g3 = d f1 / d grad u (the mixed derivatives are
 * zero for the three forms here): Laplacian g3 = kappa delta_ij; elasticity
 * g3 = lambda delta_ci delta_c'j + mu (delta_cc' delta_ij + delta_cj
 * delta_ic'); mass g0 = kappa. The matrix is written from this definition,
 * not from the residual routine.
 *
 * Assembly (Section 2: the global residual is the sum over elements of the
 * element vectors mapped back through the element restriction E_e, the
 * transpose of the closure): F[v][c] = sum over (e, b) with conn[e][b] = v of
 * R_e[b*N_comp + c], summed element by element in increasing e, from zero.
 * Its adjoint is the restriction itself: the closure of a vertex field.
 *
 * Layouts (structure of arrays, n = n_elem):
 *   coords [n_vert][dim], conn [n_elem][dim+1] (0-based),
 *   inv_j [dim*dim][n] (row k*dim+i), det_j [n],
 *   u, w, elem_vec [N_b*N_comp][n] (row b*N_comp+c),
 *   coef [N_coef][N_w][n], N_w = N_q (points), N_b (P1) or 1 (P0),
 *   elem_mat [N_bt*N_bt][n] (row r*N_bt + s, r = b*N_comp + c the test
 *   function, s = b'*N_comp + c' the trial function).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define OR_MAXD 3
#define OR_MAXB 20
#define OR_MAXQ 11
#define OR_MAXC 3
#define OR_MAXCOEF 2

enum { OR_LAPLACE = 0, OR_ELASTICITY = 1, OR_MASS = 2 };
enum { OR_RULE_TRI3 = 0, OR_RULE_TET4 = 1, OR_RULE_CENTROID = 2, OR_RULE_TRI6 = 3, OR_RULE_TET11 = 4 };
enum { OR_COEF_QUAD = 0, OR_COEF_P1 = 1, OR_COEF_P0 = 2 };

int fem_oracle_n_qpts(int dim, int rule)
{
    if (dim != 2 && dim != 3) return -1;
    if (rule == OR_RULE_TRI3) return dim == 2 ? 3 : -1;
    if (rule == OR_RULE_TET4) return dim == 3 ? 4 : -1;
    if (rule == OR_RULE_CENTROID) return 1;
    if (rule == OR_RULE_TRI6) return dim == 2 ? 6 : -1;
    if (rule == OR_RULE_TET11) return dim == 3 ? 11 : -1;
    return -1;
}

/* Quadrature points xi[q][dim] on the unit simplex and weights wts[q].
 * Returns the number of points, or -1 for an unknown (dim, rule). */
int fem_oracle_rule(int dim, int rule, double *xi, double *wts)
{
    int nq = fem_oracle_n_qpts(dim, rule);
    if (nq < 0) return -1;
    double lam[OR_MAXQ][OR_MAXB];
    double wq[OR_MAXQ];
    for (int q = 0; q < nq; ++q) {
        for (int b = 0; b <= dim; ++b) {
            if (rule == OR_RULE_TRI3)
                lam[q][b] = (b == q) ? 2.0 / 3.0 : 1.0 / 6.0;
            else if (rule == OR_RULE_TET4)
                lam[q][b] = (b == q) ? (5.0 + 3.0 * sqrt(5.0)) / 20.0 : (5.0 - sqrt(5.0)) / 20.0;
            else
                lam[q][b] = 1.0 / (double)(dim + 1);
        }
        if (rule == OR_RULE_TRI3) wq[q] = 1.0 / 6.0;
        else if (rule == OR_RULE_TET4) wq[q] = 1.0 / 24.0;
        else wq[q] = (dim == 2) ? 0.5 : 1.0 / 6.0;
    }
    if (rule == OR_RULE_TRI6) {
        /* degree 4, two orbits of three points; point q (and q + 3) carries
         * the distinguished barycentric value at vertex q */
        const double a1 = 0.108103018168070227363341492234, b1 = 0.5 * (1.0 - a1);
        const double a2 = 0.816847572980458513080857073195, b2 = 0.5 * (1.0 - a2);
        const double w1 = 0.5 * 0.223381589678011465944710768628, w2 = 0.5 * 0.109951743655321867388622564704;
        for (int q = 0; q < 3; ++q)
            for (int b = 0; b < 3; ++b) {
                lam[q][b] = (b == q) ? a1 : b1;
                lam[q + 3][b] = (b == q) ? a2 : b2;
            }
        for (int q = 0; q < 3; ++q) { wq[q] = w1; wq[q + 3] = w2; }
    } else if (rule == OR_RULE_TET11) {
        /* degree 4: the centroid (negative weight), four points with 11/14 at
         * one vertex, six points with (1 + sqrt(5/14))/4 at the two vertices
         * of an edge, edges in lexicographic order */
        const double s = sqrt(5.0 / 14.0), a = 0.25 * (1.0 + s), b = 0.25 * (1.0 - s);
        for (int v = 0; v < 4; ++v) lam[0][v] = 0.25;
        wq[0] = -148.0 / 1875.0 / 6.0;
        for (int q = 0; q < 4; ++q) {
            for (int v = 0; v < 4; ++v) lam[q + 1][v] = (v == q) ? 11.0 / 14.0 : 1.0 / 14.0;
            wq[q + 1] = 343.0 / 7500.0 / 6.0;
        }
        int q = 5;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j, ++q) {
                for (int v = 0; v < 4; ++v) lam[q][v] = (v == i || v == j) ? a : b;
                wq[q] = 56.0 / 375.0 / 6.0;
            }
    }
    for (int q = 0; q < nq; ++q) {
        /* reference coordinates are the barycentric weights of vertices 1..d */
        for (int k = 0; k < dim; ++k) xi[q * dim + k] = lam[q][k + 1];
        wts[q] = wq[q];
    }
    return nq;
}

/* Lagrange basis of order 1, 2 or 3 on the unit simplex, in barycentric
 * coordinates lam_0 = 1 - sum xi, lam_k = xi_k (grad lam_0 = -1,
 * grad lam_k = e_k). Order 1: phi_b = lam_b. Order 2: vertex functions
 * lam_b (2 lam_b - 1), b = 0..d, then edge functions 4 lam_i lam_j for the
 * edges (i, j), i < j, in lexicographic order. Order 3 (nodes at barycentric
 * multiples of 1/3): vertex functions lam (3 lam - 1)(3 lam - 2) / 2; per
 * edge (i, j), lexicographic, (9/2) lam_i lam_j (3 lam_i - 1) (the node at
 * 2/3 lam_i) then (9/2) lam_i lam_j (3 lam_j - 1); per face (i, j, k),
 * lexicographic, 27 lam_i lam_j lam_k. Gradients follow from the chain rule
 * through the barycentric coordinates. */
static int or_nbasis(int dim, int order)
{
    if (order == 1) return dim + 1;
    if (order == 2) return (dim + 1) * (dim + 2) / 2;
    return (dim + 1) * (dim + 2) * (dim + 3) / 6;
}

static void or_grad_lam(int dim, int v, double g[OR_MAXD])
{
    for (int k = 0; k < dim; ++k) g[k] = (v == 0) ? -1.0 : (v - 1 == k ? 1.0 : 0.0);
}

static void or_basis(int dim, int order, const double *xi, double *phi, double dphi[OR_MAXB][OR_MAXD])
{
    double lam[OR_MAXD + 1], gl[OR_MAXD + 1][OR_MAXD];
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += xi[k];
    lam[0] = 1.0 - s;
    for (int k = 0; k < dim; ++k) lam[k + 1] = xi[k];
    for (int v = 0; v <= dim; ++v) or_grad_lam(dim, v, gl[v]);
    if (order == 1) {
        for (int b = 0; b <= dim; ++b) {
            phi[b] = lam[b];
            for (int k = 0; k < dim; ++k) dphi[b][k] = gl[b][k];
        }
        return;
    }
    if (order == 3) {
        /* derivative of each function with respect to each lam_v, then the
         * chain rule */
        double dl[OR_MAXB][OR_MAXD + 1];
        for (int b = 0; b < OR_MAXB; ++b)
            for (int v = 0; v <= dim; ++v) dl[b][v] = 0.0;
        int b = 0;
        for (int v = 0; v <= dim; ++v, ++b) {
            const double l = lam[v];
            phi[b] = 0.5 * l * (3.0 * l - 1.0) * (3.0 * l - 2.0);
            dl[b][v] = 0.5 * (27.0 * l * l - 18.0 * l + 2.0);
        }
        for (int i = 0; i <= dim; ++i)
            for (int j = i + 1; j <= dim; ++j)
                for (int s = 0; s < 2; ++s, ++b) {
                    const int a = s == 0 ? i : j, o = s == 0 ? j : i;  /* node nearer a */
                    phi[b] = 4.5 * lam[a] * lam[o] * (3.0 * lam[a] - 1.0);
                    dl[b][a] = 4.5 * lam[o] * (6.0 * lam[a] - 1.0);
                    dl[b][o] = 4.5 * lam[a] * (3.0 * lam[a] - 1.0);
                }
        for (int i = 0; i <= dim; ++i)
            for (int j = i + 1; j <= dim; ++j)
                for (int k = j + 1; k <= dim; ++k, ++b) {
                    phi[b] = 27.0 * lam[i] * lam[j] * lam[k];
                    dl[b][i] = 27.0 * lam[j] * lam[k];
                    dl[b][j] = 27.0 * lam[i] * lam[k];
                    dl[b][k] = 27.0 * lam[i] * lam[j];
                }
        for (int c = 0; c < b; ++c)
            for (int k = 0; k < dim; ++k) {
                double g = 0.0;
                for (int v = 0; v <= dim; ++v) g += dl[c][v] * gl[v][k];
                dphi[c][k] = g;
            }
        return;
    }
    for (int b = 0; b <= dim; ++b) {
        phi[b] = lam[b] * (2.0 * lam[b] - 1.0);
        for (int k = 0; k < dim; ++k) dphi[b][k] = (4.0 * lam[b] - 1.0) * gl[b][k];
    }
    int b = dim + 1;
    for (int i = 0; i <= dim; ++i)
        for (int j = i + 1; j <= dim; ++j, ++b) {
            phi[b] = 4.0 * lam[i] * lam[j];
            for (int k = 0; k < dim; ++k) dphi[b][k] = 4.0 * (lam[i] * gl[j][k] + lam[j] * gl[i][k]);
        }
}

/* Tabulation at the quadrature points: B[q][b] = phi_b(xi_q),
 * D[q][b][k] = d phi_b / d xi_k (xi_q) for the basis of u (order 1 to 3),
 * and B1[q][b] = lam_b(xi_q), the P1 basis a P1 coefficient lives in. */
typedef struct {
    int dim, order, nb, nq;
    double w[OR_MAXQ];
    double B[OR_MAXQ][OR_MAXB];
    double D[OR_MAXQ][OR_MAXB][OR_MAXD];
    double B1[OR_MAXQ][OR_MAXD + 1];
} or_tab;

static int or_tabulate(int dim, int rule, int order, or_tab *t)
{
    double xi[OR_MAXQ * OR_MAXD];
    if (order < 1 || order > 3) return -1;
    int nq = fem_oracle_rule(dim, rule, xi, t->w);
    if (nq < 0) return -1;
    t->dim = dim;
    t->order = order;
    t->nb = or_nbasis(dim, order);
    t->nq = nq;
    for (int q = 0; q < nq; ++q) {
        double d1[OR_MAXB][OR_MAXD];
        or_basis(dim, order, xi + q * dim, t->B[q], t->D[q]);
        or_basis(dim, 1, xi + q * dim, t->B1[q], d1);
    }
    return nq;
}

static int or_ncomp(int dim, int physics) { return physics == OR_ELASTICITY ? dim : 1; }
static int or_ncoef(int physics) { return physics == OR_ELASTICITY ? 2 : 1; }
static int or_physics_ok(int physics)
{
    return physics == OR_LAPLACE || physics == OR_ELASTICITY || physics == OR_MASS;
}

/* Words of one coefficient field per element, or -1 for an unknown space
 * (a P1 coefficient has the d+1 vertex values whatever the order of u). */
static int or_coef_words(int space, int dim, int nq)
{
    if (space == OR_COEF_QUAD) return nq;
    if (space == OR_COEF_P1) return dim + 1;
    if (space == OR_COEF_P0) return 1;
    return -1;
}

/* Coefficient values at the quadrature points, cq[m][q], from the element's
 * coefficient words a[m][k] in their space. */
static void or_coef_at_points(const or_tab *t, int space, int ncoef, double a[OR_MAXCOEF][OR_MAXB + OR_MAXQ],
                              double cq[OR_MAXCOEF][OR_MAXQ], int absmode)
{
    for (int m = 0; m < ncoef; ++m)
        for (int q = 0; q < t->nq; ++q) {
            if (space == OR_COEF_QUAD) {
                cq[m][q] = a[m][q];
            } else if (space == OR_COEF_P1) {
                double v = 0.0;
                for (int b = 0; b <= t->dim; ++b) v += (absmode ? fabs(t->B1[q][b]) : t->B1[q][b]) * a[m][b];
                cq[m][q] = v;
            } else {
                cq[m][q] = a[m][0];
            }
        }
}

/* Pointwise physics at one quadrature point.
 * uq[c], gu[c][i] = d u_c / d x_i, cq[m] = coefficient m at this point.
 * Outputs f0[c] and f1[c][i]. In absmode every input is already >= 0. */
static void or_physics(int dim, int physics, const double *uq, double gu[OR_MAXC][OR_MAXD],
                       const double *cq, double *f0, double f1[OR_MAXC][OR_MAXD])
{
    int nc = or_ncomp(dim, physics);
    for (int c = 0; c < nc; ++c) {
        f0[c] = 0.0;
        for (int i = 0; i < dim; ++i) f1[c][i] = 0.0;
    }
    if (physics == OR_LAPLACE) {
        for (int i = 0; i < dim; ++i) f1[0][i] = cq[0] * gu[0][i];
    } else if (physics == OR_ELASTICITY) {
        double eps[OR_MAXC][OR_MAXD];
        double tr = 0.0;
        for (int c = 0; c < dim; ++c)
            for (int i = 0; i < dim; ++i) eps[c][i] = 0.5 * (gu[c][i] + gu[i][c]);
        for (int i = 0; i < dim; ++i) tr += eps[i][i];
        for (int c = 0; c < dim; ++c)
            for (int i = 0; i < dim; ++i)
                f1[c][i] = (c == i ? cq[0] * tr : 0.0) + 2.0 * cq[1] * eps[c][i];
    } else { /* OR_MASS */
        f0[0] = cq[0] * uq[0];
    }
}

/* Residual of one element (Eq. (2) bracket).
 * ij[k][i] = invJ, sdet = |det J|, ub[b][c] nodal values, cf[m][q] coefficients.
 * R[b][c] is overwritten. */
static void or_element(const or_tab *t, int physics, double ij[OR_MAXD][OR_MAXD], double sdet,
                       double ub[OR_MAXB][OR_MAXC], double cf[OR_MAXCOEF][OR_MAXQ],
                       double R[OR_MAXB][OR_MAXC], int absmode)
{
    int dim = t->dim, nb = t->nb;
    int nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics);
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < nc; ++c) R[b][c] = 0.0;
    for (int q = 0; q < t->nq; ++q) {
        double G[OR_MAXB][OR_MAXD];   /* physical basis gradients J^{-T} grad phi_b */
        double Bq[OR_MAXB];
        for (int b = 0; b < nb; ++b) {
            Bq[b] = absmode ? fabs(t->B[q][b]) : t->B[q][b];
            for (int i = 0; i < dim; ++i) {
                double g = 0.0;
                for (int k = 0; k < dim; ++k) {
                    double d = absmode ? fabs(t->D[q][b][k]) : t->D[q][b][k];
                    g += ij[k][i] * d;
                }
                G[b][i] = g;
            }
        }
        double uq[OR_MAXC], gu[OR_MAXC][OR_MAXD];
        for (int c = 0; c < nc; ++c) {
            uq[c] = 0.0;
            for (int b = 0; b < nb; ++b) uq[c] += Bq[b] * ub[b][c];
            for (int i = 0; i < dim; ++i) {
                gu[c][i] = 0.0;
                for (int b = 0; b < nb; ++b) gu[c][i] += ub[b][c] * G[b][i];
            }
        }
        double cq[OR_MAXCOEF] = {0.0, 0.0};
        for (int m = 0; m < ncoef; ++m) cq[m] = cf[m][q];
        double f0[OR_MAXC], f1[OR_MAXC][OR_MAXD];
        or_physics(dim, physics, uq, gu, cq, f0, f1);
        double s = (absmode ? fabs(t->w[q]) : t->w[q]) * sdet;
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) {
                double v = Bq[b] * f0[c];
                for (int i = 0; i < dim; ++i) v += G[b][i] * f1[c][i];
                R[b][c] += s * v;
            }
    }
}

/* Affine geometry of one element from its vertices.
 * x[b][i] vertex coordinates. Returns det J; fills ij[k][i] = (J^{-1})[k][i]. */
static double or_geometry_one(int dim, double x[OR_MAXB][OR_MAXD], double ij[OR_MAXD][OR_MAXD])
{
    double J[OR_MAXD][OR_MAXD] = {{0.0}};
    for (int i = 0; i < dim; ++i)
        for (int k = 0; k < dim; ++k) J[i][k] = x[k + 1][i] - x[0][i];
    double det;
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        ij[0][0] = J[1][1] / det;
        ij[0][1] = -J[0][1] / det;
        ij[1][0] = -J[1][0] / det;
        ij[1][1] = J[0][0] / det;
    } else {
        /* cofactors C[i][k] of J; inverse = C^T / det */
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) ij[k][i] = C[i][k] / det;
    }
    return det;
}

/* Geometry for all elements. Returns the number of degenerate elements
 * (det J == 0 or not finite), or -1 on bad arguments / out-of-range vertex. */
int64_t fem_oracle_geometry(int dim, int64_t n_elem, int64_t n_vert, const double *coords,
                            const int32_t *conn, double *inv_j, double *det_j)
{
    if ((dim != 2 && dim != 3) || n_elem < 0 || n_vert < 0) return -1;
    int nb = dim + 1;
    int64_t ndeg = 0;
    for (int64_t e = 0; e < n_elem; ++e) {
        double x[OR_MAXB][OR_MAXD], ij[OR_MAXD][OR_MAXD];
        for (int b = 0; b < nb; ++b) {
            int64_t v = conn[e * nb + b];
            if (v < 0 || v >= n_vert) return -1;
            for (int i = 0; i < dim; ++i) x[b][i] = coords[v * dim + i];
        }
        double det = or_geometry_one(dim, x, ij);
        if (det == 0.0 || !isfinite(det)) ++ndeg;
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < dim; ++i) inv_j[(int64_t)(k * dim + i) * n_elem + e] = ij[k][i];
        det_j[e] = det;
    }
    return ndeg;
}

/* Element residuals from precomputed geometry for Lagrange elements of the
 * given order (1 to 3; closure rows b*N_comp + c with the node order of
 * or_basis). Returns 0, or -1 on bad arguments. absmode != 0 gives the
 * absolute-value bound described above. */
int fem_oracle_integrate_p(int order, int dim, int physics, int rule, int space, int64_t n_elem,
                           const double *inv_j, const double *det_j, const double *u, const double *coef,
                           double *elem_vec, int absmode)
{
    or_tab t;
    if (!or_physics_ok(physics) || n_elem < 0 || or_tabulate(dim, rule, order, &t) < 0) return -1;
    int nb = t.nb, nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics);
    int nw = or_coef_words(space, dim, t.nq);
    if (nw < 0) return -1;
    int64_t n = n_elem;
    for (int64_t e = 0; e < n; ++e) {
        double ij[OR_MAXD][OR_MAXD], ub[OR_MAXB][OR_MAXC], cf[OR_MAXCOEF][OR_MAXQ], R[OR_MAXB][OR_MAXC];
        double a[OR_MAXCOEF][OR_MAXB + OR_MAXQ];
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < dim; ++i) {
                double v = inv_j[(int64_t)(k * dim + i) * n + e];
                ij[k][i] = absmode ? fabs(v) : v;
            }
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) {
                double v = u[(int64_t)(b * nc + c) * n + e];
                ub[b][c] = absmode ? fabs(v) : v;
            }
        for (int m = 0; m < ncoef; ++m)
            for (int k = 0; k < nw; ++k) {
                double v = coef[(int64_t)(m * nw + k) * n + e];
                a[m][k] = absmode ? fabs(v) : v;
            }
        or_coef_at_points(&t, space, ncoef, a, cf, absmode);
        or_element(&t, physics, ij, fabs(det_j[e]), ub, cf, R, absmode);
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) elem_vec[(int64_t)(b * nc + c) * n + e] = R[b][c];
    }
    return 0;
}

/* Coordinates and connectivity to element residuals, one element at a time
 * (geometry, then integration). Returns the number of degenerate elements,
 * or -1 on bad arguments. */
int64_t fem_oracle_residual(int dim, int physics, int rule, int space, int64_t n_elem, int64_t n_vert,
                            const double *coords, const int32_t *conn, const double *u,
                            const double *coef, double *elem_vec)
{
    or_tab t;
    if (!or_physics_ok(physics) || n_elem < 0 || n_vert < 0 || or_tabulate(dim, rule, 1, &t) < 0)
        return -1;
    int nb = t.nb, nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics);
    int nw = or_coef_words(space, dim, t.nq);
    if (nw < 0) return -1;
    int64_t n = n_elem, ndeg = 0;
    for (int64_t e = 0; e < n; ++e) {
        double x[OR_MAXB][OR_MAXD], ij[OR_MAXD][OR_MAXD];
        double ub[OR_MAXB][OR_MAXC], cf[OR_MAXCOEF][OR_MAXQ], R[OR_MAXB][OR_MAXC];
        double a[OR_MAXCOEF][OR_MAXB + OR_MAXQ];
        for (int b = 0; b < nb; ++b) {
            int64_t v = conn[e * nb + b];
            if (v < 0 || v >= n_vert) return -1;
            for (int i = 0; i < dim; ++i) x[b][i] = coords[v * dim + i];
        }
        double det = or_geometry_one(dim, x, ij);
        if (det == 0.0 || !isfinite(det)) ++ndeg;
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) ub[b][c] = u[(int64_t)(b * nc + c) * n + e];
        for (int m = 0; m < ncoef; ++m)
            for (int k = 0; k < nw; ++k) a[m][k] = coef[(int64_t)(m * nw + k) * n + e];
        or_coef_at_points(&t, space, ncoef, a, cf, 0);
        or_element(&t, physics, ij, fabs(det), ub, cf, R, 0);
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) elem_vec[(int64_t)(b * nc + c) * n + e] = R[b][c];
    }
    return ndeg;
}

/* Adjoint of L = sum_e w_e . R_e. du [N_bt][n] and dcoef [N_coef][N_q][n]
 * may each be NULL. Returns 0, or -1 on bad arguments. */
int fem_oracle_backward_p(int order, int dim, int physics, int rule, int space, int64_t n_elem,
                          const double *inv_j, const double *det_j, const double *u, const double *coef,
                          const double *w, double *du, double *dcoef)
{
    or_tab t;
    if (!or_physics_ok(physics) || n_elem < 0 || or_tabulate(dim, rule, order, &t) < 0) return -1;
    int nb = t.nb, nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics);
    int nw = or_coef_words(space, dim, t.nq);
    if (nw < 0) return -1;
    int64_t n = n_elem;
    for (int64_t e = 0; e < n; ++e) {
        double ij[OR_MAXD][OR_MAXD], ub[OR_MAXB][OR_MAXC], wb[OR_MAXB][OR_MAXC];
        double cf[OR_MAXCOEF][OR_MAXQ], R[OR_MAXB][OR_MAXC];
        double a[OR_MAXCOEF][OR_MAXB + OR_MAXQ];
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < dim; ++i) ij[k][i] = inv_j[(int64_t)(k * dim + i) * n + e];
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) {
                ub[b][c] = u[(int64_t)(b * nc + c) * n + e];
                wb[b][c] = w[(int64_t)(b * nc + c) * n + e];
            }
        for (int m = 0; m < ncoef; ++m)
            for (int k = 0; k < nw; ++k) a[m][k] = coef[(int64_t)(m * nw + k) * n + e];
        or_coef_at_points(&t, space, ncoef, a, cf, 0);
        double sdet = fabs(det_j[e]);
        if (du) {
            /* dL/du_j = w . R(unit_j): R is linear in u */
            for (int j = 0; j < nb * nc; ++j) {
                double unit[OR_MAXB][OR_MAXC];
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c) unit[b][c] = (b * nc + c == j) ? 1.0 : 0.0;
                or_element(&t, physics, ij, sdet, unit, cf, R, 0);
                double s = 0.0;
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c) s += wb[b][c] * R[b][c];
                du[(int64_t)j * n + e] = s;
            }
        }
        if (dcoef) {
            /* dL/dcoef_{m,k} = w . R(coef = unit_{m,k}): R is linear in the
             * coefficient words, whatever their space */
            for (int m = 0; m < ncoef; ++m)
                for (int k = 0; k < nw; ++k) {
                    double unit[OR_MAXCOEF][OR_MAXB + OR_MAXQ], uq[OR_MAXCOEF][OR_MAXQ];
                    for (int mm = 0; mm < ncoef; ++mm)
                        for (int kk = 0; kk < nw; ++kk) unit[mm][kk] = (mm == m && kk == k) ? 1.0 : 0.0;
                    or_coef_at_points(&t, space, ncoef, unit, uq, 0);
                    or_element(&t, physics, ij, sdet, ub, uq, R, 0);
                    double s = 0.0;
                    for (int b = 0; b < nb; ++b)
                        for (int c = 0; c < nc; ++c) s += wb[b][c] * R[b][c];
                    dcoef[(int64_t)(m * nw + k) * n + e] = s;
                }
        }
    }
    return 0;
}

/* Pointwise derivatives of the physics at one quadrature point from the
 * coefficients cq[m] there: g0[c][c'] = d f0_c / d u_c' and
 * g3[c][i][c'][j] = d f1_{c,i} / d (d u_c' / d x_j). In absmode the
 * coefficients are already >= 0 and every term is added with its sign
 * dropped. */
static void or_physics_jac(int dim, int physics, const double *cq, double g0[OR_MAXC][OR_MAXC],
                           double g3[OR_MAXC][OR_MAXD][OR_MAXC][OR_MAXD])
{
    memset(g0, 0, sizeof(double) * OR_MAXC * OR_MAXC);
    memset(g3, 0, sizeof(double) * OR_MAXC * OR_MAXD * OR_MAXC * OR_MAXD);
    if (physics == OR_LAPLACE) {
        for (int i = 0; i < dim; ++i) g3[0][i][0][i] = cq[0];
    } else if (physics == OR_ELASTICITY) {
        /* f1_ci = lambda tr(eps) delta_ci + 2 mu eps_ci, eps_ci = (du_c/dx_i + du_i/dx_c) / 2 */
        for (int c = 0; c < dim; ++c)
            for (int i = 0; i < dim; ++i)
                for (int cp = 0; cp < dim; ++cp)
                    for (int j = 0; j < dim; ++j) {
                        double v = 0.0;
                        if (c == i && cp == j) v += cq[0];
                        if (c == cp && i == j) v += cq[1];
                        if (c == j && i == cp) v += cq[1];
                        g3[c][i][cp][j] = v;
                    }
    } else { /* OR_MASS: f0 = kappa u */
        g0[0][0] = cq[0];
    }
}

/* Element matrix of one element; ij[k][i] = invJ, sdet = |det J|,
 * cf[m][q] coefficients at the points. K[r][s] is overwritten. */
static void or_element_jac(const or_tab *t, int physics, double ij[OR_MAXD][OR_MAXD], double sdet,
                           double cf[OR_MAXCOEF][OR_MAXQ], double K[OR_MAXB * OR_MAXC][OR_MAXB * OR_MAXC],
                           int absmode)
{
    int dim = t->dim, nb = t->nb;
    int nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics), nbt = nb * nc;
    for (int r = 0; r < nbt; ++r)
        for (int s = 0; s < nbt; ++s) K[r][s] = 0.0;
    for (int q = 0; q < t->nq; ++q) {
        double G[OR_MAXB][OR_MAXD], Bq[OR_MAXB];
        for (int b = 0; b < nb; ++b) {
            Bq[b] = absmode ? fabs(t->B[q][b]) : t->B[q][b];
            for (int i = 0; i < dim; ++i) {
                double g = 0.0;
                for (int k = 0; k < dim; ++k) {
                    double d = absmode ? fabs(t->D[q][b][k]) : t->D[q][b][k];
                    g += ij[k][i] * d;
                }
                G[b][i] = g;
            }
        }
        double cq[OR_MAXCOEF] = {0.0, 0.0};
        for (int m = 0; m < ncoef; ++m) cq[m] = cf[m][q];
        double g0[OR_MAXC][OR_MAXC], g3[OR_MAXC][OR_MAXD][OR_MAXC][OR_MAXD];
        or_physics_jac(dim, physics, cq, g0, g3);
        double s = (absmode ? fabs(t->w[q]) : t->w[q]) * sdet;
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c)
                for (int bp = 0; bp < nb; ++bp)
                    for (int cp = 0; cp < nc; ++cp) {
                        double v = Bq[b] * g0[c][cp] * Bq[bp];
                        for (int i = 0; i < dim; ++i)
                            for (int j = 0; j < dim; ++j) v += G[b][i] * g3[c][i][cp][j] * G[bp][j];
                        K[b * nc + c][bp * nc + cp] += s * v;
                    }
    }
}

/* Element matrices elem_mat [N_bt*N_bt][n] from precomputed geometry for
 * Lagrange elements of the given order (1 to 3). Returns 0, or -1 on bad
 * arguments. absmode != 0 gives the absolute-value bound. */
int fem_oracle_jacobian_p(int order, int dim, int physics, int rule, int space, int64_t n_elem,
                          const double *inv_j, const double *det_j, const double *coef, double *elem_mat,
                          int absmode)
{
    or_tab t;
    if (!or_physics_ok(physics) || n_elem < 0 || or_tabulate(dim, rule, order, &t) < 0) return -1;
    int nb = t.nb, nc = or_ncomp(dim, physics), ncoef = or_ncoef(physics), nbt = nb * nc;
    int nw = or_coef_words(space, dim, t.nq);
    if (nw < 0) return -1;
    int64_t n = n_elem;
    for (int64_t e = 0; e < n; ++e) {
        double ij[OR_MAXD][OR_MAXD], cf[OR_MAXCOEF][OR_MAXQ], a[OR_MAXCOEF][OR_MAXB + OR_MAXQ];
        double K[OR_MAXB * OR_MAXC][OR_MAXB * OR_MAXC];
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < dim; ++i) {
                double v = inv_j[(int64_t)(k * dim + i) * n + e];
                ij[k][i] = absmode ? fabs(v) : v;
            }
        for (int m = 0; m < ncoef; ++m)
            for (int k = 0; k < nw; ++k) {
                double v = coef[(int64_t)(m * nw + k) * n + e];
                a[m][k] = absmode ? fabs(v) : v;
            }
        or_coef_at_points(&t, space, ncoef, a, cf, absmode);
        or_element_jac(&t, physics, ij, fabs(det_j[e]), cf, K, absmode);
        for (int r = 0; r < nbt; ++r)
            for (int s = 0; s < nbt; ++s) elem_mat[(int64_t)(r * nbt + s) * n + e] = K[r][s];
    }
    return 0;
}

/* Global residual F [n_vert][n_comp] = sum_e E_e^T R_e from element vectors
 * elem_vec [(dim+1)*n_comp][n_elem]. Elements are added in increasing order.
 * Returns 0, or -1 on bad arguments or a vertex index out of range. */
int fem_oracle_assemble(int dim, int n_comp, int64_t n_elem, int64_t n_vert, const int32_t *conn,
                        const double *elem_vec, double *out)
{
    if ((dim != 2 && dim != 3) || n_comp < 1 || n_comp > OR_MAXC || n_elem < 0 || n_vert < 0) return -1;
    int nb = dim + 1;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int b = 0; b < nb; ++b) {
            int32_t v = conn[e * nb + b];
            if (v < 0 || v >= n_vert) return -1;
        }
    for (int64_t i = 0; i < n_vert * n_comp; ++i) out[i] = 0.0;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int b = 0; b < nb; ++b) {
            int64_t v = conn[e * nb + b];
            for (int c = 0; c < n_comp; ++c) out[v * n_comp + c] += elem_vec[(int64_t)(b * n_comp + c) * n_elem + e];
        }
    return 0;
}

/* Element restriction (the closure): elem_vec[(b*n_comp + c)][e] =
 * vert[conn[e][b]][c]. Returns 0, or -1 on bad arguments or a vertex index
 * out of range. */
int fem_oracle_restrict(int dim, int n_comp, int64_t n_elem, int64_t n_vert, const int32_t *conn,
                        const double *vert, double *elem_vec)
{
    if ((dim != 2 && dim != 3) || n_comp < 1 || n_comp > OR_MAXC || n_elem < 0 || n_vert < 0) return -1;
    int nb = dim + 1;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int b = 0; b < nb; ++b) {
            int64_t v = conn[e * nb + b];
            if (v < 0 || v >= n_vert) return -1;
            for (int c = 0; c < n_comp; ++c) elem_vec[(int64_t)(b * n_comp + c) * n_elem + e] = vert[v * n_comp + c];
        }
    return 0;
}

/* Order-1 forms of the two routines above (P1 elements). */
int fem_oracle_integrate(int dim, int physics, int rule, int space, int64_t n_elem, const double *inv_j,
                         const double *det_j, const double *u, const double *coef,
                         double *elem_vec, int absmode)
{
    return fem_oracle_integrate_p(1, dim, physics, rule, space, n_elem, inv_j, det_j, u, coef, elem_vec, absmode);
}

int fem_oracle_backward(int dim, int physics, int rule, int space, int64_t n_elem, const double *inv_j,
                        const double *det_j, const double *u, const double *coef,
                        const double *w, double *du, double *dcoef)
{
    return fem_oracle_backward_p(1, dim, physics, rule, space, n_elem, inv_j, det_j, u, coef, w, du, dcoef);
}
