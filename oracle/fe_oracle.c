/*
 * fe_oracle.c -- plain, slow CPU oracle for linear (P1) finite element assembly of
 * the Poisson problem, written from L. Chen, "Programming of Finite Element Methods
 * in MATLAB".
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
 * leg of the benchmark are the only code that may load this file.  It shares no
 * code, header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Everything is IEEE double precision, single-threaded, in plain loops:
 *   - local stiffness through the affine map of the reference simplex, gradients
 *     by solving B x = G with Gaussian elimination (Section 3.1.1), generalised
 *     from triangles to tetrahedra in the same way;
 *   - triplets (i, j, s) collected element by element, local row then local column
 *     (Section 3.1.2), then one call of a `sparse` routine that sorts them stably by
 *     (row, column) and adds duplicates left to right (Section 2.2);
 *   - load vector: 2-D three edge-midpoint rule (Section 3.2 and Section 4); 3-D
 *     symmetric four-point rule of degree two (the paper names a 4-point rule but
 *     lists none; the reading used here is recorded in the design notes); on
 *     request the one-point (centroid) or the trapezoidal (vertex) rule of Section 4;
 *   - Dirichlet lifting b <- b - A u_D and Neumann side integrals by the midpoint
 *     (2-D) / centroid (3-D) rule (Section 3.3);
 *   - solve on the free nodes (equation (directsolve)): dense Cholesky when small,
 *     plain Jacobi-preconditioned CG otherwise;
 *   - adjoint gradient dJ/dkappa_t = -|t| grad(lambda_h) . grad(u_h) on t.
 *
 * Array layout: node[c*N + k], elem[a*NT + t] (0-based), bdflag[a*NT + t];
 * face a of an element is opposite its local vertex a (Section 1.2).
 * Return codes: 0 ok, -1 invalid argument, -2 bad element (measure <= 0 or not
 * finite), -3 unsupported (dimension, boundary type 3), -7 no convergence.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EMESH (-2)
#define OR_EUNSUPPORTED (-3)
#define OR_ENOCONV (-7)

/* kinds of a data function (source f, Dirichlet g_D, Neumann g_N) */
#define OR_FN_ZERO 0
#define OR_FN_CONST 1
#define OR_FN_LINEAR 2
#define OR_FN_SINPROD 3
#define OR_FN_DUDN_SINPROD 4
#define OR_FN_NODAL 5

typedef struct {
    int32_t kind;
    double c[4];
    const double *nodal;
} or_fn;

static const double OR_PI = 3.14159265358979323846;

/* Value of a data function at point x (dim coordinates).  `bary`/`verts` give the
 * point's barycentric coordinates in an element with vertices verts[0..nv-1], used
 * only by the NODAL kind (piecewise-linear interpolation of nodal values).
 * `nrm` is the outward unit normal (only for DUDN_SINPROD). */
static double fn_eval(const or_fn *fn, int dim, const double *x, int nv, const double *bary,
                      const int32_t *verts, const double *nrm)
{
    if (!fn) return 0.0;
    switch (fn->kind) {
    case OR_FN_ZERO:
        return 0.0;
    case OR_FN_CONST:
        return fn->c[0];
    case OR_FN_LINEAR: {
        double v = fn->c[0];
        for (int c = 0; c < dim; ++c) v += fn->c[1 + c] * x[c];
        return v;
    }
    case OR_FN_SINPROD: {
        double v = fn->c[0];
        for (int c = 0; c < dim; ++c) v *= sin(OR_PI * x[c]);
        return v;
    }
    case OR_FN_DUDN_SINPROD: {
        /* c0 * grad(prod_c sin(pi x_c)) . n */
        double s = 0.0;
        for (int c = 0; c < dim; ++c) {
            double g = OR_PI * cos(OR_PI * x[c]);
            for (int e = 0; e < dim; ++e)
                if (e != c) g *= sin(OR_PI * x[e]);
            s += g * nrm[c];
        }
        return fn->c[0] * s;
    }
    case OR_FN_NODAL: {
        double v = 0.0;
        for (int a = 0; a < nv; ++a) v += bary[a] * fn->nodal[verts[a]];
        return v;
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------- */
/* sparse(i, j, s, m, n): stable sort by (row, column), then add duplicates.  */
/* ------------------------------------------------------------------------- */

typedef struct {
    const int64_t *ii, *jj;
} or_keys;

static int key_less(const or_keys *k, int64_t p, int64_t q)
{
    if (k->ii[p] != k->ii[q]) return k->ii[p] < k->ii[q];
    return k->jj[p] < k->jj[q];
}

/* top-down merge sort of index array idx[lo, hi) (stable) */
static void merge_sort(const or_keys *k, int64_t *idx, int64_t *tmp, int64_t lo, int64_t hi)
{
    if (hi - lo < 2) return;
    int64_t mid = lo + (hi - lo) / 2;
    merge_sort(k, idx, tmp, lo, mid);
    merge_sort(k, idx, tmp, mid, hi);
    int64_t a = lo, b = mid, o = lo;
    while (a < mid && b < hi) {
        /* take from the right run only when strictly smaller: keeps equal keys in order */
        if (key_less(k, idx[b], idx[a])) tmp[o++] = idx[b++];
        else tmp[o++] = idx[a++];
    }
    while (a < mid) tmp[o++] = idx[a++];
    while (b < hi) tmp[o++] = idx[b++];
    memcpy(idx + lo, tmp + lo, (size_t)(hi - lo) * sizeof(int64_t));
}

/* Compressed-row form of the m x n matrix with triplets (ii[k], jj[k], ss[k]),
 * duplicates added in their input order.  rowptr has m+1 entries; colind/val need
 * room for nz entries.  *nnz receives the number of distinct (row, col) pairs.
 * Entries that add up to zero are kept (the pattern depends on the indices only). */
int oracle_coo_to_csr(int64_t m, int64_t n, int64_t nz, const int64_t *ii, const int64_t *jj,
                      const double *ss, int64_t *rowptr, int64_t *colind, double *val, int64_t *nnz)
{
    if (m < 0 || n < 0 || nz < 0) return OR_EINVAL;
    for (int64_t k = 0; k < nz; ++k)
        if (ii[k] < 0 || ii[k] >= m || jj[k] < 0 || jj[k] >= n) return OR_EINVAL;
    int64_t *idx = malloc((size_t)(nz > 0 ? nz : 1) * sizeof(int64_t));
    int64_t *tmp = malloc((size_t)(nz > 0 ? nz : 1) * sizeof(int64_t));
    if (!idx || !tmp) { free(idx); free(tmp); return OR_EINVAL; }
    for (int64_t k = 0; k < nz; ++k) idx[k] = k;
    or_keys keys = {ii, jj};
    merge_sort(&keys, idx, tmp, 0, nz);
    for (int64_t r = 0; r <= m; ++r) rowptr[r] = 0;
    int64_t out = -1;
    for (int64_t q = 0; q < nz; ++q) {
        int64_t k = idx[q];
        if (out >= 0 && ii[idx[q - 1]] == ii[k] && jj[idx[q - 1]] == jj[k]) {
            val[out] += ss[k];
        } else {
            ++out;
            colind[out] = jj[k];
            val[out] = ss[k];
            rowptr[ii[k] + 1] += 1;
        }
    }
    for (int64_t r = 0; r < m; ++r) rowptr[r + 1] += rowptr[r];
    *nnz = out + 1;
    free(idx);
    free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Local quantities on one simplex (Section 3.1.1).                          */
/* ------------------------------------------------------------------------- */

/* Solve the d x d system M X = R (R has ncol columns, column-major in r[c*d + row])
 * by Gaussian elimination with partial pivoting; M is overwritten. Returns 0, or -1
 * if a pivot is exactly zero. */
static int gauss_solve(int d, double *M /* row-major d x d */, double *r, int ncol)
{
    for (int k = 0; k < d; ++k) {
        int p = k;
        for (int i = k + 1; i < d; ++i)
            if (fabs(M[i * d + k]) > fabs(M[p * d + k])) p = i;
        if (M[p * d + k] == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < d; ++j) {
                double t = M[k * d + j]; M[k * d + j] = M[p * d + j]; M[p * d + j] = t;
            }
            for (int c = 0; c < ncol; ++c) {
                double t = r[c * d + k]; r[c * d + k] = r[c * d + p]; r[c * d + p] = t;
            }
        }
        for (int i = k + 1; i < d; ++i) {
            double l = M[i * d + k] / M[k * d + k];
            for (int j = k; j < d; ++j) M[i * d + j] -= l * M[k * d + j];
            for (int c = 0; c < ncol; ++c) r[c * d + i] -= l * r[c * d + k];
        }
    }
    for (int c = 0; c < ncol; ++c) {
        for (int i = d - 1; i >= 0; --i) {
            double s = r[c * d + i];
            for (int j = i + 1; j < d; ++j) s -= M[i * d + j] * r[c * d + j];
            r[c * d + i] = s / M[i * d + i];
        }
    }
    return 0;
}

/* Determinant of a d x d row-major matrix (d = 2 or 3) by cofactor expansion. */
static double det_small(int d, const double *M)
{
    if (d == 2) return M[0] * M[3] - M[1] * M[2];
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* For the simplex with vertex coordinates p[a*dim + c] (a = 0..dim):
 *   signed measure: det[x_2 - x_1, ..., x_{d+1} - x_1] / d!  (positive for the
 *                   orientation required in Section 1.1),
 *   measure:        |det B| / d!, B rows x_k - x_{d+1}, k = 1..d,
 *   grad[a*dim+c]:  gradient of barycentric coordinate lambda_a, from B X = G with
 *                   G = [I_d | -1] (gradients of the reference barycentrics),
 *   K[a*(d+1)+b]:   measure * grad lambda_a . grad lambda_b.
 * Returns -2 if the signed measure is not positive and finite. */
int oracle_local_stiffness(int dim, const double *p, double *K, double *grad, double *measure,
                           double *signed_measure)
{
    if (dim != 2 && dim != 3) return OR_EUNSUPPORTED;
    const int nv = dim + 1;
    double E[9], B[9], R[12];
    for (int k = 0; k < dim; ++k)
        for (int c = 0; c < dim; ++c) E[k * dim + c] = p[(k + 1) * dim + c] - p[c];
    double fact = (dim == 2) ? 2.0 : 6.0;
    double sgn = det_small(dim, E) / fact;
    if (signed_measure) *signed_measure = sgn;
    if (!(sgn > 0.0) || !isfinite(sgn)) return OR_EMESH;
    for (int k = 0; k < dim; ++k)
        for (int c = 0; c < dim; ++c) B[k * dim + c] = p[k * dim + c] - p[dim * dim + c];
    double area = fabs(det_small(dim, B)) / fact;
    /* right-hand sides: columns of G = [I_d | -1] */
    for (int a = 0; a < nv; ++a)
        for (int c = 0; c < dim; ++c) R[a * dim + c] = (a < dim) ? (a == c ? 1.0 : 0.0) : -1.0;
    if (gauss_solve(dim, B, R, nv) != 0) return OR_EMESH;
    for (int a = 0; a < nv; ++a)
        for (int c = 0; c < dim; ++c) grad[a * dim + c] = R[a * dim + c];
    for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
            double s = 0.0;
            for (int c = 0; c < dim; ++c) s += grad[a * dim + c] * grad[b * dim + c];
            K[a * nv + b] = area * s;
        }
    *measure = area;
    return OR_OK;
}

static void gather_coords(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                          int64_t t, double *p, int32_t *verts)
{
    for (int a = 0; a <= dim; ++a) {
        int32_t v = elem[(int64_t)a * NT + t];
        verts[a] = v;
        for (int c = 0; c < dim; ++c) p[a * dim + c] = node[(int64_t)c * N + v];
    }
}

/* ------------------------------------------------------------------------- */
/* Assembly of A, b and the boundary conditions (Sections 3.1-3.3).           */
/* ------------------------------------------------------------------------- */

/* Inputs: dim (2|3), N, NT, node, elem, bdflag (may be NULL), kappa (may be NULL:
 * all ones), data functions f, g_D, g_N (each may be NULL: zero).
 * Outputs (caller-allocated, nnz_cap >= (dim+1)^2 * NT):
 *   rowptr[N+1], colind[nnz_cap], val[nnz_cap]  CSR of A (duplicates summed)
 *   val_bc[nnz_cap]  A with Dirichlet rows and columns set to the identity
 *   b[N]        lifted right-hand side: free rows f + g_N terms - (A u_D), Dirichlet rows g_D
 *   b_load[N]   load plus Neumann terms before lifting
 *   is_d[N]     1 for Dirichlet nodes
 *   b_scale[N]  sum of |load and Neumann terms| entering b_load[i] (a size for
 *               rounding tolerances)
 *   *nnz        number of stored entries
 */
/* Robin sides (bdflag 3) carry kappa grad(u).n + alpha u = g_R: the side mass term
 * alpha int_F u v joins A and int_F g_R v joins b.  load_rule selects the quadrature
 * of int_t f phi_a (Section 4): OR_LOAD_DEFAULT the rules above, OR_LOAD_CENTROID
 * the one-point rule f(c_t) phi_a(c_t) |t| = f(c_t) |t| / (d+1), OR_LOAD_TRAPEZOID
 * the vertex rule sum_e f(x_e) phi_a(x_e) |t| / (d+1) = f(x_a) |t| / (d+1).
 * oracle_assemble_robin is the default rule; oracle_assemble is also alpha = 0,
 * g_R = 0. */
#define OR_LOAD_DEFAULT 0
#define OR_LOAD_CENTROID 1
#define OR_LOAD_TRAPEZOID 2
int oracle_assemble_rule(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                         const int8_t *bdflag, const double *kappa, const or_fn *f, const or_fn *gD,
                         const or_fn *gN, const or_fn *gR, double alpha_r, int load_rule, int64_t nnz_cap,
                         int64_t *rowptr, int64_t *colind, double *val, double *val_bc, double *b,
                         double *b_load, uint8_t *is_d, double *b_scale, int64_t *nnz);

int oracle_assemble_robin(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                          const int8_t *bdflag, const double *kappa, const or_fn *f, const or_fn *gD,
                          const or_fn *gN, const or_fn *gR, double alpha_r, int64_t nnz_cap,
                          int64_t *rowptr, int64_t *colind, double *val, double *val_bc, double *b,
                          double *b_load, uint8_t *is_d, double *b_scale, int64_t *nnz)
{
    return oracle_assemble_rule(dim, N, NT, node, elem, bdflag, kappa, f, gD, gN, gR, alpha_r, OR_LOAD_DEFAULT,
                                nnz_cap, rowptr, colind, val, val_bc, b, b_load, is_d, b_scale, nnz);
}

int oracle_assemble(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                    const int8_t *bdflag, const double *kappa, const or_fn *f, const or_fn *gD,
                    const or_fn *gN, int64_t nnz_cap, int64_t *rowptr, int64_t *colind, double *val,
                    double *val_bc, double *b, double *b_load, uint8_t *is_d, double *b_scale,
                    int64_t *nnz)
{
    return oracle_assemble_robin(dim, N, NT, node, elem, bdflag, kappa, f, gD, gN, NULL, 0.0, nnz_cap,
                                 rowptr, colind, val, val_bc, b, b_load, is_d, b_scale, nnz);
}

/* Measure of the side opposite local vertex a and its outward unit normal, from the
 * gradient of lambda_a: |t| = |F| h / d with h = 1 / |grad lambda_a|. */
static double side_measure(int dim, double meas, const double *G, int a, double *nrm)
{
    double gn = 0.0;
    for (int c = 0; c < dim; ++c) gn += G[a * dim + c] * G[a * dim + c];
    gn = sqrt(gn);
    for (int c = 0; c < dim; ++c) nrm[c] = -G[a * dim + c] / gn;
    return dim * meas * gn;
}

int oracle_assemble_rule(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                         const int8_t *bdflag, const double *kappa, const or_fn *f, const or_fn *gD,
                         const or_fn *gN, const or_fn *gR, double alpha_r, int load_rule, int64_t nnz_cap,
                         int64_t *rowptr, int64_t *colind, double *val, double *val_bc, double *b,
                         double *b_load, uint8_t *is_d, double *b_scale, int64_t *nnz)
{
    if (dim != 2 && dim != 3) return OR_EUNSUPPORTED;
    const int nv = dim + 1;
    if (N <= 0 || NT < 0 || nnz_cap < (int64_t)nv * nv * NT) return OR_EINVAL;
    if (load_rule != OR_LOAD_DEFAULT && load_rule != OR_LOAD_CENTROID && load_rule != OR_LOAD_TRAPEZOID)
        return OR_EINVAL;
    if (!(alpha_r >= 0.0) || !isfinite(alpha_r)) return OR_EINVAL;
    for (int64_t k = 0; k < (int64_t)nv * NT; ++k)
        if (elem[k] < 0 || elem[k] >= N) return OR_EINVAL;
    int64_t nrobin = 0;
    if (bdflag)
        for (int64_t k = 0; k < (int64_t)nv * NT; ++k) {
            if (bdflag[k] < 0 || bdflag[k] > 3) return OR_EINVAL;
            if (bdflag[k] == 3) ++nrobin;
        }
    if (kappa)
        for (int64_t t = 0; t < NT; ++t)
            if (!(kappa[t] > 0.0) || !isfinite(kappa[t])) return OR_EINVAL;

    const int64_t ns = (int64_t)nv * nv * NT + nrobin * dim * dim;
    int64_t *ii = malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
    int64_t *jj = malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
    double *ss = malloc((size_t)(ns > 0 ? ns : 1) * sizeof(double));
    double *bt = malloc((size_t)(nv * NT > 0 ? nv * NT : 1) * sizeof(double));
    double *area = malloc((size_t)(NT > 0 ? NT : 1) * sizeof(double));
    if (!ii || !jj || !ss || !bt || !area) {
        free(ii); free(jj); free(ss); free(bt); free(area);
        return OR_EINVAL;
    }
    int status = OR_OK;
    double p[12], K[16], G[12], meas, sgn;
    int32_t verts[4];

    /* Stiffness triplets, element by element (Section 3.1.2). */
    int64_t idx = 0;
    for (int64_t t = 0; t < NT && status == OR_OK; ++t) {
        gather_coords(dim, N, NT, node, elem, t, p, verts);
        status = oracle_local_stiffness(dim, p, K, G, &meas, &sgn);
        if (status != OR_OK) break;
        area[t] = meas;
        double kt = kappa ? kappa[t] : 1.0;
        for (int a = 0; a < nv; ++a)
            for (int c = 0; c < nv; ++c) {
                ii[idx] = verts[a];
                jj[idx] = verts[c];
                ss[idx] = kt * K[a * nv + c];
                ++idx;
            }
    }
    if (status != OR_OK) goto done;
    /* Robin side mass matrices alpha |F| (1 + delta_ij) / (d (d+1)) on the side's d
     * vertices, in the stacked side order (sides opposite vertex 1, then 2, ...). */
    for (int a = 0; a < nv && status == OR_OK && nrobin > 0; ++a)
        for (int64_t t = 0; t < NT; ++t) {
            if (bdflag[(int64_t)a * NT + t] != 3) continue;
            gather_coords(dim, N, NT, node, elem, t, p, verts);
            status = oracle_local_stiffness(dim, p, K, G, &meas, &sgn);
            if (status != OR_OK) break;
            double nrm[3];
            const double fmeas = side_measure(dim, meas, G, a, nrm);
            for (int e = 0; e < nv; ++e) {
                if (e == a) continue;
                for (int e2 = 0; e2 < nv; ++e2) {
                    if (e2 == a) continue;
                    ii[idx] = verts[e];
                    jj[idx] = verts[e2];
                    ss[idx] = alpha_r * fmeas * (e == e2 ? 2.0 : 1.0) / (dim * (dim + 1));
                    ++idx;
                }
            }
        }
    if (status != OR_OK) goto done;
    status = oracle_coo_to_csr(N, N, idx, ii, jj, ss, rowptr, colind, val, nnz);
    if (status != OR_OK) goto done;

    /* Load vector (Section 3.2): per-element contributions bt[a*NT + t]. */
    for (int64_t t = 0; t < NT; ++t) {
        gather_coords(dim, N, NT, node, elem, t, p, verts);
        if (load_rule == OR_LOAD_CENTROID) {
            /* one-point rule at the barycentre c_t, where every phi_a is 1/(d+1) */
            double x[3] = {0, 0, 0}, bary[4];
            for (int e = 0; e < nv; ++e) {
                bary[e] = 1.0 / nv;
                for (int c = 0; c < dim; ++c) x[c] += p[e * dim + c] / nv;
            }
            const double fc = fn_eval(f, dim, x, nv, bary, verts, NULL);
            for (int a = 0; a < nv; ++a) bt[a * NT + t] = area[t] * fc / nv;
        } else if (load_rule == OR_LOAD_TRAPEZOID) {
            /* vertex rule: at x_e only phi_e is non-zero (and equal to 1) */
            for (int a = 0; a < nv; ++a) {
                double bary[4];
                for (int e = 0; e < nv; ++e) bary[e] = (e == a) ? 1.0 : 0.0;
                const double fa = fn_eval(f, dim, p + a * dim, nv, bary, verts, NULL);
                bt[a * NT + t] = area[t] * fa / nv;
            }
        } else if (dim == 2) {
            /* mid_a = midpoint of the edge opposite vertex a; three-midpoint rule */
            double mid[3][2], fm[3], bary[3];
            for (int a = 0; a < 3; ++a) {
                int u = (a + 1) % 3, w = (a + 2) % 3;
                for (int c = 0; c < 2; ++c) mid[a][c] = (p[u * 2 + c] + p[w * 2 + c]) / 2;
                for (int e = 0; e < 3; ++e) bary[e] = (e == a) ? 0.0 : 0.5;
                fm[a] = fn_eval(f, 2, mid[a], 3, bary, verts, NULL);
            }
            for (int a = 0; a < 3; ++a) {
                int u = (a + 1) % 3, w = (a + 2) % 3;
                bt[a * NT + t] = area[t] * (fm[u] + fm[w]) / 6;
            }
        } else {
            /* symmetric 4-point rule of degree 2: point k has barycentrics alpha at
             * vertex k and beta elsewhere, weight |t|/4 */
            const double alpha = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
            const double beta = (5.0 - sqrt(5.0)) / 20.0;
            double fq[4];
            for (int k = 0; k < 4; ++k) {
                double x[3] = {0, 0, 0}, bary[4];
                for (int e = 0; e < 4; ++e) {
                    bary[e] = (e == k) ? alpha : beta;
                    for (int c = 0; c < 3; ++c) x[c] += bary[e] * p[e * 3 + c];
                }
                fq[k] = fn_eval(f, 3, x, 4, bary, verts, NULL);
            }
            for (int a = 0; a < 4; ++a) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += fq[k] * ((k == a) ? alpha : beta);
                bt[a * NT + t] = area[t] * s / 4;
            }
        }
    }
    /* accumarray over the stacked list [vertex-1 terms; vertex-2 terms; ...] */
    for (int64_t i = 0; i < N; ++i) { b[i] = 0.0; b_scale[i] = 0.0; is_d[i] = 0; }
    for (int a = 0; a < nv; ++a)
        for (int64_t t = 0; t < NT; ++t) {
            int32_t v = elem[(int64_t)a * NT + t];
            b[v] += bt[a * NT + t];
            b_scale[v] += fabs(bt[a * NT + t]);
        }

    /* Neumann (type 2) and Robin (type 3) sides (Section 3.3): midpoint (2-D) /
     * centroid (3-D) rule for g_N, g_R.  Sides are taken in the stacked order [faces
     * opposite vertex 1; opposite vertex 2; ...]. */
    if (bdflag) {
        for (int a = 0; a < nv; ++a)
            for (int64_t t = 0; t < NT; ++t) {
                const int8_t code = bdflag[(int64_t)a * NT + t];
                if (code != 2 && code != 3) continue;
                gather_coords(dim, N, NT, node, elem, t, p, verts);
                status = oracle_local_stiffness(dim, p, K, G, &meas, &sgn);
                if (status != OR_OK) goto done;
                /* outward unit normal of the face opposite a, and the face measure */
                double nrm[3];
                const double fmeas = side_measure(dim, meas, G, a, nrm);
                double x[3] = {0, 0, 0}, bary[4];
                for (int e = 0; e < nv; ++e) {
                    bary[e] = (e == a) ? 0.0 : 1.0 / dim;
                    for (int c = 0; c < dim; ++c) x[c] += bary[e] * p[e * dim + c];
                }
                double g = fn_eval(code == 2 ? gN : gR, dim, x, nv, bary, verts, nrm);
                double share = fmeas * g / dim;
                for (int e = 0; e < nv; ++e) {
                    if (e == a) continue;
                    b[verts[e]] += share;
                    b_scale[verts[e]] += fabs(share);
                }
            }
        /* Dirichlet nodes: vertices of sides of type 1 */
        for (int a = 0; a < nv; ++a)
            for (int64_t t = 0; t < NT; ++t)
                if (bdflag[(int64_t)a * NT + t] == 1)
                    for (int e = 0; e < nv; ++e)
                        if (e != a) is_d[elem[(int64_t)e * NT + t]] = 1;
    }
    for (int64_t i = 0; i < N; ++i) b_load[i] = b[i];

    /* Lifting: u_D = g_D at Dirichlet nodes, b <- b - A u_D, then b_D = u_D. */
    {
        double *uD = calloc((size_t)N, sizeof(double));
        if (!uD) { status = OR_EINVAL; goto done; }
        for (int64_t i = 0; i < N; ++i)
            if (is_d[i]) {
                double x[3];
                for (int c = 0; c < dim; ++c) x[c] = node[(int64_t)c * N + i];
                double one = 1.0;
                int32_t self = (int32_t)i;
                uD[i] = fn_eval(gD, dim, x, 1, &one, &self, NULL);
            }
        for (int64_t i = 0; i < N; ++i) {
            double s = 0.0;
            for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) s += val[q] * uD[colind[q]];
            if (is_d[i]) b[i] = uD[i];
            else b[i] -= s;
        }
        for (int64_t i = 0; i < N; ++i)
            for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
                int64_t j = colind[q];
                if (is_d[i] || is_d[j]) val_bc[q] = (i == j) ? 1.0 : 0.0;
                else val_bc[q] = val[q];
            }
        free(uD);
    }
done:
    free(ii); free(jj); free(ss); free(bt); free(area);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Solve (equation (directsolve)).                                           */
/* ------------------------------------------------------------------------- */

static void csr_matvec(int64_t N, const int64_t *rowptr, const int64_t *colind, const double *val,
                       const double *x, double *y)
{
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) s += val[q] * x[colind[q]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* Solve A_bc u = b where A_bc has identity rows/columns at Dirichlet nodes
 * (is_d[i] = 1); u holds the Dirichlet values on entry at those nodes.
 * method 0: dense Cholesky of A(free, free) (requires n_free <= 6000);
 * method 1: Jacobi-preconditioned CG from x0 = u, stopping when ||r|| <= rtol ||b||.
 * *iters and *relres report the CG iteration count and final ||b - A u|| / ||b||. */
int oracle_solve(int64_t N, const int64_t *rowptr, const int64_t *colind, const double *val_bc,
                 const double *b, const uint8_t *is_d, double *u, double rtol, int64_t maxit,
                 int method, int64_t *iters, double *relres)
{
    int status = OR_OK;
    *iters = 0;
    if (method == 0) {
        int64_t *fid = malloc((size_t)N * sizeof(int64_t));
        int64_t nf = 0;
        for (int64_t i = 0; i < N; ++i) fid[i] = is_d[i] ? -1 : nf++;
        if (nf > 6000) { free(fid); return OR_EINVAL; }
        double *L = calloc((size_t)(nf * nf + 1), sizeof(double));
        double *y = calloc((size_t)(nf + 1), sizeof(double));
        for (int64_t i = 0; i < N; ++i) {
            if (fid[i] < 0) { u[i] = b[i]; continue; }
            y[fid[i]] = b[i];
            for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
                if (fid[colind[q]] >= 0) L[fid[i] * nf + fid[colind[q]]] += val_bc[q];
        }
        /* Cholesky A = L L^T in place (lower triangle) */
        for (int64_t j = 0; j < nf && status == OR_OK; ++j) {
            double d = L[j * nf + j];
            for (int64_t k = 0; k < j; ++k) d -= L[j * nf + k] * L[j * nf + k];
            if (!(d > 0.0)) { status = OR_EMESH; break; }
            d = sqrt(d);
            L[j * nf + j] = d;
            for (int64_t i = j + 1; i < nf; ++i) {
                double s = L[i * nf + j];
                for (int64_t k = 0; k < j; ++k) s -= L[i * nf + k] * L[j * nf + k];
                L[i * nf + j] = s / d;
            }
        }
        if (status == OR_OK) {
            for (int64_t i = 0; i < nf; ++i) {
                double s = y[i];
                for (int64_t k = 0; k < i; ++k) s -= L[i * nf + k] * y[k];
                y[i] = s / L[i * nf + i];
            }
            for (int64_t i = nf - 1; i >= 0; --i) {
                double s = y[i];
                for (int64_t k = i + 1; k < nf; ++k) s -= L[k * nf + i] * y[k];
                y[i] = s / L[i * nf + i];
            }
            for (int64_t i = 0; i < N; ++i)
                if (fid[i] >= 0) u[i] = y[fid[i]];
        }
        free(fid); free(L); free(y);
    } else {
        double *r = malloc((size_t)N * sizeof(double));
        double *z = malloc((size_t)N * sizeof(double));
        double *pp = malloc((size_t)N * sizeof(double));
        double *q = malloc((size_t)N * sizeof(double));
        double *dg = malloc((size_t)N * sizeof(double));
        for (int64_t i = 0; i < N; ++i) {
            dg[i] = 1.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colind[k] == i) dg[i] = val_bc[k];
        }
        csr_matvec(N, rowptr, colind, val_bc, u, q);
        for (int64_t i = 0; i < N; ++i) { r[i] = b[i] - q[i]; z[i] = r[i] / dg[i]; pp[i] = z[i]; }
        double bn = sqrt(dot(N, b, b));
        if (bn == 0.0) bn = 1.0;
        double rz = dot(N, r, z);
        int64_t it = 0;
        while (sqrt(dot(N, r, r)) > rtol * bn) {
            if (it >= maxit) { status = OR_ENOCONV; break; }
            csr_matvec(N, rowptr, colind, val_bc, pp, q);
            double alpha = rz / dot(N, pp, q);
            for (int64_t i = 0; i < N; ++i) { u[i] += alpha * pp[i]; r[i] -= alpha * q[i]; }
            for (int64_t i = 0; i < N; ++i) z[i] = r[i] / dg[i];
            double rz2 = dot(N, r, z);
            double beta = rz2 / rz;
            rz = rz2;
            for (int64_t i = 0; i < N; ++i) pp[i] = z[i] + beta * pp[i];
            ++it;
        }
        *iters = it;
        free(r); free(z); free(pp); free(q); free(dg);
    }
    /* true residual */
    {
        double *q = malloc((size_t)N * sizeof(double));
        csr_matvec(N, rowptr, colind, val_bc, u, q);
        double rn = 0.0, bn = 0.0;
        for (int64_t i = 0; i < N; ++i) { rn += (b[i] - q[i]) * (b[i] - q[i]); bn += b[i] * b[i]; }
        *relres = sqrt(rn) / (bn > 0 ? sqrt(bn) : 1.0);
        free(q);
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* Adjoint gradient.                                                          */
/* ------------------------------------------------------------------------- */

/* g[t] = -|t| (sum_a lam[v_a] grad lambda_a) . (sum_a u[v_a] grad lambda_a):
 * the derivative of J(kappa) = 1/2 ||u - u_obs||^2 with respect to kappa_t when
 * A(free,free) lam(free) = (u - u_obs)(free) and lam = 0 at Dirichlet nodes,
 * because dA/dkappa_t is the unit-coefficient local stiffness of t. */
int oracle_grad(int dim, int64_t N, int64_t NT, const double *node, const int32_t *elem,
                const double *u, const double *lam, double *g)
{
    if (dim != 2 && dim != 3) return OR_EUNSUPPORTED;
    const int nv = dim + 1;
    double p[12], K[16], G[12], meas, sgn;
    int32_t verts[4];
    for (int64_t t = 0; t < NT; ++t) {
        gather_coords(dim, N, NT, node, elem, t, p, verts);
        int st = oracle_local_stiffness(dim, p, K, G, &meas, &sgn);
        if (st != OR_OK) return st;
        double gu[3] = {0, 0, 0}, gl[3] = {0, 0, 0};
        for (int a = 0; a < nv; ++a)
            for (int c = 0; c < dim; ++c) {
                gu[c] += u[verts[a]] * G[a * dim + c];
                gl[c] += lam[verts[a]] * G[a * dim + c];
            }
        double s = 0.0;
        for (int c = 0; c < dim; ++c) s += gl[c] * gu[c];
        g[t] = -meas * s;
    }
    (void)nv;
    return OR_OK;
}

/* y = A x for a CSR matrix (64-bit indices). */
int oracle_spmv(int64_t N, const int64_t *rowptr, const int64_t *colind, const double *val,
                const double *x, double *y)
{
    csr_matvec(N, rowptr, colind, val, x, y);
    return OR_OK;
}
