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
 * Everything is IEEE double precision, single-threaded, in plain loops, and each
 * quantity is computed from its definition:
 *   - barycentric coordinates lambda_a of a simplex are the affine functions with
 *     lambda_a(x_b) = delta_ab; their gradients come from that (d+1) x (d+1)
 *     linear system (rows [1, x_b]) by Gaussian elimination with partial pivoting,
 *     and |t| = |det| / d! of the same matrix;
 *   - a_ij = sum over the elements t containing i and j of
 *     kappa_t |t| grad(lambda_i) . grad(lambda_j) (Section 3.1), added into a
 *     sorted per-row list of (column, value) entries, elements in ascending order,
 *     so duplicates are summed as `sparse` does (Section 2.2) without forming
 *     triplets; pairs whose sum is zero stay stored;
 *   - load integrals int_t f lambda_a by a quadrature rule given as points in
 *     barycentric coordinates and weights, lambda_a read off the point's
 *     barycentrics (Sections 3.2 and 4): 2-D the three edge midpoints, 3-D the
 *     symmetric four-point rule of degree two (the paper names a 4-point rule but
 *     lists none; the reading used here is recorded in the design notes), and on
 *     request the one-point (centroid) or the vertex (trapezoidal) rule;
 *   - Dirichlet lifting b <- b - A u_D, Neumann and Robin side integrals by the
 *     one-point rule at the side's midpoint (2-D) / centroid (3-D) (Section 3.3);
 *   - solve on the free nodes (equation (directsolve)): dense Cholesky when small,
 *     plain Jacobi-preconditioned CG otherwise;
 *   - adjoint gradient dJ/dkappa_t = -|t| grad(lambda_h) . grad(u_h) on t.
 * The compressed-row conversion of a triplet list (oracle_coo_to_csr, the `sparse`
 * of Section 2.1) is kept as a routine of its own, checked on the paper's example.
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

/* quadrature of the load integrals (Section 4) */
#define OR_LOAD_DEFAULT 0
#define OR_LOAD_CENTROID 1
#define OR_LOAD_TRAPEZOID 2

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
 * if a pivot is exactly zero.  (d <= 4) */
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

/* For the simplex with vertex coordinates p[a*dim + c] (a = 0..dim):
 *   lambda_a(x) = c_a + grad_a . x with lambda_a(x_b) = delta_ab, i.e. the columns
 *   of the inverse of M (row b = [1, x_b]): M [c_a; grad_a] = e_a;
 *   signed measure: det M / d!  (= det[x_2 - x_1, ..., x_{d+1} - x_1] / d!,
 *                   positive for the orientation required in Section 1.1),
 *   measure:        |det M| / d!,
 *   grad[a*dim+c]:  gradient of lambda_a,
 *   K[a*(d+1)+b]:   measure * grad lambda_a . grad lambda_b  (the element's
 *                   unit-coefficient stiffness, int_t grad lambda_a . grad lambda_b).
 * Returns -2 if the signed measure is not positive and finite. */
int oracle_local_stiffness(int dim, const double *p, double *K, double *grad, double *measure,
                           double *signed_measure)
{
    if (dim != 2 && dim != 3) return OR_EUNSUPPORTED;
    const int nv = dim + 1;
    double M[16], X[16];
    for (int b = 0; b < nv; ++b) {
        M[b * nv] = 1.0;
        for (int c = 0; c < dim; ++c) M[b * nv + 1 + c] = p[b * dim + c];
    }
    /* the determinant from the elimination's pivots (with the sign of the row swaps) */
    double det = 1.0;
    {
        double W[16];
        memcpy(W, M, sizeof(double) * (size_t)(nv * nv));
        for (int k = 0; k < nv; ++k) {
            int piv = k;
            for (int i = k + 1; i < nv; ++i)
                if (fabs(W[i * nv + k]) > fabs(W[piv * nv + k])) piv = i;
            if (W[piv * nv + k] == 0.0) { det = 0.0; break; }
            if (piv != k) {
                for (int j = 0; j < nv; ++j) {
                    double t = W[k * nv + j]; W[k * nv + j] = W[piv * nv + j]; W[piv * nv + j] = t;
                }
                det = -det;
            }
            det *= W[k * nv + k];
            for (int i = k + 1; i < nv; ++i) {
                double l = W[i * nv + k] / W[k * nv + k];
                for (int j = k; j < nv; ++j) W[i * nv + j] -= l * W[k * nv + j];
            }
        }
    }
    const double fact = (dim == 2) ? 2.0 : 6.0;
    const double sgn = det / fact;
    if (signed_measure) *signed_measure = sgn;
    if (!(sgn > 0.0) || !isfinite(sgn)) return OR_EMESH;
    /* columns of M^-1: right-hand sides e_a, stored column-major X[a*nv + row] */
    for (int a = 0; a < nv; ++a)
        for (int r = 0; r < nv; ++r) X[a * nv + r] = (a == r) ? 1.0 : 0.0;
    if (gauss_solve(nv, M, X, nv) != 0) return OR_EMESH;
    for (int a = 0; a < nv; ++a)
        for (int c = 0; c < dim; ++c) grad[a * dim + c] = X[a * nv + 1 + c];
    const double area = fabs(det) / fact;
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

/* The rows of A being summed: row i's entries (column, value), sorted by column,
 * in slot [off[i], off[i] + n[i]) of one pool; a row can hold no more than the
 * vertex itself plus d columns per incident element, which sizes its slot. */
typedef struct {
    int64_t *off, *n, *col;
    double *val;
} or_rows;

/* a_ij += v: the entry of column j is found by bisection, or inserted in order. */
static void row_add(or_rows *R, int64_t i, int64_t j, double v)
{
    int64_t *c = R->col + R->off[i];
    double *w = R->val + R->off[i];
    const int64_t n = R->n[i];
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (c[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    if (lo < n && c[lo] == j) {
        w[lo] += v;
        return;
    }
    for (int64_t k = n; k > lo; --k) {
        c[k] = c[k - 1];
        w[k] = w[k - 1];
    }
    c[lo] = j;
    w[lo] = v;
    R->n[i] = n + 1;
}

/* A quadrature rule on a simplex: npt points in barycentric coordinates bary[q][e]
 * and weights w[q] relative to the measure (they sum to 1). */
typedef struct {
    int npt;
    double bary[4][4];
    double w[4];
} or_rule;

/* The load rule of Sections 3.2 and 4 for dimension dim. */
static or_rule load_quadrature(int dim, int load_rule)
{
    or_rule R;
    memset(&R, 0, sizeof(R));
    const int nv = dim + 1;
    if (load_rule == OR_LOAD_CENTROID) {          /* one point: the barycentre */
        R.npt = 1;
        for (int e = 0; e < nv; ++e) R.bary[0][e] = 1.0 / nv;
        R.w[0] = 1.0;
    } else if (load_rule == OR_LOAD_TRAPEZOID) {  /* the vertices, equal weights */
        R.npt = nv;
        for (int q = 0; q < nv; ++q) {
            R.bary[q][q] = 1.0;
            R.w[q] = 1.0 / nv;
        }
    } else if (dim == 2) {                        /* the three edge midpoints */
        R.npt = 3;
        for (int q = 0; q < 3; ++q) {
            for (int e = 0; e < 3; ++e) R.bary[q][e] = (e == q) ? 0.0 : 0.5;
            R.w[q] = 1.0 / 3.0;
        }
    } else {                                      /* (alpha, beta, beta, beta) and permutations */
        const double alpha = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
        const double beta = (5.0 - sqrt(5.0)) / 20.0;
        R.npt = 4;
        for (int q = 0; q < 4; ++q) {
            for (int e = 0; e < 4; ++e) R.bary[q][e] = (e == q) ? alpha : beta;
            R.w[q] = 0.25;
        }
    }
    return R;
}

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

    or_rows rows;
    rows.off = calloc((size_t)N + 1, sizeof(int64_t));
    rows.n = calloc((size_t)N, sizeof(int64_t));
    double *area = malloc((size_t)(NT > 0 ? NT : 1) * sizeof(double));
    rows.col = NULL;
    rows.val = NULL;
    if (rows.off && rows.n && area) {
        /* slot sizes: 1 + d per incidence of the vertex */
        for (int64_t i = 0; i < N; ++i) rows.off[i + 1] = 1;
        for (int64_t k = 0; k < (int64_t)nv * NT; ++k) rows.off[elem[k] + 1] += dim;
        for (int64_t i = 0; i < N; ++i) rows.off[i + 1] += rows.off[i];
        rows.col = malloc((size_t)rows.off[N] * sizeof(int64_t));
        rows.val = malloc((size_t)rows.off[N] * sizeof(double));
    }
    if (!rows.off || !rows.n || !area || !rows.col || !rows.val) {
        free(rows.off); free(rows.n); free(rows.col); free(rows.val); free(area);
        return OR_EINVAL;
    }
    int status = OR_OK;
    double p[12], K[16], G[12], meas, sgn;
    int32_t verts[4];

    /* a_ij = sum_t kappa_t int_t grad lambda_i . grad lambda_j, elements in order. */
    for (int64_t t = 0; t < NT && status == OR_OK; ++t) {
        gather_coords(dim, N, NT, node, elem, t, p, verts);
        status = oracle_local_stiffness(dim, p, K, G, &meas, &sgn);
        if (status != OR_OK) break;
        area[t] = meas;
        double kt = kappa ? kappa[t] : 1.0;
        for (int a = 0; a < nv; ++a)
            for (int c = 0; c < nv; ++c) row_add(&rows, verts[a], verts[c], kt * K[a * nv + c]);
    }
    if (status != OR_OK) goto done;
    /* Robin sides: alpha int_F lambda_i lambda_j = alpha |F| (1 + delta_ij) / (d (d+1))
     * on the side's d vertices (sides opposite vertex 1, then 2, ...). */
    for (int a = 0; a < nv && status == OR_OK && nrobin > 0; ++a)
        for (int64_t t = 0; t < NT && status == OR_OK; ++t) {
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
                    row_add(&rows, verts[e], verts[e2], alpha_r * fmeas * (e == e2 ? 2.0 : 1.0) / (dim * (dim + 1)));
                }
            }
        }
    if (status != OR_OK) goto done;
    /* the rows, in order, are the compressed-row matrix */
    rowptr[0] = 0;
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t q = 0; q < rows.n[i]; ++q) {
            colind[rowptr[i] + q] = rows.col[rows.off[i] + q];
            val[rowptr[i] + q] = rows.val[rows.off[i] + q];
        }
        rowptr[i + 1] = rowptr[i] + rows.n[i];
    }
    *nnz = rowptr[N];

    /* Load vector: b_a += |t| sum_q w_q f(x_q) lambda_a(x_q), with x_q and lambda_a(x_q)
     * from the point's barycentric coordinates (nodal f: its linear interpolant). */
    for (int64_t i = 0; i < N; ++i) { b[i] = 0.0; b_scale[i] = 0.0; is_d[i] = 0; }
    {
        const or_rule R = load_quadrature(dim, load_rule);
        for (int64_t t = 0; t < NT; ++t) {
            gather_coords(dim, N, NT, node, elem, t, p, verts);
            double fq[4];
            for (int q = 0; q < R.npt; ++q) {
                double x[3] = {0, 0, 0};
                for (int e = 0; e < nv; ++e)
                    for (int c = 0; c < dim; ++c) x[c] += R.bary[q][e] * p[e * dim + c];
                fq[q] = fn_eval(f, dim, x, nv, R.bary[q], verts, NULL);
            }
            for (int a = 0; a < nv; ++a) {
                double s = 0.0;
                for (int q = 0; q < R.npt; ++q) s += R.w[q] * fq[q] * R.bary[q][a];
                const double ba = area[t] * s;
                b[verts[a]] += ba;
                b_scale[verts[a]] += fabs(ba);
            }
        }
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
    free(rows.off); free(rows.n); free(rows.col); free(rows.val); free(area);
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
