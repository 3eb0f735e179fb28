/*
 * femhip.h -- C interface of the MI355X (gfx950) library for linear (P1) finite
 * element assembly of the Poisson problem, its solve and its adjoint gradient.
 *
 * The method is the one of L. Chen, "Programming of Finite Element Methods in
 * MATLAB": mesh arrays node/elem/bdFlag (Section 1), a sparse matrix built from
 * element contributions whose duplicate (i, j) entries are added (Sections 2.2 and
 * 3.1), a load vector by quadrature (Section 3.2), Dirichlet and Neumann boundary
 * conditions (Section 3.3) and a solve on the free nodes (equation (directsolve)).
 * The problem solved is -div(kappa grad u) = f with kappa constant on each element;
 * kappa = 1 gives the paper's problem (PoissonEq).
 *
 * Conventions shared by every entry point
 *  - Arrays marked "device" live in GPU memory and are owned by the caller; the
 *    library never allocates or frees device memory.  Host pointers are marked.
 *  - Indices are 0-based int32.  Sizes are int64 but must fit the int32 index
 *    space: n_node, n_elem*(dim+1), and nnz below 2^31 (else FE_EOVERFLOW).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work
 *    is enqueued on it and returns before it finishes, except where a call is
 *    documented as synchronizing.
 *  - Every function returns an fe_status; outputs are unspecified on error.  A
 *    problem found by a kernel (bad element, bad kappa) is recorded in the plan and
 *    reported by fe_plan_status(), which synchronizes.
 *  - A plan must not be used by two streams at the same time.
 */
#ifndef FEMHIP_H
#define FEMHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fe_status {
    FE_OK = 0,
    FE_EINVAL = -1,        /* bad argument: NULL pointer, bad size, index out of range, kappa <= 0 */
    FE_EMESH = -2,         /* element with non-positive or non-finite measure, repeated vertex */
    FE_EUNSUPPORTED = -3,  /* dim not 2 or 3 */
    FE_EOVERFLOW = -4,     /* a count exceeds the int32 index space */
    FE_ESIZE = -5,         /* workspace smaller than the size query returned */
    FE_EHIP = -6,          /* a HIP runtime call failed */
    FE_ENOCONV = -7,       /* the iteration limit was reached before the tolerance */
    FE_ELIMIT = -8         /* a fixed capacity exceeded: see the function */
} fe_status;

/* Boundary side types (Section 1.2).  Side a of an element is opposite local vertex a. */
enum { FE_BD_INTERIOR = 0, FE_BD_DIRICHLET = 1, FE_BD_NEUMANN = 2, FE_BD_ROBIN = 3 };

/* A simplicial mesh (Section 1.1), structure-of-arrays (MATLAB's column-major
 * node(N,d) and elem(NT,d+1)).  Every element must be positively oriented:
 * det[x_2 - x_1, ..., x_{d+1} - x_1] > 0 (counter-clockwise triangles, right-hand
 * rule for tetrahedra). */
typedef struct fe_mesh {
    int32_t dim;            /* 2 (triangles) or 3 (tetrahedra) */
    int64_t n_node;         /* N */
    int64_t n_elem;         /* NT */
    const double *node;     /* device, dim*N:      node[c*N + k] = coordinate c of vertex k */
    const int32_t *elem;    /* device, (dim+1)*NT: elem[a*NT + t] = vertex a of element t */
    const int8_t *bdflag;   /* device, (dim+1)*NT: type of side a of t (0, 1, 2); NULL = all 0 */
} fe_mesh;

/* Data functions: source f, Dirichlet value g_D, Neumann flux g_N = kappa du/dn. */
enum {
    FE_FN_ZERO = 0,          /* 0 */
    FE_FN_CONST = 1,         /* c0 */
    FE_FN_LINEAR = 2,        /* c0 + c1 x + c2 y (+ c3 z) */
    FE_FN_SINPROD = 3,       /* c0 * prod_c sin(pi x_c) */
    FE_FN_DUDN_SINPROD = 4,  /* c0 * grad(prod_c sin(pi x_c)) . n, n the outward unit normal (g_N only) */
    FE_FN_NODAL = 5          /* piecewise-linear interpolant of nodal[0..N-1] (device array) */
};

/* Quadrature of the load integrals int_t f phi_i (Section 4). */
enum {
    FE_LOAD_DEFAULT = 0,    /* 2-D three edge midpoints, 3-D symmetric four-point rule (degree 2) */
    FE_LOAD_CENTROID = 1,   /* one-point rule: |t| f(c_t) / (d+1) to every vertex of t (degree 1) */
    FE_LOAD_TRAPEZOID = 2   /* vertex (trapezoidal) rule: |t| f(x_i) / (d+1) to vertex i (degree 1) */
};

typedef struct fe_fn {
    int32_t kind;
    double c[4];
    const double *nodal;    /* device, N values; used by FE_FN_NODAL only */
} fe_fn;

typedef struct fe_plan fe_plan;   /* opaque, host-side; refers to the caller's workspace */

typedef struct fe_plan_info {
    int32_t dim;
    int64_t n_node, n_elem;
    int64_t nnz;            /* stored entries of A (all pairs of vertices sharing an element) */
    int64_t n_inc;          /* (dim+1)*n_elem vertex-element incidences */
    int32_t max_row;        /* longest row of A */
    int32_t max_deg;        /* most elements around one vertex */
    int64_t n_dirichlet;    /* Dirichlet nodes */
    int32_t sort_runs;      /* 1 if the labels follow the element order (the incidence sort found
                               runs of equal buckets in neighbouring elements): the sort aggregates
                               its counter updates per wavefront and rows are processed in label
                               order; else 0 (a choice of kernels; results do not depend on it) */
    int32_t n_long;         /* rows with more than 32 (2-D) / 64 (3-D) stored entries, which take
                               the long-row kernels (one workgroup per row) */
} fe_plan_info;

/* Library version string (host, static). */
const char *fe_version(void);
/* Human-readable name of a status code (host, static). */
const char *fe_status_string(int status);

/* ---------------------------------------------------------------------------
 * Symbolic phase: everything that depends only on elem and bdflag.
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace a plan for `mesh` needs (host arithmetic only; the
 * node pointer is not read).  The workspace must stay allocated and untouched by
 * the caller until fe_plan_destroy(). */
int fe_plan_workspace_bytes(const fe_mesh *mesh, size_t *bytes);

/* Build the plan for the topology of `mesh` (elem, bdflag; node is not read):
 * vertex-to-element incidence lists in a fixed order, the row pattern of A and
 * the Dirichlet node set (vertices of sides of type 1, Section 3.3).  The stored
 * pattern of A is every pair of vertices that share an element (Section 3.1.2),
 * including pairs whose sum of contributions is zero.  Synchronizes `stream` once
 * and returns nnz in *nnz (host).  The plan keeps pointers to mesh->elem and
 * mesh->bdflag, which must stay valid and unchanged while the plan lives.
 * Errors: FE_EINVAL (NULL, sizes, vertex index out of range, bdflag code not in
 * 0..3), FE_EUNSUPPORTED (dim), FE_EMESH (repeated vertex in an
 * element), FE_EOVERFLOW, FE_ESIZE, FE_EHIP, and FE_ELIMIT when the mesh exceeds
 * a capacity: more than 2^29 vertices in use by elements, or a vertex in more than
 * 4095 (2-D) / 2730 (3-D) elements (a row's candidate columns, dim per incident
 * element plus the vertex itself, must fit 8192 LDS slots). */
int fe_plan_create(const fe_mesh *mesh, void *ws, size_t ws_bytes, fe_plan **plan, int64_t *nnz,
                   void *stream);

/* Write the compressed-row pattern of A: rowptr (device, N+1, rowptr[0] = 0) and
 * colind (device, nnz; columns strictly ascending within each row).  A is
 * structurally symmetric, so these arrays are also its compressed-column pattern. */
int fe_plan_pattern(fe_plan *plan, int32_t *rowptr, int32_t *colind, void *stream);

/* Launch setting of the numeric phase: rows per workgroup of the row kernels of
 * fe_assemble* (64, 128 or 256; 0 = the default, the widest block whose row
 * accumulators fit 32 KB of LDS).  Results do not depend on it (each row is summed
 * by one thread in a fixed order).  Host only; a batch built on this plan recaptures
 * its graph on its next call.  FE_EINVAL for other values. */
int fe_plan_set_launch(fe_plan *plan, int32_t rows_per_block);

/* Fill *info (host). */
int fe_plan_get_info(const fe_plan *plan, fe_plan_info *info);

/* Synchronize `stream` and return the first problem recorded by a kernel of this
 * plan since the last call (FE_EMESH for an element of non-positive or non-finite
 * measure, FE_EINVAL for kappa <= 0 or non-finite), then clear it. */
int fe_plan_status(fe_plan *plan, void *stream);

/* Release the host-side plan object (the workspace is the caller's). */
int fe_plan_destroy(fe_plan *plan);

/* ---------------------------------------------------------------------------
 * Numeric phase (Sections 3.1.3, 3.2, 3.3).
 * ------------------------------------------------------------------------- */

/* Assemble, in the plan's pattern:
 *   val[nnz]     A, a_ij = sum over elements t of kappa_t |t| grad(lambda_i).grad(lambda_j)
 *                with grad(lambda_i) = n_i / (d! |t|) (equation (dlambda)),
 *   b_load[N]    load plus Neumann terms: 2-D three edge-midpoint rule, 3-D symmetric
 *                four-point rule of degree 2 (exact closed form for FE_FN_NODAL);
 *                Neumann sides by the midpoint (2-D) / centroid (3-D) rule,
 *   b[N]         lifted right-hand side: b_load - A u_D on free rows, g_D at Dirichlet rows,
 *   val_bc[nnz]  A with Dirichlet rows and columns replaced by the identity, so that
 *                val_bc u = b is the full-size form of A(free,free) u = b(free),
 *   is_dirichlet[N]  1 at Dirichlet nodes, else 0.
 * node: device coordinates (same layout as fe_mesh.node).  kappa: device, NT values
 * > 0, or NULL for kappa = 1.  f, g_d, g_n: host structs, NULL = zero.  val and b are
 * required; val_bc, b_load and is_dirichlet may be NULL.  Duplicates are added in
 * ascending element order, so results are bitwise reproducible.  Robin sides (bdflag
 * 3) are treated as kappa grad(u).n = 0 here; see fe_assemble_robin. */
int fe_assemble(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                const fe_fn *g_d, const fe_fn *g_n, double *val, double *val_bc, double *b,
                double *b_load, uint8_t *is_dirichlet, void *stream);

/* As fe_assemble, with Robin sides (bdflag 3, Section 1.2) carrying
 * kappa grad(u).n + robin_alpha u = g_r: the side mass term robin_alpha |F| (1 +
 * delta_ij) / (d (d+1)) joins A on the side's vertices (and is lifted like the
 * stiffness at Dirichlet vertices), and g_r enters b_load by the midpoint (2-D) /
 * centroid (3-D) rule, as g_n does.  robin_alpha >= 0 (else FE_EINVAL); g_r may be
 * NULL (zero).  fe_assemble is this call with robin_alpha = 0 and g_r = NULL. */
int fe_assemble_robin(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                      const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r, double robin_alpha,
                      double *val, double *val_bc, double *b, double *b_load,
                      uint8_t *is_dirichlet, void *stream);

/* As fe_assemble_robin, with the load integrals int_t f phi_i taken by load_rule
 * (FE_LOAD_*, Section 4; any other value: FE_EINVAL).  The side terms of g_n and g_r
 * keep their rules.  fe_assemble_robin is this call with FE_LOAD_DEFAULT. */
int fe_assemble_quad(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                     const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r, double robin_alpha,
                     int32_t load_rule, double *val, double *val_bc, double *b, double *b_load,
                     uint8_t *is_dirichlet, void *stream);

/* ---------------------------------------------------------------------------
 * Symmetric storage: the upper triangle of A (Section 3.1.3, the remark on
 * symmetry: the local matrices are symmetric, so the entries j >= i hold A).
 * ------------------------------------------------------------------------- */

/* The pattern of triu(A) (diagonal included) from the pattern of A (rowptr,
 * colind from fe_plan_pattern, device): rowptr_u (device, N+1, 16-byte aligned) and
 * colind_u (device, nnz_u; label order, columns ascending), and vidx (device, nnz):
 * for every entry q of A's pattern, the position in the upper storage of the entry
 * (column >= row) or of its mirror across the diagonal (column < row), so A's value
 * q is val_u[vidx[q]].  Call once with colind_u = vidx = NULL to get *nnz_u (host;
 * rowptr_u is filled), then with both allocated.  Synchronizes.  FE_EINVAL for NULL
 * arguments, a misaligned rowptr_u, only one of colind_u and vidx, or a plan whose
 * pattern was not yet written. */
int fe_plan_upper(fe_plan *plan, const int32_t *rowptr, const int32_t *colind, int32_t *rowptr_u,
                  int32_t *colind_u, int32_t *vidx, int64_t *nnz_u, void *stream);

/* As fe_assemble_quad, with the matrices written in the symmetric storage of
 * fe_plan_upper: val_u[nnz_u] = triu(A), val_bc_u[nnz_u] = triu(A_bc) (nullable).
 * The values are bitwise those of the same entries of fe_assemble_quad's val and
 * val_bc; b, b_load and is_dirichlet are the same arrays.  rowptr_u: device, from
 * fe_plan_upper. */
int fe_assemble_upper(fe_plan *plan, const int32_t *rowptr_u, const double *node, const double *kappa,
                      const fe_fn *f, const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r,
                      double robin_alpha, int32_t load_rule, double *val_u, double *val_bc_u, double *b,
                      double *b_load, uint8_t *is_dirichlet, void *stream);

/* y = A x for A in symmetric storage: A's pattern (rowptr, colind: n rows, device)
 * with the values val_u[vidx[q]] (fe_plan_upper).  Row sums run in column order, as
 * in fe_spmv. */
int fe_spmv_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const int32_t *vidx,
                const double *val_u, const double *x, double *y, void *stream);

/* y = A x for a CSR matrix (device arrays; n rows). */
int fe_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
            const double *x, double *y, void *stream);

/* out[i] = mask[i] ? a[i] : b[i] for i < n (device arrays; a or b NULL reads as 0).
 * With mask = is_dirichlet it forms the start vector of a solve (g_D at Dirichlet
 * rows, 0 elsewhere: a = b from fe_assemble, b = NULL) and the adjoint right-hand
 * side (dJ/du at free rows, 0 at Dirichlet rows: a = NULL, b = dJ/du).  out may
 * alias a or b. */
int fe_select(int64_t n, const uint8_t *mask, const double *a, const double *b, double *out,
              void *stream);

/* ---------------------------------------------------------------------------
 * Solve (replaces the direct solve of equation (directsolve)).
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace fe_solve needs for n unknowns. */
int fe_solve_workspace_bytes(int64_t n, size_t *bytes);

/* Jacobi-preconditioned conjugate gradients for the symmetric positive definite
 * CSR matrix (rowptr, colind, val), typically val_bc from fe_assemble.  u (device,
 * n) holds x0 on entry (with the Dirichlet values at Dirichlet rows) and the
 * solution on return.  Stops when ||b - A u||_2 <= rtol ||b||_2 (recurrence
 * residual) or after maxit iterations (FE_ENOCONV).  Synchronizes; *iters and
 * *relres (host) receive the iteration count and the final recurrence ratio.
 * Dot products use a fixed reduction order, so results are bitwise reproducible. */
int fe_solve(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
             const double *b, double *u, double rtol, int32_t maxit, void *ws, size_t ws_bytes,
             int32_t *iters, double *relres, void *stream);

/* fe_solve for A_bc in symmetric storage (val_u = val_bc_u of fe_assemble_upper;
 * rowptr, colind, vidx as for fe_spmv_sym).  Arguments, workspace, stopping rule,
 * synchronization and errors as for fe_solve. */
int fe_solve_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const int32_t *vidx,
                 const double *val_u, const double *b, double *u, double rtol, int32_t maxit, void *ws,
                 size_t ws_bytes, int32_t *iters, double *relres, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): fe_solve without a workspace
 * argument.  Its workspace is a fixed 64 MiB device array inside the library, one
 * per GPU, held until the process ends; its device address is looked up on the
 * first call on each device.  The call allocates nothing (no hipMalloc, no
 * allocating library routine).  Arguments, stopping rule, results (bit for bit),
 * synchronization and errors are those of fe_solve, plus FE_ELIMIT for n above
 * FE_SOLVE_NOALLOC_MAX_N.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams or two host threads) race and must
 * be serialized by the caller. */
#define FE_SOLVE_NOALLOC_MAX_N 1310720
int fe_solve_noalloc(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                     const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                     double *relres, void *stream);

/* ---------------------------------------------------------------------------
 * Pure Neumann problem (Section 3.3, equations (compatible) and (meanb)).
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace fe_neumann_solve needs for this plan and nnz stored
 * entries. */
int fe_neumann_workspace_bytes(const fe_plan *plan, int64_t nnz, size_t *bytes);

/* Solve A u = b when every boundary side is Neumann (the plan has no Dirichlet
 * vertex, else FE_EINVAL).  val, b: from fe_assemble (A, not A_bc).  The method's
 * steps: b' = b - mean(b) (the discrete compatibility condition); u = 0 at vertex
 * 0 and Jacobi-PCG on the other rows (A with row and column 0 replaced by the
 * identity, b'_0 = 0); then u <- u - c with c = sum_t |t| mean(u(elem_t)) / sum_t
 * |t|, so u has zero mean.  u (device, N) is output only.  *iters and *relres as for
 * fe_solve (relative to ||b'||), *mean_b receives mean(b) (may be NULL).  node:
 * device coordinates; ws: 256-byte aligned, at least the queried size.
 * Synchronizes.  FE_ENOCONV if maxit was reached (u is still shifted). */
int fe_neumann_solve(fe_plan *plan, const double *node, const int32_t *rowptr,
                     const int32_t *colind, const double *val, const double *b, double *u,
                     double rtol, int32_t maxit, void *ws, size_t ws_bytes, int32_t *iters,
                     double *relres, double *mean_b, void *stream);

/* ---------------------------------------------------------------------------
 * Adjoint gradient.
 * ------------------------------------------------------------------------- */

/* g[t] = -|t| grad(lam_h) . grad(u_h) on every element t (device arrays: u, lam of
 * length N, g of length NT).  With A(free,free) lam(free) = dJ/du(free) and lam = 0
 * at Dirichlet nodes this is dJ/dkappa_t, since dA/dkappa_t is the unit-coefficient
 * local stiffness of t (Section 3.1). */
int fe_grad(fe_plan *plan, const double *node, const double *u, const double *lam, double *g,
            void *stream);

/* ---------------------------------------------------------------------------
 * Batches of independent problems (many meshes, one launch).
 *
 * A batch is the disjoint union of its instances: the caller concatenates the
 * instances' node arrays (vertex labels of instance k offset by off[k]) and element
 * arrays (labels offset accordingly), and builds one plan for the union.  The
 * union's A_bc is block diagonal, one block per instance, so one fe_assemble call
 * assembles every instance at once (each instance's rows bitwise equal to those of
 * its own plan).  The batched solve runs Jacobi-PCG on every block with its own
 * scalars and stopping test in one persistent kernel; each instance's iterates are
 * bitwise equal to fe_solve on that block alone.  At most 4096 instances.
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace for n rows in n_inst instances (FE_ELIMIT above 4096). */
int fe_batch_solve_workspace_bytes(int64_t n, int32_t n_inst, size_t *bytes);

/* Solve every diagonal block of the CSR matrix (rowptr, colind, val) (device, n =
 * inst_row_off[n_inst] rows).  inst_row_off: host, n_inst + 1 nondecreasing row
 * offsets starting at 0; block k is rows [inst_row_off[k], inst_row_off[k+1]) and
 * must not couple to other rows.  u: x0 on entry, solutions on return.  Instance k
 * stops when its recurrence residual drops to rtol times ||b_k||_2, or after maxit
 * iterations.  blocks_per_cu: workgroups per compute unit of the persistent grid
 * (0 picks a default; above what fits, or above 4, the most verified co-resident on
 * MI355X, FE_EINVAL); units_per_step: 256-row units
 * each workgroup processes together (1, 2 or 4; 0 picks a default).  Neither
 * changes any result bit.  iters, relres: host arrays of
 * n_inst (may be NULL).  ws: 256-byte aligned device workspace of at least the
 * queried size.  Synchronizes.  Returns FE_ENOCONV if an instance hit maxit,
 * FE_EINVAL for a non-positive diagonal entry, FE_ELIMIT if the device-wide wait
 * timed out (the grid was not co-resident). */
int fe_batch_solve(int32_t n_inst, const int64_t *inst_row_off, const int32_t *rowptr,
                   const int32_t *colind, const double *val, const double *b, double *u,
                   double rtol, int32_t maxit, int32_t blocks_per_cu, int32_t units_per_step,
                   void *ws, size_t ws_bytes, int32_t *iters, double *relres, void *stream);

typedef struct fe_batch fe_batch;   /* opaque; refers to the caller's plan and workspace */

typedef struct fe_batch_info {
    int32_t n_inst, n_units;        /* instances; 256-row reduction units over all of them */
    int64_t n_rows;
    int32_t grid;                   /* workgroups of the persistent solve kernel */
    int32_t blocks_per_cu;
    int32_t max_blocks_per_cu;      /* most workgroups per compute unit at this units_per_step */
    int32_t units_per_step;
    int32_t cooperative;            /* 1 if the captured solve node is a cooperative launch (read
                                       back from the graph node), 0 if not */
    int32_t captures;               /* graph captures so far */
} fe_batch_info;

/* Batched assemble + solve replayed from one captured hipGraph.  plan: a plan of the
 * union mesh with its pattern built (fe_plan_pattern); inst_node_off: host, n_inst
 * + 1 vertex offsets with inst_node_off[n_inst] = N.  ws: as for fe_batch_solve
 * with n = N.  The plan and ws stay owned by the caller and must outlive the batch.
 * Synchronizes (uploads the instance table). */
int fe_batch_create(fe_plan *plan, int32_t n_inst, const int64_t *inst_node_off,
                    int32_t blocks_per_cu, int32_t units_per_step, void *ws, size_t ws_bytes,
                    fe_batch **batch, void *stream);

/* Change the persistent grid (as for fe_batch_solve, 0 = default); the next
 * fe_batch_assemble_solve captures a new graph. */
int fe_batch_set_grid(fe_batch *batch, int32_t blocks_per_cu, int32_t units_per_step);

int fe_batch_get_info(const fe_batch *batch, fe_batch_info *info);

/* Assemble the union (as fe_assemble with b_load = NULL), set the start vector u =
 * g_D at Dirichlet rows and 0 elsewhere (as fe_select), and solve every instance
 * (as fe_batch_solve on val_bc, b), all as one graph launch.  The graph is captured
 * on the first call and again whenever a pointer, function or scalar argument
 * differs from the previous call; otherwise it is replayed.  u (device, N): the
 * solutions on return.  iters, relres: host, n_inst each (may be NULL).
 * Synchronizes; also reports fe_plan_status. */
int fe_batch_assemble_solve(fe_batch *batch, const double *node, const double *kappa,
                            const fe_fn *f, const fe_fn *g_d, const fe_fn *g_n,
                            const int32_t *rowptr, const int32_t *colind, double *val,
                            double *val_bc, double *b, double *u, double rtol, int32_t maxit,
                            int32_t *iters, double *relres, void *stream);

int fe_batch_destroy(fe_batch *batch);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support).
 * ------------------------------------------------------------------------- */

typedef struct fe_prof_entry {
    char name[40];                  /* kernel name */
    int64_t launches;
    double total_ms, min_ms, max_ms;  /* per launch, from HIP events on the launch stream */
} fe_prof_entry;

/* Enable (on != 0) or disable timing and drop the records kept so far (disabling
 * also destroys the timer's HIP events, so none outlives its use).  While
 * enabled, each launch of the library's kernels is bracketed by two HIP events
 * recorded on its stream (launches into a capturing stream are skipped).  Process
 * wide; do not call it while another thread launches library work. */
int fe_prof_enable(int on);

/* Synchronize the recorded events, aggregate them by kernel name into out[0..cap)
 * (*count receives the number of distinct kernels, which may exceed cap), and drop
 * the records. */
int fe_prof_read(fe_prof_entry *out, int32_t cap, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif /* FEMHIP_H */
