// solve.hip -- CSR SpMV and Jacobi-preconditioned conjugate gradients (FP64).
//
// Stands in for the direct solve A(free,free) \ b(free) of equation (directsolve):
// with the Dirichlet rows and columns of A replaced by the identity and b = g_D
// there, A_bc u = b is the same system at full size and is symmetric positive
// definite, so CG applies.
//
// One CG iteration is two row kernels, each followed by a one-block kernel that
// adds its partial sums:
//   K_A: p = z + beta p_old (row i), q = A p computed as A (z + beta p_old) on the
//        fly (so no grid-wide barrier is needed between the two), partial p.q
//   K_A': alpha = r.z / p.q
//   K_B: x += alpha p, r -= alpha q, z = r / diag(A), partials r.z and r.r
//   K_B': beta, the stopping test, the iteration count
// Partials are added in index order, so every reduction has a fixed order and
// results are bitwise repeatable.  The kernel boundaries make every block's
// partial visible to the summing kernel; no device-scope fence or atomic runs
// inside the row kernels (one per workgroup would serialize on the L2s).
// Scalars live in device memory; the host launches iterations in chunks and reads
// the "done" flag once per chunk, kernels after convergence return at once.
#include <mutex>

#include "cg_common.h"

namespace {

constexpr int SB = CG_UNIT;   // threads per block, one row per thread

enum { S_RZ = 0, S_RR, S_BB, S_ALPHA, S_BETA, S_TOL2, S_PQ, S_RZ_ODD, S_NSCAL = 8 };

// r.z of iteration j (fused form): even j in S_RZ, odd j in S_RZ_ODD, so a kernel
// can read r.z of the previous iteration while its block 0 stores the current one.
FE_DEV int rz_slot(int32_t j) { return (j & 1) ? S_RZ_ODD : S_RZ; }

// Systems of at most FUSE_NB blocks use the fused form: each row kernel first adds
// the partial sums of the previous row kernel itself (every block, the same fixed
// order, so every block gets the same bits), which halves the launches per
// iteration.  Larger systems run the separate one-block summing kernels.
constexpr int32_t FUSE_NB = 1024;
enum { F_DONE = 0, F_ITER, F_BAD, F_NFLAG = 8 };

struct SolveWs {
    double *r, *z, *p0, *p1, *q, *dinv;
    double *part;      // 3 * nblocks
    double *scal;      // S_NSCAL
    int32_t *flag;     // F_NFLAG
};

size_t ws_layout(int64_t n, SolveWs *w, char *base)
{
    const int64_t nb = cdiv(n > 0 ? n : 1, SB);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return base ? base + at : nullptr;
    };
    char *r = take(sizeof(double) * n), *z = take(sizeof(double) * n), *p0 = take(sizeof(double) * n),
         *p1 = take(sizeof(double) * n), *q = take(sizeof(double) * n), *d = take(sizeof(double) * n),
         *part = take(sizeof(double) * 3 * nb), *scal = take(sizeof(double) * S_NSCAL),
         *flag = take(sizeof(int32_t) * F_NFLAG);
    if (w) {
        w->r = (double *)r; w->z = (double *)z; w->p0 = (double *)p0; w->p1 = (double *)p1;
        w->q = (double *)q; w->dinv = (double *)d; w->part = (double *)part; w->scal = (double *)scal;
        w->flag = (int32_t *)flag;
    }
    return o;
}

template <bool IND>
__global__ __launch_bounds__(SB) void k_spmv(int32_t n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ colind, const double *__restrict__ val,
                                             const double *__restrict__ x, double *__restrict__ y,
                                             const int32_t *__restrict__ vidx)
{
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    if (i >= n) return;
    // the row in chunks of 8 entries: all of a chunk's column indices and values,
    // then all its gathers of x, then the products in column order (the same sum
    // whatever the chunk size)
    constexpr int CH = 8;
    const int32_t e = rowptr[i + 1];
    double s = 0.0;
    for (int32_t q0 = rowptr[i]; q0 < e; q0 += CH) {
        int32_t c[CH];
        double v[CH], xv[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t)
            if (q0 + t < e) {
                c[t] = colind[q0 + t];
                v[t] = cg_value<IND>(val, vidx, q0 + t);
            }
#pragma unroll
        for (int t = 0; t < CH; ++t)
            if (q0 + t < e) xv[t] = x[c[t]];
#pragma unroll
        for (int t = 0; t < CH; ++t)
            if (q0 + t < e) s += v[t] * xv[t];
    }
    y[i] = s;
}

// diag(A)^-1, r = b - A x, z = r * dinv, p_old = 0; partials r.z, r.r, b.b.
// IND: values through vidx (symmetric upper-triangle storage), here and below.
template <bool IND>
__global__ __launch_bounds__(SB) void k_cg_init(int32_t n, const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ colind, const double *__restrict__ val,
                                                const double *__restrict__ b, const double *__restrict__ x,
                                                double *r, double *z, double *p0, double *dinv, double *part,
                                                int32_t *flag, const int32_t *__restrict__ vidx)
{
    __shared__ double lds[SB / 64];
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (i < n) {
        double ri, d;
        cg_init_row<IND>(i, rowptr, colind, val, b, x, &ri, &d, vidx);
        if (!(d > 0.0)) atomicOr(flag + F_BAD, 1);
        const double di = 1.0 / d;
        dinv[i] = di;
        r[i] = ri;
        z[i] = ri * di;
        p0[i] = 0.0;
        rz = ri * ri * di;
        rr = ri * ri;
        bb = b[i] * b[i];
    }
    const int32_t nb = gridDim.x;
    double s0 = block_sum<SB>(rz, lds);
    double s1 = block_sum<SB>(rr, lds);
    double s2 = block_sum<SB>(bb, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nb + blockIdx.x] = s1;
        part[2 * nb + blockIdx.x] = s2;
    }
}

// One block: r.z, r.r, b.b from the partials; tolerance and initial stopping test.
__global__ __launch_bounds__(SB) void k_cg_init_sum(int32_t nb, const double *part, double *scal, int32_t *flag,
                                                    double rtol)
{
    __shared__ double lds[SB / 64];
    const double RZ = cg_sum_partials(part, nb, lds);
    const double RR = cg_sum_partials(part + nb, nb, lds);
    const double BB = cg_sum_partials(part + 2 * nb, nb, lds);
    if (threadIdx.x == 0) {
        const double bn2 = BB > 0.0 ? BB : 1.0;
        scal[S_RZ] = RZ;
        scal[S_RR] = RR;
        scal[S_BB] = bn2;
        scal[S_TOL2] = rtol * rtol * bn2;
        scal[S_BETA] = 0.0;
        scal[S_ALPHA] = 0.0;
        flag[F_ITER] = 0;
        flag[F_DONE] = (RR <= rtol * rtol * bn2) ? 1 : 0;
    }
}

// p = z + beta p_old; q = A p (as A z + beta A p_old); partial p.q.
template <bool IND>
__global__ __launch_bounds__(SB) void k_cg_a(int32_t n, const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ colind, const double *__restrict__ val,
                                             const double *__restrict__ z, const double *__restrict__ pold,
                                             double *__restrict__ pnew, double *__restrict__ qv, double *part,
                                             const double *scal, const int32_t *flag,
                                             const int32_t *__restrict__ vidx)
{
    __shared__ double lds[SB / 64];
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const double beta = scal[S_BETA];
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    double pq = 0.0;
    if (i < n) {
        const bool ok = true;
        double s;
        cg_apply_rows<1, 8, IND>(&i, &ok, rowptr, colind, val, z, pold, &beta, &s, vidx);
        const double pi = z[i] + beta * pold[i];
        pnew[i] = pi;
        qv[i] = s;
        pq = pi * s;
    }
    const double bs = block_sum<SB>(pq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// One block: alpha = r.z / p.q.
__global__ __launch_bounds__(SB) void k_cg_a_sum(int32_t nb, const double *part, double *scal, const int32_t *flag)
{
    __shared__ double lds[SB / 64];
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const double PQ = cg_sum_partials(part, nb, lds);
    if (threadIdx.x == 0) {
        scal[S_PQ] = PQ;
        scal[S_ALPHA] = scal[S_RZ] / PQ;
    }
}

// x += alpha p; r -= alpha q; z = r dinv; partials r.z, r.r.
__global__ __launch_bounds__(SB) void k_cg_b(int32_t n, double *__restrict__ x, const double *__restrict__ p,
                                             const double *__restrict__ qv, double *__restrict__ r,
                                             double *__restrict__ z, const double *__restrict__ dinv, double *part,
                                             const double *scal, const int32_t *flag)
{
    __shared__ double lds[SB / 64];
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const double alpha = scal[S_ALPHA];
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * qv[i];
        const double zi = ri * dinv[i];
        r[i] = ri;
        z[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    const int32_t nb = gridDim.x;
    const double s0 = block_sum<SB>(rz, lds);
    const double s1 = block_sum<SB>(rr, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nb + blockIdx.x] = s1;
    }
}

// One block: beta = r.z_new / r.z_old, the stopping test and the iteration count.
__global__ __launch_bounds__(SB) void k_cg_b_sum(int32_t nb, const double *part, double *scal, int32_t *flag)
{
    __shared__ double lds[SB / 64];
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const double RZ = cg_sum_partials(part, nb, lds);
    const double RR = cg_sum_partials(part + nb, nb, lds);
    if (threadIdx.x == 0) {
        scal[S_BETA] = RZ / scal[S_RZ];
        scal[S_RZ] = RZ;
        scal[S_RR] = RR;
        flag[F_ITER] += 1;
        if (RR <= scal[S_TOL2]) flag[F_DONE] = 1;
    }
}

// Fused K_A of iteration it: r.z and r.r of the previous K_B from its partials,
// beta and the stopping test (recorded by block 0), then p = z + beta p_old,
// q = A p and the partial p.q.  check_only: record the stopping test and stop.
template <bool IND>
__global__ __launch_bounds__(SB) void k_cg_a_fused(int32_t n, int32_t it, int32_t check_only,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind, const double *__restrict__ val,
                                                   const double *__restrict__ z, const double *__restrict__ pold,
                                                   double *__restrict__ pnew, double *__restrict__ qv, double *part,
                                                   double *scal, int32_t *flag, const int32_t *__restrict__ vidx)
{
    __shared__ double lds[SB / 64];
    __shared__ double bc[2];
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const int32_t nb = gridDim.x;
    double beta = 0.0;
    bool done = false;
    if (it > 0) {
        const double RZ = cg_sum_partials(part + nb, nb, lds);
        const double RR = cg_sum_partials(part + 2 * nb, nb, lds);
        if (threadIdx.x == 0) {
            bc[0] = RZ;
            bc[1] = RR;
        }
        __syncthreads();
        const double rz = bc[0], rr = bc[1];
        beta = rz / scal[rz_slot(it - 1)];
        done = rr <= scal[S_TOL2];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[rz_slot(it)] = rz;
            scal[S_RR] = rr;
            scal[S_BETA] = beta;
            if (done) {
                flag[F_DONE] = 1;
                flag[F_ITER] = it;
            }
        }
    }
    if (done || check_only) return;
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    double pq = 0.0;
    if (i < n) {
        const bool ok = true;
        double sv;
        cg_apply_rows<1, 8, IND>(&i, &ok, rowptr, colind, val, z, pold, &beta, &sv, vidx);
        const double pi = z[i] + beta * pold[i];
        pnew[i] = pi;
        qv[i] = sv;
        pq = pi * sv;
    }
    const double bs = block_sum<SB>(pq, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// Fused K_B of iteration it: alpha = r.z / p.q from the partials of K_A, then
// x += alpha p, r -= alpha q, z = r / diag and the partials r.z, r.r.
__global__ __launch_bounds__(SB) void k_cg_b_fused(int32_t n, int32_t it, double *__restrict__ x,
                                                   const double *__restrict__ p, const double *__restrict__ qv,
                                                   double *__restrict__ r, double *__restrict__ z,
                                                   const double *__restrict__ dinv, double *part, double *scal,
                                                   int32_t *flag)
{
    __shared__ double lds[SB / 64];
    __shared__ double bc;
    if (*(volatile const int32_t *)(flag + F_DONE)) return;
    const int32_t nb = gridDim.x;
    const double PQ = cg_sum_partials(part, nb, lds);
    if (threadIdx.x == 0) bc = PQ;
    __syncthreads();
    const double alpha = scal[rz_slot(it)] / bc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_PQ] = bc;
        scal[S_ALPHA] = alpha;
        flag[F_ITER] = it + 1;
    }
    const int32_t i = blockIdx.x * SB + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * qv[i];
        const double zi = ri * dinv[i];
        r[i] = ri;
        z[i] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    const double s0 = block_sum<SB>(rz, lds);
    const double s1 = block_sum<SB>(rr, lds);
    if (threadIdx.x == 0) {
        part[nb + blockIdx.x] = s0;
        part[2 * nb + blockIdx.x] = s1;
    }
}

}  // namespace

extern "C" int fe_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, const double *x,
                       double *y, void *stream)
{
    if (n < 0 || n >= INT32_MAX) return FE_EINVAL;
    if (n == 0) return FE_OK;
    if (!rowptr || !colind || !val || !x || !y) return FE_EINVAL;
    FE_TIMED("k_spmv", static_cast<hipStream_t>(stream),
             hipLaunchKernelGGL(k_spmv<false>, dim3((unsigned)cdiv(n, SB)), dim3(SB), 0,
                                static_cast<hipStream_t>(stream), (int32_t)n, rowptr, colind, val, x, y, nullptr));
    return fe_launch_check();
}

extern "C" int fe_spmv_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const int32_t *vidx,
                           const double *val_u, const double *x, double *y, void *stream)
{
    if (n < 0 || n >= INT32_MAX) return FE_EINVAL;
    if (n == 0) return FE_OK;
    if (!rowptr || !colind || !vidx || !val_u || !x || !y) return FE_EINVAL;
    FE_TIMED("k_spmv_sym", static_cast<hipStream_t>(stream),
             hipLaunchKernelGGL(k_spmv<true>, dim3((unsigned)cdiv(n, SB)), dim3(SB), 0,
                                static_cast<hipStream_t>(stream), (int32_t)n, rowptr, colind, val_u, x, y, vidx));
    return fe_launch_check();
}

extern "C" int fe_solve_workspace_bytes(int64_t n, size_t *bytes)
{
    if (n < 0 || n >= INT32_MAX || !bytes) return FE_EINVAL;
    *bytes = ws_layout(n, nullptr, nullptr);
    return FE_OK;
}

// The iteration itself, on a workspace already laid out by ws_layout.
template <bool IND>
static int solve_run(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, const double *b,
                     double *u, double rtol, int32_t maxit, const SolveWs &W, int32_t *iters, double *relres,
                     hipStream_t s, const int32_t *vidx)
{
    const int32_t nn = (int32_t)n;
    const unsigned nb = (unsigned)cdiv(n, SB);
    int rc;
    if ((rc = fe_fill_i32(W.flag, F_NFLAG, 0, s))) return rc;
    FE_TIMED("k_cg_init", s,
             hipLaunchKernelGGL(k_cg_init<IND>, dim3(nb), dim3(SB), 0, s, nn, rowptr, colind, val, b,
                                (const double *)u, W.r, W.z, W.p0, W.dinv, W.part, W.flag, vidx));
    FE_TIMED("k_cg_init_sum", s,
             hipLaunchKernelGGL(k_cg_init_sum, dim3(1), dim3(SB), 0, s, (int32_t)nb, (const double *)W.part, W.scal,
                                W.flag, rtol));
    if ((rc = fe_launch_check())) return rc;
    int32_t fl[F_NFLAG];
    double sc[S_NSCAL];
    int32_t launched = 0;
    int parity = 0;
    const int CHUNK = 32;
    const bool fused = nb <= (unsigned)FUSE_NB;
    for (;;) {
        FE_HIP_CHECK(hipMemcpyAsync(fl, W.flag, sizeof(fl), hipMemcpyDeviceToHost, s));
        FE_HIP_CHECK(hipStreamSynchronize(s));
        if (fl[F_BAD]) return FE_EINVAL;          // non-positive diagonal: not SPD
        if (fl[F_DONE] || launched >= maxit) break;
        const int32_t chunk = (maxit - launched < CHUNK) ? (maxit - launched) : CHUNK;
        for (int32_t c = 0; c < chunk; ++c) {
            double *pold = parity ? W.p1 : W.p0;
            double *pnew = parity ? W.p0 : W.p1;
            if (fused) {
                const int32_t it = launched + c;
                FE_TIMED("k_cg_a_fused", s,
                         hipLaunchKernelGGL(k_cg_a_fused<IND>, dim3(nb), dim3(SB), 0, s, nn, it, 0, rowptr, colind, val,
                                            (const double *)W.z, (const double *)pold, pnew, W.q, W.part, W.scal,
                                            W.flag, vidx));
                FE_TIMED("k_cg_b_fused", s,
                         hipLaunchKernelGGL(k_cg_b_fused, dim3(nb), dim3(SB), 0, s, nn, it, u, (const double *)pnew,
                                            (const double *)W.q, W.r, W.z, (const double *)W.dinv, W.part, W.scal,
                                            W.flag));
            } else {
                FE_TIMED("k_cg_a", s,
                         hipLaunchKernelGGL(k_cg_a<IND>, dim3(nb), dim3(SB), 0, s, nn, rowptr, colind, val,
                                            (const double *)W.z, (const double *)pold, pnew, W.q, W.part,
                                            (const double *)W.scal, (const int32_t *)W.flag, vidx));
                FE_TIMED("k_cg_a_sum", s,
                         hipLaunchKernelGGL(k_cg_a_sum, dim3(1), dim3(SB), 0, s, (int32_t)nb, (const double *)W.part,
                                            W.scal, (const int32_t *)W.flag));
                FE_TIMED("k_cg_b", s,
                         hipLaunchKernelGGL(k_cg_b, dim3(nb), dim3(SB), 0, s, nn, u, (const double *)pnew,
                                            (const double *)W.q, W.r, W.z, (const double *)W.dinv, W.part,
                                            (const double *)W.scal, (const int32_t *)W.flag));
                FE_TIMED("k_cg_b_sum", s,
                         hipLaunchKernelGGL(k_cg_b_sum, dim3(1), dim3(SB), 0, s, (int32_t)nb, (const double *)W.part,
                                            W.scal, W.flag));
            }
            parity ^= 1;
        }
        if ((rc = fe_launch_check())) return rc;
        launched += chunk;
        if (fused && launched >= maxit) {
            // the stopping test after the last iteration (no further work)
            FE_TIMED("k_cg_a_fused", s,
                     hipLaunchKernelGGL(k_cg_a_fused<IND>, dim3(nb), dim3(SB), 0, s, nn, launched, 1, rowptr, colind,
                                        val, (const double *)W.z, (const double *)W.p0, W.p1, W.q, W.part, W.scal,
                                        W.flag, vidx));
            if ((rc = fe_launch_check())) return rc;
        }
    }
    FE_HIP_CHECK(hipMemcpyAsync(sc, W.scal, sizeof(sc), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    *iters = fl[F_ITER];
    *relres = sqrt(sc[S_RR] / sc[S_BB]);
    return fl[F_DONE] ? FE_OK : FE_ENOCONV;
}

static bool solve_args_ok(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                          const double *b, double *u, double rtol, int32_t maxit, int32_t *iters, double *relres)
{
    if (n <= 0 || n >= INT32_MAX || maxit < 0 || !(rtol >= 0.0)) return false;
    return rowptr && colind && val && b && u && iters && relres;
}

extern "C" int fe_solve(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val, const double *b,
                        double *u, double rtol, int32_t maxit, void *ws, size_t ws_bytes, int32_t *iters,
                        double *relres, void *stream)
{
    if (!solve_args_ok(n, rowptr, colind, val, b, u, rtol, maxit, iters, relres) || !ws) return FE_EINVAL;
    if ((uintptr_t)ws & 255) return FE_EINVAL;
    SolveWs W;
    const size_t need = ws_layout(n, &W, static_cast<char *>(ws));
    if (ws_bytes < need) return FE_ESIZE;
    return solve_run<false>(n, rowptr, colind, val, b, u, rtol, maxit, W, iters, relres,
                            static_cast<hipStream_t>(stream), nullptr);
}

extern "C" int fe_solve_sym(int64_t n, const int32_t *rowptr, const int32_t *colind, const int32_t *vidx,
                            const double *val_u, const double *b, double *u, double rtol, int32_t maxit, void *ws,
                            size_t ws_bytes, int32_t *iters, double *relres, void *stream)
{
    if (!solve_args_ok(n, rowptr, colind, val_u, b, u, rtol, maxit, iters, relres) || !vidx || !ws) return FE_EINVAL;
    if ((uintptr_t)ws & 255) return FE_EINVAL;
    SolveWs W;
    const size_t need = ws_layout(n, &W, static_cast<char *>(ws));
    if (ws_bytes < need) return FE_ESIZE;
    return solve_run<true>(n, rowptr, colind, val_u, b, u, rtol, maxit, W, iters, relres,
                           static_cast<hipStream_t>(stream), vidx);
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a fixed device array of this file.
//
// The array's name is only a host-side stand-in for it; its device address is
// looked up with hipGetSymbolAddress, once per device (with that device current),
// and only that address is handed to kernels.  Every call on one device reuses
// that device's array: the flags are cleared by a fill kernel at the start of each
// solve, and every other vector and partial is written before it is read, so
// nothing of an earlier call leaks into a later one.  Calls that overlap on one
// device (two streams or two host threads) race on the array.
// ---------------------------------------------------------------------------
static_assert(FE_SOLVE_NOALLOC_MAX_N < INT32_MAX, "row limit");
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;

static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES];   // device address of `scratch` per device, once looked up
}  // namespace

// Device address of this device's array, looked up on its first use.
static int scratch_ptr(void **out)
{
    int dev = -1;
    FE_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return FE_ELIMIT;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        FE_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return FE_EHIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return FE_OK;
}

extern "C" int fe_solve_noalloc(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                                const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                                double *relres, void *stream)
{
    if (!solve_args_ok(n, rowptr, colind, val, b, u, rtol, maxit, iters, relres)) return FE_EINVAL;
    if (n > FE_SOLVE_NOALLOC_MAX_N || ws_layout(n, nullptr, nullptr) > NOALLOC_BYTES) return FE_ELIMIT;
    void *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    SolveWs W;
    ws_layout(n, &W, static_cast<char *>(base));
    return solve_run<false>(n, rowptr, colind, val, b, u, rtol, maxit, W, iters, relres,
                            static_cast<hipStream_t>(stream), nullptr);
}
