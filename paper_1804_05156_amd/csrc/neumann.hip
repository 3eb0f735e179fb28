// neumann.hip -- the pure Neumann problem (Section 3.3, equations (compatible) and
// (meanb)).
//
// With Neumann data on the whole boundary A is only semi-definite (its kernel is
// the constants) and A u = b is solvable only when b sums to zero.  The steps are
// those of the method:
//   1. b' = b - mean(b)                       (enforces the discrete compatibility)
//   2. fix u = 0 at vertex 0, solve the other rows: A_pin u = b' with row and column
//      0 of A replaced by the identity and b'_0 = 0 (freeNode = 2:N)
//   3. u <- u - c, c = sum_t |t| mean(u(elem_t)) / sum_t |t|   (zero mean)
// Every sum is a fixed-order tree of per-block partials, so the result is bitwise
// repeatable.
#include "cg_common.h"

namespace {

constexpr int NB = 256;
constexpr int NPART = 8192;   // blocks of the reduction kernels at most (grid-stride beyond)

struct NeuWs {
    double *val_pin, *b, *part, *scal;
    char *solve_ws;
    size_t solve_bytes;
};

size_t neu_layout(int64_t N, int64_t nnz, NeuWs *w, char *base)
{
    size_t sb = 0;
    fe_solve_workspace_bytes(N, &sb);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return base ? base + at : nullptr;
    };
    char *vp = take(8 * (size_t)(nnz > 0 ? nnz : 1)), *b = take(8 * (size_t)N), *part = take(8 * 2 * (size_t)NPART),
         *scal = take(8 * 8), *sw = take(sb);
    if (w) {
        w->val_pin = (double *)vp; w->b = (double *)b; w->part = (double *)part; w->scal = (double *)scal;
        w->solve_ws = sw; w->solve_bytes = sb;
    }
    return o;
}

// Partial sums of x over a grid-stride range: block b adds x[b*NB + t + k*NB*G].
__global__ __launch_bounds__(NB) void k_sum_partials(int64_t n, const double *__restrict__ x, double *part)
{
    __shared__ double lds[NB / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x; i < n; i += (int64_t)gridDim.x * NB) v += x[i];
    const double s = block_sum<NB>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One block: scal[0] = (sum of part) / n.
__global__ __launch_bounds__(NB) void k_mean(int32_t nb, const double *part, double n, double *scal)
{
    __shared__ double lds[NB / 64];
    const double s = cg_sum_partials(part, nb, lds);
    if (threadIdx.x == 0) scal[0] = s / n;
}

// b' = b - mean(b), then b'_pin = 0.
__global__ __launch_bounds__(NB) void k_shift_b(int64_t n, const double *__restrict__ b, const double *scal,
                                                int32_t pin, double *__restrict__ out)
{
    const double m = scal[0];
    for (int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x; i < n; i += (int64_t)gridDim.x * NB)
        out[i] = (i == pin) ? 0.0 : b[i] - m;
}

// A with row and column `pin` replaced by those of the identity (one thread per row).
__global__ __launch_bounds__(NB) void k_pin(int32_t n, const int32_t *__restrict__ rowptr,
                                            const int32_t *__restrict__ colind, const double *__restrict__ val,
                                            int32_t pin, double *__restrict__ out)
{
    const int32_t i = blockIdx.x * NB + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t c = colind[q];
        out[q] = (i == pin) ? (c == pin ? 1.0 : 0.0) : (c == pin ? 0.0 : val[q]);
    }
}

// Per block: sum of |t| * mean(u(elem_t)) and of |t| over a grid-stride range.
template <int DIM>
__global__ __launch_bounds__(NB) void k_area_mean(int32_t N, int32_t NT, const int32_t *__restrict__ elem,
                                                  const double *__restrict__ node, const double *__restrict__ u,
                                                  double *part)
{
    __shared__ double lds[2 * (NB / 64)];
    constexpr int NV = DIM + 1;
    double su = 0.0, sa = 0.0;
    for (int32_t t = blockIdx.x * NB + threadIdx.x; t < NT; t += gridDim.x * NB) {
        int32_t v[NV];
        double x[NV][DIM];
        double um = 0.0;
        for (int a = 0; a < NV; ++a) {
            v[a] = elem[(int64_t)a * NT + t];
            for (int c = 0; c < DIM; ++c) x[a][c] = node[(int64_t)c * N + v[a]];
            um += u[v[a]];
        }
        double meas;
        if (DIM == 2) {
            meas = 0.5 * fabs((x[1][0] - x[0][0]) * (x[2][1] - x[0][1]) - (x[2][0] - x[0][0]) * (x[1][1] - x[0][1]));
        } else {
            double e[3][3];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) e[a][c] = x[a + 1][c] - x[0][c];
            const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                               e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                               e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
            meas = fabs(det) / 6.0;
        }
        su += meas * (um / NV);
        sa += meas;
    }
    double w[2] = {su, sa};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 2; ++k) {
        for (int off = 32; off > 0; off >>= 1) w[k] += __shfl_xor(w[k], off, 64);
        if (lane == 0) lds[k * (NB / 64) + wid] = w[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 2; ++k) {
            double s = 0.0;
            for (int q = 0; q < NB / 64; ++q) s += lds[k * (NB / 64) + q];
            part[k * NPART + blockIdx.x] = s;
        }
}

// One block: scal[1] = c = (sum |t| mean u) / (sum |t|).
__global__ __launch_bounds__(NB) void k_area_mean_sum(int32_t nb, const double *part, double *scal)
{
    __shared__ double lds[NB / 64];
    const double su = cg_sum_partials(part, nb, lds);
    const double sa = cg_sum_partials(part + NPART, nb, lds);
    if (threadIdx.x == 0) scal[1] = su / sa;
}

__global__ __launch_bounds__(NB) void k_sub_c(int64_t n, const double *scal, double *u)
{
    const double c = scal[1];
    for (int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x; i < n; i += (int64_t)gridDim.x * NB) u[i] -= c;
}

unsigned grid_of(int64_t n)
{
    int64_t g = cdiv(n > 0 ? n : 1, NB);
    return (unsigned)(g < NPART ? g : NPART);
}

}  // namespace

extern "C" int fe_neumann_workspace_bytes(const fe_plan *plan, int64_t nnz, size_t *bytes)
{
    if (!plan || !bytes || nnz < 0) return FE_EINVAL;
    *bytes = neu_layout(plan->N, nnz, nullptr, nullptr);
    return FE_OK;
}

extern "C" int fe_neumann_solve(fe_plan *plan, const double *node, const int32_t *rowptr, const int32_t *colind,
                                const double *val, const double *b, double *u, double rtol, int32_t maxit, void *ws,
                                size_t ws_bytes, int32_t *iters, double *relres, double *mean_b, void *stream)
{
    if (!plan || !node || !rowptr || !colind || !val || !b || !u || !ws || !iters || !relres) return FE_EINVAL;
    if (!plan->pattern_done || plan->ndir != 0) return FE_EINVAL;   // pure Neumann: no Dirichlet vertex
    if ((uintptr_t)ws & 255) return FE_EINVAL;
    const int64_t N = plan->N, NT = plan->NT;
    NeuWs W;
    if (ws_bytes < neu_layout(N, plan->nnz, &W, static_cast<char *>(ws))) return FE_ESIZE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t pin = 0;
    int rc;
    const unsigned gn = grid_of(N), ge = grid_of(NT);
    // 1. b' = b - mean(b), b'_pin = 0
    FE_TIMED("k_sum_partials", s, hipLaunchKernelGGL(k_sum_partials, dim3(gn), dim3(NB), 0, s, N, b, W.part));
    FE_TIMED("k_mean", s, hipLaunchKernelGGL(k_mean, dim3(1), dim3(NB), 0, s, (int32_t)gn, (const double *)W.part,
                                             (double)N, W.scal));
    FE_TIMED("k_shift_b", s, hipLaunchKernelGGL(k_shift_b, dim3(gn), dim3(NB), 0, s, N, b, (const double *)W.scal, pin,
                                                W.b));
    // 2. pinned matrix, zero start vector, PCG on the other rows
    FE_TIMED("k_pin", s, hipLaunchKernelGGL(k_pin, dim3((unsigned)cdiv(N, NB)), dim3(NB), 0, s, (int32_t)N, rowptr,
                                            colind, val, pin, W.val_pin));
    if ((rc = fe_fill_f64(u, N, 0.0, s))) return rc;
    if ((rc = fe_launch_check())) return rc;
    rc = fe_solve(N, rowptr, colind, W.val_pin, W.b, u, rtol, maxit, W.solve_ws, W.solve_bytes, iters, relres,
                  stream);
    if (rc != FE_OK && rc != FE_ENOCONV) return rc;
    // 3. zero mean: u -= sum |t| mean(u(elem_t)) / sum |t|
    if (plan->dim == 2)
        FE_TIMED("k_area_mean", s, hipLaunchKernelGGL(k_area_mean<2>, dim3(ge), dim3(NB), 0, s, (int32_t)N,
                                                      (int32_t)NT, plan->elem, node, (const double *)u, W.part));
    else
        FE_TIMED("k_area_mean", s, hipLaunchKernelGGL(k_area_mean<3>, dim3(ge), dim3(NB), 0, s, (int32_t)N,
                                                      (int32_t)NT, plan->elem, node, (const double *)u, W.part));
    FE_TIMED("k_area_mean_sum", s, hipLaunchKernelGGL(k_area_mean_sum, dim3(1), dim3(NB), 0, s, (int32_t)ge,
                                                      (const double *)W.part, W.scal));
    FE_TIMED("k_sub_c", s, hipLaunchKernelGGL(k_sub_c, dim3(gn), dim3(NB), 0, s, N, (const double *)W.scal, u));
    int rc2 = fe_launch_check();
    if (rc2) return rc2;
    double mb = 0.0;   // (scal[0] still holds mean(b))
    FE_HIP_CHECK(hipMemcpyAsync(&mb, W.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (mean_b) *mean_b = mb;
    return rc;
}
