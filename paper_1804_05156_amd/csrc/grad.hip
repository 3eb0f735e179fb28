// grad.hip -- adjoint gradient of J(kappa) = 1/2 ||u - u_obs||^2, one thread per element.
//
// A = sum_t kappa_t K_t with K_t the unit-coefficient local stiffness, so
// dA/dkappa_t = K_t.  With A(free,free) lam(free) = (u - u_obs)(free) and lam = 0
// at Dirichlet nodes, dJ/dkappa_t = -lam^T K_t u = -|t| grad(lam_h) . grad(u_h),
// and with grad(lambda_c) = n_c / (d! |t|) (equation (dlambda)):
//     g_t = -(sum_c lam_c n_c) . (sum_c u_c n_c) / (d!^2 |t|).
// In 2-D the rotated edge vectors can be replaced by the edge vectors themselves
// (a rotation keeps dot products).
#include "fe_internal.h"

namespace {

constexpr int GB = 256;

__global__ __launch_bounds__(GB) void k_grad_2d(int32_t N, int32_t NT, const int32_t *__restrict__ elem,
                                                const double *__restrict__ node, const double *__restrict__ u,
                                                const double *__restrict__ lam, double *__restrict__ g,
                                                int32_t *status)
{
    const int32_t t = blockIdx.x * GB + threadIdx.x;
    if (t >= NT) return;
    int32_t v[3];
    double x[3], y[3];
    for (int c = 0; c < 3; ++c) {
        v[c] = elem[(int64_t)c * NT + t];
        x[c] = node[v[c]];
        y[c] = node[(int64_t)N + v[c]];
    }
    // edge vector opposite vertex c: x_{c-1} - x_{c+1}
    double ex[3], ey[3];
    for (int c = 0; c < 3; ++c) {
        const int cp = (c + 1) % 3, cm = (c + 2) % 3;
        ex[c] = x[cm] - x[cp];
        ey[c] = y[cm] - y[cp];
    }
    const double area2 = ex[1] * ey[2] - ey[1] * ex[2];
    if (!(area2 > 0.0) || !isfinite(area2)) atomicOr(status + ST_ERR, ERR_MEASURE);
    double gux = 0.0, guy = 0.0, glx = 0.0, gly = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double uc = u[v[c]], lc = lam[v[c]];
        gux += uc * ex[c];
        guy += uc * ey[c];
        glx += lc * ex[c];
        gly += lc * ey[c];
    }
    g[t] = -(glx * gux + gly * guy) / (2.0 * area2);
}

FE_DEV void cross3g(const double *p, const double *q, double *w)
{
    w[0] = p[1] * q[2] - p[2] * q[1];
    w[1] = p[2] * q[0] - p[0] * q[2];
    w[2] = p[0] * q[1] - p[1] * q[0];
}

__global__ __launch_bounds__(GB) void k_grad_3d(int32_t N, int32_t NT, const int32_t *__restrict__ elem,
                                                const double *__restrict__ node, const double *__restrict__ u,
                                                const double *__restrict__ lam, double *__restrict__ g,
                                                int32_t *status)
{
    const int32_t t = blockIdx.x * GB + threadIdx.x;
    if (t >= NT) return;
    int32_t v[4];
    double X[4][3];
    for (int c = 0; c < 4; ++c) {
        v[c] = elem[(int64_t)c * NT + t];
        for (int k = 0; k < 3; ++k) X[c][k] = node[(int64_t)k * N + v[c]];
    }
    double d10[3], d20[3], d30[3], d31[3], d21[3];
    for (int k = 0; k < 3; ++k) {
        d10[k] = X[1][k] - X[0][k];
        d20[k] = X[2][k] - X[0][k];
        d30[k] = X[3][k] - X[0][k];
        d31[k] = X[3][k] - X[1][k];
        d21[k] = X[2][k] - X[1][k];
    }
    double n[4][3];
    cross3g(d31, d21, n[0]);
    cross3g(d20, d30, n[1]);
    cross3g(d30, d10, n[2]);
    cross3g(d10, d20, n[3]);
    const double vol6 = n[3][0] * d30[0] + n[3][1] * d30[1] + n[3][2] * d30[2];
    if (!(vol6 > 0.0) || !isfinite(vol6)) atomicOr(status + ST_ERR, ERR_MEASURE);
    double gu[3] = {0, 0, 0}, gl[3] = {0, 0, 0};
    for (int c = 0; c < 4; ++c) {
        const double uc = u[v[c]], lc = lam[v[c]];
        for (int k = 0; k < 3; ++k) {
            gu[k] += uc * n[c][k];
            gl[k] += lc * n[c][k];
        }
    }
    g[t] = -(gl[0] * gu[0] + gl[1] * gu[1] + gl[2] * gu[2]) / (6.0 * vol6);
}

}  // namespace

extern "C" int fe_grad(fe_plan *plan, const double *node, const double *u, const double *lam, double *g,
                       void *stream)
{
    if (!plan || !node || !u || !lam || (!g && plan->NT > 0)) return FE_EINVAL;
    if (plan->NT == 0) return FE_OK;
    const unsigned nb = (unsigned)cdiv(plan->NT, GB);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan->dim == 2)
        FE_TIMED("k_grad_2d", s,
                 hipLaunchKernelGGL(k_grad_2d, dim3(nb), dim3(GB), 0, s, (int32_t)plan->N, (int32_t)plan->NT, plan->elem, node,
                               u, lam, g, plan->status));
    else
        FE_TIMED("k_grad_3d", s,
                 hipLaunchKernelGGL(k_grad_3d, dim3(nb), dim3(GB), 0, s, (int32_t)plan->N, (int32_t)plan->NT, plan->elem, node,
                               u, lam, g, plan->status));
    return fe_launch_check();
}
