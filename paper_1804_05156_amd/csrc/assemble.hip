// assemble.hip -- numeric phase: stiffness values, load vector and boundary
// conditions, one thread per row of A.
//
// A row i of A is the sum, over the elements t around vertex i, of row a of the
// local matrix of t (a = local index of i in t):
//     K_t[a][b] = kappa_t n_a . n_b / (d!^2 |t|)            (equation (dlambda))
// with n_c the scaled inward normal of the side opposite local vertex c (edge
// rotation in 2-D, cross product of two side edges in 3-D, Section 3.1.3).  The
// thread walks the row's incidence list (ascending element index, from the plan),
// recomputes the element geometry from the coordinates, and adds row a into an
// LDS accumulator slot per stored column.  This is the `sparse` duplicate sum of
// Section 2.2 done per row, in a fixed order, with no atomics and no triplet array.
// The same walk adds the load term of Section 3.2, the Neumann side terms and the
// Dirichlet lifting of Section 3.3, so A, A_bc and b come out of one kernel.
#include "fe_internal.h"

namespace {

struct AsmArgs {
    int32_t N, NT;
    const int32_t *elem;
    const double *node;
    const double *kappa;
    const int32_t *pi, *pincptr, *pinc, *prow_start;
    const uint32_t *pmeta, *prow_info;
    DevFn f, gd, gn;
    double *val, *val_bc, *b, *b_load;
    uint8_t *isd_out;
    int32_t *status;
};

template <int DIM> FE_DEV void load_xy(const double *node, int32_t N, int32_t v, double *x)
{
    for (int c = 0; c < DIM; ++c) x[c] = node[(int64_t)c * N + v];
}

// Value of g_D at vertex v with coordinates x.
template <int DIM> FE_DEV double dirichlet_value(const DevFn &g, int32_t v, const double *x)
{
    if (g.kind == FE_FN_NODAL) return g.nodal[v];
    return fn_point<DIM>(g, x);
}

// ----------------------------------------------------------------------------- 2-D
// Local vertices are rotated so the row's vertex comes first: X0 = x_a,
// X1 = x_{a+1}, X2 = x_{a+2} (indices mod 3).  A cyclic rotation keeps the
// orientation, so with E0 = X2 - X1, E1 = X0 - X2, E2 = X1 - X0 (the edge vectors
// opposite X0, X1, X2) the doubled area is E1 x E2 > 0 and K[0][c] =
// kappa E0 . Ec / (2 * doubled area).
template <int ROWCAP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_assemble_2d(AsmArgs A)
{
    __shared__ double acc[ROWCAP * BLOCK];
    const int tid = threadIdx.x;
    const int32_t k = blockIdx.x * BLOCK + tid;
    if (k >= A.N) return;
    const int32_t i = A.pi[k];
    const int32_t s = A.pincptr[k], e = A.pincptr[k + 1];
    const int32_t rs = A.prow_start[k];
    const uint32_t info = A.prow_info[k];
    const int len = info & 0xff, diag = (info >> 8) & 0xff;
    const bool rowd = (info >> 16) & 1;
    for (int c = 0; c < len; ++c) acc[c * BLOCK + tid] = 0.0;
    double X0[2];
    load_xy<2>(A.node, A.N, i, X0);
    double bsum = 0.0, lift = 0.0;
    uint64_t dmask = 0;
    int32_t err = 0;
    const bool nodal_f = A.f.kind == FE_FN_NODAL;
    for (int32_t p = s; p < e; ++p) {
        const int32_t key = A.pinc[p];
        const uint32_t meta = A.pmeta[p];
        const int32_t t = key / 3;
        const int a = key - 3 * t;
        const int b1 = (a == 2) ? 0 : a + 1;
        const int b2 = (a == 0) ? 2 : a - 1;
        const int32_t v1 = A.elem[(int64_t)b1 * A.NT + t];
        const int32_t v2 = A.elem[(int64_t)b2 * A.NT + t];
        double X1[2], X2[2];
        load_xy<2>(A.node, A.N, v1, X1);
        load_xy<2>(A.node, A.N, v2, X2);
        const double E0x = X2[0] - X1[0], E0y = X2[1] - X1[1];
        const double E1x = X0[0] - X2[0], E1y = X0[1] - X2[1];
        const double E2x = X1[0] - X0[0], E2y = X1[1] - X0[1];
        const double area2 = E1x * E2y - E1y * E2x;        // 2|t|
        const double kt = A.kappa ? A.kappa[t] : 1.0;
        if (!(area2 > 0.0) || !isfinite(area2)) err |= ERR_MEASURE;
        if (!(kt > 0.0) || !isfinite(kt)) err |= ERR_KAPPA;
        const double sc = kt / (2.0 * area2);
        const double k00 = sc * (E0x * E0x + E0y * E0y);
        const double k01 = sc * (E0x * E1x + E0y * E1y);
        const double k02 = sc * (E0x * E2x + E0y * E2y);
        const int o1 = (meta >> Meta<3>::OFF) & 0xff;
        const int o2 = (meta >> (Meta<3>::OFF + 8)) & 0xff;
        acc[diag * BLOCK + tid] += k00;
        acc[o1 * BLOCK + tid] += k01;
        acc[o2 * BLOCK + tid] += k02;
        // load: |t| (f(m1) + f(m2)) / 6, m1 = (X2+X0)/2, m2 = (X0+X1)/2 (Section 3.2)
        if (A.f.kind != FE_FN_ZERO) {
            double f1, f2;
            if (nodal_f) {
                const double fa = A.f.nodal[i], g1 = A.f.nodal[v1], g2 = A.f.nodal[v2];
                f1 = 0.5 * (g2 + fa);
                f2 = 0.5 * (fa + g1);
            } else {
                const double m1[2] = {0.5 * (X2[0] + X0[0]), 0.5 * (X2[1] + X0[1])};
                const double m2[2] = {0.5 * (X0[0] + X1[0]), 0.5 * (X0[1] + X1[1])};
                f1 = fn_point<2>(A.f, m1);
                f2 = fn_point<2>(A.f, m2);
            }
            bsum += area2 * (f1 + f2) / 12.0;
        }
        // Neumann sides through vertex a: the side opposite X1 (X2-X0) and opposite X2 (X0-X1)
        const uint32_t nb = (meta >> Meta<3>::NBIT) & 3u;
        if (nb) {
            for (int jj = 0; jj < 2; ++jj) {
                if (!((nb >> jj) & 1u)) continue;
                const double *Xo = jj == 0 ? X2 : X1;              // other end of the side
                const double ex = jj == 0 ? E1x : E2x, ey = jj == 0 ? E1y : E2y;
                const double L = sqrt(ex * ex + ey * ey);
                const double mid[2] = {0.5 * (X0[0] + Xo[0]), 0.5 * (X0[1] + Xo[1])};
                double g;
                if (A.gn.kind == FE_FN_DUDN_SINPROD) {
                    // inward normal of the side = its edge vector rotated counter-clockwise
                    const double nrm[2] = {ey / L, -ex / L};           // outward unit normal
                    g = fn_dudn<2>(A.gn, mid, nrm);
                } else if (A.gn.kind == FE_FN_NODAL) {
                    const int32_t vo = jj == 0 ? v2 : v1;
                    g = 0.5 * (A.gn.nodal[i] + A.gn.nodal[vo]);
                } else {
                    g = fn_point<2>(A.gn, mid);
                }
                bsum += L * g / 2.0;
            }
        }
        // Dirichlet columns: record them and lift b by K[a][c] u_D(c)
        const uint32_t db = (meta >> Meta<3>::DBIT) & 3u;
        if (db) {
            if (db & 1u) {
                dmask |= 1ull << o1;
                if (A.gd.kind != FE_FN_ZERO) lift += k01 * dirichlet_value<2>(A.gd, v1, X1);
            }
            if (db & 2u) {
                dmask |= 1ull << o2;
                if (A.gd.kind != FE_FN_ZERO) lift += k02 * dirichlet_value<2>(A.gd, v2, X2);
            }
        }
    }
    if (err) atomicOr(A.status + ST_ERR, err);
    for (int c = 0; c < len; ++c) A.val[rs + c] = acc[c * BLOCK + tid];
    if (A.val_bc) {
        for (int c = 0; c < len; ++c) {
            double v = acc[c * BLOCK + tid];
            if (rowd) v = (c == diag) ? 1.0 : 0.0;
            else if ((dmask >> c) & 1ull) v = 0.0;
            A.val_bc[rs + c] = v;
        }
    }
    if (A.b_load) A.b_load[i] = bsum;
    A.b[i] = rowd ? dirichlet_value<2>(A.gd, i, X0) : bsum - lift;
    if (A.isd_out) A.isd_out[i] = rowd ? 1 : 0;
}

// ----------------------------------------------------------------------------- 3-D
// Local vertices are taken in the even order Y0 = x_a, Y1..Y3 = x_{fe_other(a, .)},
// which keeps the orientation.  Sides opposite Y0..Y3 follow the paper's face list
// [1 3 2], [0 2 3], [0 3 1], [0 1 2]; n_f = (Y_F1 - Y_F0) x (Y_F2 - Y_F0) is the
// inward normal of a positively oriented tetrahedron, 6|t| = n_3 . (Y3 - Y0) and
// K[0][q] = kappa n_0 . n_q / (6 * 6|t|).
FE_DEV void cross3(const double *u, const double *v, double *w)
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

FE_DEV double dot3(const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

template <int ROWCAP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_assemble_3d(AsmArgs A)
{
    __shared__ double acc[ROWCAP * BLOCK];
    const int tid = threadIdx.x;
    const int32_t k = blockIdx.x * BLOCK + tid;
    if (k >= A.N) return;
    const int32_t i = A.pi[k];
    const int32_t s = A.pincptr[k], e = A.pincptr[k + 1];
    const int32_t rs = A.prow_start[k];
    const uint32_t info = A.prow_info[k];
    const int len = info & 0xff, diag = (info >> 8) & 0xff;
    const bool rowd = (info >> 16) & 1;
    for (int c = 0; c < len; ++c) acc[c * BLOCK + tid] = 0.0;
    double Y[4][3];
    load_xy<3>(A.node, A.N, i, Y[0]);
    double bsum = 0.0, lift = 0.0;
    uint64_t dmask = 0;
    int32_t err = 0;
    const double alpha = 0.58541019662496845446;   // (5 + 3 sqrt 5) / 20
    const double beta = 0.13819660112501051518;    // (5 - sqrt 5) / 20
    const double fi = (A.f.kind == FE_FN_NODAL) ? A.f.nodal[i] : 0.0;
    for (int32_t p = s; p < e; ++p) {
        const int32_t key = A.pinc[p];
        const uint32_t meta = A.pmeta[p];
        const int32_t t = key >> 2;
        const int a = key & 3;
        int32_t v[4];
        v[0] = i;
#pragma unroll
        for (int q = 1; q < 4; ++q) {
            v[q] = A.elem[(int64_t)fe_other<4>(a, q - 1) * A.NT + t];
            load_xy<3>(A.node, A.N, v[q], Y[q]);
        }
        double d10[3], d20[3], d30[3], d31[3], d21[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d10[c] = Y[1][c] - Y[0][c];
            d20[c] = Y[2][c] - Y[0][c];
            d30[c] = Y[3][c] - Y[0][c];
            d31[c] = Y[3][c] - Y[1][c];
            d21[c] = Y[2][c] - Y[1][c];
        }
        double n[4][3];
        cross3(d31, d21, n[0]);   // side [1 3 2]
        cross3(d20, d30, n[1]);   // side [0 2 3]
        cross3(d30, d10, n[2]);   // side [0 3 1]
        cross3(d10, d20, n[3]);   // side [0 1 2]
        const double vol6 = dot3(n[3], d30);
        const double kt = A.kappa ? A.kappa[t] : 1.0;
        if (!(vol6 > 0.0) || !isfinite(vol6)) err |= ERR_MEASURE;
        if (!(kt > 0.0) || !isfinite(kt)) err |= ERR_KAPPA;
        const double sc = kt / (6.0 * vol6);
        double kr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) kr[q] = sc * dot3(n[0], n[q]);
        acc[diag * BLOCK + tid] += kr[0];
        int off[3];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            off[jj] = (meta >> (Meta<4>::OFF + 8 * jj)) & 0xff;
            acc[off[jj] * BLOCK + tid] += kr[jj + 1];
        }
        const double vol = vol6 / 6.0;
        // load (Section 3.2): symmetric 4-point rule; exact closed form for nodal f
        if (A.f.kind == FE_FN_NODAL) {
            const double sf = fi + A.f.nodal[v[1]] + A.f.nodal[v[2]] + A.f.nodal[v[3]];
            bsum += vol * (fi + sf) / 20.0;
        } else if (A.f.kind != FE_FN_ZERO) {
            double S[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) S[c] = Y[0][c] + Y[1][c] + Y[2][c] + Y[3][c];
            double q = 0.0;
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) {
                double pt[3];
                for (int c = 0; c < 3; ++c) pt[c] = beta * S[c] + (alpha - beta) * Y[kq][c];
                q += fn_point<3>(A.f, pt) * (kq == 0 ? alpha : beta);
            }
            bsum += vol * q / 4.0;
        }
        // Neumann sides containing Y0: the sides opposite Y1, Y2, Y3
        const uint32_t nb = (meta >> Meta<4>::NBIT) & 7u;
        if (nb) {
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                if (!((nb >> jj) & 1u)) continue;
                const int fq = jj + 1;
                const double nn = sqrt(dot3(n[fq], n[fq]));
                const double area = 0.5 * nn;
                double cen[3];
                for (int c = 0; c < 3; ++c) cen[c] = (Y[0][c] + Y[1][c] + Y[2][c] + Y[3][c] - Y[fq][c]) / 3.0;
                double g;
                if (A.gn.kind == FE_FN_DUDN_SINPROD) {
                    const double nrm[3] = {-n[fq][0] / nn, -n[fq][1] / nn, -n[fq][2] / nn};
                    g = fn_dudn<3>(A.gn, cen, nrm);
                } else if (A.gn.kind == FE_FN_NODAL) {
                    double sg = 0.0;
                    for (int c = 0; c < 4; ++c)
                        if (c != fq) sg += A.gn.nodal[v[c]];
                    g = sg / 3.0;
                } else {
                    g = fn_point<3>(A.gn, cen);
                }
                bsum += area * g / 3.0;
            }
        }
        const uint32_t db = (meta >> Meta<4>::DBIT) & 7u;
        if (db) {
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                if (!((db >> jj) & 1u)) continue;
                dmask |= 1ull << off[jj];
                if (A.gd.kind != FE_FN_ZERO) lift += kr[jj + 1] * dirichlet_value<3>(A.gd, v[jj + 1], Y[jj + 1]);
            }
        }
    }
    if (err) atomicOr(A.status + ST_ERR, err);
    for (int c = 0; c < len; ++c) A.val[rs + c] = acc[c * BLOCK + tid];
    if (A.val_bc) {
        for (int c = 0; c < len; ++c) {
            double v = acc[c * BLOCK + tid];
            if (rowd) v = (c == diag) ? 1.0 : 0.0;
            else if ((dmask >> c) & 1ull) v = 0.0;
            A.val_bc[rs + c] = v;
        }
    }
    if (A.b_load) A.b_load[i] = bsum;
    A.b[i] = rowd ? dirichlet_value<3>(A.gd, i, Y[0]) : bsum - lift;
    if (A.isd_out) A.isd_out[i] = rowd ? 1 : 0;
}

template <int ROWCAP, int BLOCK> int launch(int dim, const AsmArgs &A, hipStream_t s)
{
    const unsigned g = (unsigned)cdiv(A.N, BLOCK);
    if (dim == 2) hipLaunchKernelGGL((k_assemble_2d<ROWCAP, BLOCK>), dim3(g), dim3(BLOCK), 0, s, A);
    else hipLaunchKernelGGL((k_assemble_3d<ROWCAP, BLOCK>), dim3(g), dim3(BLOCK), 0, s, A);
    return fe_launch_check();
}

}  // namespace

extern "C" int fe_assemble(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                           const fe_fn *g_d, const fe_fn *g_n, double *val, double *val_bc, double *b,
                           double *b_load, uint8_t *is_dirichlet, void *stream)
{
    if (!plan || !node || !val || !b) return FE_EINVAL;
    if (!plan->pattern_done) return FE_EINVAL;
    if (!devfn_valid(f, false) || !devfn_valid(g_d, false) || !devfn_valid(g_n, true)) return FE_EINVAL;
    AsmArgs A{};
    A.N = (int32_t)plan->N;
    A.NT = (int32_t)plan->NT;
    A.elem = plan->elem;
    A.node = node;
    A.kappa = kappa;
    A.pi = plan->pi;
    A.pincptr = plan->pincptr;
    A.pinc = plan->pinc;
    A.prow_start = plan->prow_start;
    A.pmeta = plan->pmeta;
    A.prow_info = plan->prow_info;
    A.f = make_devfn(f);
    A.gd = make_devfn(g_d);
    A.gn = make_devfn(g_n);
    A.val = val;
    A.val_bc = val_bc;
    A.b = b;
    A.b_load = b_load;
    A.isd_out = is_dirichlet;
    A.status = plan->status;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int mr = plan->max_row;
    if (mr <= 16) return launch<16, 256>(plan->dim, A, s);
    if (mr <= 32) return launch<32, 128>(plan->dim, A, s);
    return launch<64, 64>(plan->dim, A, s);
}
