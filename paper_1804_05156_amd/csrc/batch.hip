// batch.hip -- many independent systems solved by one persistent launch.
//
// A batch of meshes is assembled as one mesh (their disjoint union, vertex and
// element labels offset per instance), so the plan and assembly kernels apply
// unchanged and produce a block-diagonal A_bc.  Each diagonal block (instance) is
// then solved by Jacobi-preconditioned CG with its own scalars and its own stopping
// test, all instances advancing together inside one kernel:
//   phase A: for every 256-row unit of a running instance, p = z + beta p_old,
//            q = A p, partial p.q; the instance's last unit to finish computes alpha;
//   phase B: x += alpha p, r -= alpha q, z = r / diag, partials r.z and r.r; the
//            last unit computes beta and the stopping test.
// Device-wide barriers separate the phases.  Units, reduction trees and the order
// of every sum are those of the single-system solve, so each instance reproduces
// fe_solve on its own block bit for bit, whatever the grid size.
//
// Work distribution: every block keeps in LDS the list of instances still running
// with the prefix sum of their unit counts, and walks the virtual unit range
// [0, units of running instances) with a grid stride, so converged instances cost
// nothing.  The list changes only when an instance converges (phase B); each block
// rebuilds it after the barrier that follows.
//
// Every device-wide wait is bounded: a block that waits longer than the limit
// (blocks not co-resident) raises an abort flag that every block checks in its
// waits and after each barrier, so the grid always drains.
#include <cstring>
#include <new>
#include <vector>

#include "cg_common.h"

namespace {

constexpr int BB = CG_UNIT;
constexpr int32_t MAX_INST = 4096;

enum { BS_RZ = 0, BS_RR, BS_BB, BS_ALPHA, BS_BETA, BS_TOL2, BS_COUNT = 8 };   // doubles per instance
enum { BF_DONE = 0, BF_ITER, BF_TICKET, BF_BAD, BF_COUNT = 4 };                // ints per instance
enum { BAR_COUNT = 0, BAR_GEN, BAR_ABORT, BAR_ACTIVE, BAR_WORDS = 8 };

struct BatchArgs {
    int32_t n_inst;
    const int4 *inst;     // per instance: (first unit, unit count, first row, end row)
    const int32_t *rowptr, *colind;
    const double *val, *b;
    double *x, *r, *z, *p0, *p1, *q, *dinv;
    double *part;         // 3 * total units
    double *scal;         // BS_COUNT * n_inst
    int32_t *flag;        // BF_COUNT * n_inst
    uint32_t *bar;        // BAR_WORDS
    int32_t n_units;
    double rtol;
    int32_t maxit;
    int64_t spin_limit;   // in s_memrealtime ticks (100 MHz)
};

FE_DEV uint32_t ld_acquire(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
FE_DEV int32_t ld_i32(const int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
FE_DEV double ld_f64(const double *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Generation barrier over the whole grid with a bounded wait.  Every thread
// publishes its own writes before the arrival and acquires after the release.
FE_DEV void grid_barrier(uint32_t *bar, int64_t spin_limit)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t gen = ld_acquire(bar + BAR_GEN);
        const uint32_t arrived = __hip_atomic_fetch_add(bar + BAR_COUNT, 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(bar + BAR_COUNT, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + BAR_GEN, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (ld_acquire(bar + BAR_GEN) == gen) {
                if (ld_acquire(bar + BAR_ABORT)) break;
                __builtin_amdgcn_s_sleep(2);
                if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > spin_limit) {
                    __hip_atomic_fetch_or(bar + BAR_ABORT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
    }
    __syncthreads();
    __threadfence();
}

// LDS list of running instances: ainst[j] = (instance, first unit, first row, end
// row), pre[j] = units of the running instances before j, pre[nact] = total.
struct Active {
    int4 *ainst;
    int32_t *pre;
    int32_t nact, units;
};

FE_DEV void build_active(const BatchArgs &A, Active &L, int32_t *scan_lds)
{
    int32_t nact = 0, base = 0;
    for (int32_t k0 = 0; k0 < A.n_inst; k0 += BB) {
        const int32_t k = k0 + threadIdx.x;
        int4 in = make_int4(0, 0, 0, 0);
        int32_t act = 0;
        if (k < A.n_inst) {
            in = A.inst[k];
            act = (in.y > 0 && ld_i32(A.flag + BF_COUNT * k + BF_DONE) == 0) ? 1 : 0;
        }
        int32_t tot_act, tot_units;
        const int32_t pos = block_exclusive_i32<BB>(act, scan_lds, &tot_act);
        const int32_t upre = block_exclusive_i32<BB>(act ? in.y : 0, scan_lds, &tot_units);
        if (act) {
            L.ainst[nact + pos] = make_int4(k, in.x, in.z, in.w);
            L.pre[nact + pos] = base + upre;
        }
        nact += tot_act;
        base += tot_units;
    }
    if (threadIdx.x == 0) L.pre[nact] = base;
    __syncthreads();
    L.nact = nact;
    L.units = base;
}

// Virtual unit v -> running-instance slot j (largest j with pre[j] <= v).
FE_DEV int32_t find_slot(const Active &L, int32_t v)
{
    int32_t lo = 0, hi = L.nact - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (L.pre[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Unit {
    int32_t inst, u0, u, row0, row1, count;   // u0: the instance's first unit
};

FE_DEV Unit unit_of(const Active &L, int32_t v)
{
    const int32_t j = find_slot(L, v);
    const int4 a = L.ainst[j];
    const int32_t local = v - L.pre[j];
    Unit t;
    t.inst = a.x;
    t.u0 = a.y;
    t.u = a.y + local;
    t.row0 = a.z + local * BB;
    t.row1 = (a.w - t.row0 < BB) ? a.w : t.row0 + BB;
    t.count = L.pre[j + 1] - L.pre[j];
    return t;
}

__global__ __launch_bounds__(BB) void k_batch_pcg(BatchArgs A)
{
    extern __shared__ int4 dyn[];
    __shared__ double lds[BB / 64];
    __shared__ int32_t scan_lds[2 * BB / 64];
    __shared__ int s_stop;
    Active L;
    L.ainst = dyn;
    L.pre = reinterpret_cast<int32_t *>(dyn + A.n_inst);
    const int32_t U = A.n_units;
    const int32_t G = gridDim.x;
    // blocks b and b + 8 run on the same XCD: give each XCD a contiguous range of units
    const int32_t vb = (G % 8 == 0) ? (int32_t)(blockIdx.x % 8) * (G / 8) + (int32_t)(blockIdx.x / 8)
                                    : (int32_t)blockIdx.x;
    build_active(A, L, scan_lds);
    // ---- initial residual, diagonal, z = r / diag, p_old = 0
    for (int32_t v = vb; v < L.units; v += G) {
        const Unit t = unit_of(L, v);
        const int32_t i = t.row0 + threadIdx.x;
        double rz = 0.0, rr = 0.0, bb = 0.0;
        if (i < t.row1) {
            double ri, d;
            cg_init_row(i, A.rowptr, A.colind, A.val, A.b, A.x, &ri, &d);
            if (!(d > 0.0)) atomicOr(A.flag + BF_COUNT * t.inst + BF_BAD, 1);
            const double di = 1.0 / d;
            A.dinv[i] = di;
            A.r[i] = ri;
            A.z[i] = ri * di;
            A.p0[i] = 0.0;
            rz = ri * ri * di;
            rr = ri * ri;
            bb = A.b[i] * A.b[i];
        }
        const double s0 = block_sum<BB>(rz, lds);
        const double s1 = block_sum<BB>(rr, lds);
        const double s2 = block_sum<BB>(bb, lds);
        if (threadIdx.x == 0) {
            A.part[t.u] = s0;
            A.part[U + t.u] = s1;
            A.part[2 * U + t.u] = s2;
        }
        if (cg_last_arrival(A.flag + BF_COUNT * t.inst + BF_TICKET, t.count)) {
            const double RZ = cg_sum_partials(A.part + t.u0, t.count, lds);
            const double RR = cg_sum_partials(A.part + U + t.u0, t.count, lds);
            const double BBv = cg_sum_partials(A.part + 2 * U + t.u0, t.count, lds);
            if (threadIdx.x == 0) {
                double *sc = A.scal + BS_COUNT * t.inst;
                int32_t *fl = A.flag + BF_COUNT * t.inst;
                const double bn2 = BBv > 0.0 ? BBv : 1.0;
                sc[BS_RZ] = RZ;
                sc[BS_RR] = RR;
                sc[BS_BB] = bn2;
                sc[BS_TOL2] = A.rtol * A.rtol * bn2;
                sc[BS_BETA] = 0.0;
                sc[BS_ALPHA] = 0.0;
                fl[BF_ITER] = 0;
                if (RR <= A.rtol * A.rtol * bn2) {
                    fl[BF_DONE] = 1;
                    __hip_atomic_fetch_sub(A.bar + BAR_ACTIVE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    grid_barrier(A.bar, A.spin_limit);
    uint32_t seen = 0xffffffffu;
    for (int32_t it = 0; it < A.maxit; ++it) {
        if (threadIdx.x == 0) {
            const uint32_t act = ld_acquire(A.bar + BAR_ACTIVE);
            s_stop = ld_acquire(A.bar + BAR_ABORT) ? 2 : (act == 0 ? 1 : 0);
            if (act != seen) s_stop |= 4;
            seen = act;
        }
        __syncthreads();
        const int stop = s_stop;
        __syncthreads();
        if (stop & 3) break;
        if (stop & 4) build_active(A, L, scan_lds);
        const double *pold = (it & 1) ? A.p1 : A.p0;
        double *pnew = (it & 1) ? A.p0 : A.p1;
        // ---- phase A
        for (int32_t v = vb; v < L.units; v += G) {
            const Unit t = unit_of(L, v);
            const double beta = ld_f64(A.scal + BS_COUNT * t.inst + BS_BETA);
            const int32_t i = t.row0 + threadIdx.x;
            double pq = 0.0;
            if (i < t.row1) {
                const double s = cg_apply_row(i, A.rowptr, A.colind, A.val, A.z, pold, beta);
                const double pi = A.z[i] + beta * pold[i];
                pnew[i] = pi;
                A.q[i] = s;
                pq = pi * s;
            }
            const double bs = block_sum<BB>(pq, lds);
            if (threadIdx.x == 0) A.part[t.u] = bs;
            if (cg_last_arrival(A.flag + BF_COUNT * t.inst + BF_TICKET, t.count)) {
                const double PQ = cg_sum_partials(A.part + t.u0, t.count, lds);
                if (threadIdx.x == 0) {
                    double *sc = A.scal + BS_COUNT * t.inst;
                    sc[BS_ALPHA] = sc[BS_RZ] / PQ;
                }
            }
        }
        grid_barrier(A.bar, A.spin_limit);
        if (ld_acquire(A.bar + BAR_ABORT)) break;
        // ---- phase B
        for (int32_t v = vb; v < L.units; v += G) {
            const Unit t = unit_of(L, v);
            const double alpha = ld_f64(A.scal + BS_COUNT * t.inst + BS_ALPHA);
            const int32_t i = t.row0 + threadIdx.x;
            double rz = 0.0, rr = 0.0;
            if (i < t.row1) {
                A.x[i] += alpha * pnew[i];
                const double ri = A.r[i] - alpha * A.q[i];
                const double zi = ri * A.dinv[i];
                A.r[i] = ri;
                A.z[i] = zi;
                rz = ri * zi;
                rr = ri * ri;
            }
            const double s0 = block_sum<BB>(rz, lds);
            const double s1 = block_sum<BB>(rr, lds);
            if (threadIdx.x == 0) {
                A.part[U + t.u] = s0;
                A.part[2 * U + t.u] = s1;
            }
            if (cg_last_arrival(A.flag + BF_COUNT * t.inst + BF_TICKET, t.count)) {
                const double RZ = cg_sum_partials(A.part + U + t.u0, t.count, lds);
                const double RR = cg_sum_partials(A.part + 2 * U + t.u0, t.count, lds);
                if (threadIdx.x == 0) {
                    double *sc = A.scal + BS_COUNT * t.inst;
                    int32_t *fl = A.flag + BF_COUNT * t.inst;
                    sc[BS_BETA] = RZ / sc[BS_RZ];
                    sc[BS_RZ] = RZ;
                    sc[BS_RR] = RR;
                    fl[BF_ITER] += 1;
                    if (RR <= sc[BS_TOL2]) {
                        fl[BF_DONE] = 1;
                        __hip_atomic_fetch_sub(A.bar + BAR_ACTIVE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
        grid_barrier(A.bar, A.spin_limit);
        if (ld_acquire(A.bar + BAR_ABORT)) break;
    }
}

// Barrier words and per-instance flags to their start values (a kernel, so that the
// reset can sit inside a captured graph).
__global__ void k_batch_reset(uint32_t *bar, int32_t *flag, int32_t n_inst, uint32_t active)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < BAR_WORDS) bar[k] = (k == BAR_ACTIVE) ? active : 0u;
    if (k < BF_COUNT * n_inst) flag[k] = 0;
}

struct BatchWs {
    double *r, *z, *p0, *p1, *q, *dinv, *part, *scal;
    int32_t *flag;
    uint32_t *bar;
    int4 *inst;
    uint8_t *isd;         // Dirichlet mask of the graph path
};

int64_t max_units(int64_t n, int32_t n_inst) { return n / CG_UNIT + n_inst; }

size_t batch_layout(int64_t n, int32_t n_inst, BatchWs *w, char *base)
{
    const int64_t U = max_units(n, n_inst);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return base ? base + at : nullptr;
    };
    char *r = take(8 * (size_t)n), *z = take(8 * (size_t)n), *p0 = take(8 * (size_t)n), *p1 = take(8 * (size_t)n),
         *q = take(8 * (size_t)n), *d = take(8 * (size_t)n), *part = take(8 * 3 * (size_t)U),
         *scal = take(8 * BS_COUNT * (size_t)n_inst), *flag = take(4 * BF_COUNT * (size_t)n_inst),
         *bar = take(4 * BAR_WORDS), *inst = take(16 * (size_t)n_inst), *isd = take((size_t)n);
    if (w) {
        w->r = (double *)r; w->z = (double *)z; w->p0 = (double *)p0; w->p1 = (double *)p1; w->q = (double *)q;
        w->dinv = (double *)d; w->part = (double *)part; w->scal = (double *)scal; w->flag = (int32_t *)flag;
        w->bar = (uint32_t *)bar; w->inst = (int4 *)inst; w->isd = (uint8_t *)isd;
    }
    return o;
}

size_t dyn_lds_bytes(int32_t n_inst) { return 16 * (size_t)n_inst + 4 * ((size_t)n_inst + 1); }

}  // namespace

// Host side of one batched solve: the instance table, the grid, the launch.
struct fe_batch_solver {
    int32_t n_inst = 0, n_units = 0, grid = 0, blocks_per_cu = 0, max_per_cu = 0;
    int64_t n = 0;
    size_t lds = 0;
    BatchWs W{};
    std::vector<int4> inst;
    uint32_t active = 0;
};

static int batch_set_grid(fe_batch_solver *S, int32_t blocks_per_cu)
{
    if (blocks_per_cu < 0) return FE_EINVAL;
    int dev = 0, cus = 0, per = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(&k_batch_pcg), BB,
                                                              S->lds));
    if (per < 1) return FE_ELIMIT;
    S->max_per_cu = per;
    int32_t want = blocks_per_cu ? blocks_per_cu : (per < 4 ? per : 4);
    if (want > per) return FE_ELIMIT;
    int64_t g = (int64_t)cus * want;
    if (g > S->n_units) g = S->n_units;
    S->grid = (int32_t)(g > 0 ? g : 1);
    S->blocks_per_cu = want;
    return FE_OK;
}

static int batch_prepare(fe_batch_solver *S, int32_t n_inst, const int64_t *off, void *ws, size_t ws_bytes,
                         int32_t blocks_per_cu)
{
    if (n_inst <= 0 || n_inst > MAX_INST || !off || !ws) return n_inst > MAX_INST ? FE_ELIMIT : FE_EINVAL;
    const int64_t n = off[n_inst];
    if (off[0] != 0 || n <= 0 || n >= INT32_MAX) return FE_EINVAL;
    for (int32_t k = 0; k < n_inst; ++k)
        if (off[k + 1] < off[k]) return FE_EINVAL;
    if ((uintptr_t)ws & 255) return FE_EINVAL;
    if (ws_bytes < batch_layout(n, n_inst, nullptr, nullptr)) return FE_ESIZE;
    batch_layout(n, n_inst, &S->W, static_cast<char *>(ws));
    S->n = n;
    S->n_inst = n_inst;
    S->inst.assign(n_inst, make_int4(0, 0, 0, 0));
    S->active = 0;
    int32_t units = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        const int32_t r0 = (int32_t)off[k], r1 = (int32_t)off[k + 1];
        const int32_t cnt = (int32_t)cdiv(r1 - r0, CG_UNIT);
        S->inst[k] = make_int4(units, cnt, r0, r1);
        units += cnt;
        if (cnt > 0) ++S->active;
    }
    S->n_units = units;
    S->lds = dyn_lds_bytes(n_inst);
    return batch_set_grid(S, blocks_per_cu);
}

static int batch_upload(fe_batch_solver *S, hipStream_t s)
{
    FE_HIP_CHECK(hipMemcpyAsync(S->W.inst, S->inst.data(), sizeof(int4) * S->inst.size(), hipMemcpyHostToDevice, s));
    return FE_OK;
}

// Enqueue the state reset and the solve kernel (no host synchronization).
static int batch_enqueue(fe_batch_solver *S, const int32_t *rowptr, const int32_t *colind, const double *val,
                         const double *b, double *u, double rtol, int32_t maxit, hipStream_t s, bool cooperative)
{
    const int32_t nfill = BF_COUNT * S->n_inst > BAR_WORDS ? BF_COUNT * S->n_inst : BAR_WORDS;
    hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)cdiv(nfill, 256)), dim3(256), 0, s, S->W.bar, S->W.flag,
                       S->n_inst, S->active);
    FE_HIP_CHECK(hipGetLastError());
    BatchArgs A{};
    A.n_inst = S->n_inst;
    A.inst = S->W.inst;
    A.rowptr = rowptr;
    A.colind = colind;
    A.val = val;
    A.b = b;
    A.x = u;
    A.r = S->W.r;
    A.z = S->W.z;
    A.p0 = S->W.p0;
    A.p1 = S->W.p1;
    A.q = S->W.q;
    A.dinv = S->W.dinv;
    A.part = S->W.part;
    A.scal = S->W.scal;
    A.flag = S->W.flag;
    A.bar = S->W.bar;
    A.n_units = S->n_units;
    A.rtol = rtol;
    A.maxit = maxit;
    A.spin_limit = 500000000;   // 5 s at 100 MHz
    if (cooperative) {
        void *args[] = {&A};
        FE_HIP_CHECK(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_batch_pcg),
                                                dim3((unsigned)S->grid), dim3(BB), args, (unsigned)S->lds, s));
    } else {
        hipLaunchKernelGGL(k_batch_pcg, dim3((unsigned)S->grid), dim3(BB), S->lds, s, A);
        FE_HIP_CHECK(hipGetLastError());
    }
    return FE_OK;
}

// Read back per-instance results (synchronizes).
static int batch_results(fe_batch_solver *S, int32_t *iters, double *relres, hipStream_t s)
{
    std::vector<int32_t> fl((size_t)BF_COUNT * S->n_inst);
    std::vector<double> sc((size_t)BS_COUNT * S->n_inst);
    uint32_t bar[BAR_WORDS];
    FE_HIP_CHECK(hipMemcpyAsync(fl.data(), S->W.flag, sizeof(int32_t) * fl.size(), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipMemcpyAsync(sc.data(), S->W.scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipMemcpyAsync(bar, S->W.bar, sizeof(bar), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (bar[BAR_ABORT]) return FE_ELIMIT;
    int rc = FE_OK;
    for (int32_t k = 0; k < S->n_inst; ++k) {
        const int32_t *f = fl.data() + BF_COUNT * k;
        const double *c = sc.data() + BS_COUNT * k;
        const bool empty = S->inst[k].y == 0;
        if (f[BF_BAD]) rc = FE_EINVAL;
        if (iters) iters[k] = f[BF_ITER];
        if (relres) relres[k] = empty ? 0.0 : sqrt(c[BS_RR] / c[BS_BB]);
        if (!empty && !f[BF_DONE] && rc == FE_OK) rc = FE_ENOCONV;
    }
    return rc;
}

extern "C" int fe_batch_solve_workspace_bytes(int64_t n, int32_t n_inst, size_t *bytes)
{
    if (n <= 0 || n >= INT32_MAX || n_inst <= 0 || !bytes) return FE_EINVAL;
    if (n_inst > MAX_INST) return FE_ELIMIT;
    *bytes = batch_layout(n, n_inst, nullptr, nullptr);
    return FE_OK;
}

extern "C" int fe_batch_solve(int32_t n_inst, const int64_t *inst_row_off, const int32_t *rowptr,
                              const int32_t *colind, const double *val, const double *b, double *u, double rtol,
                              int32_t maxit, int32_t blocks_per_cu, void *ws, size_t ws_bytes, int32_t *iters,
                              double *relres, void *stream)
{
    if (!rowptr || !colind || !val || !b || !u || maxit < 0 || !(rtol >= 0.0)) return FE_EINVAL;
    fe_batch_solver S;
    int rc = batch_prepare(&S, n_inst, inst_row_off, ws, ws_bytes, blocks_per_cu);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = batch_upload(&S, s))) return rc;
    if ((rc = batch_enqueue(&S, rowptr, colind, val, b, u, rtol, maxit, s, true))) return rc;
    return batch_results(&S, iters, relres, s);
}

// ---------------------------------------------------------------------------
// Graph path: assembly of the whole batch plus the batched solve, captured into a
// hipGraph on first use and replayed while the arguments stay the same.
// ---------------------------------------------------------------------------
struct fe_batch {
    fe_plan *plan = nullptr;
    fe_batch_solver S;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t cooperative = 0, captures = 0;
    // the arguments the graph was captured with
    const double *node = nullptr, *kappa = nullptr;
    fe_fn f{}, gd{}, gn{};
    bool hf = false, hgd = false, hgn = false;
    double *val = nullptr, *val_bc = nullptr, *b = nullptr, *u = nullptr;
    const int32_t *rowptr = nullptr, *colind = nullptr;
    double rtol = 0.0;
    int32_t maxit = 0;
};

static bool same_fn(const fe_fn *a, bool has, const fe_fn &b)
{
    if (!a) return !has;
    return has && memcmp(a, &b, sizeof(fe_fn)) == 0;
}

static void drop_graph(fe_batch *B)
{
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

static int capture(fe_batch *B, const double *node, const double *kappa, const fe_fn *f, const fe_fn *g_d,
                   const fe_fn *g_n, const int32_t *rowptr, const int32_t *colind, double *val, double *val_bc,
                   double *b, double *u, double rtol, int32_t maxit, bool cooperative)
{
    hipStream_t cs;
    FE_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int rc = FE_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = FE_EHIP;
    if (rc == FE_OK) rc = fe_assemble(B->plan, node, kappa, f, g_d, g_n, val, val_bc, b, nullptr, B->S.W.isd, cs);
    if (rc == FE_OK) rc = fe_select(B->S.n, B->S.W.isd, b, nullptr, u, cs);   // start vector: g_D, else 0
    if (rc == FE_OK) rc = batch_enqueue(&B->S, rowptr, colind, val_bc, b, u, rtol, maxit, cs, cooperative);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (rc == FE_OK && (e != hipSuccess || !g)) rc = FE_EHIP;
    hipGraphExec_t x = nullptr;
    if (rc == FE_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) rc = FE_EHIP;
    if (rc != FE_OK) {
        (void)hipGetLastError();
        if (g) hipGraphDestroy(g);
        return rc;
    }
    B->graph = g;
    B->exec = x;
    B->cooperative = cooperative ? 1 : 0;
    ++B->captures;
    return FE_OK;
}

extern "C" int fe_batch_create(fe_plan *plan, int32_t n_inst, const int64_t *inst_node_off, int32_t blocks_per_cu,
                               void *ws, size_t ws_bytes, fe_batch **out, void *stream)
{
    if (!plan || !out || !inst_node_off || n_inst <= 0) return FE_EINVAL;
    if (inst_node_off[n_inst] != plan->N) return FE_EINVAL;
    fe_batch *B = new (std::nothrow) fe_batch();
    if (!B) return FE_EINVAL;
    int rc = batch_prepare(&B->S, n_inst, inst_node_off, ws, ws_bytes, blocks_per_cu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rc == FE_OK) rc = batch_upload(&B->S, s);
    if (rc == FE_OK && hipStreamSynchronize(s) != hipSuccess) rc = FE_EHIP;
    if (rc) {
        delete B;
        return rc;
    }
    B->plan = plan;
    *out = B;
    return FE_OK;
}

extern "C" int fe_batch_set_grid(fe_batch *B, int32_t blocks_per_cu)
{
    if (!B) return FE_EINVAL;
    const int32_t old = B->S.blocks_per_cu;
    int rc = batch_set_grid(&B->S, blocks_per_cu);
    if (rc) {
        batch_set_grid(&B->S, old);
        return rc;
    }
    drop_graph(B);
    return FE_OK;
}

extern "C" int fe_batch_get_info(const fe_batch *B, fe_batch_info *info)
{
    if (!B || !info) return FE_EINVAL;
    info->n_inst = B->S.n_inst;
    info->n_units = B->S.n_units;
    info->n_rows = B->S.n;
    info->grid = B->S.grid;
    info->blocks_per_cu = B->S.blocks_per_cu;
    info->max_blocks_per_cu = B->S.max_per_cu;
    info->cooperative = B->cooperative;
    info->captures = B->captures;
    return FE_OK;
}

extern "C" int fe_batch_assemble_solve(fe_batch *B, const double *node, const double *kappa, const fe_fn *f,
                                       const fe_fn *g_d, const fe_fn *g_n, const int32_t *rowptr,
                                       const int32_t *colind, double *val, double *val_bc, double *b, double *u,
                                       double rtol, int32_t maxit, int32_t *iters, double *relres, void *stream)
{
    if (!B || !node || !kappa || !rowptr || !colind || !val || !val_bc || !b || !u || maxit < 0 || !(rtol >= 0.0))
        return FE_EINVAL;
    if (!B->plan->pattern_done) return FE_EINVAL;
    if (!devfn_valid(f, false) || !devfn_valid(g_d, false) || !devfn_valid(g_n, true)) return FE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool same = B->exec && B->node == node && B->kappa == kappa && same_fn(f, B->hf, B->f) &&
                      same_fn(g_d, B->hgd, B->gd) && same_fn(g_n, B->hgn, B->gn) && B->rowptr == rowptr &&
                      B->colind == colind && B->val == val && B->val_bc == val_bc && B->b == b && B->u == u &&
                      B->rtol == rtol && B->maxit == maxit;
    if (!same) {
        drop_graph(B);
        int rc = capture(B, node, kappa, f, g_d, g_n, rowptr, colind, val, val_bc, b, u, rtol, maxit, true);
        if (rc != FE_OK) rc = capture(B, node, kappa, f, g_d, g_n, rowptr, colind, val, val_bc, b, u, rtol, maxit,
                                      false);
        if (rc != FE_OK) return rc;
        B->node = node;
        B->kappa = kappa;
        B->hf = f != nullptr;
        B->hgd = g_d != nullptr;
        B->hgn = g_n != nullptr;
        if (f) B->f = *f;
        if (g_d) B->gd = *g_d;
        if (g_n) B->gn = *g_n;
        B->rowptr = rowptr;
        B->colind = colind;
        B->val = val;
        B->val_bc = val_bc;
        B->b = b;
        B->u = u;
        B->rtol = rtol;
        B->maxit = maxit;
    }
    FE_HIP_CHECK(hipGraphLaunch(B->exec, s));
    int rc = batch_results(&B->S, iters, relres, s);
    const int st = fe_plan_status(B->plan, stream);
    return st != FE_OK ? st : rc;
}

extern "C" int fe_batch_destroy(fe_batch *B)
{
    if (!B) return FE_OK;
    drop_graph(B);
    delete B;
    return FE_OK;
}
