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

enum { BS_RR = 0, BS_BB, BS_COUNT = 2 };                 // doubles per instance (reported)
enum { BF_DONE = 0, BF_ITER, BF_BAD, BF_COUNT = 4 };     // ints per instance
// Barrier words: top-level count, generation, abort flag, running instances, then
// one arrival counter per group of blocks (blocks b with b % NGROUP == g), each in
// its own 256-byte line.
constexpr int NGROUP = 8;
enum { BAR_TOP = 0, BAR_GEN = 1, BAR_ABORT = 2, BAR_ACTIVE = 3, BAR_GROUP = 64, BAR_GSTRIDE = 64 };
constexpr int BAR_WORDS = BAR_GROUP + NGROUP * BAR_GSTRIDE;

struct BatchArgs {
    int32_t n_inst, n_units;
    const int4 *inst;     // per instance: (first unit, unit count, first row, end row)
    const int32_t *rowptr, *colind;
    const double *val, *b;
    double *x, *r, *z, *p0, *p1, *q, *dinv;
    double *pq, *rz[2], *rr[2], *bbp;   // per-unit partial sums
    double *scal;         // BS_COUNT * n_inst
    int32_t *flag;        // BF_COUNT * n_inst
    uint32_t *bar;        // BAR_WORDS
    double rtol;
    int32_t maxit;
    int64_t spin_limit;   // in s_memrealtime ticks (100 MHz)
};

FE_DEV uint32_t ld_u32(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
FE_DEV int32_t ld_i32(const int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Device-wide barrier with a bounded wait.  Arrivals count first per group of
// blocks, then the last block of each group counts at the top; only thread 0 of a
// block issues the device-scope release and acquire (the block's other threads are
// ordered through the workgroup barriers around it).
FE_DEV void grid_barrier(uint32_t *bar, int64_t spin_limit)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t G = gridDim.x;
        const uint32_t g = blockIdx.x % NGROUP;
        const uint32_t ng = G / NGROUP + (g < G % NGROUP ? 1u : 0u);
        const uint32_t ngroups = G < (uint32_t)NGROUP ? G : (uint32_t)NGROUP;
        uint32_t *cnt = bar + BAR_GROUP + BAR_GSTRIDE * g;
        const uint32_t gen = ld_u32(bar + BAR_GEN);
        bool released = false;
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ng - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(bar + BAR_TOP, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                ngroups - 1) {
                __hip_atomic_store(bar + BAR_TOP, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(bar + BAR_GEN, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (ld_u32(bar + BAR_GEN) == gen) {
                if (ld_u32(bar + BAR_ABORT)) break;
                __builtin_amdgcn_s_sleep(1);
                if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > spin_limit) {
                    __hip_atomic_fetch_or(bar + BAR_ABORT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// NV block sums at once, each with block_sum's wavefront tree and wave order, so each
// result equals block_sum of that value.  Results valid in thread 0.
template <int NV> FE_DEV void block_sum_n(double *v, double *lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        if (lane == 0) lds[k * (BB / 64) + wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < BB / 64; ++w) s += lds[k * (BB / 64) + w];
            v[k] = s;
        }
    __syncthreads();
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

struct Unit {
    int32_t inst, u0, u, row0, row1, count;   // u0: the instance's first unit
};

// Virtual unit v (0 <= v < L.units) -> its instance and rows.
FE_DEV Unit unit_of(const Active &L, int32_t v)
{
    int32_t lo = 0, hi = L.nact - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (L.pre[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    const int4 a = L.ainst[lo];
    const int32_t local = v - L.pre[lo];
    Unit t;
    t.inst = a.x;
    t.u0 = a.y;
    t.u = a.y + local;
    t.row0 = a.z + local * BB;
    t.row1 = (a.w - t.row0 < BB) ? a.w : t.row0 + BB;
    t.count = L.pre[lo + 1] - L.pre[lo];
    return t;
}

// Sums over an instance's units of up to four partial arrays, each in the fixed
// order of cg_sum_partials; broadcast to every thread through `bc`.
template <int NV>
FE_DEV void instance_sums(const double *const *arr, int32_t u0, int32_t count, double *lds, double *bc, double *out)
{
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        v[k] = 0.0;
        for (int32_t j = threadIdx.x; j < count; j += BB) v[k] += arr[k][u0 + j];
    }
    block_sum_n<NV>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) bc[k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = bc[k];
    __syncthreads();
}

// This block's contiguous share of the running units.
FE_DEV void block_range(int32_t units, int32_t vb, int32_t *v0, int32_t *v1)
{
    const int32_t per = (int32_t)((units + gridDim.x - 1) / gridDim.x);
    const int64_t a = (int64_t)vb * per;
    *v0 = (int32_t)(a < units ? a : units);
    *v1 = (*v0 + per < units) ? *v0 + per : units;
}

// Record the stopping state of instance k (one block per instance does this).
FE_DEV void record(const BatchArgs &A, int32_t k, bool done, int32_t iters, double RR, double BBv)
{
    int32_t *fl = A.flag + BF_COUNT * k;
    A.scal[BS_COUNT * k + BS_RR] = RR;
    A.scal[BS_COUNT * k + BS_BB] = BBv;
    fl[BF_ITER] = iters;
    if (done) {
        fl[BF_DONE] = 1;
        __hip_atomic_fetch_sub(A.bar + BAR_ACTIVE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// K units per step: every thread owns row t of each of the K units, so K independent
// row walks overlap their loads; reductions stay per unit.  CH: entries per chunk of
// the row walk (fewer registers for smaller chunks, hence more workgroups per CU).
template <int K, int CH>
__global__ __launch_bounds__(BB) void k_batch_pcg(BatchArgs A)
{
    extern __shared__ int4 dyn[];
    __shared__ double lds[4 * K * (BB / 64)];
    __shared__ double bc[4];
    __shared__ int32_t scan_lds[2 * (BB / 64)];
    __shared__ int32_t s_flag;
    Active L;
    L.ainst = dyn;
    L.pre = reinterpret_cast<int32_t *>(dyn + A.n_inst);
    const int32_t G = gridDim.x;
    // blocks b and b + 8 run on the same XCD: give each XCD a contiguous range of units
    const int32_t vb = (G % 8 == 0) ? (int32_t)(blockIdx.x % 8) * (G / 8) + (int32_t)(blockIdx.x / 8)
                                    : (int32_t)blockIdx.x;
    const int tid = threadIdx.x;
    uint32_t seen = 0;
    if (tid == 0) seen = ld_u32(A.bar + BAR_ACTIVE);
    build_active(A, L, scan_lds);
    int32_t v0, v1;
    block_range(L.units, vb, &v0, &v1);

    // ---- r = b - A x, diag, z = r / diag, p_old = 0; partials r.z, r.r, b.b
    for (int32_t v = v0; v < v1; v += K) {
        Unit t[K];
        double red[3 * K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            red[3 * j] = red[3 * j + 1] = red[3 * j + 2] = 0.0;
            if (v + j >= v1) continue;
            t[j] = unit_of(L, v + j);
            const int32_t i = t[j].row0 + tid;
            if (i < t[j].row1) {
                double ri, d;
                cg_init_row(i, A.rowptr, A.colind, A.val, A.b, A.x, &ri, &d);
                if (!(d > 0.0)) atomicOr(A.flag + BF_COUNT * t[j].inst + BF_BAD, 1);
                const double di = 1.0 / d;
                A.dinv[i] = di;
                A.r[i] = ri;
                A.z[i] = ri * di;
                A.p0[i] = 0.0;
                red[3 * j] = ri * ri * di;
                red[3 * j + 1] = ri * ri;
                red[3 * j + 2] = A.b[i] * A.b[i];
            }
        }
        block_sum_n<3 * K>(red, lds);
        if (tid == 0)
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (v + j < v1) {
                    A.rz[0][t[j].u] = red[3 * j];
                    A.rr[0][t[j].u] = red[3 * j + 1];
                    A.bbp[t[j].u] = red[3 * j + 2];
                }
    }
    grid_barrier(A.bar, A.spin_limit);

    int32_t it = 0;
    for (; it < A.maxit; ++it) {
        if (tid == 0) {
            const uint32_t act = ld_u32(A.bar + BAR_ACTIVE);
            s_flag = (ld_u32(A.bar + BAR_ABORT) ? 2 : 0) | (act == 0 ? 1 : 0) | (act != seen ? 4 : 0);
            seen = act;
        }
        __syncthreads();
        const int32_t fl = s_flag;
        __syncthreads();
        if (fl & 3) break;
        if (fl & 4) {
            build_active(A, L, scan_lds);
            block_range(L.units, vb, &v0, &v1);
        }
        const int cur = it & 1;
        const double *pold = cur ? A.p1 : A.p0;
        double *pnew = cur ? A.p0 : A.p1;
        // ---- phase A: stopping test and beta per instance; p = z + beta p_old, q = A p
        int32_t ci = -1;
        double c_beta = 0.0;
        bool c_done = false;
        for (int32_t v = v0; v < v1; v += K) {
            Unit t[K];
            bool ok[K];
            double beta[K];
            int32_t rows[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                ok[j] = false;
                beta[j] = 0.0;
                rows[j] = 0;
                if (v + j >= v1) continue;
                t[j] = unit_of(L, v + j);
                if (t[j].inst != ci) {
                    const double *arr[4] = {A.rz[cur], A.rr[cur], A.bbp, A.rz[cur ^ 1]};
                    double S[4];
                    instance_sums<4>(arr, t[j].u0, t[j].count, lds, bc, S);
                    const double bn2 = S[2] > 0.0 ? S[2] : 1.0;
                    ci = t[j].inst;
                    c_done = S[1] <= A.rtol * A.rtol * bn2;
                    c_beta = it == 0 ? 0.0 : S[0] / S[3];
                    // the block holding the instance's first unit records the result
                    if (c_done && tid == 0 && t[j].u == t[j].u0) record(A, ci, true, it, S[1], bn2);
                }
                rows[j] = t[j].row0 + tid;
                ok[j] = !c_done && rows[j] < t[j].row1;
                beta[j] = c_beta;
                if (c_done) t[j].count = 0;   // mark: no partial for this slot
            }
            double s[K];
            cg_apply_rows<K, CH>(rows, ok, A.rowptr, A.colind, A.val, A.z, pold, beta, s);
            double red[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                red[j] = 0.0;
                if (ok[j]) {
                    const int32_t i = rows[j];
                    const double pi = A.z[i] + beta[j] * pold[i];
                    pnew[i] = pi;
                    A.q[i] = s[j];
                    red[j] = pi * s[j];
                }
            }
            block_sum_n<K>(red, lds);
            if (tid == 0)
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if (v + j < v1 && t[j].count > 0) A.pq[t[j].u] = red[j];
        }
        grid_barrier(A.bar, A.spin_limit);
        if (ld_u32(A.bar + BAR_ABORT)) break;
        // ---- phase B: alpha per instance; x += alpha p, r -= alpha q, z = r / diag
        ci = -1;
        double c_alpha = 0.0;
        c_done = false;
        for (int32_t v = v0; v < v1; v += K) {
            Unit t[K];
            bool ok[K];
            double alpha[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                ok[j] = false;
                alpha[j] = 0.0;
                if (v + j >= v1) continue;
                t[j] = unit_of(L, v + j);
                if (t[j].inst != ci) {
                    ci = t[j].inst;
                    c_done = ld_i32(A.flag + BF_COUNT * ci + BF_DONE) != 0;
                    if (!c_done) {
                        const double *arr[2] = {A.pq, A.rz[cur]};
                        double S[2];
                        instance_sums<2>(arr, t[j].u0, t[j].count, lds, bc, S);
                        c_alpha = S[1] / S[0];
                    }
                }
                ok[j] = !c_done && t[j].row0 + tid < t[j].row1;
                alpha[j] = c_alpha;
                if (c_done) t[j].count = 0;
            }
            double red[2 * K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                red[2 * j] = red[2 * j + 1] = 0.0;
                if (ok[j]) {
                    const int32_t i = t[j].row0 + tid;
                    A.x[i] += alpha[j] * pnew[i];
                    const double ri = A.r[i] - alpha[j] * A.q[i];
                    const double zi = ri * A.dinv[i];
                    A.r[i] = ri;
                    A.z[i] = zi;
                    red[2 * j] = ri * zi;
                    red[2 * j + 1] = ri * ri;
                }
            }
            block_sum_n<2 * K>(red, lds);
            if (tid == 0)
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if (v + j < v1 && t[j].count > 0) {
                        A.rz[cur ^ 1][t[j].u] = red[2 * j];
                        A.rr[cur ^ 1][t[j].u] = red[2 * j + 1];
                    }
        }
        grid_barrier(A.bar, A.spin_limit);
        if (ld_u32(A.bar + BAR_ABORT)) break;
    }
    // ---- iteration limit reached: final stopping test of the instances still running
    if (it == A.maxit && !ld_u32(A.bar + BAR_ABORT)) {
        if (tid == 0) {
            const uint32_t act = ld_u32(A.bar + BAR_ACTIVE);
            s_flag = act != seen ? 4 : 0;
        }
        __syncthreads();
        const int32_t fl = s_flag;
        __syncthreads();
        if (fl & 4) {
            build_active(A, L, scan_lds);
            block_range(L.units, vb, &v0, &v1);
        }
        const int cur = it & 1;
        for (int32_t v = v0; v < v1; ++v) {
            const Unit t = unit_of(L, v);
            if (t.u != t.u0) continue;
            const double *arr[2] = {A.rr[cur], A.bbp};
            double S[2];
            instance_sums<2>(arr, t.u0, t.count, lds, bc, S);
            const double bn2 = S[1] > 0.0 ? S[1] : 1.0;
            if (tid == 0) record(A, t.inst, S[0] <= A.rtol * A.rtol * bn2, it, S[0], bn2);
        }
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

constexpr int NPART = 6;   // pq, rz[2], rr[2], bb

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
         *q = take(8 * (size_t)n), *d = take(8 * (size_t)n), *part = take(8 * NPART * (size_t)U),
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

// The instantiation for K units per step at `per_cu` workgroups per compute unit:
// one unit per step takes 8-entry row chunks up to 4 workgroups per compute unit
// and 4-entry chunks (fewer registers) for 5.
const void *pcg_kernel(int K, int per_cu)
{
    if (K == 1) {
        if (per_cu <= 4) return reinterpret_cast<const void *>(&k_batch_pcg<1, 8>);
        return reinterpret_cast<const void *>(&k_batch_pcg<1, 4>);
    }
    if (K == 2) return reinterpret_cast<const void *>(&k_batch_pcg<2, 2>);
    return reinterpret_cast<const void *>(&k_batch_pcg<4, 2>);
}

}  // namespace

// Host side of one batched solve: the instance table, the grid, the launch.
struct fe_batch_solver {
    int32_t n_inst = 0, n_units = 0, grid = 0, blocks_per_cu = 0, max_per_cu = 0, units_per_step = 0;
    int64_t n = 0;
    size_t lds = 0;
    BatchWs W{};
    std::vector<int4> inst;
    uint32_t active = 0;
};

// Most workgroups per compute unit that a grid of the persistent kernel may use:
// the largest count that has always run co-resident on MI355X (4).  Grids of 7 per
// compute unit (the 2-entry row chunk: 68 VGPRs, no scratch, a few KB of LDS) and
// of 5 (the 4-entry chunk: 86 VGPRs) passed the occupancy query but were not all
// resident at once (5 ran once, then failed in later runs): the bounded
// device-wide wait expired.  The kernels' resources do not explain that, so grids
// above the verified count are refused rather than trusted to the query.
constexpr int32_t BATCH_VERIFIED_PER_CU = 4;

// Grid of the persistent kernel: blocks_per_cu workgroups per compute unit (0: 2)
// and units_per_step units processed together by each workgroup (1, 2 or 4; 0: 2).
static int batch_set_grid(fe_batch_solver *S, int32_t blocks_per_cu, int32_t units_per_step)
{
    if (blocks_per_cu < 0) return FE_EINVAL;
    if (units_per_step == 0) units_per_step = 2;
    if (units_per_step != 1 && units_per_step != 2 && units_per_step != 4) return FE_EINVAL;
    int dev = 0, cus = 0, per = 0, per_small = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // the most workgroups per compute unit over the instantiations of this K
    FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_small, pcg_kernel(units_per_step, 1 << 20), BB,
                                                              S->lds));
    if (per_small < 1) return FE_ELIMIT;
    if (per_small > BATCH_VERIFIED_PER_CU) per_small = BATCH_VERIFIED_PER_CU;
    int32_t want = blocks_per_cu ? blocks_per_cu : (per_small < 2 ? per_small : 2);
    FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pcg_kernel(units_per_step, want), BB, S->lds));
    if (want > per || want > BATCH_VERIFIED_PER_CU) return FE_EINVAL;   // more than fit, or than verified
    S->max_per_cu = per_small;
    S->units_per_step = units_per_step;
    int64_t g = (int64_t)cus * want;
    if (g > S->n_units) g = S->n_units;
    S->grid = (int32_t)(g > 0 ? g : 1);
    S->blocks_per_cu = want;
    return FE_OK;
}

static int batch_prepare(fe_batch_solver *S, int32_t n_inst, const int64_t *off, void *ws, size_t ws_bytes,
                         int32_t blocks_per_cu, int32_t units_per_step)
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
    return batch_set_grid(S, blocks_per_cu, units_per_step);
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
    FE_TIMED("k_batch_reset", s,
             hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)cdiv(nfill, 256)), dim3(256), 0, s, S->W.bar, S->W.flag,
                           S->n_inst, S->active));
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
    const int64_t U = S->n_units;
    A.pq = S->W.part;
    A.rz[0] = S->W.part + U;
    A.rz[1] = S->W.part + 2 * U;
    A.rr[0] = S->W.part + 3 * U;
    A.rr[1] = S->W.part + 4 * U;
    A.bbp = S->W.part + 5 * U;
    A.scal = S->W.scal;
    A.flag = S->W.flag;
    A.bar = S->W.bar;
    A.n_units = S->n_units;
    A.rtol = rtol;
    A.maxit = maxit;
    A.spin_limit = 500000000;   // 5 s at 100 MHz
    if (cooperative) {
        void *args[] = {&A};
        hipError_t e = hipSuccess;
        FE_TIMED("k_batch_pcg", s,
                 e = hipLaunchCooperativeKernel(pcg_kernel(S->units_per_step, S->blocks_per_cu),
                                                dim3((unsigned)S->grid), dim3(BB), args, (unsigned)S->lds, s));
        if (e != hipSuccess) return FE_EHIP;
    } else {
        void *args[] = {&A};
        hipError_t e = hipSuccess;
        FE_TIMED("k_batch_pcg", s,
                 e = hipLaunchKernel(pcg_kernel(S->units_per_step, S->blocks_per_cu), dim3((unsigned)S->grid),
                                     dim3(BB), args, S->lds, s));
        if (e != hipSuccess) return FE_EHIP;
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
                              int32_t maxit, int32_t blocks_per_cu, int32_t units_per_step, void *ws,
                              size_t ws_bytes, int32_t *iters, double *relres, void *stream)
{
    if (!rowptr || !colind || !val || !b || !u || maxit < 0 || !(rtol >= 0.0)) return FE_EINVAL;
    fe_batch_solver S;
    int rc = batch_prepare(&S, n_inst, inst_row_off, ws, ws_bytes, blocks_per_cu, units_per_step);
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
    int32_t launch_gen = -1;   // the plan's launch settings at capture
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

// The captured graph's persistent-solve node (the kernel and grid of the solver), or
// nullptr.
static hipGraphNode_t pcg_node(hipGraph_t g, const fe_batch_solver *S)
{
    size_t n = 0;
    if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess || n == 0) return nullptr;
    std::vector<hipGraphNode_t> nodes(n);
    if (hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return nullptr;
    const void *fn = pcg_kernel(S->units_per_step, S->blocks_per_cu);
    for (size_t i = 0; i < n; ++i) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess || kp.func != fn) continue;
        if ((int32_t)kp.gridDim.x != S->grid || (int32_t)kp.blockDim.x != BB) return nullptr;
        return nodes[i];
    }
    return nullptr;
}

// 1 if the node is a cooperative launch, 0 if not (or if the runtime cannot say).
static int32_t node_cooperative(hipGraphNode_t node)
{
    hipKernelNodeAttrValue v{};
    if (hipGraphKernelNodeGetAttribute(node, hipKernelNodeAttributeCooperative, &v) != hipSuccess) return 0;
    return v.cooperative ? 1 : 0;
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
    // The solve's node as captured: its kernel, its grid and whether it is a
    // cooperative launch, the co-residency its device-wide barrier relies on.  A
    // capture can record the cooperative launch as an ordinary kernel node; the node
    // is then marked cooperative explicitly, and the mark read back.
    int32_t coop = 0;
    hipGraphNode_t pn = nullptr;
    if (rc == FE_OK && !(pn = pcg_node(g, &B->S))) rc = FE_EHIP;   // no solve node of that kernel and grid
    if (rc == FE_OK) {
        coop = node_cooperative(pn);
        if (!coop && cooperative) {
            hipKernelNodeAttrValue v{};
            v.cooperative = 1;
            if (hipGraphKernelNodeSetAttribute(pn, hipKernelNodeAttributeCooperative, &v) == hipSuccess)
                coop = node_cooperative(pn);
            (void)hipGetLastError();
        }
    }
    hipGraphExec_t x = nullptr;
    if (rc == FE_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) rc = FE_EHIP;
    if (rc != FE_OK) {
        (void)hipGetLastError();
        if (g) hipGraphDestroy(g);
        return rc;
    }
    B->graph = g;
    B->exec = x;
    B->cooperative = coop;
    ++B->captures;
    return FE_OK;
}

extern "C" int fe_batch_create(fe_plan *plan, int32_t n_inst, const int64_t *inst_node_off, int32_t blocks_per_cu,
                               int32_t units_per_step, void *ws, size_t ws_bytes, fe_batch **out, void *stream)
{
    if (!plan || !out || !inst_node_off || n_inst <= 0) return FE_EINVAL;
    if (inst_node_off[n_inst] != plan->N) return FE_EINVAL;
    fe_batch *B = new (std::nothrow) fe_batch();
    if (!B) return FE_EINVAL;
    int rc = batch_prepare(&B->S, n_inst, inst_node_off, ws, ws_bytes, blocks_per_cu, units_per_step);
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

extern "C" int fe_batch_set_grid(fe_batch *B, int32_t blocks_per_cu, int32_t units_per_step)
{
    if (!B) return FE_EINVAL;
    const int32_t old = B->S.blocks_per_cu, oldk = B->S.units_per_step;
    int rc = batch_set_grid(&B->S, blocks_per_cu, units_per_step);
    if (rc) {
        batch_set_grid(&B->S, old, oldk);
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
    info->units_per_step = B->S.units_per_step;
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
                      B->rtol == rtol && B->maxit == maxit && B->launch_gen == B->plan->launch_gen;
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
        B->launch_gen = B->plan->launch_gen;
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
