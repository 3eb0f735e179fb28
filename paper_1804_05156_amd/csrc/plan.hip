// plan.hip -- symbolic phase: everything that depends on elem and bdflag only.
//
// The duplicate summation of `sparse` (Section 2.2) needs, for every vertex i, the
// list of element contributions to row i.  Here that list is the set of
// vertex-element incidences (t, a) with elem[a][t] = i, sorted by element, built by
// a two-level counting sort of the (dim+1)*NT incidences by vertex that uses only
// LDS atomics:
//   level 1: element chunks histogram the incidences by vertex bucket (2^bs
//            vertices per bucket) and scatter (vertex, key) pairs into buckets;
//   level 2: one block per bucket counts, places and sorts its incidences per
//            vertex entirely in LDS.
// Every per-vertex list is sorted by key t*(dim+1)+a, so sums later run in
// ascending element order whatever the thread schedule.
//
// Rows are then processed in an order chosen for memory locality, not in label
// order: vertex v gets processing position = rank of its first incidence.  For
// meshes stored element by element in a spatial order this walks the mesh in that
// order even when the vertex labels are randomly permuted, so the gathers of the
// row kernels stay within a small window.  The matrix pattern is first built in
// that order; a label-order pass then gathers whole rows into the output layout
// with coalesced stores.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>

#include "fe_internal.h"

namespace {

constexpr int EBLOCK = 256;     // element-parallel kernels
constexpr int L1B = 1024;       // threads of the level-1 kernels
constexpr int L1CH = 32768;     // elements per level-1 chunk at most
constexpr int L1CUS = 256;      // compute units: the level-1 chunk count is a multiple of it
constexpr int NBMAX = 524288;   // buckets (2^19: with 2^12 vertices each, every int32 label)
constexpr int VBMAX = 4096;     // vertices per bucket (2^bs) at most
constexpr int BKB = 256;        // threads of the bucket kernel
constexpr int BCAPMAX = 24576;  // incidences per bucket sorted in LDS at most (larger: global path)
constexpr int FINE = 1024;      // buckets per coarse bucket at most
constexpr int L1SLOTS = 512;    // coarse-to-fine blocks resident at once (2 of FB threads per CU)
constexpr int FB = 1024;        // threads of the coarse-to-fine kernel
constexpr int L1SUB = 2048;     // elements per LDS-staged sub-chunk of the level-1 scatter
static_assert(NBMAX / FINE <= L1SLOTS && L1SLOTS <= L1B, "one thread per coarse bucket in the level-1 scatter");
static_assert(L1SUB % L1B == 0, "whole sub-chunks per thread");
constexpr int RUNR = 8;         // incidences per batch in the row kernels

// Level-1 chunk of block b: contiguous chunk ranges per XCD, so the runs that
// neighbouring chunks write into one bucket are written through the same L2.
FE_DEV int32_t l1_chunk(int32_t b, int32_t nblk) { return xcd_block(b, nblk); }

// Coarse bucket of vertex v: its bucket v >> bs divided by the buckets per coarse
// bucket, as a multiply by cmul = ceil(2^32 / fine).  With q = v >> bs and
// cmul = 2^32/fine + e (0 <= e < 1), q cmul / 2^32 exceeds q / fine by less than
// 1/fine whenever q fine < 2^32, so the floor is exact: here q < NBMAX = 2^19 and
// fine <= 1024.
FE_DEV int32_t coarse_of(int32_t v, int32_t bs, uint64_t cmul)
{
    return (int32_t)(((uint64_t)(uint32_t)(v >> bs) * cmul) >> 32);
}

// Validate one element: vertex range, repeated vertices, side codes.
template <int NV>
FE_DEV int32_t check_element(const int32_t *__restrict__ elem, const int8_t *__restrict__ bd, int32_t NT, int32_t N,
                             int32_t t, int32_t *v, int8_t *code)
{
    int32_t err = 0;
    for (int a = 0; a < NV; ++a) {
        v[a] = elem[(int64_t)a * NT + t];
        if ((uint32_t)v[a] >= (uint32_t)N) err |= ERR_INDEX;
    }
    if (!err)
        for (int a = 0; a < NV; ++a)
            for (int b = a + 1; b < NV; ++b)
                if (v[a] == v[b]) err |= ERR_REPEAT;
    for (int f = 0; f < NV; ++f) {
        code[f] = bd ? bd[(int64_t)f * NT + t] : 0;
        if (code[f] < 0 || code[f] > 3) err |= ERR_BDCODE;
    }
    return err;
}

// Level 1a: validation, Dirichlet marks, histogram of incidences per coarse bucket
// (fine buckets of 2^bs vertices each).  hist1 is coarse-bucket-major:
// hist1[cb * nblk1 + chunk].  LDS: nb ints (dynamic), nb = number of coarse buckets.
template <int NV>
__global__ __launch_bounds__(L1B) void k_l1_hist(const int32_t *__restrict__ elem, const int8_t *__restrict__ bd,
                                                 int32_t NT, int32_t N, int32_t bs, uint64_t cmul, int32_t nb,
                                                 int32_t nblk1, int32_t chn, int32_t *hist1, uint8_t *isd,
                                                 int32_t *status)
{
    extern __shared__ int32_t h[];
    __shared__ int32_t block_runs;
    for (int b = threadIdx.x; b < nb; b += L1B) h[b] = 0;
    if (threadIdx.x == 0) block_runs = 0;
    __syncthreads();
    const int32_t ch = l1_chunk(blockIdx.x, nblk1);
    const int32_t t0 = ch * chn;
    const int32_t t1 = min(NT, t0 + chn);
    int32_t err = 0;
    int32_t runs = 0;   // wavefront calls with 16 or more lanes in runs of equal buckets (lane 0 counts)
    // every lane runs every trip (the counts are aggregated across the wavefront)
    for (int32_t tb = t0; tb < t1; tb += L1B) {
        const int32_t t = tb + threadIdx.x;
        int32_t v[NV];
        int8_t code[NV];
        bool ok = t < t1;
        if (ok) {
            const int32_t e = check_element<NV>(elem, bd, NT, N, t, v, code);
            err |= e;
            ok = !e;
        }
        for (int a = 0; a < NV; ++a) {
            bool r;
            wave_rank_add(h, ok ? coarse_of(v[a], bs, cmul) : 0, ok, &r);
            runs += r ? 1 : 0;
        }
        if (ok)
            for (int f = 0; f < NV; ++f)
                if (code[f] == FE_BD_DIRICHLET)
                    for (int q = 0; q < NV; ++q)
                        if (q != f) isd[v[q]] = 1;
    }
    if (err) atomicOr(status + ST_ERR, err);
    if ((threadIdx.x & 63) == 0 && runs) atomicAdd(&block_runs, runs);
    __syncthreads();
    if (threadIdx.x == 0 && block_runs) atomicAdd(status + ST_RUNS, block_runs);   // one per block
    for (int b = threadIdx.x; b < nb; b += L1B) hist1[(int64_t)b * nblk1 + ch] = h[b];
}

// Element record for label-order processing.  With the identity order the
// processing positions of an element's vertices are its labels, so elemp is the
// element array transposed to one int4 per element; each word also packs the side
// code opposite its vertex and the vertex's Dirichlet flag (EREC_CODE, EREC_DIR),
// which the final row pass would otherwise gather byte by byte.  The level-1
// scatter writes it while it reads the element array.
template <int NV>
FE_DEV void erec_words(int32_t t, const int32_t *v, int32_t NT, const int8_t *__restrict__ bd,
                       const uint8_t *__restrict__ isd, int32_t *w)
{
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        const uint32_t code = bd ? (uint32_t)bd[(int64_t)a * NT + t] : 0u;
        w[a] = v[a] | (int32_t)((code & 3u) << EREC_CODE) | (int32_t)((uint32_t)(isd[v[a]] & 1u) << EREC_DIR);
    }
}

// Level 1b: scatter (vertex, key) pairs into their coarse bucket's range.  The
// chunk is taken L1SUB elements at a time: the sub-chunk's pairs are first grouped
// by bucket in LDS (a counting sort), then stored run by run, so consecutive lanes
// store consecutive pairs of one bucket (a per-pair scattered store would cost one
// memory request per pair).  The order inside a bucket is arbitrary (LDS atomics);
// level 2 sorts it.  LDS: 2 * nb ints (dynamic), nb = number of coarse buckets.
// AGG (labels that follow the element order) also writes the element records.
template <int NV, bool AGG>
__global__ __launch_bounds__(L1B) void k_l1_scatter(const int32_t *__restrict__ elem, int32_t NT, int32_t bs,
                                                    uint64_t cmul, int32_t nb, int32_t nblk1, int32_t chn,
                                                    const int32_t *__restrict__ offs,
                                                    int2 *pairs, const int8_t *__restrict__ bd,
                                                    const uint8_t *__restrict__ isd, int4 *elemp)
{
    // Labels that follow the element order give long runs at any sub-chunk size, so
    // AGG takes half-size sub-chunks: half the LDS, twice the workgroups per CU (129^3
    // 274 -> 209 us).  Random labels need the long sub-chunks for their runs (2049^2
    // with 1024: 88 -> 111 us).
    constexpr int SUB = AGG ? L1SUB / 2 : L1SUB;
    extern __shared__ int32_t dyn[];
    __shared__ int2 buf[SUB * NV];
    __shared__ int32_t sl[2 * (L1B / 64)];
    int32_t *cur = dyn;        // next global position of each bucket
    int32_t *cnt = dyn + nb;   // sub-chunk pairs per bucket, then their LDS start
    constexpr int PER = SUB / L1B;
    const int32_t ch = l1_chunk(blockIdx.x, nblk1);
    const int tid = threadIdx.x;
    if (tid < nb) {
        cur[tid] = offs[(int64_t)tid * nblk1 + ch];
        cnt[tid] = 0;
    }
    __syncthreads();
    const int32_t t0 = ch * chn;
    const int32_t t1 = min(NT, t0 + chn);
    for (int32_t s0 = t0; s0 < t1; s0 += SUB) {
        int32_t v[PER][NV], rk[PER][NV], w[PER][NV];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int32_t t = s0 + e * L1B + tid;
#pragma unroll
            for (int a = 0; a < NV; ++a) v[e][a] = t < t1 ? elem[(int64_t)a * NT + t] : 0;
        }
        // element records: their loads go out before the ranking work, their
        // stores after it
        if (AGG)
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int32_t t = s0 + e * L1B + tid;
                if (t < t1) erec_words<NV>(t, v[e], NT, bd, isd, w[e]);
            }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int32_t t = s0 + e * L1B + tid;
#pragma unroll
            for (int a = 0; a < NV; ++a) rk[e][a] = lds_rank_add<AGG>(cnt, coarse_of(v[e][a], bs, cmul), t < t1);
        }
        if (AGG)
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int32_t t = s0 + e * L1B + tid;
                if (t < t1) elemp[t] = make_int4(w[e][0], w[e][1], w[e][2], NV == 4 ? w[e][NV - 1] : 0);
            }
        __syncthreads();
        const int32_t c = tid < nb ? cnt[tid] : 0;   // this thread's bucket count
        int32_t tot;
        const int32_t st = block_exclusive_i32<L1B>(c, sl, &tot);
        if (tid < nb) cnt[tid] = st;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int32_t t = s0 + e * L1B + tid;
            if (t < t1)
#pragma unroll
                for (int a = 0; a < NV; ++a)
                    buf[cnt[coarse_of(v[e][a], bs, cmul)] + rk[e][a]] = make_int2(v[e][a], t * NV + a);
        }
        __syncthreads();
        for (int32_t j = tid; j < tot; j += L1B) {
            const int2 pr = buf[j];
            const int32_t b = coarse_of(pr.x, bs, cmul);
            pairs[cur[b] + (j - cnt[b])] = pr;
        }
        __syncthreads();
        if (tid < nb) {
            cur[tid] += c;
            cnt[tid] = 0;
        }
        __syncthreads();
    }
}

// Level 1c: one block per coarse bucket splits it into its fine buckets: counts
// (LDS), bucket starts (fstart), then a scatter whose runs are long again.  The
// ratio fine is chosen so that all blocks are resident in one round.
template <bool AGG>
__global__ __launch_bounds__(FB) void k_l1_fine(int32_t nb, int32_t bs, int32_t fine, int32_t ncb,
                                                const int32_t *__restrict__ offs,
                                                int32_t nblk1, int64_t ninc, const int2 *__restrict__ pairs,
                                                int2 *pairs2, int32_t *fstart)
{
    static_assert(FINE <= FB, "one fine bucket per thread");
    __shared__ int32_t cnt[FINE];
    __shared__ int32_t cur[FINE];
    __shared__ int32_t sl[2 * (FB / 64)];
    const int32_t cb = blockIdx.x;
    const int32_t s = offs[(int64_t)cb * nblk1];
    const int32_t e = (cb + 1 < ncb) ? offs[(int64_t)(cb + 1) * nblk1] : (int32_t)ninc;
    if (threadIdx.x < FINE) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t fbase = cb * fine;
    for (int32_t jb = s; jb < e; jb += FB) {   // uniform trips: the counts are wavefront-aggregated
        const int32_t j = jb + threadIdx.x;
        lds_rank_add<AGG>(cnt, j < e ? (pairs[j].x >> bs) - fbase : 0, j < e);
    }
    __syncthreads();
    {
        const int f = threadIdx.x;
        int32_t tot;
        const int32_t ex = block_exclusive_i32<FB>(f < fine ? cnt[f] : 0, sl, &tot);
        if (f < fine) {
            cur[f] = s + ex;
            if (fbase + f < nb) fstart[fbase + f] = s + ex;
        }
        if (f == 0 && cb == ncb - 1) fstart[nb] = (int32_t)ninc;
    }
    __syncthreads();
    for (int32_t jb = s; jb < e; jb += FB) {
        const int32_t j = jb + threadIdx.x;
        const int2 pr = j < e ? pairs[j] : make_int2(fbase << bs, 0);
        const int32_t pos = lds_rank_add<AGG>(cur, (pr.x >> bs) - fbase, j < e);
        if (j < e) pairs2[pos] = pr;
    }
}

// Sort keys[lo, lo+n) ascending (insertion sort: lists are short).
FE_DEV void isort(int32_t *keys, int32_t lo, int32_t n)
{
    for (int32_t j = 1; j < n; ++j) {
        const int32_t x = keys[lo + j];
        int32_t m = j - 1;
        while (m >= 0 && keys[lo + m] > x) {
            keys[lo + m + 1] = keys[lo + m];
            --m;
        }
        keys[lo + m + 1] = x;
    }
}

// Sort keys[lo..lo+n) (n <= M) in registers: a bitonic network over M slots, the
// unused ones padded with INT32_MAX.  Every index is a compile-time constant once
// unrolled, so the array stays in registers; no chain of dependent LDS accesses
// as in the insertion sort.  Keys are distinct, so the result is the same.
template <int M> FE_DEV void net_sort(int32_t *keys, int32_t lo, int32_t n)
{
    int32_t a[M];
#pragma unroll
    for (int m = 0; m < M; ++m) a[m] = m < n ? keys[lo + m] : INT32_MAX;
#pragma unroll
    for (int k = 2; k <= M; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t x = a[i], y = a[l];
                    const bool up = (i & k) == 0;
                    a[i] = up ? min(x, y) : max(x, y);
                    a[l] = up ? max(x, y) : min(x, y);
                }
            }
#pragma unroll
    for (int m = 0; m < M; ++m)
        if (m < n) keys[lo + m] = a[m];
}

// One vertex list in LDS: the register network up to 32 keys, else insertion.
FE_DEV void sort_list(int32_t *keys, int32_t lo, int32_t n)
{
    if (n <= 8) net_sort<8>(keys, lo, n);
    else if (n <= 16) net_sort<16>(keys, lo, n);
    else if (n <= 32) net_sort<32>(keys, lo, n);
    else isort(keys, lo, n);
}



// Level 2: one block per bucket.  Count incidences per vertex, place them, sort
// each vertex's list, write the sorted lists, the per-vertex word (list start,
// degree, Dirichlet flag) and the first-incidence flag.  LDS holds `cap` keys and
// two counters per vertex; larger buckets are left to k_l2_bucket_global.
template <int PT>
__global__ __launch_bounds__(BKB) void k_l2_bucket(int32_t N, int32_t bs, int32_t cap,
                                                   const int32_t *__restrict__ fstart, const int2 *__restrict__ pairs,
                                                   const uint8_t *__restrict__ isd, int32_t *sorted_l, int2 *vinfo,
                                                   uint8_t *ownf)
{
    extern __shared__ int32_t dyn[];
    __shared__ int32_t sl[2 * (BKB / 64)];
    const int32_t b = blockIdx.x;
    const int32_t VB = 1 << bs;
    int32_t *keys = dyn;            // cap
    int32_t *cnt = dyn + cap;       // VB
    int32_t *cur = cnt + VB;        // VB
    const int32_t s = fstart[b], e = fstart[b + 1];
    const int32_t n = e - s;
    if (n > cap) return;
    for (int q = threadIdx.x; q < VB; q += BKB) cnt[q] = 0;
    __syncthreads();
    const int32_t vbase = b << bs;
    // PT > 0 (cap <= PT * BKB): each thread keeps its pairs (vertex offset, key) in
    // registers for the placing pass below, instead of loading them again
    int32_t vo[PT > 0 ? PT : 1], ky[PT > 0 ? PT : 1];
    if constexpr (PT > 0) {
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int32_t j = threadIdx.x + u * BKB;
            if (j < n) {
                const int2 pr = pairs[s + j];
                vo[u] = pr.x - vbase;
                ky[u] = pr.y;
            }
        }
#pragma unroll
        for (int u = 0; u < PT; ++u)
            if (threadIdx.x + u * BKB < n) atomicAdd(cnt + vo[u], 1);
    } else {
        for (int32_t j = threadIdx.x; j < n; j += BKB) atomicAdd(cnt + (pairs[s + j].x - vbase), 1);
    }
    __syncthreads();
    // exclusive scan of cnt[0..VB): each thread owns PER consecutive entries
    const int PER = (VB + BKB - 1) / BKB;
    const int q0 = threadIdx.x * PER;
    int32_t tsum = 0;
    for (int q = q0; q < q0 + PER && q < VB; ++q) tsum += cnt[q];
    int32_t tot;
    int32_t run = block_exclusive_i32<BKB>(tsum, sl, &tot);
    for (int q = q0; q < q0 + PER && q < VB; ++q) {
        const int32_t c = cnt[q];
        cur[q] = run;
        const int32_t v = vbase + q;
        if (v < N) vinfo[v] = make_int2(s + run, c | ((int32_t)isd[v] << 30));
        run += c;
    }
    __syncthreads();
    if constexpr (PT > 0) {
#pragma unroll
        for (int u = 0; u < PT; ++u)
            if (threadIdx.x + u * BKB < n) keys[atomicAdd(cur + vo[u], 1)] = ky[u];
    } else {
        for (int32_t j = threadIdx.x; j < n; j += BKB) {
            const int2 pr = pairs[s + j];
            const int32_t pos = atomicAdd(cur + (pr.x - vbase), 1);
            keys[pos] = pr.y;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < VB; q += BKB) {
        const int32_t c = cnt[q];
        if (c == 0) continue;
        const int32_t lo = cur[q] - c;   // the cursor ended at the list's end
        sort_list(keys, lo, c);
        if (ownf) ownf[keys[lo]] = 1;
    }
    __syncthreads();
    for (int32_t j = threadIdx.x; j < n; j += BKB) sorted_l[s + j] = keys[j];
}

// Level 2 for buckets above `cap` (rare: very uneven degrees): the same steps with
// the lists in global memory, one block per bucket.  `cnt` and `cursor` are
// N-sized scratch arrays.
__global__ __launch_bounds__(BKB) void k_l2_bucket_global(int32_t N, int32_t bs, int32_t cap,
                                                          const int32_t *__restrict__ fstart,
                                                          const int2 *__restrict__ pairs,
                                                          const uint8_t *__restrict__ isd, int32_t *sorted_l,
                                                          int2 *vinfo, int32_t *cnt, int32_t *cursor, uint8_t *ownf)
{
    const int32_t b = blockIdx.x;
    const int32_t VB = 1 << bs;
    const int32_t s = fstart[b], e = fstart[b + 1];
    const int32_t n = e - s;
    if (n <= cap) return;
    const int32_t vbase = b << bs;
    const int32_t vend = min(N, vbase + VB);
    for (int32_t v = vbase + threadIdx.x; v < vend; v += BKB) cnt[v] = 0;
    __syncthreads();
    for (int32_t j = threadIdx.x; j < n; j += BKB) atomicAdd(cnt + pairs[s + j].x, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = s;
        for (int32_t v = vbase; v < vend; ++v) {
            cursor[v] = run;
            run += cnt[v];
        }
    }
    __syncthreads();
    for (int32_t v = vbase + threadIdx.x; v < vend; v += BKB)
        vinfo[v] = make_int2(cursor[v], cnt[v] | ((int32_t)isd[v] << 30));
    __syncthreads();
    for (int32_t j = threadIdx.x; j < n; j += BKB) {
        const int2 pr = pairs[s + j];
        sorted_l[atomicAdd(cursor + pr.x, 1)] = pr.y;
    }
    __syncthreads();
    for (int32_t v = vbase + threadIdx.x; v < vend; v += BKB) {
        const int32_t c = cnt[v];
        if (c == 0) continue;
        const int32_t lo = cursor[v] - c;
        isort(sorted_l, lo, c);
        if (ownf) ownf[sorted_l[lo]] = 1;
    }
}


// Processing order: the vertex owned by incidence (t, a) goes to position
// ownoff[t] + (rank of a among t's owned vertices).
template <int NV>
__global__ __launch_bounds__(EBLOCK) void k_pi(const int32_t *__restrict__ elem, int32_t NT,
                                               const uint8_t *__restrict__ ownf, const int32_t *__restrict__ ownoff,
                                               const int2 *__restrict__ vinfo, int32_t *pi, int32_t *piinv,
                                               int32_t *pdeg, int32_t *inclp, uint8_t *isdp)
{
    const int32_t t = blockIdx.x * EBLOCK + threadIdx.x;
    if (t >= NT) return;
    int32_t j = ownoff[t];
    for (int a = 0; a < NV; ++a) {
        if (!ownf[(int64_t)t * NV + a]) continue;
        const int32_t v = elem[(int64_t)a * NT + t];
        const int2 vi = vinfo[v];
        pi[j] = v;
        piinv[v] = j;
        pdeg[j] = vi.y & ((1 << 30) - 1);
        inclp[j] = vi.x;
        isdp[j] = (uint8_t)((vi.y >> 30) & 1);
        ++j;
    }
}

// Vertices used by no element go after the used ones (their rows are empty); their
// relative order does not affect any value.
__global__ __launch_bounds__(EBLOCK) void k_unused(int32_t N, const int2 *__restrict__ vinfo,
                                                   const int64_t *__restrict__ nused, int32_t *pi, int32_t *piinv,
                                                   int32_t *pdeg, int32_t *inclp, uint8_t *isdp, int32_t *status)
{
    const int32_t v = blockIdx.x * EBLOCK + threadIdx.x;
    if (v >= N) return;
    if ((vinfo[v].y & ((1 << 30) - 1)) == 0) {
        const int32_t k = (int32_t)(*nused) + atomicAdd(status + ST_UNUSED, 1);
        pi[k] = v;
        piinv[v] = k;
        pdeg[k] = 0;
        inclp[k] = 0;
        isdp[k] = 0;
    }
}

// Processing order = label order, for labels that follow the element order: the
// identity permutation, and each vertex's incidence range and Dirichlet flag taken
// straight from its label-order list (the lists are contiguous in label order, so
// their starts are the exclusive prefix sums of the degrees).
__global__ __launch_bounds__(EBLOCK) void k_ident(int32_t N, int64_t ninc, const int2 *__restrict__ vinfo,
                                                  int32_t *pi, int32_t *piinv, int32_t *pincptr, int32_t *inclp,
                                                  uint8_t *isdp)
{
    const int32_t v = blockIdx.x * EBLOCK + threadIdx.x;
    if (v > N) return;
    if (v == N) {
        pincptr[N] = (int32_t)ninc;
        return;
    }
    const int2 vi = vinfo[v];
    pi[v] = v;
    piinv[v] = v;
    pincptr[v] = vi.x;
    inclp[v] = vi.x;
    isdp[v] = (uint8_t)((vi.y >> 30) & 1);
}

// Word c (0..3) of a record, by selects on the bits of c: a chain of equality tests
// compiles to branches, each of which waits for the record's load right away.
FE_DEV int32_t word_i4(const int4 &q, int c)
{
    const int32_t x = q.x, y = q.y, z = q.z, w = q.w;   // (selects of values, not of addresses)
    const int32_t lo = (c & 1) ? y : x;
    const int32_t hi = (c & 1) ? w : z;
    return (c & 2) ? hi : lo;
}
// Processing position of local vertex c of an element record.
FE_DEV int32_t sel_i4(const int4 &q, int c) { return word_i4(q, c) & EREC_POS; }

struct RowArgs {
    int32_t NT, N;
    const int32_t *elem;
    const int8_t *bd;
    const int32_t *pi, *pincptr, *inclp, *sorted_l;
    const uint8_t *isdp;
    int32_t *pinc;        // count: written; final: read (unless LBL)
    int32_t *prowptr;     // count: row lengths; final: row starts
    int32_t *elemp;       // count: written; final: read
    int32_t *colindp;     // final
    int2 *pincm;          // final
    uint32_t *prow_info;  // final
    int4 *precp;          // final
    int4 *rslot;          // 3-D register form: count: each row's column set written; final: read
    int2 *rmask;          // 3-D label-order register form: each row's Dirichlet-column mask
    int32_t *longk;       // LDS form, count: long rows appended here
    int32_t nlcap;
    const int32_t *sptr;  // 3-D sliced incidence layout (status[ST_SELL])
    int32_t *status;
};

// Sorted column set of one row, in LDS (one column of the block's array per
// thread, capacity CAP): the general form, used when a row may be long.
template <int B, int CAP> struct LdsSet {
    int32_t *cols;
    int tid, u;
    FE_DEV void init(int32_t *lds, int t, int32_t i)
    {
        cols = lds;
        tid = t;
        u = 1;
        cols[tid] = i;
    }
    // Insert c; false if the set is full.
    FE_DEV bool insert(int32_t c)
    {
        int m = 0;
        while (m < u && cols[m * B + tid] < c) ++m;
        if (m < u && cols[m * B + tid] == c) return true;
        if (u == CAP) return false;
        for (int q = u; q > m; --q) cols[q * B + tid] = cols[(q - 1) * B + tid];
        cols[m * B + tid] = c;
        ++u;
        return true;
    }
    FE_DEV int find(int32_t c) const   // position of a member
    {
        int m = 0;
        while (cols[m * B + tid] != c) ++m;
        return m;
    }
    FE_DEV int32_t at(int m) const { return cols[m * B + tid]; }
};

// The same set in CAP registers, sorted and padded with INT32_MAX.  Inserting c
// into sorted a is new[m] = max(min(a[m], c), a[m-1]) for every m (a[-1] = -inf):
// branch-free and with fixed register indices, so no LDS and no divergent loops.
// SPLIT (2-D rows, mostly at most 8 columns): while no active lane of the wavefront
// holds more than CAP/2 columns, the compares and the shift cover the lower half
// only: the upper half is padding then, which no compare can match and no shift
// needs to move.  (3-D rows fill both halves: there the vote would only cost.)
template <int CAP, bool SPLIT> struct RegSet {
    static_assert(CAP % 4 == 0, "stored as int4");
    static constexpr int HALF = CAP / 2;
    int32_t a[CAP];
    int u;
    FE_DEV void init(int32_t *, int, int32_t i)
    {
        a[0] = i;
#pragma unroll
        for (int m = 1; m < CAP; ++m) a[m] = INT32_MAX;
        u = 1;
    }
    // The whole array (padding included) to / from a row slot of CAP/4 int4.
    FE_DEV void store(int4 *slot) const
    {
#pragma unroll
        for (int q = 0; q < CAP / 4; ++q) slot[q] = make_int4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
    }
    FE_DEV void load(const int4 *slot, int n)
    {
#pragma unroll
        for (int q = 0; q < CAP / 4; ++q) {
            const int4 v = slot[q];
            a[4 * q] = v.x;
            a[4 * q + 1] = v.y;
            a[4 * q + 2] = v.z;
            a[4 * q + 3] = v.w;
        }
        u = n;
    }
    template <int W> FE_DEV bool has(int32_t c) const
    {
        bool dup = false;
#pragma unroll
        for (int m = 0; m < W; ++m) dup |= (a[m] == c);
        return dup;
    }
    template <int W> FE_DEV void shift_in(int32_t c)
    {
#pragma unroll
        for (int m = W - 1; m > 0; --m) a[m] = max(min(a[m], c), a[m - 1]);
        a[0] = min(a[0], c);
    }
    FE_DEV bool insert(int32_t c)
    {
        const bool wide = !SPLIT || __ballot(u >= HALF) != 0;   // (uniform in the wavefront)
        if (wide ? has<CAP>(c) : has<HALF>(c)) return true;
        if (u == CAP) return false;
        if (wide) shift_in<CAP>(c);
        else shift_in<HALF>(c);
        ++u;
        return true;
    }
    FE_DEV int find(int32_t c) const
    {
        const bool wide = !SPLIT || __ballot(u > HALF) != 0;
        int m = 0;
#pragma unroll
        for (int q = 0; q < HALF; ++q) m += (a[q] < c) ? 1 : 0;
        if (wide)
#pragma unroll
            for (int q = HALF; q < CAP; ++q) m += (a[q] < c) ? 1 : 0;
        return m;
    }
    FE_DEV int32_t at(int m) const   // (m is a compile-time index in the unrolled callers)
    {
        int32_t v = 0;
#pragma unroll
        for (int q = 0; q < CAP; ++q) v = (q == m) ? a[q] : v;
        return v;
    }
};

constexpr int REGCAP = 16;   // register set capacity; longer rows go to the LDS form
constexpr int REGB = 256;    // threads per block of the register form

// Per row (one thread, processing order): the sorted set of columns {i} u
// {vertices of the incident elements}.  Incidences go in batches of RUNR whose
// loads are issued together.
//   FINAL = false: copy the row's sorted incidence keys into processing order
//                  (unless LBL), record the row's position in each incident
//                  element (elemp) and write the row length (processing order).
//   FINAL = true:  write the row's columns and the per-incidence (key, metadata)
//                  words in processing order and the row record; Dirichlet flags
//                  of the columns are read in processing order through elemp, which
//                  keeps those reads local.
// REG selects the register set (capacity REGCAP): a row that does not fit sets
// ERR_RETRY and the host reruns the pass with the LDS set.  LBL: label-order
// processing (labels that follow the element order): both passes read the label-
// order lists (sorted_l), which are then local, instead of a processing-order copy,
// and take an element's vertices from its elemp record (labels, one 16-byte load)
// instead of the element array (one load per vertex); the count pass then writes
// no elemp (the level-1 scatter did).
template <int NV, bool FINAL, bool REG, bool LBL>
__global__ __launch_bounds__(REG ? REGB : RowCaps<NV>::BLOCK) void k_rows(RowArgs R)
{
    constexpr int B = REG ? REGB : RowCaps<NV>::BLOCK, COLCAP = RowCaps<NV>::COL;
    __shared__ int32_t cols[REG ? 1 : COLCAP * B];
    // 3-D register form: the finished column set is also put in LDS for the metadata
    // walk's lookups (a bisection: four LDS reads instead of 32 register compares)
    constexpr bool LFIND = REG && NV == 4;
    __shared__ int32_t sset[LFIND ? REGCAP * B : 1];
    // 3-D label-order count pass: the wavefront's rows read one contiguous range of the
    // label-order lists (both walks read it); it is loaded once into LDS with whole-line
    // loads, and the walks take their keys from there
    constexpr bool KLD = REG && NV == 4 && LBL && !FINAL;
    constexpr int KLCAP = 1536;   // keys per wavefront (64 rows of 24); longer ranges read directly
    __shared__ int32_t klds[KLD ? KLCAP * (B / 64) : 1];
    // General-path count pass: the keys a wavefront copies (its rows' incidence lists,
    // one contiguous range of pinc) are gathered in LDS and stored together, a full
    // line per store, instead of 4 bytes per lane at each row's own place
    constexpr bool STG = REG && !FINAL && !LBL;
    constexpr int KCAP = 512;   // 2-D keys per wavefront (64 rows of 8); longer ranges go direct
    constexpr int KCAPS = NV == 3 ? KCAP : 2048;   // (3-D: 64 rows of 32)
    __shared__ int32_t kst[STG ? KCAPS * (B / 64) : 1];
    // 2-D final pass, the same for a wavefront's (key, metadata) words and columns
    constexpr bool STF = REG && NV == 3 && FINAL;
    __shared__ int2 mst[STF ? KCAP * (B / 64) : 1];
    // (and, in both dimensions, the final pass's columns; 3-D: 64 rows of 16)
    constexpr int CCAP = NV == 3 ? KCAP : 1024;
    __shared__ int32_t cst[(REG && FINAL) ? CCAP * (B / 64) : 1];
    using Set = typename std::conditional<REG, RegSet<REGCAP, NV == 3>, LdsSet<B, COLCAP>>::type;
    constexpr int SETCAP = REG ? REGCAP : COLCAP;
    const int tid = threadIdx.x;
    // 3-D: contiguous rows per XCD (neighbours lie about N^(2/3) positions apart, a
    // window that interleaved blocks would need in every XCD's L2)
    const int32_t k = (NV == 4 && !FINAL ? xcd_block(blockIdx.x, gridDim.x) : (int32_t)blockIdx.x) * B + tid;
    if (k >= R.N) return;
    const int32_t i = R.pi[k];
    const int32_t s = R.pincptr[k];
    const int32_t d = R.pincptr[k + 1] - s;
    if (d == 0) {   // vertex of no element: empty row, as sparse() would give
        if (!FINAL) {
            R.prowptr[k] = 0;
        } else {
            R.prow_info[k] = 0;
            R.precp[k] = make_int4(R.prowptr[k], 0, 0, 0);
        }
        return;
    }
    // a long row (more columns than the LDS set holds) is left to k_rows_long
    if (FINAL && !REG && R.prowptr[k + 1] - R.prowptr[k] > SETCAP) return;
    const bool from_pinc = FINAL && !LBL;
    // general path: the count pass writes the element record words of this row's
    // vertex (position, side code opposite it, its Dirichlet flag)
    const int32_t rowdir = (!FINAL && !LBL && R.isdp[k]) ? (int32_t)(1u << EREC_DIR) : 0;
    const int32_t src = from_pinc ? s : R.inclp[k];
    const int32_t *klist = from_pinc ? R.pinc : R.sorted_l;
    Set set;
    bool ok = true;
    const int32_t *kl = klist + src;   // this row's keys
    if constexpr (KLD) {
        const uint64_t act = __ballot(1);
        const int last = 63 - __clzll((long long)act);
        const int32_t kb = __builtin_amdgcn_readfirstlane(src);
        const int32_t kn = __builtin_amdgcn_readfirstlane(__shfl(src + d, last)) - kb;
        if (kn <= KLCAP) {
            int32_t *kw = klds + __builtin_amdgcn_readfirstlane(tid >> 6) * KLCAP;
            const int nact = __popcll(act);
            const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
            for (int32_t j = r; j < kn; j += nact) kw[j] = klist[kb + j];
            wave_lds_sync();
            kl = kw + (src - kb);
        }
    }
    // the wavefront's range of pinc (its active lanes' rows are consecutive positions)
    // (wavefront-uniform values, read through the first lane so they sit in scalar
    // registers)
    int32_t *wk = kst + (STG ? __builtin_amdgcn_readfirstlane(tid >> 6) * KCAPS : 0);
    int32_t wbase = 0, wlen = 0;
    bool staged = false;
    if constexpr (STG) {
        const uint64_t act = __ballot(1);
        const int last = 63 - __clzll((long long)act);
        wbase = __builtin_amdgcn_readfirstlane(s);
        wlen = __builtin_amdgcn_readfirstlane(__shfl(s + d, last) - wbase);
        staged = wlen <= KCAPS;
    }
    // The side codes and Dirichlet flags of an incidence's other vertices, three bits
    // each (code, then flag), from its element record.  Taken as soon as the record is
    // loaded, so that its four registers are free again while the set is formed
    // (2-D final pass: 107 -> 84 VGPRs, 4 -> 5 waves per SIMD, 287 -> 278 us).
    static_assert(EREC_DIR == EREC_CODE + 2, "code and flag are adjacent");
    auto flags_of = [&](int32_t key, const int4 &ep) -> uint32_t {
        const int a = key % NV;
        uint32_t fl = 0;
#pragma unroll
        for (int jj = 0; jj < NV - 1; ++jj)
            fl |= (((uint32_t)word_i4(ep, fe_other<NV>(a, jj)) >> EREC_CODE) & 7u) << (3 * jj);
        return fl;
    };
    // Metadata word of one incidence (local vertex, column offsets of the other
    // vertices, Dirichlet / Neumann / Robin bits), from its key, the flags above and
    // the other vertices' labels; adds its Dirichlet columns to dmask.
    auto meta_of = [&](int32_t key, uint32_t fl, const int32_t *c, uint64_t &dmask) -> uint32_t {
        const int a = key % NV;
        uint32_t meta = (uint32_t)a;
#pragma unroll
        for (int jj = 0; jj < NV - 1; ++jj) {
            const uint32_t wb = (fl >> (3 * jj)) << EREC_CODE;   // packed code and flag
            const int m = set.find(c[jj]);                       // present by construction
            meta |= (uint32_t)m << (Meta<NV>::OFF + Meta<NV>::OB * jj);
            if ((wb >> EREC_DIR) & 1u) {
                meta |= 1u << (Meta<NV>::DBIT + jj);
                dmask |= 1ull << m;
            }
            const uint32_t code = (wb >> EREC_CODE) & 3u;
            if (code == FE_BD_NEUMANN) meta |= 1u << (Meta<NV>::NBIT + jj);
            if (code == FE_BD_ROBIN) meta |= 1u << (Meta<NV>::RBIT + jj);
        }
        return meta;
    };
    // Final pass: the row's columns and its row record.
    auto finish = [&](uint64_t dmask, int32_t *cw = nullptr) {   // cw: columns to LDS, at ps - cw's base
        const int u = set.u;
        const int32_t ps = R.prowptr[k];
        int diag = 0;
#pragma unroll
        for (int m = 0; m < SETCAP; ++m) {
            if (m >= u) break;
            const int32_t c = set.at(m);
            if (cw) cw[m] = c;
            else R.colindp[ps + m] = c;
            if (c == i) diag = m;
        }
        const uint32_t info = (uint32_t)u | ((uint32_t)diag << 8) | ((uint32_t)(R.isdp[k] ? 1 : 0) << 16);
        R.prow_info[k] = info;
        R.precp[k] = make_int4(ps, (int32_t)info, (int32_t)(uint32_t)dmask, (int32_t)(uint32_t)(dmask >> 32));
    };
    // 2-D final pass, rows of at most RUNR incidences (nearly every row): one walk.
    // The keys, element records and labels loaded to form the column set stay in
    // registers for the metadata words, instead of a second walk that loads them again.
    constexpr bool FUSE = FINAL && REG && NV == 3;
    if constexpr (FUSE) {
        // the wavefront's ranges of pincm and colindp, staged when every row takes
        // the one walk and both ranges fit
        const uint64_t act = __ballot(1);
        const int last = 63 - __clzll((long long)act);
        const int32_t ps0 = R.prowptr[k], pe0 = R.prowptr[k + 1];
        const int32_t mb = __builtin_amdgcn_readfirstlane(s);
        const int32_t ml = __builtin_amdgcn_readfirstlane(__shfl(s + d, last)) - mb;
        const int32_t cb = __builtin_amdgcn_readfirstlane(ps0);
        const int32_t cl = __builtin_amdgcn_readfirstlane(__shfl(pe0, last)) - cb;
        const bool stg = __all(d <= RUNR) && ml <= KCAP && cl <= CCAP;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
        int2 *mw = mst + wv * KCAP;
        int32_t *cw = cst + wv * CCAP;
        if (d <= RUNR) {
            int32_t key[RUNR];
            uint32_t fl[RUNR];
            int32_t c[RUNR][NV - 1];
            const int4 *ep4 = reinterpret_cast<const int4 *>(R.elemp);
            set.init(cols, tid, i);
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (q < d) key[q] = klist[src + q];
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (q < d) {
                    const int32_t t = key[q] / NV;
                    const int a = key[q] - t * NV;
                    const int4 ep = ep4[t];
                    fl[q] = flags_of(key[q], ep);
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj)
                        c[q][jj] = LBL ? sel_i4(ep, fe_other<NV>(a, jj)) : R.elem[(int64_t)fe_other<NV>(a, jj) * R.NT + t];
                }
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (q < d)
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj) ok = ok && set.insert(c[q][jj]);
            if (!ok) {
                atomicOr(R.status + ST_ERR, ERR_RETRY);
                return;
            }
            uint64_t dmask = 0;
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (q < d) {
                    const int2 w = make_int2(key[q], (int32_t)meta_of(key[q], fl[q], c[q], dmask));
                    if (stg) mw[s - mb + q] = w;
                    else R.pincm[s + q] = w;
                }
            finish(dmask, stg ? cw + (ps0 - cb) : nullptr);
            if (stg) {
                // (the active lanes share the stores; a row whose set overflowed left,
                // and the pass is rerun)
                wave_lds_sync();
                const uint64_t a2 = __ballot(1);
                const int nact = __popcll(a2);
                const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(a2 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)a2, 0u));
                for (int32_t j = r; j < ml; j += nact) R.pincm[mb + j] = mw[j];
                for (int32_t j = r; j < cl; j += nact) R.colindp[cb + j] = cw[j];
            }
            return;
        }
    }
    // 3-D rows (about 24 incidences, 15 columns): the count pass stores the register
    // set and the final pass loads it instead of walking the incidences again.  In
    // 2-D (6 incidences) the stores cost the count pass more than the walk costs.
    constexpr bool SLOT = REG && NV == 4;
    if constexpr (FINAL && SLOT) {
        // the count pass left the row's column set in its slot
        set.load(R.rslot + (int64_t)k * (REGCAP / 4), R.prowptr[k + 1] - R.prowptr[k]);
    } else {
        set.init(cols, tid, i);
        for (int32_t j0 = 0; j0 < d && ok; j0 += RUNR) {
            int32_t key[RUNR];
            int32_t c[RUNR][NV - 1];
            int32_t code[RUNR];
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d) key[q] = kl[j0 + q];
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d) {
                    const int32_t t = key[q] / NV;
                    const int a = key[q] - t * NV;
                    if (!FINAL && !LBL) code[q] = R.bd ? (int32_t)(R.bd[(int64_t)a * R.NT + t] & 3) : 0;
                    if (LBL) {
                        const int4 e4 = reinterpret_cast<const int4 *>(R.elemp)[t];
#pragma unroll
                        for (int jj = 0; jj < NV - 1; ++jj) c[q][jj] = sel_i4(e4, fe_other<NV>(a, jj));
                    } else {
#pragma unroll
                        for (int jj = 0; jj < NV - 1; ++jj)
                            c[q][jj] = R.elem[(int64_t)fe_other<NV>(a, jj) * R.NT + t];
                    }
                }
            if (!FINAL && !LBL)   // stores after all of the batch's loads
#pragma unroll
                for (int q = 0; q < RUNR; ++q)
                    if (j0 + q < d) {
                        const int32_t t = key[q] / NV;
                        const int a = key[q] - t * NV;
                        if (staged) wk[s - wbase + j0 + q] = key[q];
                        else R.pinc[s + j0 + q] = key[q];
                        R.elemp[(int64_t)t * 4 + a] = k | (int32_t)((uint32_t)code[q] << EREC_CODE) | rowdir;
                    }
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d)
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj) ok = ok && set.insert(c[q][jj]);
        }
    }
    if constexpr (STG) {
        // (every lane of the wavefront that walked a row is here: the active lanes share
        // the stores; a row whose set overflowed stops early, and the pass is rerun)
        if (staged) {
            wave_lds_sync();
            const uint64_t act = __ballot(1);
            const int nact = __popcll(act);
            const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
            for (int32_t j = r; j < wlen; j += nact) R.pinc[wbase + j] = wk[j];
        }
    }
    if (!ok) {
        if (REG) {
            atomicOr(R.status + ST_ERR, ERR_RETRY);
        } else if (!FINAL) {
            // a long row: k_rows_long counts it (and writes its incidences' words)
            const int32_t j = atomicAdd(R.status + ST_NLONG, 1);
            if (j < R.nlcap) R.longk[j] = k;
            else atomicOr(R.status + ST_ERR, ERR_LIMIT);
        }
        if (!FINAL) R.prowptr[k] = 0;
        return;
    }
    // The metadata words of every incidence of the row to pincm; returns the row's
    // Dirichlet-column mask.
    auto meta_walk2 = [&]() -> uint64_t {
        uint64_t dmask = 0;
        const int4 *ep4 = reinterpret_cast<const int4 *>(R.elemp);
        const bool sell = NV == 4 && R.status[ST_SELL] != 0;
        for (int32_t j0 = 0; j0 < d; j0 += RUNR) {
            int32_t key[RUNR];
            uint32_t fl[RUNR];
            int32_t c[RUNR][NV - 1];
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d) key[q] = klist[src + j0 + q];
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d) {
                    const int32_t t = key[q] / NV;
                    const int a = key[q] - t * NV;
                    const int4 ep = ep4[t];
                    fl[q] = flags_of(key[q], ep);
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj) {
                        const int b = fe_other<NV>(a, jj);
                        // labels (LBL: the record's processing positions are the labels)
                        c[q][jj] = LBL ? (int32_t)((uint32_t)word_i4(ep, b) & EREC_POS) : R.elem[(int64_t)b * R.NT + t];
                    }
                }
#pragma unroll
            for (int q = 0; q < RUNR; ++q)
                if (j0 + q < d)
                    R.pincm[inc_at(sell, R.sptr, s, k, j0 + q)] = make_int2(key[q], (int32_t)meta_of(key[q], fl[q], c[q], dmask));
        }
        return dmask;
    };
    auto meta_walk3 = [&]() -> uint64_t {
        // Batches of 6 in the count pass (label-order processing): 90 VGPRs and 5 waves
        // per SIMD (129^3: 639 us).  With 8, 110 VGPRs and 4 waves (645 us; 148 and 3
        // waves, 691 us, before the packed flags); with 4, 70 VGPRs and 7 waves (695 us:
        // more rows in flight than the L2 serves well); 3 or 2 hold too few loads in
        // flight.
        constexpr int MB = FINAL ? RUNR : 6;
        uint64_t dmask = 0;
        const int4 *ep4 = reinterpret_cast<const int4 *>(R.elemp);
        const bool sell = NV == 4 && R.status[ST_SELL] != 0;
        for (int32_t j0 = 0; j0 < d; j0 += MB) {
            int32_t key[MB];
            int4 ep[MB];
            int32_t c[MB][NV - 1];
            uint32_t fl[MB];
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (j0 + q < d) key[q] = kl[j0 + q];
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (j0 + q < d) {
                    const int32_t t = key[q] / NV;
                    const int a = key[q] - t * NV;
                    ep[q] = ep4[t];
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj) {
                        const int b = fe_other<NV>(a, jj);
                        if (!LBL) c[q][jj] = R.elem[(int64_t)b * R.NT + t];   // labels (LBL: from ep[q])
                    }
                }
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (j0 + q < d) {
                    const int a = key[q] % NV;
                    fl[q] = flags_of(key[q], ep[q]);
                    if (LBL)
#pragma unroll
                        for (int jj = 0; jj < NV - 1; ++jj)   // processing position = label
                            c[q][jj] = sel_i4(ep[q], fe_other<NV>(a, jj));
                }
#pragma unroll
            for (int q = 0; q < MB; ++q)
                if (j0 + q < d) {
                    uint32_t meta = (uint32_t)(key[q] % NV);
#pragma unroll
                    for (int jj = 0; jj < NV - 1; ++jj) {
                        int m;   // present by construction
                        if constexpr (LFIND) {
                            const int32_t cc = c[q][jj];
                            m = (sset[7 * B + tid] < cc) ? 8 : 0;
                            m += (sset[(m + 3) * B + tid] < cc) ? 4 : 0;
                            m += (sset[(m + 1) * B + tid] < cc) ? 2 : 0;
                            m += (sset[m * B + tid] < cc) ? 1 : 0;
                        } else {
                            m = set.find(c[q][jj]);
                        }
                        meta |= (uint32_t)m << (Meta<NV>::OFF + Meta<NV>::OB * jj);
                        const uint32_t f3 = (fl[q] >> (3 * jj)) & 7u;   // code, then the flag
                        if (f3 >> 2) {
                            meta |= 1u << (Meta<NV>::DBIT + jj);
                            dmask |= 1ull << m;
                        }
                        if ((f3 & 3u) == FE_BD_NEUMANN) meta |= 1u << (Meta<NV>::NBIT + jj);
                        if ((f3 & 3u) == FE_BD_ROBIN) meta |= 1u << (Meta<NV>::RBIT + jj);
                    }
                    R.pincm[inc_at(sell, R.sptr, s, k, j0 + q)] = make_int2(key[q], (int32_t)meta);
                }
        }
        return dmask;
    };
    // (3-D keeps the walk whose loads, codes and offsets run as separate loops: that
    // schedule holds more of a batch's loads in flight than the per-incidence form)
    auto meta_walk = [&]() -> uint64_t {
        if constexpr (LFIND) {
#pragma unroll
            for (int q = 0; q < REGCAP; ++q) sset[q * B + tid] = set.a[q];   // sorted, padded
        }
        if constexpr (NV == 4) return meta_walk3();
        else return meta_walk2();
    };
    // 3-D label-order processing with stored sets: the count pass writes the
    // metadata while the row's element records are still in cache, and the final
    // pass only writes the columns and the row record.
    constexpr bool MERGE = LBL && SLOT;
    if (!FINAL) {
        if constexpr (MERGE) {
            const uint64_t dm = meta_walk();   // (puts the set in sset first)
            R.rmask[k] = make_int2((int32_t)(uint32_t)dm, (int32_t)(uint32_t)(dm >> 32));
        } else if constexpr (SLOT) {
            // (general path: the wavefront's part of the key-copy buffer, free again)
            static_assert(!SLOT || MERGE || KCAPS >= 64 * REGCAP, "room for the sets");
            wave_lds_sync();
#pragma unroll
            for (int q = 0; q < REGCAP; ++q) wk[q * 64 + (tid & 63)] = set.a[q];
        }
        if constexpr (SLOT) {
            // the wavefront's slots (64 rows of REGCAP words, contiguous) stored together
            // from the LDS copy of the sets; rows of lanes that left early (no
            // incidences: never read; an overflowed set: the pass is rerun) get whatever
            // their LDS column holds
            wave_lds_sync();
            const uint64_t act = __ballot(1);
            const int nact = __popcll(act);
            const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
            const int32_t kw0 = __builtin_amdgcn_readfirstlane(k - (tid & 63));
            const int nw = min(64, R.N - kw0) * REGCAP;
            constexpr int CS = MERGE ? B : 64;   // stride of a set's words
            const int32_t *col = MERGE ? sset + (tid & ~63) : wk;
            int32_t *slot = reinterpret_cast<int32_t *>(R.rslot) + (int64_t)kw0 * REGCAP;
            for (int j = r; j < nw; j += nact) slot[j] = col[(j % REGCAP) * CS + j / REGCAP];
        }
        R.prowptr[k] = set.u;
        return;
    }
    if constexpr (FINAL) {
        uint64_t dmask;
        if constexpr (MERGE) {
            const int2 mm = R.rmask[k];
            dmask = (uint64_t)(uint32_t)mm.x | ((uint64_t)(uint32_t)mm.y << 32);
        } else {
            dmask = meta_walk();
        }
        if constexpr (REG && NV == 4) {
            // the wavefront's columns gathered in LDS and stored together (the active
            // lanes share the stores; a row whose set overflowed left, and the pass is
            // rerun)
            const uint64_t act = __ballot(1);
            const int last = 63 - __clzll((long long)act);
            const int32_t ps0 = R.prowptr[k];
            const int32_t cb = __builtin_amdgcn_readfirstlane(ps0);
            const int32_t cl = __builtin_amdgcn_readfirstlane(__shfl(R.prowptr[k + 1], last)) - cb;
            if (cl <= CCAP) {
                int32_t *cw = cst + __builtin_amdgcn_readfirstlane(tid >> 6) * CCAP;
                finish(dmask, cw + (ps0 - cb));
                wave_lds_sync();
                const int nact = __popcll(act);
                const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
                for (int32_t j = r; j < cl; j += nact) R.colindp[cb + j] = cw[j];
                return;
            }
        }
        finish(dmask);
    }
}

// Sliced incidence layout (3-D): SELLW times the longest row of each slice of SELLW
// processing positions, then (one block) the depth W of every slice, the longest
// row of all, in sptr[0], and the choice of layout: sliced if the padded total fits
// pincm.
__global__ __launch_bounds__(256) void k_sell_len(int32_t N, const int32_t *__restrict__ pincptr, int32_t *sptr)
{
    const int32_t sl = blockIdx.x * 256 + threadIdx.x;
    const int32_t k0 = sl * SELLW;
    if (k0 >= N) return;
    const int32_t k1 = min(N, k0 + SELLW);
    int32_t m = 0;
    for (int32_t k = k0; k < k1; ++k) m = max(m, pincptr[k + 1] - pincptr[k]);
    sptr[sl] = SELLW * m;
}

__global__ __launch_bounds__(1024) void k_sell_choose(int32_t nsl, int64_t cap, int32_t *sptr, int32_t *status)
{
    __shared__ int32_t m;
    if (threadIdx.x == 0) m = 0;
    __syncthreads();
    int32_t w = 0;
    for (int32_t i = threadIdx.x; i < nsl; i += 1024) w = max(w, sptr[i]);
    atomicMax(&m, w);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t W = m / SELLW;
        sptr[0] = W;
        status[ST_SELL] = ((int64_t)nsl * SELLW * W <= cap) ? 1 : 0;
    }
}

// Long rows: rows with more columns than the LDS column set holds (a vertex with
// more than 31 neighbours in 2-D, 63 in 3-D).  One workgroup per long row forms the
// row's column set from all its incidences at once: the other vertices of every
// incident element and the vertex itself go to LDS, are sorted by a bitonic network
// and made unique.  The count form (FINAL false) records the length and, in the
// general path, writes what the count pass writes for every incidence (the
// processing-order key copy and the element record word).  The final form writes
// the columns, each incidence's metadata word (local vertex and Dirichlet /
// Neumann / Robin bits; no column offsets: the numeric long-row kernel finds them
// by search) and the row record, with INFO_LONG and the length and diagonal offset
// in the record's .z and .w.  The count form loops over the long rows counted on
// the device (any grid); the final form takes one block per row.
constexpr int LB = 256;

template <int NV, bool FINAL, bool LBL>
__global__ __launch_bounds__(LB) void k_rows_long(RowArgs R)
{
    __shared__ int32_t cand[LCAND];
    __shared__ int32_t sl[2 * (LB / 64)];
    __shared__ int32_t sh_diag;
    const int32_t nlong = min(R.status[ST_NLONG], R.nlcap);
    const int4 *ep4 = reinterpret_cast<const int4 *>(R.elemp);
    for (int32_t r = blockIdx.x; r < nlong; r += gridDim.x) {
        const int32_t k = R.longk[r];
        const int32_t i = R.pi[k];
        const int32_t s = R.pincptr[k];
        const int32_t d = R.pincptr[k + 1] - s;
        const int32_t nc = (NV - 1) * d + 1;
        if (nc > LCAND) {   // block-uniform
            if (threadIdx.x == 0) atomicOr(R.status + ST_ERR, ERR_LIMIT);
            continue;
        }
        const bool from_pinc = FINAL && !LBL;
        const int32_t src = from_pinc ? s : R.inclp[k];
        const int32_t *klist = from_pinc ? R.pinc : R.sorted_l;
        const int32_t rowdir = (!FINAL && !LBL && R.isdp[k]) ? (int32_t)(1u << EREC_DIR) : 0;
        int32_t M = 1;
        while (M < nc) M <<= 1;
        for (int32_t j = threadIdx.x; j < d; j += LB) {
            const int32_t key = klist[src + j];
            const int32_t t = key / NV;
            const int a = key - t * NV;
            int4 e4 = make_int4(0, 0, 0, 0);
            if (LBL) e4 = ep4[t];
#pragma unroll
            for (int jj = 0; jj < NV - 1; ++jj)
                cand[(NV - 1) * j + jj] = LBL ? sel_i4(e4, fe_other<NV>(a, jj))
                                              : R.elem[(int64_t)fe_other<NV>(a, jj) * R.NT + t];
            if (!FINAL && !LBL) {
                const int32_t code = R.bd ? (int32_t)(R.bd[(int64_t)a * R.NT + t] & 3) : 0;
                R.pinc[s + j] = key;
                R.elemp[(int64_t)t * 4 + a] = k | (int32_t)((uint32_t)code << EREC_CODE) | rowdir;
            }
        }
        for (int32_t j = (NV - 1) * d + threadIdx.x; j < M; j += LB) cand[j] = (j == (NV - 1) * d) ? i : INT32_MAX;
        __syncthreads();
        for (int32_t kk = 2; kk <= M; kk <<= 1)
            for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int32_t x = threadIdx.x; x < M; x += LB) {
                    const int32_t l = x ^ jj;
                    if (l > x) {
                        const int32_t p = cand[x], q = cand[l];
                        if (((x & kk) == 0) ? p > q : p < q) {
                            cand[x] = q;
                            cand[l] = p;
                        }
                    }
                }
                __syncthreads();
            }
        const int32_t ps = FINAL ? R.prowptr[k] : 0;
        int32_t u = 0;
        for (int32_t x0 = 0; x0 < M; x0 += LB) {
            const int32_t x = x0 + threadIdx.x;
            const int32_t c = x < M ? cand[x] : INT32_MAX;
            const bool first = c != INT32_MAX && (x == 0 || cand[x - 1] != c);
            int32_t tot;
            const int32_t ex = block_exclusive_i32<LB>(first ? 1 : 0, sl, &tot);
            if (FINAL && first) {
                R.colindp[ps + u + ex] = c;
                if (c == i) sh_diag = u + ex;
            }
            u += tot;
        }
        if (!FINAL) {
            if (threadIdx.x == 0) R.prowptr[k] = u;
            __syncthreads();
            continue;
        }
        const bool sell = NV == 4 && R.status[ST_SELL] != 0;
        for (int32_t j = threadIdx.x; j < d; j += LB) {
            const int32_t key = klist[src + j];
            const int32_t t = key / NV;
            const int a = key - t * NV;
            const int4 ep = ep4[t];
            uint32_t meta = (uint32_t)a;
#pragma unroll
            for (int jj = 0; jj < NV - 1; ++jj) {
                const uint32_t wb = (uint32_t)word_i4(ep, fe_other<NV>(a, jj));
                const uint32_t code = (wb >> EREC_CODE) & 3u;
                if ((wb >> EREC_DIR) & 1u) meta |= 1u << (Meta<NV>::DBIT + jj);
                if (code == FE_BD_NEUMANN) meta |= 1u << (Meta<NV>::NBIT + jj);
                if (code == FE_BD_ROBIN) meta |= 1u << (Meta<NV>::RBIT + jj);
            }
            R.pincm[inc_at(sell, R.sptr, s, k, j)] = make_int2(key, (int32_t)meta);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t info = INFO_LONG | ((uint32_t)(R.isdp[k] ? 1 : 0) << 16);
            R.prow_info[k] = info;
            R.precp[k] = make_int4(ps, (int32_t)info, u, sh_diag);
        }
        __syncthreads();
    }
}

// Label-order row records and lengths: rowrec[i] = precp[piinv[i]], rowlen[i] =
// its length (one gather per row; the stores are coalesced).
__global__ __launch_bounds__(256) void k_label_rows(int32_t N, const int32_t *__restrict__ piinv,
                                                    const int4 *__restrict__ precp, int4 *rowrec, int32_t *rowlen)
{
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int4 r = precp[piinv[i]];
    rowrec[i] = r;
    rowlen[i] = (r.y & INFO_LONG) ? r.z : (r.y & 0xff);
}

// Label-order copy of the column indices from the processing-order rows: one
// wavefront per 64 consecutive label rows, each lane writing consecutive entries
// of their (contiguous) output range, so the stores are fully coalesced; the reads
// gather whole rows of the processing-order copy.
__global__ __launch_bounds__(256) void k_pattern_to_label(int32_t N, const int32_t *__restrict__ rowptr,
                                                          const int4 *__restrict__ rowrec,
                                                          const int32_t *__restrict__ colindp, int32_t *colind)
{
    __shared__ int32_t sdst[4][65];
    __shared__ int32_t ssrc[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t i0 = (blockIdx.x * 4 + w) * 64;
    const int32_t i = i0 + lane;
    sdst[w][lane] = rowptr[min(i, N)];
    ssrc[w][lane] = (i < N) ? rowrec[i].x : 0;
    if (lane == 0) sdst[w][64] = rowptr[min(i0 + 64, N)];
    __syncthreads();
    const int32_t base = sdst[w][0];
    const int32_t total = sdst[w][64] - base;
    // CU gathers per lane in flight, then their stores
    constexpr int CU = 4;
    for (int32_t e0 = lane; e0 < total; e0 += 64 * CU) {
        int32_t v[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int32_t e = e0 + 64 * u;
            if (e >= total) break;
            const int32_t pos = base + e;
            int lo = 0, hi = 63;   // last row r with sdst[r] <= pos
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sdst[w][mid] <= pos) lo = mid;
                else hi = mid - 1;
            }
            v[u] = colindp[ssrc[w][lo] + (pos - sdst[w][lo])];
        }
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (e0 + 64 * u < total) colind[base + e0 + 64 * u] = v[u];
    }
}

// Row statistics without same-address atomics: per-block partials (max row length,
// max incidences per vertex, Dirichlet count), then one block combines them.
constexpr int STB = 256;

FE_DEV void block_reduce3(int64_t &mr, int64_t &md, int64_t &nd, int64_t *lds)
{
    for (int off = 32; off > 0; off >>= 1) {
        mr = max(mr, (int64_t)__shfl_xor(mr, off, 64));
        md = max(md, (int64_t)__shfl_xor(md, off, 64));
        nd += (int64_t)__shfl_xor(nd, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        lds[wid] = mr;
        lds[STB / 64 + wid] = md;
        lds[2 * (STB / 64) + wid] = nd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mr = lds[0];
        md = lds[STB / 64];
        nd = lds[2 * (STB / 64)];
        for (int w = 1; w < STB / 64; ++w) {
            mr = max(mr, lds[w]);
            md = max(md, lds[STB / 64 + w]);
            nd += lds[2 * (STB / 64) + w];
        }
    }
}

// Statistics over processing-order arrays: row lengths (prowptr after its scan),
// incidences per vertex (pincptr), Dirichlet flags; a grid-stride loop keeps the
// number of block partials small for the one-block combine.
__global__ __launch_bounds__(STB) void k_stats_partial(int32_t N, const int32_t *__restrict__ prowptr,
                                                       const int32_t *__restrict__ pincptr,
                                                       const uint8_t *__restrict__ isdp, int64_t *part)
{
    __shared__ int64_t lds[3 * (STB / 64)];
    int64_t mr = 0, md = 0, nd = 0;
    for (int32_t k = blockIdx.x * STB + threadIdx.x; k < N; k += gridDim.x * STB) {
        mr = max(mr, (int64_t)(prowptr[k + 1] - prowptr[k]));
        md = max(md, (int64_t)(pincptr[k + 1] - pincptr[k]));
        nd += isdp[k];
    }
    block_reduce3(mr, md, nd, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = mr;
        part[3 * blockIdx.x + 1] = md;
        part[3 * blockIdx.x + 2] = nd;
    }
}

__global__ __launch_bounds__(STB) void k_stats_final(int32_t nb, const int64_t *__restrict__ part, int32_t *status)
{
    __shared__ int64_t lds[3 * (STB / 64)];
    int64_t mr = 0, md = 0, nd = 0;
    for (int32_t b = threadIdx.x; b < nb; b += STB) {
        mr = max(mr, part[3 * b]);
        md = max(md, part[3 * b + 1]);
        nd += part[3 * b + 2];
    }
    block_reduce3(mr, md, nd, lds);
    if (threadIdx.x == 0) {
        status[ST_MAXROW] = (int32_t)mr;
        status[ST_MAXDEG] = (int32_t)md;
        status[ST_NDIR] = (int32_t)nd;
    }
}

// Bucket size: about 4096 incidences per bucket on average, at most NBMAX buckets.
struct Buckets {
    int32_t bs, nb, fine, ncb, nblk1, chn;   // chn: elements per level-1 chunk
    uint64_t cmul;   // ceil(2^32 / fine)
};

Buckets choose_buckets(int64_t N, int64_t NT, int nv)
{
    Buckets B{};
    const double avg = N > 0 ? (double)nv * (double)NT / (double)N : 1.0;
    int bs = 0;
    while (bs < 12 && (double)(1 << (bs + 1)) * avg <= 4096.0) ++bs;
    if (bs < 4) bs = 4;
    while (bs < 12 && cdiv(N, (int64_t)1 << bs) > NBMAX) ++bs;
    B.bs = bs;
    B.nb = (int32_t)cdiv(N, (int64_t)1 << bs);
    // Buckets per coarse bucket: as few as keep the coarse-to-fine kernel's blocks
    // within one resident round, so that round is as full as it can be (129^3 Kuhn
    // cube: 494 blocks instead of 263, 381 -> 263 us; 2049^2 grid: 483 instead of
    // 257, 182 -> 169 us, for 7 us more in the level-1 scatter, whose runs get
    // shorter with more coarse buckets).
    B.fine = (int32_t)(B.nb > L1SLOTS ? cdiv(B.nb, L1SLOTS) : 1);
    B.ncb = (int32_t)cdiv(B.nb, B.fine);
    B.cmul = ((uint64_t)1 << 32) / (uint64_t)B.fine + (((uint64_t)1 << 32) % (uint64_t)B.fine ? 1 : 0);
    // level-1 chunks: a whole number of chunks per CU (129^3: 512 chunks of 24576
    // elements instead of 384 of 32768, which left half of the CUs with one chunk and
    // half with two; 2049^2 keeps 256 of 32768), in multiples of the LDS sub-chunk
    const int64_t nt = NT > 0 ? NT : 1;
    const int64_t want = cdiv(cdiv(nt, (int64_t)L1CH), (int64_t)L1CUS) * L1CUS;
    const int64_t ch = cdiv(cdiv(nt, want), (int64_t)L1SUB) * L1SUB;
    B.chn = (int32_t)ch;
    B.nblk1 = (int32_t)cdiv(nt, ch);
    return B;
}

// Capacity of pincm: the incidences, and in 3-D half as many more for the padding
// of the sliced layout (a mesh whose padded size exceeds it keeps the row-major
// one: every row padded to the longest, so for a mesh whose longest row is more
// than 1.5 times the average).
int64_t pincm_cap(int64_t ninc, int nv)
{
    if (nv != 4) return ninc;
    const int64_t c = ninc + ninc / 2 + (int64_t)SELLW * SELLW;
    return c < (int64_t)INT32_MAX ? c : (int64_t)INT32_MAX;
}

// Upper bound of the number of stored entries: every element adds at most
// nv*(nv-1) off-diagonal entries.
int64_t nnz_bound(int64_t N, int64_t NT, int nv) { return N + NT * nv * (nv - 1); }

// Capacity of the long-row list: a long row has more than COL columns, so its vertex
// is in at least COL / (nv - 1) elements.
int64_t long_cap(int64_t N, int64_t NT, int nv)
{
    const int64_t col = nv == 3 ? RowCaps<3>::COL : RowCaps<4>::COL;
    const int64_t per = cdiv(col, nv - 1);
    const int64_t c = (int64_t)nv * NT / per + 1;
    return c < N ? c : N;
}

enum {
    W_STATUS, W_TOTALS, W_PART, W_VINFO, W_INCLP, W_ISD, W_ISDP, W_OWNF, W_HIST1, W_OWNCNT, W_PI, W_PIINV,
    W_PINCPTR, W_PINC, W_PINCM, W_ELEMP, W_ROWLEN, W_PROWPTR, W_PROWINFO, W_PRECP, W_ROWREC, W_XYP, W_FP,
    W_VALP, W_STATPART, W_SORTED, W_PAIRS2, W_FSTART, W_RSLOT, W_RMASK, W_LONGK, W_SPTR, W_COUNT
};

struct Layout {
    size_t off[W_COUNT];
    size_t total;
};

// Workspace layout (every array 256-byte aligned).  The level-1 pairs share memory
// with pincm (dead before the final row pass writes pincm); the level-2 global
// path borrows rowlen and prowptr as scratch.
Layout plan_layout(int64_t N, int64_t NT, int nv)
{
    const int64_t ninc = (int64_t)nv * NT;
    const Buckets Bk = choose_buckets(N, NT, nv);
    const int64_t nh = (int64_t)Bk.ncb * Bk.nblk1 + 1;
    int64_t nscan = N;
    if (NT > nscan) nscan = NT;
    if (nh > nscan) nscan = nh;
    size_t sz[W_COUNT];
    sz[W_STATUS] = sizeof(int32_t) * ST_COUNT;
    sz[W_TOTALS] = sizeof(int64_t) * 8;
    sz[W_PART] = sizeof(int64_t) * (size_t)(fe_scan_part_elems(nscan) + 1);
    sz[W_VINFO] = sizeof(int2) * (size_t)N;
    sz[W_INCLP] = sizeof(int32_t) * (size_t)N;
    sz[W_ISD] = sizeof(uint8_t) * (size_t)N;
    sz[W_ISDP] = sizeof(uint8_t) * (size_t)N;
    sz[W_OWNF] = sizeof(uint8_t) * (size_t)ninc;
    sz[W_HIST1] = sizeof(int32_t) * (size_t)nh;
    sz[W_OWNCNT] = sizeof(int32_t) * (size_t)(NT + 1);
    sz[W_PI] = sizeof(int32_t) * (size_t)N;
    sz[W_PIINV] = sizeof(int32_t) * (size_t)N;
    sz[W_PINCPTR] = sizeof(int32_t) * (size_t)(N + 1);
    sz[W_PINC] = sizeof(int32_t) * (size_t)ninc;
    sz[W_PINCM] = sizeof(int2) * (size_t)pincm_cap(ninc, nv);
    sz[W_ELEMP] = sizeof(int32_t) * 4 * (size_t)NT;
    sz[W_ROWLEN] = sizeof(int32_t) * (size_t)(N + 1);
    sz[W_PROWPTR] = sizeof(int32_t) * (size_t)(N + 1);
    sz[W_PROWINFO] = sizeof(uint32_t) * (size_t)N;
    sz[W_PRECP] = sizeof(int4) * (size_t)N;
    sz[W_ROWREC] = sizeof(int4) * (size_t)N;
    sz[W_XYP] = sizeof(double) * 4 * (size_t)N;
    sz[W_FP] = sizeof(double) * (size_t)N;
    sz[W_VALP] = sizeof(double) * (size_t)(nnz_bound(N, NT, nv) + 2 * N);
    sz[W_STATPART] = sizeof(int64_t) * 3 * (size_t)(cdiv(N, STB) + 1);
    sz[W_SORTED] = sizeof(int32_t) * (size_t)ninc;
    sz[W_PAIRS2] = sizeof(int2) * (size_t)ninc;
    sz[W_FSTART] = sizeof(int32_t) * (size_t)(Bk.nb + 1);
    sz[W_RMASK] = nv == 4 ? sizeof(int2) * (size_t)N : 0;
    sz[W_RSLOT] = nv == 4 ? sizeof(int32_t) * (size_t)REGCAP * (size_t)N : 0;   // 3-D row slots
    sz[W_LONGK] = sizeof(int32_t) * (size_t)long_cap(N, NT, nv);
    sz[W_SPTR] = nv == 4 ? sizeof(int32_t) * (size_t)(cdiv(N, SELLW) + 1) : 0;
    Layout L{};
    size_t o = 0;
    for (int k = 0; k < W_COUNT; ++k) {
        L.off[k] = o;
        o += align256(sz[k]);
    }
    L.total = o;
    return L;
}

int check_mesh(const fe_mesh *m)
{
    if (!m) return FE_EINVAL;
    if (m->dim != 2 && m->dim != 3) return FE_EUNSUPPORTED;
    if (m->n_node <= 0 || m->n_elem < 0) return FE_EINVAL;
    const int64_t nv = m->dim + 1;
    if (m->n_node >= INT32_MAX || m->n_elem >= INT32_MAX / nv) return FE_EOVERFLOW;
    static_assert((int64_t)VBMAX * NBMAX >= (int64_t)INT32_MAX, "every int32 label has a bucket");
    return FE_OK;
}

RowArgs row_args(fe_plan *P)
{
    RowArgs R{};
    R.NT = (int32_t)P->NT;
    R.N = (int32_t)P->N;
    R.elem = P->elem;
    R.bd = P->bdflag;
    R.pi = P->pi;
    R.pincptr = P->pincptr;
    R.inclp = P->inclp;
    R.sorted_l = P->sorted_l;
    R.isdp = P->isdp;
    R.pinc = P->pinc;
    R.prowptr = P->prowptr;
    R.elemp = P->elemp;
    R.colindp = reinterpret_cast<int32_t *>(P->valp);
    R.pincm = P->pincm;
    R.prow_info = P->prow_info;
    R.precp = P->precp;
    R.rslot = P->rslot;
    R.rmask = P->rmask;
    R.longk = P->longk;
    R.nlcap = P->nlcap;
    R.sptr = P->sptr;
    R.status = P->status;
    return R;
}

// Launch a row pass.  Labels that follow the element order (the sort found runs)
// make the label-order lists local in processing order: both passes read them
// directly (LBL).  Scattered labels make them random reads, and the count pass
// copies them into processing order for the final pass.
template <int NV, bool FINAL> void launch_rows(const fe_plan *P, const RowArgs &R, hipStream_t s)
{
    const int32_t N = (int32_t)P->N;
    const char *name = FINAL ? "k_rows_final" : "k_rows_count";
    const dim3 greg((unsigned)cdiv(N, REGB)), glds((unsigned)cdiv(N, RowCaps<NV>::BLOCK));
    if (P->rows_reg && P->l1_agg)
        FE_TIMED(name, s, hipLaunchKernelGGL((k_rows<NV, FINAL, true, true>), greg, dim3(REGB), 0, s, R));
    else if (P->rows_reg)
        FE_TIMED(name, s, hipLaunchKernelGGL((k_rows<NV, FINAL, true, false>), greg, dim3(REGB), 0, s, R));
    else if (P->l1_agg)
        FE_TIMED(name, s,
                 hipLaunchKernelGGL((k_rows<NV, FINAL, false, true>), glds, dim3(RowCaps<NV>::BLOCK), 0, s, R));
    else
        FE_TIMED(name, s,
                 hipLaunchKernelGGL((k_rows<NV, FINAL, false, false>), glds, dim3(RowCaps<NV>::BLOCK), 0, s, R));
}

template <int NV> int plan_build(fe_plan *P, hipStream_t s)
{
    const int32_t N = (int32_t)P->N, NT = (int32_t)P->NT;
    const unsigned eg = (unsigned)cdiv(NT > 0 ? NT : 1, EBLOCK);
    const unsigned ng = (unsigned)cdiv(N, EBLOCK);
    const int64_t nh = (int64_t)P->ncb * P->nblk1;
    const size_t l1lds = sizeof(int32_t) * (size_t)P->ncb;
    int rc;
    if ((rc = fe_fill_i32(P->status, ST_COUNT, 0, s))) return rc;
    if ((rc = fe_fill_u8(P->isd, N, 0, s))) return rc;
    // (vinfo needs no clearing: the bucket kernels write it for every vertex)
    if (NT > 0)
        FE_TIMED("k_l1_hist", s,
                 hipLaunchKernelGGL(k_l1_hist<NV>, dim3((unsigned)P->nblk1), dim3(L1B), l1lds, s, P->elem, P->bdflag, NT, N,
                               P->bs, P->cmul, P->ncb, P->nblk1, P->chn, P->hist1, P->isd, P->status));
    if ((rc = fe_launch_check())) return rc;
    // Vertex indices are validated by the histogram kernel only: stop here, before
    // any kernel uses elem entries as addresses, if one was out of range.
    int32_t st0[ST_RUNS + 1];
    FE_HIP_CHECK(hipMemcpyAsync(st0, P->status, sizeof(st0), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (st0[ST_ERR]) return fe_status_from_bits(st0[ST_ERR]);
    if (NT > 0) {
        // Labels that follow the element order put runs of equal buckets in
        // neighbouring lanes; then the level-1 kernels aggregate their LDS counter
        // updates per wavefront.  The histogram kernel counted its wavefront calls
        // that found such runs.
        int64_t calls = 0;
        for (int64_t ch = 0; ch < P->nblk1; ++ch) {
            const int64_t len = std::min<int64_t>(P->chn, (int64_t)NT - ch * P->chn);
            calls += cdiv(len, L1B) * NV * (L1B / 64);
        }
        // (label-order processing stores labels as positions in the element records)
        P->l1_agg = 2 * (int64_t)st0[ST_RUNS] > calls && (int64_t)N <= (int64_t)EREC_POS + 1;
        if ((rc = fe_scan_exclusive(P->hist1, P->hist1, nh, P->totals + 4, P->part, P->status, s))) return rc;
        if (P->l1_agg) {
            FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_l1_scatter<NV, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * l1lds)));
            FE_TIMED("k_l1_scatter", s,
                     hipLaunchKernelGGL((k_l1_scatter<NV, true>), dim3((unsigned)P->nblk1), dim3(L1B), 2 * l1lds, s,
                                        P->elem, NT, P->bs, P->cmul, P->ncb, P->nblk1, P->chn, (const int32_t *)P->hist1, P->pairs,
                                        P->bdflag, (const uint8_t *)P->isd, reinterpret_cast<int4 *>(P->elemp)));
            FE_TIMED("k_l1_fine", s,
                     hipLaunchKernelGGL(k_l1_fine<true>, dim3((unsigned)P->ncb), dim3(FB), 0, s, P->nb, P->bs, P->fine, P->ncb,
                                        (const int32_t *)P->hist1, P->nblk1, P->ninc, (const int2 *)P->pairs,
                                        P->pairs2, P->fstart));
        } else {
            FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_l1_scatter<NV, false>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * l1lds)));
            FE_TIMED("k_l1_scatter", s,
                     hipLaunchKernelGGL((k_l1_scatter<NV, false>), dim3((unsigned)P->nblk1), dim3(L1B), 2 * l1lds, s,
                                        P->elem, NT, P->bs, P->cmul, P->ncb, P->nblk1, P->chn, (const int32_t *)P->hist1, P->pairs,
                                        nullptr, nullptr, nullptr));
            FE_TIMED("k_l1_fine", s,
                     hipLaunchKernelGGL(k_l1_fine<false>, dim3((unsigned)P->ncb), dim3(FB), 0, s, P->nb, P->bs, P->fine, P->ncb,
                                        (const int32_t *)P->hist1, P->nblk1, P->ninc, (const int2 *)P->pairs,
                                        P->pairs2, P->fstart));
        }
        // first-incidence flags, for the processing order of the general path
        uint8_t *ownf = P->l1_agg ? nullptr : P->ownf;
        if (ownf && (rc = fe_fill_u8(ownf, P->ninc, 0, s))) return rc;
        // LDS capacity per bucket: 1.5 times the average bucket, at least 2048 keys
        int64_t cap = cdiv(3 * P->ninc, 2 * (int64_t)P->nb);
        cap = cdiv(cap, 1024) * 1024;
        if (cap < 2048) cap = 2048;
        if (cap > BCAPMAX) cap = BCAPMAX;
        const size_t lds = sizeof(int32_t) * ((size_t)cap + 2 * ((size_t)1 << P->bs));
        // Pairs per thread held in registers between the counting and placing passes
        // (129^3: 239 -> 211 us; 2049^2 unchanged, 157 -> 159 us, so 2-D keeps the
        // second load)
        constexpr int L2PT = 20;
        if (P->dim == 3 && cap <= (int64_t)L2PT * BKB) {
            FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_l2_bucket<L2PT>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            FE_TIMED("k_l2_bucket", s,
                     hipLaunchKernelGGL(k_l2_bucket<L2PT>, dim3((unsigned)P->nb), dim3(BKB), lds, s, N, P->bs,
                                        (int32_t)cap, (const int32_t *)P->fstart, (const int2 *)P->pairs2,
                                        (const uint8_t *)P->isd, P->sorted_l, P->vinfo, ownf));
        } else {
            FE_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_l2_bucket<0>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            FE_TIMED("k_l2_bucket", s,
                     hipLaunchKernelGGL(k_l2_bucket<0>, dim3((unsigned)P->nb), dim3(BKB), lds, s, N, P->bs,
                                        (int32_t)cap, (const int32_t *)P->fstart, (const int2 *)P->pairs2,
                                        (const uint8_t *)P->isd, P->sorted_l, P->vinfo, ownf));
        }
        FE_TIMED("k_l2_bucket_global", s,
                 hipLaunchKernelGGL(k_l2_bucket_global, dim3((unsigned)P->nb), dim3(BKB), 0, s, N, P->bs, (int32_t)cap,
                               (const int32_t *)P->fstart, (const int2 *)P->pairs2, (const uint8_t *)P->isd,
                               P->sorted_l, P->vinfo, P->rowlen, P->prowptr, ownf));
        if ((rc = fe_launch_check())) return rc;
    }
    if (P->l1_agg) {
        // labels follow the element order: process rows in label order
        FE_TIMED("k_ident", s,
                 hipLaunchKernelGGL(k_ident, dim3((unsigned)cdiv(N + 1, EBLOCK)), dim3(EBLOCK), 0, s, N, P->ninc,
                                    (const int2 *)P->vinfo, P->pi, P->piinv, P->pincptr, P->inclp, P->isdp));
        if ((rc = fe_launch_check())) return rc;
    } else {
        // processing position = rank of the vertex's first incidence (element order)
        // first incidences per element, scanned straight from the flags
        if ((rc = fe_scan_exclusive_flags(P->ownf, NV, P->owncnt, NT, P->totals + 0, P->part, P->status, s))) return rc;
        if (NT > 0)
            FE_TIMED("k_pi", s,
                     hipLaunchKernelGGL(k_pi<NV>, dim3(eg), dim3(EBLOCK), 0, s, P->elem, NT, (const uint8_t *)P->ownf,
                                        (const int32_t *)P->owncnt, (const int2 *)P->vinfo, P->pi, P->piinv,
                                        P->pincptr, P->inclp, P->isdp));
        FE_TIMED("k_unused", s,
                 hipLaunchKernelGGL(k_unused, dim3(ng), dim3(EBLOCK), 0, s, N, (const int2 *)P->vinfo,
                                    (const int64_t *)(P->totals + 0), P->pi, P->piinv, P->pincptr, P->inclp, P->isdp,
                                    P->status));
        if ((rc = fe_launch_check())) return rc;
        if ((rc = fe_scan_exclusive(P->pincptr, P->pincptr, N, P->totals + 1, P->part, P->status, s))) return rc;
    }
    if (NV == 4) {
        // the sliced incidence layout, if its padded size fits pincm
        const int64_t nsl = cdiv(N, SELLW);
        FE_TIMED("k_sell_len", s,
                 hipLaunchKernelGGL(k_sell_len, dim3((unsigned)cdiv(nsl, 256)), dim3(256), 0, s, N,
                                    (const int32_t *)P->pincptr, P->sptr));
        FE_TIMED("k_sell_choose", s,
                 hipLaunchKernelGGL(k_sell_choose, dim3(1), dim3(1024), 0, s, (int32_t)nsl, pincm_cap(P->ninc, NV),
                                    P->sptr, P->status));
        if ((rc = fe_launch_check())) return rc;
    }
    const RowArgs R = row_args(P);
    // the row pass with the register column set; rows too long for it make the pass
    // run again with the LDS set (both give the same sets)
    P->rows_reg = 1;
    for (int attempt = 0; attempt < 2; ++attempt) {
        launch_rows<NV, false>(P, R, s);
        if (!P->rows_reg) {
            // rows beyond the LDS set: counted by k_rows_long (the grid loops over
            // however many the count pass found, none for most meshes)
            const unsigned lg = (unsigned)std::min<int64_t>(P->nlcap, 1024);
            if (P->l1_agg)
                FE_TIMED("k_rows_long_count", s,
                         hipLaunchKernelGGL((k_rows_long<NV, false, true>), dim3(lg), dim3(LB), 0, s, R));
            else
                FE_TIMED("k_rows_long_count", s,
                         hipLaunchKernelGGL((k_rows_long<NV, false, false>), dim3(lg), dim3(LB), 0, s, R));
        }
        if ((rc = fe_launch_check())) return rc;
        if ((rc = fe_scan_exclusive(P->prowptr, P->prowptr, N, P->totals + 2, P->part, P->status, s))) return rc;
        const unsigned sb = (unsigned)(cdiv(N, STB) < 1024 ? cdiv(N, STB) : 1024);   // grid-stride beyond
        FE_TIMED("k_stats_partial", s,
                 hipLaunchKernelGGL(k_stats_partial, dim3(sb), dim3(STB), 0, s, N, (const int32_t *)P->prowptr,
                                    (const int32_t *)P->pincptr, (const uint8_t *)P->isdp, P->stat_part));
        FE_TIMED("k_stats_final", s,
                 hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(STB), 0, s, (int32_t)sb,
                                    (const int64_t *)P->stat_part, P->status));
        if ((rc = fe_launch_check())) return rc;
        int32_t st[ST_COUNT];
        int64_t tot[8];
        FE_HIP_CHECK(hipMemcpyAsync(st, P->status, sizeof(st), hipMemcpyDeviceToHost, s));
        FE_HIP_CHECK(hipMemcpyAsync(tot, P->totals, sizeof(tot), hipMemcpyDeviceToHost, s));
        FE_HIP_CHECK(hipStreamSynchronize(s));
        if (st[ST_ERR] & ERR_RETRY) {
            if (!P->rows_reg) return FE_EHIP;
            P->rows_reg = 0;
            if ((rc = fe_fill_i32(P->status + ST_ERR, 1, st[ST_ERR] & ~ERR_RETRY, s))) return rc;
            continue;
        }
        if (st[ST_ERR]) return fe_status_from_bits(st[ST_ERR]);
        P->nlong = st[ST_NLONG];
        P->nnz = tot[2];
        P->max_row = st[ST_MAXROW];
        P->max_deg = st[ST_MAXDEG];
        P->ndir = st[ST_NDIR];
        if (!P->l1_agg && tot[1] != P->ninc) return FE_EHIP;   // every incidence must be placed
        // the element records hold 29-bit positions of the vertices in use
        if (!P->l1_agg && tot[0] > (int64_t)EREC_POS + 1) return FE_ELIMIT;
        if (P->nnz > P->nnz_max) return FE_EHIP;
        return FE_OK;
    }
    return FE_EHIP;
}

template <int NV> int plan_pattern(fe_plan *P, int32_t *rowptr, int32_t *colind, hipStream_t s)
{
    const int32_t N = (int32_t)P->N;
    RowArgs R = row_args(P);
    if (P->l1_agg) {
        // processing order = label order: the final pass writes the caller's column
        // indices, and the row pointer is the processing-order one
        R.colindp = colind;
        launch_rows<NV, true>(P, R, s);
        if (P->nlong > 0)
            FE_TIMED("k_rows_long_final", s,
                     hipLaunchKernelGGL((k_rows_long<NV, true, true>), dim3((unsigned)P->nlong), dim3(LB), 0, s, R));
        int rc;
        if ((rc = fe_launch_check())) return rc;
        FE_HIP_CHECK(hipMemcpyAsync(rowptr, P->prowptr, sizeof(int32_t) * (size_t)(N + 1), hipMemcpyDeviceToDevice, s));
        return FE_OK;
    }
    launch_rows<NV, true>(P, R, s);
    if (P->nlong > 0)
        FE_TIMED("k_rows_long_final", s,
                 hipLaunchKernelGGL((k_rows_long<NV, true, false>), dim3((unsigned)P->nlong), dim3(LB), 0, s, R));
    FE_TIMED("k_label_rows", s,
             hipLaunchKernelGGL(k_label_rows, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, s, N, (const int32_t *)P->piinv,
                           (const int4 *)P->precp, P->rowrec, P->rowlen));
    int rc;
    if ((rc = fe_launch_check())) return rc;
    if ((rc = fe_scan_exclusive(P->rowlen, P->rowlen, N, P->totals + 3, P->part, P->status, s))) return rc;
    FE_HIP_CHECK(hipMemcpyAsync(rowptr, P->rowlen, sizeof(int32_t) * (size_t)(N + 1), hipMemcpyDeviceToDevice, s));
    FE_TIMED("k_pattern_to_label", s,
             hipLaunchKernelGGL(k_pattern_to_label, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, s, N,
                           (const int32_t *)P->rowlen, (const int4 *)P->rowrec, (const int32_t *)R.colindp, colind));
    return fe_launch_check();
}

}  // namespace

extern "C" int fe_plan_workspace_bytes(const fe_mesh *mesh, size_t *bytes)
{
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!bytes) return FE_EINVAL;
    *bytes = plan_layout(mesh->n_node, mesh->n_elem, mesh->dim + 1).total;
    return FE_OK;
}

extern "C" int fe_plan_create(const fe_mesh *mesh, void *ws, size_t ws_bytes, fe_plan **plan, int64_t *nnz,
                              void *stream)
{
    int rc = check_mesh(mesh);
    if (rc) return rc;
    if (!ws || !plan || !mesh->elem) return FE_EINVAL;
    if ((uintptr_t)ws & 255) return FE_EINVAL;
    const int nv = mesh->dim + 1;
    Layout L = plan_layout(mesh->n_node, mesh->n_elem, nv);
    if (ws_bytes < L.total) return FE_ESIZE;
    fe_plan *P = new (std::nothrow) fe_plan();
    if (!P) return FE_EINVAL;
    char *base = static_cast<char *>(ws);
    const Buckets Bk = choose_buckets(mesh->n_node, mesh->n_elem, nv);
    P->dim = mesh->dim;
    P->nv = nv;
    P->N = mesh->n_node;
    P->NT = mesh->n_elem;
    P->ninc = (int64_t)nv * mesh->n_elem;
    P->elem = mesh->elem;
    P->bdflag = mesh->bdflag;
    P->bs = Bk.bs;
    P->fine = Bk.fine;
    P->cmul = Bk.cmul;
    P->nb = Bk.nb;
    P->ncb = Bk.ncb;
    P->nblk1 = Bk.nblk1;
    P->chn = Bk.chn;
    P->status = reinterpret_cast<int32_t *>(base + L.off[W_STATUS]);
    P->totals = reinterpret_cast<int64_t *>(base + L.off[W_TOTALS]);
    P->part = reinterpret_cast<int64_t *>(base + L.off[W_PART]);
    P->vinfo = reinterpret_cast<int2 *>(base + L.off[W_VINFO]);
    P->inclp = reinterpret_cast<int32_t *>(base + L.off[W_INCLP]);
    P->isd = reinterpret_cast<uint8_t *>(base + L.off[W_ISD]);
    P->isdp = reinterpret_cast<uint8_t *>(base + L.off[W_ISDP]);
    P->ownf = reinterpret_cast<uint8_t *>(base + L.off[W_OWNF]);
    P->hist1 = reinterpret_cast<int32_t *>(base + L.off[W_HIST1]);
    P->owncnt = reinterpret_cast<int32_t *>(base + L.off[W_OWNCNT]);
    P->pi = reinterpret_cast<int32_t *>(base + L.off[W_PI]);
    P->piinv = reinterpret_cast<int32_t *>(base + L.off[W_PIINV]);
    P->pincptr = reinterpret_cast<int32_t *>(base + L.off[W_PINCPTR]);
    P->pinc = reinterpret_cast<int32_t *>(base + L.off[W_PINC]);
    P->pincm = reinterpret_cast<int2 *>(base + L.off[W_PINCM]);
    P->pairs = P->pincm;
    P->elemp = reinterpret_cast<int32_t *>(base + L.off[W_ELEMP]);
    P->rowlen = reinterpret_cast<int32_t *>(base + L.off[W_ROWLEN]);
    P->prowptr = reinterpret_cast<int32_t *>(base + L.off[W_PROWPTR]);
    P->prow_info = reinterpret_cast<uint32_t *>(base + L.off[W_PROWINFO]);
    P->precp = reinterpret_cast<int4 *>(base + L.off[W_PRECP]);
    P->rowrec = reinterpret_cast<int4 *>(base + L.off[W_ROWREC]);
    P->xyp = reinterpret_cast<double *>(base + L.off[W_XYP]);
    P->fp = reinterpret_cast<double *>(base + L.off[W_FP]);
    P->valp = reinterpret_cast<double *>(base + L.off[W_VALP]);
    P->stat_part = reinterpret_cast<int64_t *>(base + L.off[W_STATPART]);
    P->sorted_l = reinterpret_cast<int32_t *>(base + L.off[W_SORTED]);
    P->pairs2 = reinterpret_cast<int2 *>(base + L.off[W_PAIRS2]);
    P->fstart = reinterpret_cast<int32_t *>(base + L.off[W_FSTART]);
    P->rslot = reinterpret_cast<int4 *>(base + L.off[W_RSLOT]);
    P->rmask = reinterpret_cast<int2 *>(base + L.off[W_RMASK]);
    P->longk = reinterpret_cast<int32_t *>(base + L.off[W_LONGK]);
    P->sptr = reinterpret_cast<int32_t *>(base + L.off[W_SPTR]);
    P->nlcap = (int32_t)long_cap(mesh->n_node, mesh->n_elem, nv);
    P->nlong = 0;
    P->nnz_max = nnz_bound(mesh->n_node, mesh->n_elem, nv);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = (nv == 3) ? plan_build<3>(P, s) : plan_build<4>(P, s);
    if (rc) {
        delete P;
        return rc;
    }
    if (nnz) *nnz = P->nnz;
    *plan = P;
    return FE_OK;
}

extern "C" int fe_plan_pattern(fe_plan *plan, int32_t *rowptr, int32_t *colind, void *stream)
{
    if (!plan || !rowptr || (!colind && plan->nnz > 0)) return FE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = (plan->nv == 3) ? plan_pattern<3>(plan, rowptr, colind, s) : plan_pattern<4>(plan, rowptr, colind, s);
    if (rc == FE_OK) plan->pattern_done = 1;
    return rc;
}

extern "C" int fe_plan_set_launch(fe_plan *plan, int32_t rows_per_block)
{
    if (!plan) return FE_EINVAL;
    if (rows_per_block != 0 && rows_per_block != 64 && rows_per_block != 128 && rows_per_block != 256)
        return FE_EINVAL;
    if (plan->asm_block != rows_per_block) {
        plan->asm_block = rows_per_block;
        ++plan->launch_gen;
    }
    return FE_OK;
}

extern "C" int fe_plan_get_info(const fe_plan *plan, fe_plan_info *info)
{
    if (!plan || !info) return FE_EINVAL;
    info->dim = plan->dim;
    info->n_node = plan->N;
    info->n_elem = plan->NT;
    info->nnz = plan->nnz;
    info->n_inc = plan->ninc;
    info->max_row = plan->max_row;
    info->max_deg = plan->max_deg;
    info->n_dirichlet = plan->ndir;
    info->sort_runs = plan->l1_agg;
    info->n_long = plan->nlong;
    return FE_OK;
}

extern "C" int fe_plan_status(fe_plan *plan, void *stream)
{
    if (!plan) return FE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t err = 0;
    FE_HIP_CHECK(hipMemcpyAsync(&err, plan->status + ST_ERR, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (err) {
        int rc = fe_fill_i32(plan->status + ST_ERR, 1, 0, s);
        if (rc) return rc;
        FE_HIP_CHECK(hipStreamSynchronize(s));
    }
    return fe_status_from_bits(err);
}

extern "C" int fe_plan_destroy(fe_plan *plan)
{
    delete plan;
    return FE_OK;
}
