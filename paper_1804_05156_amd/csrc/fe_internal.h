// fe_internal.h -- internal declarations of the HIP library (gfx950 only).
//
// Device helpers, the plan object and its workspace layout, shared by the
// library's .hip translation units.  Nothing here is part of the C interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "femhip.h"

// ---------------------------------------------------------------------------
// Error bits recorded by kernels in plan->status[ST_ERR].
// ---------------------------------------------------------------------------
enum : int32_t {
    ERR_INDEX = 1,      // vertex index outside [0, N)
    ERR_BDCODE = 2,     // bdflag not in 0..3
    ERR_ROBIN = 4,      // bdflag 3
    ERR_REPEAT = 8,     // an element lists a vertex twice
    ERR_MEASURE = 16,   // element measure not positive / not finite
    ERR_KAPPA = 32,     // kappa not positive / not finite
    ERR_LIMIT = 64,     // a row exceeds the fixed per-row capacity
    ERR_OVERFLOW = 128, // a prefix sum exceeds the int32 range
    ERR_RETRY = 256     // internal: a row did not fit the register column set
};

// Slots of the device status array.
enum { ST_ERR = 0, ST_UNUSED = 1, ST_MAXROW = 2, ST_MAXDEG = 3, ST_NDIR = 4, ST_RUNS = 5, ST_NLONG = 6,
       ST_SELL = 7, ST_COUNT = 16 };

// Layout of the per-incidence (key, metadata) words, pincm.  Row-major: row k's
// incidences at pincptr[k] .. pincptr[k+1].  Sliced (3-D plans whose padded size
// fits, status word ST_SELL set): rows grouped in slices of SELLW consecutive
// processing positions, every slice W incidences deep (W = the most incidences of
// any row, in sptr[0]), incidence q of row k at (k / SELLW) SELLW W + SELLW q +
// k % SELLW.  A wavefront's rows are one slice, so its q-th loads and stores are
// contiguous, and the address needs no per-row load (W is one word for the whole
// grid, held by the scalar cache).
constexpr int SELLW = 64;
__device__ __forceinline__ int64_t inc_at(bool sell, const int32_t *sptr, int32_t s, int32_t k, int32_t q)
{
    return sell ? (int64_t)(k >> 6) * SELLW * sptr[0] + (int64_t)SELLW * q + (k & (SELLW - 1)) : (int64_t)s + q;
}

// Per-row capacity (stored columns, the vertex itself included) of the row kernels
// and the numeric kernels, and their block sizes.  Longer rows ("long rows") are
// handled by kernels of their own, one workgroup per row, whose LDS holds up to
// LCAND candidate columns: (dim) * (incidences of the vertex) + 1 <= LCAND.
constexpr int LCAND = 8192;
template <int NV> struct RowCaps;
template <> struct RowCaps<3> { static constexpr int COL = 32, BLOCK = 128; };
template <> struct RowCaps<4> { static constexpr int COL = 64, BLOCK = 64; };

// Incidence metadata word (one per vertex-element incidence, in row order):
//   bits 0-1                  local index a of the row's vertex in the element
//   bits OFF+OB*j .. +OB-1    offset within the row of the column of local vertex
//                             fe_other<NV>(a, j), j = 0..NV-2 (OB = 5 bits in 2-D,
//                             6 in 3-D: rows hold at most 32 / 64 columns)
//   bit  DBIT+j               that vertex is a Dirichlet node
//   bit  NBIT+j               the side opposite that vertex is a Neumann side
//   bit  RBIT+j               the side opposite that vertex is a Robin side
//                             (the sides opposite the other vertices are the sides
//                             that contain vertex a)
template <int NV> struct Meta {
    static constexpr int OFF = 2;
    static constexpr int OB = NV == 3 ? 5 : 6;
    static constexpr uint32_t OMASK = (1u << OB) - 1;
    static constexpr int DBIT = OFF + OB * (NV - 1);
    static constexpr int NBIT = DBIT + (NV - 1);
    static constexpr int RBIT = NBIT + (NV - 1);
};
static_assert(Meta<4>::RBIT + 3 <= 32, "metadata word overflow");

// Local order used for the row of local vertex a: the element's vertices are
// taken as (a, other(a,0), ..., other(a,NV-2)), an even permutation of the stored
// order, so the element keeps its positive orientation.  2-D: cyclic rotation.
// 3-D: (0,1,2,3), (1,2,0,3), (2,0,1,3), (3,0,2,1).
template <int NV> __host__ __device__ __forceinline__ int fe_other(int a, int jj)
{
    if (NV == 3) return (a + 1 + jj) % 3;
    // 2 bits per entry, entry (a, jj) at bit 2*(3a + jj)
    constexpr uint32_t T = (1u << 0) | (2u << 2) | (3u << 4) |    // a = 0: 1 2 3
                           (2u << 6) | (0u << 8) | (3u << 10) |   // a = 1: 2 0 3
                           (0u << 12) | (1u << 14) | (3u << 16) | // a = 2: 0 1 3
                           (0u << 18) | (2u << 20) | (1u << 22);  // a = 3: 0 2 1
    return (int)((T >> (2 * (3 * a + jj))) & 3u);
}

// Row info word (one per row, in processing order): bits 0-7 row length,
// bits 8-15 offset of the diagonal, bit 16 the row's vertex is a Dirichlet node,
// bit 17 (INFO_LONG) a long row: length and diagonal offset are then kept in the
// row record's .z and .w (in place of the Dirichlet-column mask) and bits 0-15 are 0.
constexpr uint32_t INFO_LONG = 1u << 17;

struct fe_plan {
    int32_t dim, nv;
    int64_t N, NT, ninc;
    const int32_t *elem;
    const int8_t *bdflag;
    int32_t bs, nb, nblk1;   // bucket shift (2^bs vertices per bucket), bucket count, level-1 chunks
    int32_t chn;             // elements per level-1 chunk
    // device arrays inside the caller's workspace
    int32_t *status;      // ST_COUNT ints
    int64_t *totals;      // scan totals (4 slots)
    int64_t *part;        // scan partials
    int2 *vinfo;          // N      per vertex (label order): (start of its sorted list in
                          //        sorted_l, incident elements | Dirichlet flag << 30)
    int32_t *inclp;       // N      start of the sorted list (processing order)
    uint8_t *isd;         // N      Dirichlet flag (label order)
    uint8_t *isdp;        // N      Dirichlet flag (processing order)
    int4 *precp;          // N      row record (processing order), see rowrec
    int4 *rslot;          // 4*N    3-D: each row's column set (register form, padded), count -> final pass
    int2 *rmask;          // N      3-D label-order register form: row Dirichlet-column masks, count -> final
    uint8_t *ownf;        // ninc   1 if incidence t*nv+a is the first one of its vertex
    int32_t *hist1;       // nb*nblk1+1  level-1 bucket histogram (bucket-major) -> offsets
    int2 *pairs;          // ninc   (vertex, key) grouped by coarse bucket (shares memory with pincm)
    int2 *pairs2;         // ninc   (vertex, key) grouped by bucket
    int32_t *fstart;      // nb+1   first incidence of each bucket in pairs2
    int32_t ncb;          // coarse buckets (fine buckets each, the last maybe fewer)
    int32_t fine;         // buckets per coarse bucket (1..32)
    uint64_t cmul;        // ceil(2^32 / fine): coarse bucket = ((v >> bs) * cmul) >> 32
    int32_t *sorted_l;    // ninc   keys grouped by vertex label, ascending
    int32_t *owncnt;      // NT+1   vertices whose first incidence is in element t -> offsets
    int32_t *pi;          // N      processing order -> vertex label
    int32_t *piinv;       // N      vertex label -> processing position
    int32_t *pincptr;     // N+1    incidence ranges in processing order
    int32_t *pinc;        // ninc   incidence keys t*nv+a, ascending within a row
    int2 *pincm;          // pcap   (key, metadata word) per incidence, processing order (see inc_at)
    int32_t *sptr;        // N/64+1 3-D: the longest row of each slice, then sptr[0] = the
                          //        depth W of every slice of the sliced layout
    int32_t *elemp;       // 4*NT   processing positions of each element's vertices (AoS),
                          //        see EREC_POS
    int32_t *rowlen;      // N+1    row lengths (label order) -> row pointer (label order)
    int32_t *prowptr;     // N+1    row lengths (processing order) -> row pointer of the
                          //        processing-order copy of the matrix
    uint32_t *prow_info;  // N      row info word (processing order)
    int4 *rowrec;         // N      per label row: (processing-order start, info word, Dirichlet
                          //        column mask low, high 32 bits)
    double *xyp;          // 4*N    numeric scratch: coordinates in processing order
    double *fp;           // N      numeric scratch: nodal source values in processing order
    double *valp;         // nnz_max+2N numeric scratch: processing-order rows, row k at
                          //        prowptr[k] + 2k holding its values then (b, b_load); the
                          //        pattern pass keeps its column indices here as int32
    int64_t nnz_max;      // capacity of valp
    int64_t *stat_part;   // per-block partial statistics
    int32_t *longk;       // nlcap  processing positions of the long rows
    int32_t nlcap;        // capacity of longk
    int32_t nlong;        // long rows (host copy)
    // host copies
    int64_t nnz, ndir;
    int32_t max_row, max_deg;
    int rows_reg;         // the row passes use the register column set
    int l1_agg;           // labels follow the element order: the level-1 kernels aggregate LDS
                          // counter updates per wavefront, the row passes read the label-order
                          // lists, and rows are processed in label order (identity pi)
    int pattern_done;
    int32_t asm_block;    // rows per workgroup of the numeric row kernels (0: by row width)
    int32_t launch_gen;   // bumped whenever a launch setting changes (captured graphs recapture)
};

// ---------------------------------------------------------------------------
// Small device helpers.
// ---------------------------------------------------------------------------
#define FE_DEV __device__ __forceinline__

struct DevFn {
    int32_t kind;
    double c0, c1, c2, c3;
    const double *nodal;
};

static inline DevFn make_devfn(const fe_fn *f)
{
    DevFn d{};
    if (!f) { d.kind = FE_FN_ZERO; return d; }
    d.kind = f->kind;
    d.c0 = f->c[0]; d.c1 = f->c[1]; d.c2 = f->c[2]; d.c3 = f->c[3];
    d.nodal = f->nodal;
    return d;
}

static inline bool devfn_valid(const fe_fn *f, bool allow_dudn)
{
    if (!f) return true;
    if (f->kind < FE_FN_ZERO || f->kind > FE_FN_NODAL) return false;
    if (f->kind == FE_FN_DUDN_SINPROD && !allow_dudn) return false;
    if (f->kind == FE_FN_NODAL && !f->nodal) return false;
    return true;
}

// Value of a point-evaluable data function (not NODAL, not DUDN) at x.
template <int DIM> FE_DEV double fn_point(const DevFn &f, const double *x)
{
    switch (f.kind) {
    case FE_FN_CONST: return f.c0;
    case FE_FN_LINEAR: {
        double v = f.c0 + f.c1 * x[0] + f.c2 * x[1];
        if (DIM == 3) v += f.c3 * x[2];
        return v;
    }
    case FE_FN_SINPROD: {
        double v = f.c0 * sinpi(x[0]) * sinpi(x[1]);
        if (DIM == 3) v *= sinpi(x[2]);
        return v;
    }
    default: return 0.0;
    }
}

// c0 * grad(prod sin(pi x_c)) . nrm
template <int DIM> FE_DEV double fn_dudn(const DevFn &f, const double *x, const double *nrm)
{
    double s[DIM], c[DIM];
    for (int k = 0; k < DIM; ++k) { s[k] = sinpi(x[k]); c[k] = cospi(x[k]); }
    const double pi = 3.14159265358979323846;
    double acc = 0.0;
    for (int k = 0; k < DIM; ++k) {
        double g = pi * c[k];
        for (int e = 0; e < DIM; ++e)
            if (e != k) g *= s[e];
        acc += g * nrm[k];
    }
    return f.c0 * acc;
}

// Deterministic block-wide sum (fixed combination order) of one double per thread.
// `lds` needs BLOCK/64 doubles.  Every thread of the block must call it.
// Order the LDS accesses of one wavefront: every lane's earlier LDS stores are seen
// by every lane's later loads (for work shared within a wavefront, with no workgroup
// barrier).
FE_DEV void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int BLOCK> FE_DEV double block_sum(double v, double *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    __syncthreads();
    return s;   // valid in thread 0
}

// LDS counter increments aggregated over a wavefront: lanes with equal keys in a
// run of consecutive active lanes make one atomicAdd(cnt + key, run length) (issued
// by the run's first lane), so a key shared by many lanes costs one atomic instead
// of one per lane.  When no lane repeats its neighbour's key every lane adds its own
// 1.  *runs is set (the same in every lane) when at least 16 lanes continue a run:
// the statistic by which the plan picks the aggregated kernels.  Returns, for an active lane, a
// distinct rank within its key: the counter's old value plus the lane's place in
// its run (as a per-lane atomicAdd(cnt + key, 1) would, in another order).  Every
// lane of the wavefront must call it, inactive ones with active = false (their
// result is meaningless).
FE_DEV int32_t wave_rank_add(int32_t *cnt, int32_t key, bool active, bool *runs)
{
    const int lane = threadIdx.x & 63;
    const uint64_t act = __ballot(active);
    const int32_t kprev = __shfl_up(key, 1, 64);
    const bool cont = active && lane > 0 && ((act >> (lane - 1)) & 1ull) && kprev == key;
    const uint64_t conts = __ballot(cont);
    *runs = __popcll((long long)conts) >= 16;
    if (conts == 0) return active ? atomicAdd(cnt + key, 1) : 0;   // wavefront-uniform branch
    const uint64_t heads = act & ~conts;
    const bool head = active && !cont;
    const uint64_t stops = heads | ~act;                        // lanes that do not continue a run
    const uint64_t after = lane == 63 ? 0ull : stops >> (lane + 1);
    const int32_t len = after ? __ffsll((long long)after) : 64 - lane;
    int32_t base = 0;
    if (head) base = atomicAdd(cnt + key, len);
    const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const int hl = upto ? 63 - __clzll((long long)upto) : lane;  // this lane's run head
    return __shfl(base, hl, 64) + (lane - hl);
}

// Per-lane LDS counter increment (AGG false) or the wavefront-aggregated one above
// (AGG true; then every lane of the wavefront must call it).
// Element records (elemp, one int4 per element): word a holds the processing
// position of vertex a in its low 29 bits, the side code of the face opposite
// vertex a in bits 29-30 and the Dirichlet flag of vertex a in bit 31.  Positions
// of vertices in use are below 2^29 (a plan with more vertices in use is refused);
// unused vertices never appear in a record.
constexpr int32_t EREC_POS = (1 << 29) - 1;
constexpr int EREC_CODE = 29, EREC_DIR = 31;

// Logical block of hardware block b in a grid of nblk.  Blocks are dealt to the 8
// XCDs round-robin (b, b + 8, ... share one XCD and its L2); this bijection gives
// every XCD a contiguous range of logical blocks, so blocks that run together on
// one XCD work on neighbouring data.
FE_DEV int32_t xcd_block(int32_t b, int32_t nblk)
{
    const int32_t q = nblk / 8, r = nblk % 8, x = b % 8;
    return x * q + min(x, r) + b / 8;
}

template <bool AGG> FE_DEV int32_t lds_rank_add(int32_t *cnt, int32_t key, bool active)
{
    if (!AGG) return active ? atomicAdd(cnt + key, 1) : 0;
    bool runs;
    return wave_rank_add(cnt, key, active, &runs);
}

// Exclusive scan of one int per thread over a block of BLOCK threads (BLOCK a
// multiple of 64); *total receives the block sum.  `lds` needs 2*BLOCK/64 ints.
// Every thread of the block must call it.
template <int BLOCK> FE_DEV int32_t block_exclusive_i32(int32_t v, int32_t *lds, int32_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int NW = BLOCK / 64;
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int32_t w = (lane < NW) ? lds[lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(w, off, 64);
            if (lane >= off) w += y;
        }
        if (lane < NW) lds[NW + lane] = w;
    }
    __syncthreads();
    const int32_t pre = (wid > 0) ? lds[NW + wid - 1] : 0;
    *total = lds[2 * NW - 1];
    __syncthreads();
    return pre + x - v;
}

// ---------------------------------------------------------------------------
// Host helpers.
// ---------------------------------------------------------------------------
#define FE_HIP_CHECK(expr)                                  \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return FE_EHIP;               \
    } while (0)

static inline int fe_launch_check()
{
    return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

// Optional per-kernel event timing (prof.hip): FE_TIMED(name, stream, launch...)
// brackets one launch with events on its stream when timing is enabled.
int fe_prof_begin(const char *name, hipStream_t s);
void fe_prof_end(int tok, hipStream_t s);
#define FE_TIMED(name, stream, ...)                          \
    do {                                                     \
        const int fe_prof_tok_ = fe_prof_begin(name, stream); \
        __VA_ARGS__;                                         \
        fe_prof_end(fe_prof_tok_, stream);                   \
    } while (0)

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Exclusive prefix sum of in[0..n) into out[0..n] (out[n] = total, in may equal out).
// The 64-bit total is also stored at *total_dev; ERR_OVERFLOW is set in *status if
// it does not fit int32.  `part` needs fe_scan_part_elems(n) int64 entries.
int64_t fe_scan_part_elems(int64_t n);
// The same scan over per-entry counts of flag bytes: entry i is the sum of the nv
// (3 or 4) bytes flags[nv*i .. nv*i + nv); flags 4-byte aligned.
int fe_scan_exclusive_flags(const uint8_t *flags, int nv, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part,
                            int32_t *status, hipStream_t s);
int fe_scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part,
                      int32_t *status, hipStream_t s);

// Fill helpers (kernels, so they are safe to record in a graph).
int fe_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int fe_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
int fe_fill_f64(double *p, int64_t n, double v, hipStream_t s);

int fe_status_from_bits(int32_t bits);
