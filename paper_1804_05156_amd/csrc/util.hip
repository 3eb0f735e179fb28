// util.hip -- prefix sum, fill kernels and status helpers of the library.
#include "fe_internal.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_CHUNKS = 4;                        // one int4 per thread per chunk
constexpr int SCAN_CHUNK = SCAN_BLOCK * 4;            // 1024 elements
constexpr int SCAN_TILE = SCAN_CHUNKS * SCAN_CHUNK;   // 4096 elements per block
// Up to this many tiles the apply kernel sums its predecessors' partials itself
// (at most 32 KB of L2-resident reads per block); beyond it a one-block kernel
// scans the partials first.
constexpr int64_t SCAN_DIRECT_TILES = 4096;

// Inclusive scan across the 64 lanes of a wavefront.
FE_DEV int64_t wave_inclusive(int64_t x)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive block scan of one value per thread; *total receives the block sum.
template <int BLOCK = SCAN_BLOCK> FE_DEV int64_t block_exclusive(int64_t v, int64_t *lds, int64_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int NW = BLOCK / 64;
    int64_t inc = wave_inclusive(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int64_t w = (lane < NW) ? lds[lane] : 0;
        w = wave_inclusive(w);
        if (lane < NW) lds[NW + lane] = w;
    }
    __syncthreads();
    int64_t pre = (wid > 0) ? lds[NW + wid - 1] : 0;
    *total = lds[NW + NW - 1];
    __syncthreads();
    return pre + inc - v;
}

// A tile is SCAN_CHUNKS chunks of 1024 elements; in each chunk thread t holds
// elements 4t..4t+3, so every load and store of a wavefront is contiguous.
// FL = 0: int32 input.  FL = 3 or 4: element i is the sum of the FL bytes
// in[FL*i .. FL*i + FL) (per-element flag counts, read as 32-bit words).
template <int FL> FE_DEV int32_t in_at(const void *in, int64_t i)
{
    if constexpr (FL == 0) {
        return static_cast<const int32_t *>(in)[i];
    } else {
        const uint8_t *f = static_cast<const uint8_t *>(in) + (int64_t)FL * i;
        int32_t s = 0;
#pragma unroll
        for (int a = 0; a < FL; ++a) s += f[a];
        return s;
    }
}

template <int FL> FE_DEV void load_tile(const void *in, int64_t n, int64_t tile0, int4 q[SCAN_CHUNKS])
{
    for (int c = 0; c < SCAN_CHUNKS; ++c) {
        const int64_t base = tile0 + (int64_t)c * SCAN_CHUNK + 4 * (int64_t)threadIdx.x;
        if (base + 4 <= n) {
            if constexpr (FL == 0) {
                q[c] = *reinterpret_cast<const int4 *>(static_cast<const int32_t *>(in) + base);
            } else {
                // 4 elements = FL aligned words (base is a multiple of 4)
                const uint32_t *p = reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(in) + FL * base);
                uint32_t w[FL];
#pragma unroll
                for (int j = 0; j < FL; ++j) w[j] = p[j];
                int32_t e[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    e[k] = 0;
#pragma unroll
                    for (int a = 0; a < FL; ++a) {
                        const int j = k * FL + a;
                        e[k] += (int32_t)((w[j >> 2] >> (8 * (j & 3))) & 0xffu);
                    }
                }
                q[c] = make_int4(e[0], e[1], e[2], e[3]);
            }
        } else {
            q[c].x = (base + 0 < n) ? in_at<FL>(in, base + 0) : 0;
            q[c].y = (base + 1 < n) ? in_at<FL>(in, base + 1) : 0;
            q[c].z = (base + 2 < n) ? in_at<FL>(in, base + 2) : 0;
            q[c].w = (base + 3 < n) ? in_at<FL>(in, base + 3) : 0;
        }
    }
}

FE_DEV int64_t sum4(int4 q) { return (int64_t)q.x + q.y + q.z + q.w; }

template <int FL>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const void *in, int64_t n, int64_t *part)
{
    __shared__ int64_t lds[2 * (SCAN_BLOCK / 64)];
    int4 q[SCAN_CHUNKS];
    load_tile<FL>(in, n, (int64_t)blockIdx.x * SCAN_TILE, q);
    int64_t s = 0;
    for (int c = 0; c < SCAN_CHUNKS; ++c) s += sum4(q[c]);
    int64_t tot;
    block_exclusive(s, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// The scan's total: to *total_dev and out[n], with the int32 overflow check.
FE_DEV void scan_total(int64_t carry, int64_t *total_dev, int32_t *out, int64_t n, int32_t *status)
{
    *total_dev = carry;
    if (carry > INT32_MAX) atomicOr(status + ST_ERR, ERR_OVERFLOW);
    out[n] = (int32_t)carry;
}

// One block: exclusive scan of part[0..nb) in place (for more than
// SCAN_DIRECT_TILES tiles).  Each thread owns a contiguous run of partials: a
// serial sum, one block scan of the run sums, then a serial pass writing the
// run's offsets.
constexpr int SP_BLOCK = 1024;

__global__ __launch_bounds__(SP_BLOCK) void k_scan_partials(int64_t *part, int64_t nb, int64_t *total_dev,
                                                            int32_t *out, int64_t n, int32_t *status)
{
    __shared__ int64_t lds[2 * (SP_BLOCK / 64)];
    const int64_t per = (nb + SP_BLOCK - 1) / SP_BLOCK;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    const int64_t b1 = (b0 + per < nb) ? b0 + per : nb;
    int64_t s = 0;
    for (int64_t k = b0; k < b1; ++k) s += part[k];
    int64_t carry;
    int64_t ex = block_exclusive<SP_BLOCK>(s, lds, &carry);
    for (int64_t k = b0; k < b1; ++k) {
        const int64_t v = part[k];
        part[k] = ex;
        ex += v;
    }
    if (threadIdx.x == 0) scan_total(carry, total_dev, out, n, status);
}

// DIRECT: part[] holds the tile sums and block b adds part[0..b) itself; the
// last block also writes the total.  Otherwise part[] already holds the tiles'
// exclusive offsets.
template <bool DIRECT, int FL>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const void *in, int32_t *out, int64_t n,
                                                           const int64_t *part, int64_t *total_dev, int32_t *status)
{
    __shared__ int64_t lds[2 * (SCAN_BLOCK / 64)];
    const int64_t tile0 = (int64_t)blockIdx.x * SCAN_TILE;
    int4 q[SCAN_CHUNKS];
    load_tile<FL>(in, n, tile0, q);
    int64_t carry;
    if (DIRECT) {
        int64_t s = 0;
        for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += SCAN_BLOCK) s += part[j];
        block_exclusive(s, lds, &carry);
    } else {
        carry = part[blockIdx.x];
    }
    for (int c = 0; c < SCAN_CHUNKS; ++c) {
        const int64_t s = sum4(q[c]);
        int64_t tot;
        int64_t ex = carry + block_exclusive(s, lds, &tot);
        carry += tot;
        int32_t o[4];
        o[0] = (int32_t)ex; ex += q[c].x;
        o[1] = (int32_t)ex; ex += q[c].y;
        o[2] = (int32_t)ex; ex += q[c].z;
        o[3] = (int32_t)ex;
        const int64_t base = tile0 + (int64_t)c * SCAN_CHUNK + 4 * (int64_t)threadIdx.x;
        if (base + 4 <= n) {
            *reinterpret_cast<int4 *>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
        } else {
            for (int k = 0; k < 4; ++k)
                if (base + k < n) out[base + k] = o[k];
        }
    }
    if (DIRECT && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) scan_total(carry, total_dev, out, n, status);
}

// p[0..n) = v: 16-byte stores over the aligned middle, element stores at the ends.
template <typename T> __global__ void k_fill(T *p, int64_t n, T v)
{
    constexpr int PER = 16 / sizeof(T);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t head = (int64_t)((16 - ((uintptr_t)p & 15)) & 15) / (int64_t)sizeof(T);
    if ((uintptr_t)p % sizeof(T)) head = n;     // misaligned element type: element stores only
    if (head > n) head = n;
    const int64_t nv = (n - head) / PER;
    for (int64_t i = tid; i < head; i += stride) p[i] = v;
    for (int64_t k = (n - head) % PER, i = tid; i < k; i += stride) p[head + nv * PER + i] = v;
    union { T e[PER]; uint4 q; } u;
    for (int k = 0; k < PER; ++k) u.e[k] = v;
    uint4 *pv = reinterpret_cast<uint4 *>(p + head);
    for (int64_t i = tid; i < nv; i += stride) pv[i] = u.q;
}

template <typename T> int fill(T *p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return FE_OK;
    int64_t blocks = cdiv(cdiv(n, 16 / (int64_t)sizeof(T)), 256);
    if (blocks > 8192) blocks = 8192;
    FE_TIMED("k_fill", s,
             hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v));
    return fe_launch_check();
}

__global__ void k_select(int64_t n, const uint8_t *__restrict__ mask, const double *a, const double *b, double *out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = mask[i] ? (a ? a[i] : 0.0) : (b ? b[i] : 0.0);
}

}  // namespace

extern "C" int fe_select(int64_t n, const uint8_t *mask, const double *a, const double *b, double *out, void *stream)
{
    if (n < 0 || (n > 0 && (!mask || !out))) return FE_EINVAL;
    if (n == 0) return FE_OK;
    int64_t blocks = cdiv(n, 256);
    if (blocks > 16384) blocks = 16384;
    FE_TIMED("k_select", static_cast<hipStream_t>(stream),
             hipLaunchKernelGGL(k_select, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), n, mask, a,
                           b, out));
    return fe_launch_check();
}

int64_t fe_scan_part_elems(int64_t n) { return cdiv(n > 0 ? n : 1, SCAN_TILE) + 1; }

namespace {

template <int FL>
int scan_exclusive(const void *in, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part, int32_t *status,
                   hipStream_t s)
{
    const int64_t nb = cdiv(n > 0 ? n : 1, SCAN_TILE);
    FE_TIMED("k_scan_reduce", s,
             hipLaunchKernelGGL(k_scan_reduce<FL>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, part));
    if (nb <= SCAN_DIRECT_TILES) {
        FE_TIMED("k_scan_apply", s,
                 hipLaunchKernelGGL((k_scan_apply<true, FL>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n,
                                    part, total_dev, status));
    } else {
        FE_TIMED("k_scan_partials", s,
                 hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SP_BLOCK), 0, s, part, nb, total_dev, out, n,
                                    status));
        FE_TIMED("k_scan_apply", s,
                 hipLaunchKernelGGL((k_scan_apply<false, FL>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n,
                                    part, total_dev, status));
    }
    return fe_launch_check();
}

}  // namespace

int fe_scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part,
                      int32_t *status, hipStream_t s)
{
    // in/out must be 16-byte aligned (workspace arrays are 256-byte aligned).
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return FE_EINVAL;
    return scan_exclusive<0>(in, out, n, total_dev, part, status, s);
}

int fe_scan_exclusive_flags(const uint8_t *flags, int nv, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part,
                            int32_t *status, hipStream_t s)
{
    if (((uintptr_t)flags & 3) || ((uintptr_t)out & 15) || (nv != 3 && nv != 4)) return FE_EINVAL;
    return nv == 3 ? scan_exclusive<3>(flags, out, n, total_dev, part, status, s)
                   : scan_exclusive<4>(flags, out, n, total_dev, part, status, s);
}

int fe_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) { return fill<int32_t>(p, n, v, s); }
int fe_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) { return fill<uint8_t>(p, n, v, s); }
int fe_fill_f64(double *p, int64_t n, double v, hipStream_t s) { return fill<double>(p, n, v, s); }

int fe_status_from_bits(int32_t bits)
{
    if (bits & ERR_OVERFLOW) return FE_EOVERFLOW;
    if (bits & (ERR_INDEX | ERR_BDCODE | ERR_KAPPA)) return FE_EINVAL;
    if (bits & ERR_ROBIN) return FE_EUNSUPPORTED;
    if (bits & (ERR_REPEAT | ERR_MEASURE)) return FE_EMESH;
    if (bits & ERR_LIMIT) return FE_ELIMIT;
    return FE_OK;
}

extern "C" const char *fe_version(void) { return "femhip 0.1 (gfx950)"; }

extern "C" const char *fe_status_string(int status)
{
    switch (status) {
    case FE_OK: return "ok";
    case FE_EINVAL: return "invalid argument";
    case FE_EMESH: return "invalid element (non-positive measure or repeated vertex)";
    case FE_EUNSUPPORTED: return "unsupported (dimension or boundary type)";
    case FE_EOVERFLOW: return "size exceeds the int32 index range";
    case FE_ESIZE: return "workspace too small";
    case FE_EHIP: return "HIP runtime error";
    case FE_ENOCONV: return "iteration limit reached before the tolerance";
    case FE_ELIMIT: return "a fixed capacity was exceeded (row width, vertex count, instances, or grid wait)";
    default: return "unknown status";
    }
}
