// util.hip -- prefix sum, fill kernels and status helpers of the library.
#include "fe_internal.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;                       // one int4 per thread
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;  // 1024 elements per block

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

FE_DEV void load_items(const int32_t *in, int64_t n, int64_t base, int32_t v[SCAN_ITEMS])
{
    if (base + SCAN_ITEMS <= n) {
        int4 q = *reinterpret_cast<const int4 *>(in + base);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = (base + k < n) ? in[base + k] : 0;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t *in, int64_t n, int64_t *part)
{
    __shared__ int64_t lds[2 * (SCAN_BLOCK / 64)];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    load_items(in, n, base, v);
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    int64_t tot;
    block_exclusive(s, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block: exclusive scan of part[0..nb), total to part[nb] and *total_dev.  Each
// thread owns a contiguous run of partials: a serial sum, one block scan of the run
// sums, then a serial pass writing the run's offsets.
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
    if (threadIdx.x == 0) {
        part[nb] = carry;
        *total_dev = carry;
        if (carry > INT32_MAX) atomicOr(status + ST_ERR, ERR_OVERFLOW);
        out[n] = (int32_t)carry;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const int32_t *in, int32_t *out, int64_t n,
                                                           const int64_t *part)
{
    __shared__ int64_t lds[2 * (SCAN_BLOCK / 64)];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    load_items(in, n, base, v);
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    int64_t tot;
    int64_t ex = block_exclusive(s, lds, &tot) + part[blockIdx.x];
    int32_t o[SCAN_ITEMS];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        o[k] = (int32_t)ex;
        ex += v[k];
    }
    if (base + SCAN_ITEMS <= n) {
        *reinterpret_cast<int4 *>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
    } else {
        for (int k = 0; k < SCAN_ITEMS; ++k)
            if (base + k < n) out[base + k] = o[k];
    }
}

template <typename T> __global__ void k_fill(T *p, int64_t n, T v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T> int fill(T *p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return FE_OK;
    int64_t blocks = cdiv(n, 256);
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

int fe_scan_exclusive(const int32_t *in, int32_t *out, int64_t n, int64_t *total_dev, int64_t *part,
                      int32_t *status, hipStream_t s)
{
    // in/out must be 16-byte aligned (workspace arrays are 256-byte aligned).
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return FE_EINVAL;
    const int64_t nb = cdiv(n > 0 ? n : 1, SCAN_TILE);
    FE_TIMED("k_scan_reduce", s,
             hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, part));
    FE_TIMED("k_scan_partials", s,
             hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SP_BLOCK), 0, s, part, nb, total_dev, out, n, status));
    FE_TIMED("k_scan_apply", s,
             hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n, part));
    return fe_launch_check();
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
