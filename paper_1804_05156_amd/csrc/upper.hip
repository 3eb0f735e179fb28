// upper.hip -- symmetric storage: the upper triangle of A (diagonal included).
//
// A is symmetric (each local matrix K_t is, Section 3.1), so its upper triangle
// holds every value; the remark on symmetry in Section 3.1.3 computes only the
// entries j >= i of each local matrix for the same reason.  Here the upper
// triangle is a CSR matrix of its own (rowptr_u, colind_u; label order, columns
// ascending), filled by fe_assemble_upper.  Row i of triu(A) is the suffix of row i
// of A that starts at its diagonal, so both patterns come from the full one:
//   k_upper_len   the suffix length of every row (a search for i in row i),
//   (prefix sum)  rowptr_u,
//   k_upper_fill  colind_u, and vidx: for every entry q of the full pattern, the
//                 position in the upper storage of that entry (j >= i) or of its
//                 mirror (j, i) (j < i; a search for i in row j).
// With vidx the full matrix is read from the upper storage as val_u[vidx[q]]: the
// symmetric-storage SpMV and PCG of solve.hip.
#include "fe_internal.h"

namespace {

constexpr int UB = 256;

FE_DEV int32_t find_col(const int32_t *__restrict__ colind, int32_t lo, int32_t hi, int32_t x)
{
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (colind[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(UB) void k_upper_len(int32_t N, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colind, int32_t *ulen)
{
    const int32_t i = blockIdx.x * UB + threadIdx.x;
    if (i >= N) return;
    const int32_t s = rowptr[i], e = rowptr[i + 1];
    ulen[i] = e - find_col(colind, s, e, i);
}

__global__ __launch_bounds__(UB) void k_upper_fill(int32_t N, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colind,
                                                   const int32_t *__restrict__ rowptr_u, int32_t *colind_u,
                                                   int32_t *vidx)
{
    const int32_t i = blockIdx.x * UB + threadIdx.x;
    if (i >= N) return;
    const int32_t s = rowptr[i], e = rowptr[i + 1];
    const int32_t us = rowptr_u[i];
    const int32_t d = e - (rowptr_u[i + 1] - us);   // position of the diagonal in the full row
    for (int32_t q = s; q < d; ++q) {
        // (i, j), j < i: its mirror (j, i) in row j of the upper storage
        const int32_t j = colind[q];
        const int32_t sj = rowptr[j], ej = rowptr[j + 1];
        const int32_t dj = ej - (rowptr_u[j + 1] - rowptr_u[j]);
        vidx[q] = rowptr_u[j] + (find_col(colind, sj, ej, i) - dj);
    }
    for (int32_t q = d; q < e; ++q) {
        colind_u[us + (q - d)] = colind[q];
        vidx[q] = us + (q - d);
    }
}

}  // namespace

extern "C" int fe_plan_upper(fe_plan *plan, const int32_t *rowptr, const int32_t *colind, int32_t *rowptr_u,
                             int32_t *colind_u, int32_t *vidx, int64_t *nnz_u, void *stream)
{
    if (!plan || !rowptr || !rowptr_u || !nnz_u || (!colind && plan->nnz > 0)) return FE_EINVAL;
    if ((colind_u == nullptr) != (vidx == nullptr)) return FE_EINVAL;
    if ((uintptr_t)rowptr_u & 15) return FE_EINVAL;
    if (!plan->pattern_done) return FE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t N = (int32_t)plan->N;
    const unsigned g = (unsigned)cdiv(N, UB);
    FE_TIMED("k_upper_len", s,
             hipLaunchKernelGGL(k_upper_len, dim3(g), dim3(UB), 0, s, N, rowptr, colind, rowptr_u));
    int rc = fe_launch_check();
    if (rc) return rc;
    if ((rc = fe_scan_exclusive(rowptr_u, rowptr_u, N, plan->totals + 5, plan->part, plan->status, s))) return rc;
    if (colind_u)
        FE_TIMED("k_upper_fill", s,
                 hipLaunchKernelGGL(k_upper_fill, dim3(g), dim3(UB), 0, s, N, rowptr, colind,
                                    (const int32_t *)rowptr_u, colind_u, vidx));
    if ((rc = fe_launch_check())) return rc;
    int32_t total = 0;
    FE_HIP_CHECK(hipMemcpyAsync(&total, rowptr_u + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    *nnz_u = total;
    return FE_OK;
}
