// cg_common.h -- the per-row arithmetic and reductions of preconditioned CG, shared
// by the single-system solve and the batched solve so that both perform the same
// operations in the same order (a batched instance reproduces the single-system
// iterates bit for bit).
#pragma once

#include "fe_internal.h"

constexpr int CG_UNIT = 256;   // rows per reduction unit (= threads per block)

// Row i at the start: r_i = b_i - (A x)_i and the diagonal entry.
FE_DEV void cg_init_row(int32_t i, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                        const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
                        double *ri, double *di)
{
    double s = 0.0, d = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t c = colind[q];
        s += val[q] * x[c];
        if (c == i) d = val[q];
    }
    *di = d;
    *ri = b[i] - s;
}

// (A p_new)_i with p_new = z + beta p_old formed on the fly.
FE_DEV double cg_apply_row(int32_t i, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                           const double *__restrict__ val, const double *__restrict__ z,
                           const double *__restrict__ pold, double beta)
{
    double s = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t c = colind[q];
        s += val[q] * (z[c] + beta * pold[c]);
    }
    return s;
}

// Sum of part[0..nb) in a fixed order: thread t adds part[t], part[t+256], ...,
// then the block tree of block_sum.  The result is valid in thread 0.
FE_DEV double cg_sum_partials(const double *part, int32_t nb, double *lds)
{
    double v = 0.0;
    for (int32_t k = threadIdx.x; k < nb; k += CG_UNIT) v += part[k];
    return block_sum<CG_UNIT>(v, lds);
}

// True in every thread of the block that arrives last at `ticket` among `count`
// arrivals; it then sees every partial written before the other arrivals.  The
// last block resets the ticket.
FE_DEV bool cg_last_arrival(int32_t *ticket, int32_t count)
{
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t prev = atomicAdd(ticket, 1);
        is_last = (prev == count - 1);
        if (is_last) *ticket = 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}
