// cg_common.h -- the per-row arithmetic and reductions of preconditioned CG, shared
// by the single-system solve and the batched solve so that both perform the same
// operations in the same order (a batched instance reproduces the single-system
// iterates bit for bit).
#pragma once

#include "fe_internal.h"

constexpr int CG_UNIT = 256;   // rows per reduction unit (= threads per block)

// Stored value of entry q of the pattern: val[q], or with IND (symmetric storage of
// the upper triangle) val[vidx[q]], the entry itself or its mirror across the
// diagonal.
template <bool IND> FE_DEV double cg_value(const double *__restrict__ val, const int32_t *__restrict__ vidx, int32_t q)
{
    return IND ? val[vidx[q]] : val[q];
}

// Row i at the start: r_i = b_i - (A x)_i and the diagonal entry.
template <bool IND = false>
FE_DEV void cg_init_row(int32_t i, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                        const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
                        double *ri, double *di, const int32_t *__restrict__ vidx = nullptr)
{
    double s = 0.0, d = 0.0;
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int32_t c = colind[q];
        const double v = cg_value<IND>(val, vidx, q);
        s += v * x[c];
        if (c == i) d = v;
    }
    *di = d;
    *ri = b[i] - s;
}

// s[j] = (A p_new)_{i[j]} with p_new = z + beta[j] p_old formed on the fly, for K rows
// at once (rows with ok[j] false are skipped).  Each row is walked in chunks of CH
// entries: all column indices and values of a chunk are loaded, then all gathers
// of z and p_old, then the products are added in column order, so the loads of a
// chunk overlap instead of forming one dependent chain per entry.  The products are
// added in column order whatever CH is, so CH never changes a result bit.
template <int K, int CH = (K >= 4 ? 2 : (K == 2 ? 4 : 8)), bool IND = false>
FE_DEV void cg_apply_rows(const int32_t *i, const bool *ok, const int32_t *__restrict__ rowptr,
                          const int32_t *__restrict__ colind, const double *__restrict__ val,
                          const double *__restrict__ z, const double *__restrict__ pold, const double *beta, double *s,
                          const int32_t *__restrict__ vidx = nullptr)
{
    int32_t q[K], e[K];
    int32_t len = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        s[j] = 0.0;
        q[j] = ok[j] ? rowptr[i[j]] : 0;
        e[j] = ok[j] ? rowptr[i[j] + 1] : 0;
        len = max(len, e[j] - q[j]);
    }
    for (int32_t m0 = 0; m0 < len; m0 += CH) {
        int32_t c[K][CH];
        double v[K][CH], zz[K][CH], pp[K][CH];
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int t = 0; t < CH; ++t)
                if (q[j] + m0 + t < e[j]) {
                    c[j][t] = colind[q[j] + m0 + t];
                    v[j][t] = cg_value<IND>(val, vidx, q[j] + m0 + t);
                }
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int t = 0; t < CH; ++t)
                if (q[j] + m0 + t < e[j]) {
                    zz[j][t] = z[c[j][t]];
                    pp[j][t] = pold[c[j][t]];
                }
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int t = 0; t < CH; ++t)
                if (q[j] + m0 + t < e[j]) s[j] += v[j][t] * (zz[j][t] + beta[j] * pp[j][t]);
    }
}

// Sum of part[0..nb) in a fixed order: thread t adds part[t], part[t+256], ...,
// then the block tree of block_sum.  The result is valid in thread 0.  The loads go
// out eight at a time ahead of their additions (the partials were just written by
// another kernel: one round trip per eight instead of one per partial).
FE_DEV double cg_sum_partials(const double *part, int32_t nb, double *lds)
{
    constexpr int PB = 8;
    double v = 0.0;
    for (int32_t k0 = threadIdx.x; k0 < nb; k0 += PB * CG_UNIT) {
        double x[PB];
#pragma unroll
        for (int q = 0; q < PB; ++q) x[q] = (k0 + q * CG_UNIT < nb) ? part[k0 + q * CG_UNIT] : 0.0;
#pragma unroll
        for (int q = 0; q < PB; ++q)
            if (k0 + q * CG_UNIT < nb) v += x[q];
    }
    return block_sum<CG_UNIT>(v, lds);
}
