// plan.hip -- symbolic phase: everything that depends on elem and bdflag only.
//
// The duplicate summation of `sparse` (Section 2.2) needs, for every vertex i, the
// list of element contributions to row i.  It is built here as a counting sort of
// the (dim+1)*NT vertex-element incidences by vertex, each list then sorted by
// element so that every sum later runs in ascending element order (this fixes the
// rounding, whatever the thread schedule).
//
// Rows are processed in an order chosen for memory locality, not in label order:
// vertex v gets processing position = rank of its first incidence (smallest
// t*nv + a).  For meshes stored element by element in a spatial order this walks
// the mesh in that order even when the vertex labels are randomly permuted, so the
// gathers of element data in the numeric kernel stay within a small window.
#include <climits>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fe_internal.h"

namespace {

constexpr int EBLOCK = 256;   // element-parallel kernels

template <int NV>
__global__ __launch_bounds__(EBLOCK) void k_sym_count(const int32_t *__restrict__ elem, const int8_t *__restrict__ bd,
                                                      int32_t NT, int32_t N, int32_t *deg, int32_t *owner,
                                                      int32_t *rank, uint8_t *isd, int32_t *status)
{
    const int32_t t = blockIdx.x * EBLOCK + threadIdx.x;
    if (t >= NT) return;
    int32_t v[NV];
    int32_t err = 0;
    for (int a = 0; a < NV; ++a) {
        v[a] = elem[(int64_t)a * NT + t];
        if ((uint32_t)v[a] >= (uint32_t)N) err |= ERR_INDEX;
    }
    if (!err)
        for (int a = 0; a < NV; ++a)
            for (int b = a + 1; b < NV; ++b)
                if (v[a] == v[b]) err |= ERR_REPEAT;
    int8_t code[NV];
    for (int f = 0; f < NV; ++f) {
        code[f] = bd ? bd[(int64_t)f * NT + t] : 0;
        if (code[f] < 0 || code[f] > 3) err |= ERR_BDCODE;
        else if (code[f] == 3) err |= ERR_ROBIN;
    }
    if (err) {
        atomicOr(status + ST_ERR, err);
        return;
    }
    for (int a = 0; a < NV; ++a) {
        rank[(int64_t)a * NT + t] = atomicAdd(deg + v[a], 1);
        atomicMin(owner + v[a], t * NV + a);
    }
    for (int f = 0; f < NV; ++f)
        if (code[f] == FE_BD_DIRICHLET)
            for (int e = 0; e < NV; ++e)
                if (e != f) isd[v[e]] = 1;
}

template <int NV>
__global__ __launch_bounds__(EBLOCK) void k_sym_own_count(const int32_t *__restrict__ elem, int32_t NT,
                                                          const int32_t *__restrict__ owner, int32_t *owncnt)
{
    const int32_t t = blockIdx.x * EBLOCK + threadIdx.x;
    if (t >= NT) return;
    int c = 0;
    for (int a = 0; a < NV; ++a) c += (owner[elem[(int64_t)a * NT + t]] == t * NV + a);
    owncnt[t] = c;
}

template <int NV>
__global__ __launch_bounds__(EBLOCK) void k_sym_pi(const int32_t *__restrict__ elem, int32_t NT,
                                                   const int32_t *__restrict__ owner, const int32_t *__restrict__ ownoff,
                                                   const int32_t *__restrict__ deg, int32_t *pi, int32_t *piinv,
                                                   int32_t *pdeg)
{
    const int32_t t = blockIdx.x * EBLOCK + threadIdx.x;
    if (t >= NT) return;
    int32_t j = ownoff[t];
    for (int a = 0; a < NV; ++a) {
        const int32_t v = elem[(int64_t)a * NT + t];
        if (owner[v] == t * NV + a) {
            pi[j] = v;
            piinv[v] = j;
            pdeg[j] = deg[v];
            ++j;
        }
    }
}

// Vertices used by no element go after the used ones (their rows are empty); their
// relative order does not affect any value.
__global__ __launch_bounds__(EBLOCK) void k_sym_unused(int32_t N, const int32_t *__restrict__ deg,
                                                       const int64_t *__restrict__ nused, int32_t *pi,
                                                       int32_t *piinv, int32_t *pdeg, int32_t *status)
{
    const int32_t v = blockIdx.x * EBLOCK + threadIdx.x;
    if (v >= N) return;
    if (deg[v] == 0) {
        const int32_t k = (int32_t)(*nused) + atomicAdd(status + ST_UNUSED, 1);
        pi[k] = v;
        piinv[v] = k;
        pdeg[k] = 0;
    }
}

template <int NV>
__global__ __launch_bounds__(EBLOCK) void k_sym_fill(const int32_t *__restrict__ elem, int32_t NT,
                                                     const int32_t *__restrict__ piinv,
                                                     const int32_t *__restrict__ pincptr,
                                                     const int32_t *__restrict__ rank, int32_t *pinc)
{
    const int32_t t = blockIdx.x * EBLOCK + threadIdx.x;
    if (t >= NT) return;
    for (int a = 0; a < NV; ++a) {
        const int32_t v = elem[(int64_t)a * NT + t];
        pinc[pincptr[piinv[v]] + rank[(int64_t)a * NT + t]] = t * NV + a;
    }
}

// Per row (one thread, processing order): sort the incidence keys ascending, then
// build the sorted set of columns {i} u {vertices of the incident elements}.
//   FINAL = false: write the row length (label order); keep the sorted keys.
//   FINAL = true:  write colind, the per-incidence metadata and the row info.
template <int NV, bool FINAL>
__global__ __launch_bounds__(RowCaps<NV>::BLOCK) void k_sym_rows(
    const int32_t *__restrict__ elem, const int8_t *__restrict__ bd, int32_t NT, int32_t N,
    const int32_t *__restrict__ pi, const int32_t *__restrict__ pincptr, int32_t *pinc, int32_t *rowlen,
    const int32_t *__restrict__ rowptr, const uint8_t *__restrict__ isd, int32_t *colind, uint32_t *pmeta,
    int32_t *prow_start, uint32_t *prow_info, int32_t *status)
{
    constexpr int B = RowCaps<NV>::BLOCK, DEGCAP = RowCaps<NV>::DEG, COLCAP = RowCaps<NV>::COL;
    __shared__ int32_t keys[DEGCAP * B];
    __shared__ int32_t cols[COLCAP * B];
    const int tid = threadIdx.x;
    const int32_t k = blockIdx.x * B + tid;
    if (k >= N) return;
    const int32_t i = pi[k];
    const int32_t s = pincptr[k];
    const int32_t d = pincptr[k + 1] - s;
    if (d == 0) {   // vertex of no element: empty row, as sparse() would give
        if (!FINAL) {
            rowlen[i] = 0;
        } else {
            prow_start[k] = rowptr[i];
            prow_info[k] = 0;
        }
        return;
    }
    if (d > DEGCAP) {
        atomicOr(status + ST_ERR, ERR_LIMIT);
        if (!FINAL) rowlen[i] = 0;
        return;
    }
    for (int j = 0; j < d; ++j) keys[j * B + tid] = pinc[s + j];
    if (!FINAL) {
        for (int j = 1; j < d; ++j) {   // insertion sort (lists are short)
            int32_t x = keys[j * B + tid];
            int m = j - 1;
            while (m >= 0 && keys[m * B + tid] > x) {
                keys[(m + 1) * B + tid] = keys[m * B + tid];
                --m;
            }
            keys[(m + 1) * B + tid] = x;
        }
        for (int j = 0; j < d; ++j) pinc[s + j] = keys[j * B + tid];
    }
    // sorted unique column set
    int u = 1;
    cols[tid] = i;
    bool over = false;
    for (int j = 0; j < d && !over; ++j) {
        const int32_t key = keys[j * B + tid];
        const int32_t t = key / NV;
        const int a = key - t * NV;
        for (int jj = 0; jj < NV - 1; ++jj) {
            const int b = fe_other<NV>(a, jj);
            const int32_t c = elem[(int64_t)b * NT + t];
            int m = 0;
            while (m < u && cols[m * B + tid] < c) ++m;
            if (m < u && cols[m * B + tid] == c) continue;
            if (u == COLCAP) { over = true; break; }
            for (int q = u; q > m; --q) cols[q * B + tid] = cols[(q - 1) * B + tid];
            cols[m * B + tid] = c;
            ++u;
        }
    }
    if (over) {
        atomicOr(status + ST_ERR, ERR_LIMIT);
        if (!FINAL) rowlen[i] = 0;
        return;
    }
    if (!FINAL) {
        rowlen[i] = u;
        atomicMax(status + ST_MAXROW, u);
        atomicMax(status + ST_MAXDEG, d);
        if (isd[i]) atomicAdd(status + ST_NDIR, 1);
        return;
    }
    const int32_t rs = rowptr[i];
    int diag = 0;
    for (int m = 0; m < u; ++m) {
        const int32_t c = cols[m * B + tid];
        colind[rs + m] = c;
        if (c == i) diag = m;
    }
    for (int j = 0; j < d; ++j) {
        const int32_t key = keys[j * B + tid];
        const int32_t t = key / NV;
        const int a = key - t * NV;
        uint32_t meta = (uint32_t)a;
        for (int jj = 0; jj < NV - 1; ++jj) {
            const int b = fe_other<NV>(a, jj);
            const int32_t c = elem[(int64_t)b * NT + t];
            int m = 0;
            while (cols[m * B + tid] != c) ++m;   // present by construction
            meta |= (uint32_t)m << (Meta<NV>::OFF + 8 * jj);
            if (isd[c]) meta |= 1u << (Meta<NV>::DBIT + jj);
            if (bd && bd[(int64_t)b * NT + t] == FE_BD_NEUMANN) meta |= 1u << (Meta<NV>::NBIT + jj);
        }
        pmeta[s + j] = meta;
    }
    prow_start[k] = rs;
    prow_info[k] = (uint32_t)u | ((uint32_t)diag << 8) | ((uint32_t)(isd[i] ? 1 : 0) << 16);
}

struct Layout {
    size_t off[20];
    size_t total;
};

// Workspace layout (every array 256-byte aligned).
Layout plan_layout(int64_t N, int64_t NT, int nv)
{
    const int64_t ninc = (int64_t)nv * NT;
    const int64_t npart = fe_scan_part_elems(N > NT ? (N > ninc ? N : ninc) : (NT > ninc ? NT : ninc));
    const size_t sz[] = {
        sizeof(int32_t) * ST_COUNT,             // 0 status
        sizeof(int64_t) * 4,                    // 1 totals
        sizeof(int64_t) * (size_t)(npart + 1),  // 2 part
        sizeof(int32_t) * (size_t)N,            // 3 deg
        sizeof(int32_t) * (size_t)N,            // 4 owner
        sizeof(uint8_t) * (size_t)N,            // 5 isd
        sizeof(int32_t) * (size_t)ninc,         // 6 rank
        sizeof(int32_t) * (size_t)(NT + 1),     // 7 owncnt
        sizeof(int32_t) * (size_t)N,            // 8 pi
        sizeof(int32_t) * (size_t)N,            // 9 piinv
        sizeof(int32_t) * (size_t)(N + 1),      // 10 pincptr
        sizeof(int32_t) * (size_t)ninc,         // 11 pinc
        sizeof(uint32_t) * (size_t)ninc,        // 12 pmeta
        sizeof(int32_t) * (size_t)(N + 1),      // 13 rowlen / rowptr
        sizeof(int32_t) * (size_t)N,            // 14 prow_start
        sizeof(uint32_t) * (size_t)N,           // 15 prow_info
    };
    Layout L{};
    size_t o = 0;
    for (int k = 0; k < 16; ++k) {
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
    return FE_OK;
}

template <int NV> int plan_build(fe_plan *P, hipStream_t s)
{
    const int32_t N = (int32_t)P->N, NT = (int32_t)P->NT;
    const unsigned eg = (unsigned)cdiv(NT > 0 ? NT : 1, EBLOCK);
    const unsigned ng = (unsigned)cdiv(N, EBLOCK);
    int rc;
    if ((rc = fe_fill_i32(P->status, ST_COUNT, 0, s))) return rc;
    if ((rc = fe_fill_i32(P->deg, N, 0, s))) return rc;
    if ((rc = fe_fill_i32(P->owner, N, INT32_MAX, s))) return rc;
    if ((rc = fe_fill_u8(P->isd, N, 0, s))) return rc;
    if (NT > 0)
        hipLaunchKernelGGL(k_sym_count<NV>, dim3(eg), dim3(EBLOCK), 0, s, P->elem, P->bdflag, NT, N, P->deg,
                           P->owner, P->rank, P->isd, P->status);
    if ((rc = fe_launch_check())) return rc;
    // Vertex indices are validated by the count kernel only: stop here, before any
    // kernel uses elem entries as addresses, if one was out of range.
    int32_t err = 0;
    FE_HIP_CHECK(hipMemcpyAsync(&err, P->status + ST_ERR, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (err) return fe_status_from_bits(err);
    if (NT > 0)
        hipLaunchKernelGGL(k_sym_own_count<NV>, dim3(eg), dim3(EBLOCK), 0, s, P->elem, NT, P->owner, P->owncnt);
    if ((rc = fe_scan_exclusive(P->owncnt, P->owncnt, NT, P->totals + 0, P->part, P->status, s))) return rc;
    if (NT > 0)
        hipLaunchKernelGGL(k_sym_pi<NV>, dim3(eg), dim3(EBLOCK), 0, s, P->elem, NT, P->owner, P->owncnt, P->deg,
                           P->pi, P->piinv, P->pincptr);
    hipLaunchKernelGGL(k_sym_unused, dim3(ng), dim3(EBLOCK), 0, s, N, P->deg, P->totals + 0, P->pi, P->piinv,
                       P->pincptr, P->status);
    if ((rc = fe_launch_check())) return rc;
    if ((rc = fe_scan_exclusive(P->pincptr, P->pincptr, N, P->totals + 1, P->part, P->status, s))) return rc;
    if (NT > 0)
        hipLaunchKernelGGL(k_sym_fill<NV>, dim3(eg), dim3(EBLOCK), 0, s, P->elem, NT, P->piinv, P->pincptr, P->rank,
                           P->pinc);
    constexpr int RB = RowCaps<NV>::BLOCK;
    hipLaunchKernelGGL((k_sym_rows<NV, false>), dim3((unsigned)cdiv(N, RB)), dim3(RB), 0, s, P->elem, P->bdflag, NT,
                       N, P->pi, P->pincptr, P->pinc, P->rowlen, (const int32_t *)nullptr, P->isd,
                       (int32_t *)nullptr, (uint32_t *)nullptr, (int32_t *)nullptr, (uint32_t *)nullptr, P->status);
    if ((rc = fe_launch_check())) return rc;
    if ((rc = fe_scan_exclusive(P->rowlen, P->rowlen, N, P->totals + 2, P->part, P->status, s))) return rc;
    int32_t st[ST_COUNT];
    int64_t tot[4];
    FE_HIP_CHECK(hipMemcpyAsync(st, P->status, sizeof(st), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipMemcpyAsync(tot, P->totals, sizeof(tot), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    if (st[ST_ERR]) return fe_status_from_bits(st[ST_ERR]);
    P->nused = tot[0];
    P->nnz = tot[2];
    P->max_row = st[ST_MAXROW];
    P->max_deg = st[ST_MAXDEG];
    P->ndir = st[ST_NDIR];
    if (tot[1] != P->ninc) return FE_EHIP;   // every incidence must be placed
    return FE_OK;
}

template <int NV> int plan_pattern(fe_plan *P, int32_t *rowptr, int32_t *colind, hipStream_t s)
{
    const int32_t N = (int32_t)P->N, NT = (int32_t)P->NT;
    FE_HIP_CHECK(hipMemcpyAsync(rowptr, P->rowlen, sizeof(int32_t) * (size_t)(N + 1), hipMemcpyDeviceToDevice, s));
    constexpr int RB = RowCaps<NV>::BLOCK;
    hipLaunchKernelGGL((k_sym_rows<NV, true>), dim3((unsigned)cdiv(N, RB)), dim3(RB), 0, s, P->elem, P->bdflag, NT, N,
                       P->pi, P->pincptr, P->pinc, (int32_t *)nullptr, (const int32_t *)P->rowlen, P->isd, colind,
                       P->pmeta, P->prow_start, P->prow_info, P->status);
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
    P->dim = mesh->dim;
    P->nv = nv;
    P->N = mesh->n_node;
    P->NT = mesh->n_elem;
    P->ninc = (int64_t)nv * mesh->n_elem;
    P->elem = mesh->elem;
    P->bdflag = mesh->bdflag;
    P->status = reinterpret_cast<int32_t *>(base + L.off[0]);
    P->totals = reinterpret_cast<int64_t *>(base + L.off[1]);
    P->part = reinterpret_cast<int64_t *>(base + L.off[2]);
    P->deg = reinterpret_cast<int32_t *>(base + L.off[3]);
    P->owner = reinterpret_cast<int32_t *>(base + L.off[4]);
    P->isd = reinterpret_cast<uint8_t *>(base + L.off[5]);
    P->rank = reinterpret_cast<int32_t *>(base + L.off[6]);
    P->owncnt = reinterpret_cast<int32_t *>(base + L.off[7]);
    P->pi = reinterpret_cast<int32_t *>(base + L.off[8]);
    P->piinv = reinterpret_cast<int32_t *>(base + L.off[9]);
    P->pincptr = reinterpret_cast<int32_t *>(base + L.off[10]);
    P->pinc = reinterpret_cast<int32_t *>(base + L.off[11]);
    P->pmeta = reinterpret_cast<uint32_t *>(base + L.off[12]);
    P->rowlen = reinterpret_cast<int32_t *>(base + L.off[13]);
    P->prow_start = reinterpret_cast<int32_t *>(base + L.off[14]);
    P->prow_info = reinterpret_cast<uint32_t *>(base + L.off[15]);
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
