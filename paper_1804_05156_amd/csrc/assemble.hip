// assemble.hip -- numeric phase: stiffness values, load vector and boundary
// conditions, one thread per row of A.
//
// A row i of A is the sum, over the elements t around vertex i, of row a of the
// local matrix of t (a = local index of i in t):
//     K_t[a][b] = kappa_t n_a . n_b / (d!^2 |t|)            (equation (dlambda))
// with n_c the scaled inward normal of the side opposite local vertex c (edge
// rotation in 2-D, cross product of two side edges in 3-D, Section 3.1.3).  The
// thread walks the row's incidence list (ascending element index, from the plan),
// recomputes the element geometry from the coordinates, and adds row a into an
// LDS accumulator slot per stored column.  This is the `sparse` duplicate sum of
// Section 2.2 done per row, in a fixed order, with no atomics and no triplet array.
// The same walk adds the load term of Section 3.2; a second walk, taken only by
// rows with a boundary bit, adds the Neumann and Robin side terms and the Dirichlet
// lifting of Section 3.3, so A, A_bc and b come out of one kernel.
//
// Memory layout.  Rows run in the plan's processing order (an order that follows
// the element order), so neighbouring threads touch neighbouring elements.  A
// prepass copies the coordinates into that order (xyp) once per call; the plan
// stores every element's vertices as processing positions (elemp).  All gathers of
// the main kernel (elemp[t], kappa[t], xyp[p]) are then spatially coherent even
// when the vertex labels are a random permutation; the only label-ordered
// accesses left are the row's own outputs.
#include <cmath>
#include <type_traits>

#include "fe_internal.h"

namespace {

struct AsmArgs {
    int32_t N, NT;
    const double *kappa;
    const int32_t *pi, *pincptr, *prowptr, *elemp;
    const int2 *pincm;
    const int32_t *sptr;   // 3-D sliced incidence layout (status[ST_SELL]; see inc_at)
    const uint32_t *prow_info;
    const double *xyp, *fp;
    DevFn f, gd, gn, gr;
    double ralpha;         // Robin coefficient alpha (kappa grad(u).n + alpha u = g_R)
    int32_t load_rule;     // FE_LOAD_*: quadrature of the load integrals
    double *valp;          // rows in processing order: row k at prowptr[k] + 2k, its values
                           // followed by (b, b_load)
    // direct: the processing order is the label order, and the rows go straight to
    // the outputs (row k of A at prowptr[k])
    int32_t direct;
    const int4 *precp;     // row records (.z, .w: Dirichlet-column mask), for val_bc
    // 3-D label-order processing with the register column set: each row's sorted
    // columns (processing positions), 16 per row, padded (the row passes' slots)
    const int32_t *rcols;
    // long rows (INFO_LONG), done by k_assemble_long: their processing positions, the
    // mesh's element array (labels), the label-order row pointer, the label-order
    // Dirichlet flags
    const int32_t *longk, *elem, *lrowptr;
    const uint8_t *isdl;
    // upper: only the upper triangle (columns from the diagonal on) is written, to
    // the symmetric storage whose label-order row starts are urowptr
    int32_t upper;
    const int32_t *urowptr;
    double *val, *val_bc, *b, *b_load;
    uint8_t *isd;
    int32_t *status;
};

// Coordinates (and nodal source values) in processing order: read in label order
// (coalesced) and write each vertex's record to its processing position (one 16-
// or 32-byte store per vertex, cheaper than gathering two 8-byte values).
template <int DIM>
__global__ __launch_bounds__(256) void k_scatter_coords(int32_t N, const int32_t *__restrict__ piinv,
                                                        const double *__restrict__ node, double *__restrict__ xyp,
                                                        const double *__restrict__ fnodal, double *__restrict__ fp)
{
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int32_t k = piinv[i];
    if (DIM == 2) {
        reinterpret_cast<double2 *>(xyp)[k] = make_double2(node[i], node[(int64_t)N + i]);
    } else {
        // (x, y), (z, nodal f): the coordinate loads of the 3-D kernel bring f along
        double2 *o = reinterpret_cast<double2 *>(xyp) + 2 * (int64_t)k;
        o[0] = make_double2(node[i], node[(int64_t)N + i]);
        o[1] = make_double2(node[2 * (int64_t)N + i], fnodal ? fnodal[i] : 0.0);
    }
    if (DIM == 2 && fnodal) fp[k] = fnodal[i];
}

template <int DIM> FE_DEV void load_label_xy(const double *node, int32_t N, int32_t v, double *x)
{
    for (int c = 0; c < DIM; ++c) x[c] = node[(int64_t)c * N + v];
}

// Value of g_D at the vertex with label v and coordinates x.
template <int DIM> FE_DEV double dirichlet_value(const DevFn &g, int32_t v, const double *x)
{
    if (g.kind == FE_FN_NODAL) return g.nodal[v];
    return fn_point<DIM>(g, x);
}

// Processing position of local vertex c of an element record (see EREC_POS).
FE_DEV int sel3(int4 q, int c) { return (c == 0 ? q.x : (c == 1 ? q.y : q.z)) & EREC_POS; }
FE_DEV int sel4(int4 q, int c) { return (c == 0 ? q.x : (c == 1 ? q.y : (c == 2 ? q.z : q.w))) & EREC_POS; }

// Write the accumulated row and its right-hand side entries, in processing order
// (consecutive threads write consecutive rows, so the stores are contiguous).
template <int BLOCK>
FE_DEV void write_row(const AsmArgs &A, const double *acc, int tid, int32_t k, int len, bool rowd, double bsum,
                      double lift, double gdi)
{
    if (A.direct) {
        // label order: A_bc replaces a Dirichlet row by the identity row and zeroes
        // Dirichlet columns (the row record holds the row's Dirichlet-column mask)
        const int4 r = A.precp[k];
        const int diag = (r.y >> 8) & 0xff;
        const int c0 = A.upper ? diag : 0;                          // first column written
        const int64_t start = A.upper ? (int64_t)A.urowptr[k] - c0 : A.prowptr[k];
        double *v = A.val + start;
        for (int c = c0; c < len; ++c) v[c] = acc[c * BLOCK + tid];
        if (A.val_bc) {
            const uint64_t dm = (uint64_t)(uint32_t)r.z | ((uint64_t)(uint32_t)r.w << 32);
            double *vb = A.val_bc + start;
            for (int c = c0; c < len; ++c) {
                double x = acc[c * BLOCK + tid];
                if (rowd) x = (c == diag) ? 1.0 : 0.0;
                else if ((dm >> c) & 1ull) x = 0.0;
                vb[c] = x;
            }
        }
        A.b[k] = rowd ? gdi : bsum - lift;
        if (A.b_load) A.b_load[k] = bsum;
        if (A.isd) A.isd[k] = (uint8_t)rowd;
        return;
    }
    double *row = A.valp + A.prowptr[k] + 2 * (int64_t)k;
    // (the upper form needs the columns from the diagonal on)
    for (int c = A.upper ? (int)((A.prow_info[k] >> 8) & 0xff) : 0; c < len; ++c) row[c] = acc[c * BLOCK + tid];
    row[len] = rowd ? gdi : bsum - lift;
    row[len + 1] = bsum;
}

// Processing-order row slots of one wavefront, written together.  Consecutive rows'
// slots (values, b, b_load) are consecutive in valp, so the wavefront's 64 slots form
// one range; each lane enters its slot's entries in an LDS map of the range, then
// the lanes walk the range on consecutive entries, which turns one partial-line
// store per lane and column into full-line stores.  Map entry: lane << 5 | column,
// column 30 for b and 31 for b_load (kept in rhs); a range longer than the map (a
// long row among the 64) takes the per-row writes.  map: (ROWCAP + 2) * 64 entries
// and rhs: 128 values, both the wavefront's own.
template <int ROWCAP, int BLOCK>
FE_DEV void write_rows_slots(const AsmArgs &A, const double *acc, uint16_t *map, double *rhs, int tid, int32_t k,
                             bool live, int len, int diag, bool rowd, double bsum, double lift, double gdi)
{
    static_assert(ROWCAP <= 16, "map entry fields");
    constexpr uint16_t NONE = 0xffff;
    const int lane = tid & 63;
    const int32_t kw0 = k - lane, kw1 = min(kw0 + 64, A.N);
    const int64_t S = (int64_t)A.prowptr[kw0] + 2 * (int64_t)kw0;
    const int32_t T = (int32_t)((int64_t)A.prowptr[kw1] + 2 * (int64_t)kw1 - S);
    if (T > (ROWCAP + 2) * 64) {   // (uniform in the wavefront: a long row among its rows)
        if (live) write_row<BLOCK>(A, acc, tid, k, len, rowd, bsum, lift, gdi);
        return;
    }
    for (int32_t p = lane; p < T; p += 64) map[p] = NONE;
    wave_lds_sync();
    if (live) {
        const int32_t base = (int32_t)((int64_t)A.prowptr[k] + 2 * (int64_t)k - S);
        // (the upper form needs the columns from the diagonal on)
        for (int c = A.upper ? diag : 0; c < len; ++c) map[base + c] = (uint16_t)((lane << 5) | c);
        map[base + len] = (uint16_t)((lane << 5) | 30);
        map[base + len + 1] = (uint16_t)((lane << 5) | 31);
        rhs[lane] = rowd ? gdi : bsum - lift;
        rhs[64 + lane] = bsum;
    }
    wave_lds_sync();
    double *out = A.valp + S;
    const double *accw = acc + (tid - lane);
    for (int32_t p = lane; p < T; p += 64) {
        const uint32_t ent = map[p];
        if (ent == NONE) continue;
        const int r = (int)(ent >> 5), c = (int)(ent & 31);
        out[p] = c < 30 ? accw[c * BLOCK + r] : rhs[(c - 30) * 64 + r];
    }
}

// Label-order rows of one wavefront, written together (label-order processing: the
// 64 rows are consecutive labels, so their outputs form one contiguous range of val
// and val_bc).  Each lane stores its row's (lane, column) pairs in an LDS map of the
// range; the lanes then walk the range on consecutive entries and store val and
// val_bc with full-line writes, instead of one partial line per lane and column.
// The map is the wavefront's own part of the stored-column array (ROWCAP ints per
// row), free once its walk is done; a range longer than the map (a long row among
// the 64) takes the per-row writes.  Map entry: lane (bits 8..13), column (0..7),
// val_bc is 0 (bit 16) or 1 (bit 17).  b, b_load and the Dirichlet mask are one word
// per row, written per lane.
template <int ROWCAP, int BLOCK>
FE_DEV void write_rows_direct(const AsmArgs &A, const double *acc, int32_t *map, int tid, int32_t k, bool live,
                              int len, int diag, bool rowd, double bsum, double lift, double gdi)
{
    static_assert(ROWCAP <= 256, "map entry fields");
    const int lane = tid & 63;
    const int32_t kw0 = k - lane, kw1 = min(kw0 + 64, A.N);
    const int32_t *rp = A.upper ? A.urowptr : A.prowptr;
    const int64_t S = rp[kw0];
    const int32_t T = (int32_t)((int64_t)rp[kw1] - S);
    const int c0 = A.upper ? diag : 0;   // first column written
    if (live) {
        A.b[k] = rowd ? gdi : bsum - lift;
        if (A.b_load) A.b_load[k] = bsum;
        if (A.isd) A.isd[k] = (uint8_t)rowd;
    }
    if (T > ROWCAP * 64) {   // (uniform in the wavefront: a long row among its rows)
        if (live) write_row<BLOCK>(A, acc, tid, k, len, rowd, bsum, lift, gdi);
        return;
    }
    for (int32_t p = lane; p < T; p += 64) map[p] = -1;   // (a long row's range stays unwritten)
    wave_lds_sync();
    if (live) {
        const int4 r = A.precp[k];
        const uint64_t dm = (uint64_t)(uint32_t)r.z | ((uint64_t)(uint32_t)r.w << 32);
        const int32_t base = (int32_t)((A.upper ? (int64_t)A.urowptr[k] - c0 : (int64_t)A.prowptr[k]) - S);
        for (int c = c0; c < len; ++c) {
            int32_t ent = (lane << 8) | c;
            if (rowd) ent |= (c == diag) ? (1 << 17) : (1 << 16);
            else if ((dm >> c) & 1ull) ent |= 1 << 16;
            map[base + c] = ent;
        }
    }
    wave_lds_sync();
    double *val = A.val + S, *vbc = A.val_bc ? A.val_bc + S : nullptr;
    const double *accw = acc + (tid - lane);
    for (int32_t p = lane; p < T; p += 64) {
        const int32_t ent = map[p];
        if (ent < 0) continue;
        const double x = accw[(ent & 0xff) * BLOCK + ((ent >> 8) & 0xff)];
        val[p] = x;
        if (vbc) vbc[p] = (ent & (1 << 17)) ? 1.0 : ((ent & (1 << 16)) ? 0.0 : x);
    }
}

// Label-order outputs from the processing-order rows: one wavefront per 64
// consecutive label rows, lanes writing consecutive entries of the rows' joint
// output range (fully coalesced stores); each source row is read once, whole.
// A_bc replaces Dirichlet rows by the identity row and zeroes Dirichlet columns
// (the row record holds the row's info word and its Dirichlet-column mask).
// UPPER: only each row's suffix from its diagonal, to the symmetric storage (rowptr
// is then its row pointer).
template <bool UPPER>
__global__ __launch_bounds__(256) void k_values_to_label(int32_t N, const int32_t *__restrict__ rowptr,
                                                         const int4 *__restrict__ rowrec,
                                                         const int32_t *__restrict__ piinv,
                                                         const double *__restrict__ valp, double *val, double *val_bc,
                                                         double *b, double *b_load, uint8_t *isd)
{
    __shared__ int32_t sdst[4][65];
    __shared__ int4 srec[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t i0 = (blockIdx.x * 4 + w) * 64;
    const int32_t i = i0 + lane;
    sdst[w][lane] = rowptr[min(i, N)];
    if (lane == 0) sdst[w][64] = rowptr[min(i0 + 64, N)];
    int4 rec = make_int4(0, 0, 0, 0);
    if (i < N) {
        rec = rowrec[i];
        if (!(rec.y & INFO_LONG)) {   // (a long row's outputs come from k_assemble_long)
            rec.x += 2 * piinv[i];                     // start of the row in valp
            const int len = rec.y & 0xff;
            const double bi = valp[rec.x + len], bl = b_load ? valp[rec.x + len + 1] : 0.0;
            b[i] = bi;
            if (b_load) b_load[i] = bl;
            if (isd) isd[i] = (uint8_t)((rec.y >> 16) & 1);
            if (UPPER) {
                // the row from its diagonal on: source, Dirichlet-column mask and the
                // diagonal's offset (0) shifted to the suffix
                const int doff = (rec.y >> 8) & 0xff;
                const uint64_t dm = ((uint64_t)(uint32_t)rec.z | ((uint64_t)(uint32_t)rec.w << 32)) >> doff;
                rec.x += doff;
                rec.y &= ~0xff00;
                rec.z = (int32_t)(uint32_t)dm;
                rec.w = (int32_t)(uint32_t)(dm >> 32);
            }
        }
    }
    srec[w][lane] = rec;
    __syncthreads();
    const int32_t base = sdst[w][0];
    const int32_t total = sdst[w][64] - base;
    // CU gathers per lane in flight, then their stores
    constexpr int CU = 4;
    for (int32_t e0 = lane; e0 < total; e0 += 64 * CU) {
        double v[CU];
        int row[CU], col[CU];
        bool lng[CU];
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
            row[u] = lo;
            col[u] = pos - sdst[w][lo];
            lng[u] = (srec[w][lo].y & INFO_LONG) != 0;
            v[u] = lng[u] ? 0.0 : valp[srec[w][lo].x + col[u]];
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int32_t e = e0 + 64 * u;
            if (e >= total) break;
            if (lng[u]) continue;
            const int32_t pos = base + e;
            val[pos] = v[u];
            if (val_bc) {
                const int4 r = srec[w][row[u]];
                const int c = col[u];
                const uint32_t info = (uint32_t)r.y;
                const uint64_t dm = (uint64_t)(uint32_t)r.z | ((uint64_t)(uint32_t)r.w << 32);
                double vb = v[u];
                if ((info >> 16) & 1u) vb = (c == (int)((info >> 8) & 0xffu)) ? 1.0 : 0.0;
                else if ((dm >> c) & 1ull) vb = 0.0;
                val_bc[pos] = vb;
            }
        }
    }
}

// ----------------------------------------------------------------------------- 2-D
// Local vertices are rotated so the row's vertex comes first: X0 = x_a,
// X1 = x_{a+1}, X2 = x_{a+2} (indices mod 3).  A cyclic rotation keeps the
// orientation, so with E0 = X2 - X1, E1 = X0 - X2, E2 = X1 - X0 (the edge vectors
// opposite X0, X1, X2) the doubled area is E1 x E2 > 0 and K[0][c] =
// kappa E0 . Ec / (2 * doubled area).
// Incidences are handled in batches of UNR whose loads are all issued before any
// arithmetic, to overlap the three dependent gathers (incidence -> element ->
// coordinates) across the batch.
template <int ROWCAP, int BLOCK, int UNR>
__global__ __launch_bounds__(BLOCK) void k_assemble_2d(AsmArgs A)
{
    __shared__ double acc[ROWCAP * BLOCK];
    constexpr bool SLOTW = ROWCAP <= 16;   // wavefront-wide slot writes (map entry fields)
    // each wavefront's own LDS: the source term at the midpoints of its rows' edges
    // during the walk (ROWCAP values per row, 8-column rows only), then its row-write
    // map and rhs values
    constexpr bool MIDC = ROWCAP <= 8;
    constexpr int WMID = MIDC ? ROWCAP * 64 : 0, WOUT = 128 + ((ROWCAP + 2) * 64 + 3) / 4;   // doubles
    constexpr int WREG = WMID > WOUT ? WMID : WOUT;
    __shared__ double wscr[SLOTW ? (BLOCK / 64) * WREG : 1];
    const int tid = threadIdx.x;
    double *wown = wscr + (SLOTW ? (tid >> 6) * WREG : 0);
    double *fmid = wown + (tid & 63);   // (column c of this lane's row at fmid[c * 64])
    const int32_t k = blockIdx.x * BLOCK + tid;
    // every thread reaches the block's row write (a barrier): rows past the end and
    // long rows (k_assemble_long) only skip the computation
    int len = 0, diag = 0;
    bool rowd = false, live = false;
    double bsum = 0.0, lift = 0.0, gdi = 0.0;
    do {
    if (k >= A.N) break;
    const int32_t s = A.pincptr[k], e = A.pincptr[k + 1];
    const uint32_t info = A.prow_info[k];
    if (info & INFO_LONG) break;
    live = true;
    len = info & 0xff;
    diag = (info >> 8) & 0xff;
    rowd = (info >> 16) & 1;
    for (int c = 0; c < len; ++c) acc[c * BLOCK + tid] = 0.0;
    const double2 X0 = reinterpret_cast<const double2 *>(A.xyp)[k];
    const double2 *xy = reinterpret_cast<const double2 *>(A.xyp);
    const int4 *ep4 = reinterpret_cast<const int4 *>(A.elemp);
    int32_t err = 0;
    const bool nodal_f = A.f.kind == FE_FN_NODAL;
    const double fi = nodal_f ? A.fp[k] : 0.0;
    double fvert = 0.0;   // f at the row's vertex (vertex rule)
    if (A.load_rule == FE_LOAD_TRAPEZOID && A.f.kind != FE_FN_ZERO) {
        const double x0[2] = {X0.x, X0.y};
        fvert = nodal_f ? fi : fn_point<2>(A.f, x0);
    }
    // incidence bits that call for the boundary walk (lifting only with g_D != 0)
    const uint32_t BND = (3u << Meta<3>::NBIT) | (3u << Meta<3>::RBIT) |
                         (A.gd.kind != FE_FN_ZERO ? 3u << Meta<3>::DBIT : 0u);
    uint32_t bmask = 0;
    // Analytic f at edge midpoints (the default rule): the midpoint of edge (i, j) is
    // met by both triangles of the edge, so its value is kept per column and computed
    // once, when the column is first met.  One evaluation per incidence covers the
    // usual case of one new column; a second runs only where both are new.  The
    // values and their sums are the same as evaluating at every incidence.
    const bool mcache = MIDC && A.load_rule == FE_LOAD_DEFAULT && A.f.kind == FE_FN_SINPROD;
    uint32_t seen = 0;   // columns whose midpoint value is in fmid
    for (int32_t p0 = s; p0 < e; p0 += UNR) {
        int2 km[UNR];
        int4 ep[UNR];
        double kt[UNR];
        double2 X1[UNR], X2[UNR];
        int p1[UNR], p2[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (p0 + u < e) km[u] = A.pincm[p0 + u];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (p0 + u < e) {
                const int32_t t = km[u].x / 3;
                ep[u] = ep4[t];
                kt[u] = A.kappa ? A.kappa[t] : 1.0;
            }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (p0 + u < e) {
                const int32_t t = km[u].x / 3;
                const int a = km[u].x - 3 * t;
                p1[u] = sel3(ep[u], a == 2 ? 0 : a + 1);
                p2[u] = sel3(ep[u], a == 0 ? 2 : a - 1);
                X1[u] = xy[p1[u]];
                X2[u] = xy[p2[u]];
            }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (p0 + u >= e) break;
            const uint32_t meta = (uint32_t)km[u].y;
            const double E0x = X2[u].x - X1[u].x, E0y = X2[u].y - X1[u].y;
            const double E1x = X0.x - X2[u].x, E1y = X0.y - X2[u].y;
            const double E2x = X1[u].x - X0.x, E2y = X1[u].y - X0.y;
            const double area2 = E1x * E2y - E1y * E2x;        // 2|t|
            if (!(area2 > 0.0) || !isfinite(area2)) err |= ERR_MEASURE;
            if (!(kt[u] > 0.0) || !isfinite(kt[u])) err |= ERR_KAPPA;
            const double sc = kt[u] / (2.0 * area2);
            const double k00 = sc * (E0x * E0x + E0y * E0y);
            const double k01 = sc * (E0x * E1x + E0y * E1y);
            const double k02 = sc * (E0x * E2x + E0y * E2y);
            const int o1 = (meta >> Meta<3>::OFF) & Meta<3>::OMASK;
            const int o2 = (meta >> (Meta<3>::OFF + Meta<3>::OB)) & Meta<3>::OMASK;
            acc[diag * BLOCK + tid] += k00;
            acc[o1 * BLOCK + tid] += k01;
            acc[o2 * BLOCK + tid] += k02;
            // load: |t| (f(m1) + f(m2)) / 6, m1 = (X2+X0)/2, m2 = (X0+X1)/2 (Section 3.2),
            // or the one-point rule |t| f(c_t) / 3, or the vertex rule |t| f(x_i) / 3
            // (Section 4)
            if (A.f.kind != FE_FN_ZERO) {
                if (A.load_rule == FE_LOAD_DEFAULT) {
                    double f1, f2;
                    if (nodal_f) {
                        f1 = 0.5 * (A.fp[p2[u]] + fi);
                        f2 = 0.5 * (fi + A.fp[p1[u]]);
                    } else if (mcache) {
                        // f1 at the midpoint towards X2 (column o2), f2 towards X1 (o1)
                        const bool n1 = !((seen >> o1) & 1u), n2 = !((seen >> o2) & 1u);
                        double fa = 0.0, fb = 0.0;
                        if (n1 || n2) {
                            const double2 Xn = n2 ? X2[u] : X1[u];
                            const double mm[2] = {0.5 * (Xn.x + X0.x), 0.5 * (Xn.y + X0.y)};
                            fa = fn_point<2>(A.f, mm);
                            const int cn = n2 ? o2 : o1;
                            fmid[cn * 64] = fa;
                            seen |= 1u << cn;
                        }
                        if (n1 && n2) {
                            const double mm[2] = {0.5 * (X0.x + X1[u].x), 0.5 * (X0.y + X1[u].y)};
                            fb = fn_point<2>(A.f, mm);
                            fmid[o1 * 64] = fb;
                            seen |= 1u << o1;
                        }
                        f1 = n2 ? fa : fmid[o2 * 64];
                        f2 = n1 ? (n2 ? fb : fa) : fmid[o1 * 64];
                    } else {
                        const double m1[2] = {0.5 * (X2[u].x + X0.x), 0.5 * (X2[u].y + X0.y)};
                        const double m2[2] = {0.5 * (X0.x + X1[u].x), 0.5 * (X0.y + X1[u].y)};
                        f1 = fn_point<2>(A.f, m1);
                        f2 = fn_point<2>(A.f, m2);
                    }
                    bsum += area2 * (f1 + f2);   // (/ 12 once per row, below)
                } else if (A.load_rule == FE_LOAD_CENTROID) {
                    double fc;
                    if (nodal_f) {
                        fc = (fi + A.fp[p1[u]] + A.fp[p2[u]]) / 3.0;
                    } else {
                        const double c[2] = {(X0.x + X1[u].x + X2[u].x) / 3.0, (X0.y + X1[u].y + X2[u].y) / 3.0};
                        fc = fn_point<2>(A.f, c);
                    }
                    bsum += area2 * fc;   // (/ 6 once per row)
                } else {
                    bsum += area2 * fvert;   // (/ 6 once per row)
                }
            }
            bmask |= meta;
        }
    }
    // the load terms were summed without their constant factor (1/12 for the
    // midpoint rule, 1/6 for the others): one division per row
    if (A.f.kind != FE_FN_ZERO) bsum /= (A.load_rule == FE_LOAD_DEFAULT ? 12.0 : 6.0);
    // Boundary terms of the row: Neumann and Robin sides through its vertex and the
    // lifting of Dirichlet neighbours.  Few rows have any, so they are added by a
    // second walk over the incidences that carry such a bit, which keeps the
    // registers of these rare paths out of the main loop.
    if (bmask & BND) {
        for (int32_t p = s; p < e; ++p) {
            const int2 kmv = A.pincm[p];
            const uint32_t meta = (uint32_t)kmv.y;
            if (!(meta & BND)) continue;
            const int32_t t = kmv.x / 3;
            const int a = kmv.x - 3 * t;
            const int4 epv = ep4[t];
            const int q1 = sel3(epv, a == 2 ? 0 : a + 1);
            const int q2 = sel3(epv, a == 0 ? 2 : a - 1);
            const double2 X1 = xy[q1], X2 = xy[q2];
            const double ktv = A.kappa ? A.kappa[t] : 1.0;
            const double E0x = X2.x - X1.x, E0y = X2.y - X1.y;
            const double E1x = X0.x - X2.x, E1y = X0.y - X2.y;
            const double E2x = X1.x - X0.x, E2y = X1.y - X0.y;
            const double area2 = E1x * E2y - E1y * E2x;
            const double sc = ktv / (2.0 * area2);
            const double k01 = sc * (E0x * E1x + E0y * E1y);
            const double k02 = sc * (E0x * E2x + E0y * E2y);
            const int o1 = (meta >> Meta<3>::OFF) & Meta<3>::OMASK;
            const int o2 = (meta >> (Meta<3>::OFF + Meta<3>::OB)) & Meta<3>::OMASK;
            // Neumann sides through the row's vertex: opposite X1 (X2-X0) and opposite X2 (X0-X1)
            const uint32_t nb = (meta >> Meta<3>::NBIT) & 3u;
            if (nb) {
                for (int jj = 0; jj < 2; ++jj) {
                    if (!((nb >> jj) & 1u)) continue;
                    const double2 Xo = jj == 0 ? X2 : X1;         // other end of the side
                    const double ex = jj == 0 ? E1x : E2x, ey = jj == 0 ? E1y : E2y;
                    const double L = sqrt(ex * ex + ey * ey);
                    const double mid[2] = {0.5 * (X0.x + Xo.x), 0.5 * (X0.y + Xo.y)};
                    double g;
                    if (A.gn.kind == FE_FN_DUDN_SINPROD) {
                        // inward normal of the side = its edge vector rotated counter-clockwise
                        const double nrm[2] = {ey / L, -ex / L};        // outward unit normal
                        g = fn_dudn<2>(A.gn, mid, nrm);
                    } else if (A.gn.kind == FE_FN_NODAL) {
                        const int32_t vo = A.pi[jj == 0 ? q2 : q1];
                        g = 0.5 * (A.gn.nodal[A.pi[k]] + A.gn.nodal[vo]);
                    } else {
                        g = fn_point<2>(A.gn, mid);
                    }
                    bsum += L * g / 2.0;
                }
            }
            const uint32_t db = (meta >> Meta<3>::DBIT) & 3u;
            // Robin sides through the row's vertex: side mass alpha |F| (1 + delta) / 6
            // (lifted like the stiffness when the other end is a Dirichlet node) and
            // g_R by the midpoint rule
            const uint32_t rb = (meta >> Meta<3>::RBIT) & 3u;
            if (rb) {
                for (int jj = 0; jj < 2; ++jj) {
                    if (!((rb >> jj) & 1u)) continue;
                    const double2 Xo = jj == 0 ? X2 : X1;         // other end of the side
                    const double ex = jj == 0 ? E1x : E2x, ey = jj == 0 ? E1y : E2y;
                    const double L = sqrt(ex * ex + ey * ey);
                    const double m1 = A.ralpha * L / 6.0;
                    acc[diag * BLOCK + tid] += A.ralpha * L / 3.0;
                    acc[(jj == 0 ? o2 : o1) * BLOCK + tid] += m1;
                    const uint32_t other_d = jj == 0 ? (db >> 1) & 1u : db & 1u;
                    if (other_d && A.gd.kind != FE_FN_ZERO) {
                        const double xo[2] = {Xo.x, Xo.y};
                        lift += m1 * dirichlet_value<2>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[jj == 0 ? q2 : q1] : 0,
                                                        xo);
                    }
                    if (A.gr.kind != FE_FN_ZERO) {
                        const double mid[2] = {0.5 * (X0.x + Xo.x), 0.5 * (X0.y + Xo.y)};
                        double g;
                        if (A.gr.kind == FE_FN_DUDN_SINPROD) {
                            const double nrm[2] = {ey / L, -ex / L};
                            g = fn_dudn<2>(A.gr, mid, nrm);
                        } else if (A.gr.kind == FE_FN_NODAL) {
                            const int32_t vo = A.pi[jj == 0 ? q2 : q1];
                            g = 0.5 * (A.gr.nodal[A.pi[k]] + A.gr.nodal[vo]);
                        } else {
                            g = fn_point<2>(A.gr, mid);
                        }
                        bsum += L * g / 2.0;
                    }
                }
            }
            // Dirichlet columns: lift b by K[0][c] u_D(c)
            if (db && A.gd.kind != FE_FN_ZERO) {
                if (db & 1u) {
                    const double x1[2] = {X1.x, X1.y};
                    lift += k01 * dirichlet_value<2>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[q1] : 0, x1);
                }
                if (db & 2u) {
                    const double x2[2] = {X2.x, X2.y};
                    lift += k02 * dirichlet_value<2>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[q2] : 0, x2);
                }
            }
        }
    }
    if (err) atomicOr(A.status + ST_ERR, err);
    if (rowd) {
        const double x0[2] = {X0.x, X0.y};
        gdi = dirichlet_value<2>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[k] : 0, x0);
    }
    } while (false);
    if constexpr (SLOTW) {
        if (!A.direct) {
            // (the wavefront's walk is done: its midpoint values are no longer needed)
            write_rows_slots<ROWCAP, BLOCK>(A, acc, reinterpret_cast<uint16_t *>(wown + 128), wown, tid, k, live, len,
                                            diag, rowd, bsum, lift, gdi);
            return;
        }
    }
    if (live) write_row<BLOCK>(A, acc, tid, k, len, rowd, bsum, lift, gdi);
}

// ----------------------------------------------------------------------------- 3-D
// Local vertices are taken in the even order Y0 = x_a, Y1..Y3 = x_{fe_other(a, .)},
// which keeps the orientation.  Sides opposite Y0..Y3 follow the paper's face list
// [1 3 2], [0 2 3], [0 3 1], [0 1 2]; n_f = (Y_F1 - Y_F0) x (Y_F2 - Y_F0) is the
// inward normal of a positively oriented tetrahedron, 6|t| = n_3 . (Y3 - Y0) and
// K[0][q] = kappa n_0 . n_q / (6 * 6|t|).  The four side vectors sum to zero, so
// n_0 = -(n_1 + n_2 + n_3).
FE_DEV void cross3(const double *u, const double *v, double *w)
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

FE_DEV double dot3(const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }


// COLS: the other vertices' positions come from the row's stored columns (LDS),
// indexed by the column offsets in each incidence's metadata word, instead of
// from a gather of the element's record: same vertices, same arithmetic.
template <int ROWCAP, int BLOCK, int UNR, bool COLS>
__global__ __launch_bounds__(BLOCK) void k_assemble_3d(AsmArgs A)
{
    __shared__ double acc[ROWCAP * BLOCK];
    // stored columns, each wavefront's rows in its own part: column q of the row of
    // lane l of wavefront w at (w * ROWCAP + q) * 64 + l (the part is later the
    // wavefront's row-write map)
    __shared__ int32_t cols[COLS ? ROWCAP * BLOCK : 1];
    const int tid = threadIdx.x;
    int32_t *mycols = cols + (COLS ? (tid >> 6) * (ROWCAP * 64) + (tid & 63) : 0);
    // contiguous rows per XCD: neighbours lie about N^(2/3) positions apart, a window
    // that interleaved blocks would need in every XCD's L2
    const int32_t k = xcd_block(blockIdx.x, gridDim.x) * BLOCK + tid;
    // every thread reaches the block's row write (a barrier): rows past the end and
    // long rows (k_assemble_long) only skip the computation
    int len = 0, diag = 0;
    bool rowd = false, live = false;
    double bsum = 0.0, lift = 0.0, gdi = 0.0;
    do {
    if (k >= A.N) break;
    const int32_t s = A.pincptr[k], e = A.pincptr[k + 1];
    const uint32_t info = A.prow_info[k];
    if (info & INFO_LONG) break;
    live = true;
    len = info & 0xff;
    diag = (info >> 8) & 0xff;
    rowd = (info >> 16) & 1;
    for (int c = 0; c < len; ++c) acc[c * BLOCK + tid] = 0.0;
    if (COLS) {
        static_assert(!COLS || ROWCAP == 16, "stored columns: 16 per row");
        const int4 *rc = reinterpret_cast<const int4 *>(A.rcols) + 4 * (int64_t)k;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 v = rc[q];
            mycols[(4 * q) * 64] = v.x;
            mycols[(4 * q + 1) * 64] = v.y;
            mycols[(4 * q + 2) * 64] = v.z;
            mycols[(4 * q + 3) * 64] = v.w;
        }
    }
    const double2 *xy = reinterpret_cast<const double2 *>(A.xyp);
    const int4 *ep4 = reinterpret_cast<const int4 *>(A.elemp);
    double Y0[3], fi;   // fi: nodal f at the row's vertex (the fourth word of its record)
    {
        const double2 q0 = xy[2 * (int64_t)k], q1 = xy[2 * (int64_t)k + 1];
        Y0[0] = q0.x; Y0[1] = q0.y; Y0[2] = q1.x;
        fi = q1.y;
    }
    int32_t err = 0;
    const double alpha = 0.58541019662496845446;   // (5 + 3 sqrt 5) / 20
    const double beta = 0.13819660112501051518;    // (5 - sqrt 5) / 20
    const bool nodal_f = A.f.kind == FE_FN_NODAL;
    double fvert = 0.0;   // f at the row's vertex (vertex rule)
    if (A.load_rule == FE_LOAD_TRAPEZOID && A.f.kind != FE_FN_ZERO) fvert = nodal_f ? fi : fn_point<3>(A.f, Y0);
    const uint32_t BND = (7u << Meta<4>::NBIT) | (7u << Meta<4>::RBIT) |
                         (A.gd.kind != FE_FN_ZERO ? 7u << Meta<4>::DBIT : 0u);
    const bool sell = A.status[ST_SELL] != 0;
    uint32_t bmask = 0;
    // One incidence: row a of K_t into the accumulators, the load term into bsum.
    auto add_inc = [&](int2 kmu, double ktu, const double (*Yu)[3], const double *Fu) {
        const uint32_t meta = (uint32_t)kmu.y;
        const double *Y1 = Yu[0], *Y2 = Yu[1], *Y3 = Yu[2];
        double d10[3], d20[3], d30[3], d31[3], d21[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d10[c] = Y1[c] - Y0[c];
            d20[c] = Y2[c] - Y0[c];
            d30[c] = Y3[c] - Y0[c];
            d31[c] = Y3[c] - Y1[c];
            d21[c] = Y2[c] - Y1[c];
        }
        double n1[3], n2[3], n3[3], n0[3];
        cross3(d20, d30, n1);   // side [0 2 3]
        cross3(d30, d10, n2);   // side [0 3 1]
        cross3(d10, d20, n3);   // side [0 1 2]
        for (int c = 0; c < 3; ++c) n0[c] = -(n1[c] + n2[c] + n3[c]);
        const double vol6 = dot3(n3, d30);
        if (!(vol6 > 0.0) || !isfinite(vol6)) err |= ERR_MEASURE;
        if (!(ktu > 0.0) || !isfinite(ktu)) err |= ERR_KAPPA;
        const double sc = ktu / (6.0 * vol6);
        const double kr0 = sc * dot3(n0, n0);
        const double kr[3] = {sc * dot3(n0, n1), sc * dot3(n0, n2), sc * dot3(n0, n3)};
        acc[diag * BLOCK + tid] += kr0;
        int off[3];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            off[jj] = (meta >> (Meta<4>::OFF + Meta<4>::OB * jj)) & Meta<4>::OMASK;
            acc[off[jj] * BLOCK + tid] += kr[jj];
        }
        // load (Section 3.2): symmetric 4-point rule; exact closed form for nodal f.
        // Section 4's one-point rule |t| f(c_t) / 4 and vertex rule |t| f(x_i) / 4 on request.
        // (Summed in units of 6|t|: the constant factor divides the row's sum once, below.)
        if (A.load_rule == FE_LOAD_CENTROID && A.f.kind != FE_FN_ZERO) {
            double fc;
            if (nodal_f) {
                fc = (fi + Fu[0] + Fu[1] + Fu[2]) / 4.0;
            } else {
                double c[3];
                for (int q = 0; q < 3; ++q) c[q] = (Y0[q] + Y1[q] + Y2[q] + Y3[q]) / 4.0;
                fc = fn_point<3>(A.f, c);
            }
            bsum += vol6 * fc;
        } else if (A.load_rule == FE_LOAD_TRAPEZOID && A.f.kind != FE_FN_ZERO) {
            bsum += vol6 * fvert;
        } else if (nodal_f) {
            const double sf = fi + Fu[0] + Fu[1] + Fu[2];
            bsum += vol6 * (fi + sf);
        } else if (A.f.kind != FE_FN_ZERO) {
            double S[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) S[c] = Y0[c] + Y1[c] + Y2[c] + Y3[c];
            double q = 0.0;
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) {
                const double *Yk = kq == 0 ? Y0 : Yu[kq - 1];
                double pt[3];
                for (int c = 0; c < 3; ++c) pt[c] = beta * S[c] + (alpha - beta) * Yk[c];
                q += fn_point<3>(A.f, pt) * (kq == 0 ? alpha : beta);
            }
            bsum += vol6 * q;
        }
        bmask |= meta;
    };
    if constexpr (COLS) {
        // Software pipeline over batches of UNR incidences: the gathers of batch j + 1
        // and the keys of batch j + 2 are in flight while batch j is added.  The wait
        // counter retires loads in issue order, so every load is issued after the ones
        // that are needed before it; the loop is unrolled twice so the two gather
        // buffers swap roles instead of being copied (a copy would wait for the loads).
        // Positions past the row's end are clamped to its last incidence: every load
        // is valid and needs no branch, and only the additions are predicated.
        if (e > s) {
            const int32_t last = e - 1 - s;
            auto walk = [&](auto has_kappa) {
                constexpr bool KAP = decltype(has_kappa)::value;
                auto ld_km = [&](int32_t q0, int2 *km) {
#pragma unroll
                    for (int u = 0; u < UNR; ++u) km[u] = A.pincm[inc_at(sell, A.sptr, s, k, min(q0 + u, last))];
                };
                // gathers of one batch: kappa and the other vertices' records, by the
                // column offsets of the metadata word (kept in m for the additions)
                auto ld_g = [&](const int2 *km, uint32_t *m, double *kt, double (*Y)[3][3], double (*F)[3]) {
#pragma unroll
                    for (int u = 0; u < UNR; ++u) {
                        kt[u] = KAP ? A.kappa[km[u].x >> 2] : 1.0;
                        m[u] = (uint32_t)km[u].y;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const int32_t pq = mycols[(int)((m[u] >> (Meta<4>::OFF + Meta<4>::OB * q)) & Meta<4>::OMASK) * 64];
                            const double2 c0 = xy[2 * (int64_t)pq], c1 = xy[2 * (int64_t)pq + 1];
                            Y[u][q][0] = c0.x; Y[u][q][1] = c0.y; Y[u][q][2] = c1.x;
                            F[u][q] = c1.y;
                        }
                    }
                };
                auto add_batch = [&](int32_t q0, const uint32_t *m, const double *kt, const double (*Y)[3][3],
                                     const double (*F)[3]) {
#pragma unroll
                    for (int u = 0; u < UNR; ++u)
                        if (q0 + u <= last) add_inc(make_int2(0, (int32_t)m[u]), kt[u], Y[u], F[u]);
                };
                int2 kmX[UNR], kmY[UNR];
                uint32_t mX[UNR], mY[UNR];
                double ktX[UNR], YX[UNR][3][3], FX[UNR][3];
                double ktY[UNR], YY[UNR][3][3], FY[UNR][3];
                ld_km(0, kmX);
                ld_km(UNR, kmY);
                ld_g(kmX, mX, ktX, YX, FX);
                ld_km(2 * UNR, kmX);
                for (int32_t q0 = 0; q0 <= last; q0 += 2 * UNR) {
                    ld_g(kmY, mY, ktY, YY, FY);
                    ld_km(q0 + 3 * UNR, kmY);
                    add_batch(q0, mX, ktX, YX, FX);
                    ld_g(kmX, mX, ktX, YX, FX);
                    ld_km(q0 + 4 * UNR, kmX);
                    add_batch(q0 + UNR, mY, ktY, YY, FY);
                }
            };
            if (A.kappa) walk(std::true_type{});
            else walk(std::false_type{});
        }
    } else {
        for (int32_t p0 = s; p0 < e; p0 += UNR) {
            int2 km[UNR];
            int4 ep[UNR];
            double kt[UNR];
            double Y[UNR][3][3], F[UNR][3];   // F: nodal f at the other vertices
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                if (p0 + u < e) km[u] = A.pincm[inc_at(sell, A.sptr, s, k, p0 - s + u)];
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                if (p0 + u < e) {
                    const int32_t t = km[u].x >> 2;
                    ep[u] = ep4[t];
                    kt[u] = A.kappa ? A.kappa[t] : 1.0;
                }
#pragma unroll
            for (int u = 0; u < UNR; ++u)
                if (p0 + u < e) {
                    const int a = km[u].x & 3;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int pq = sel4(ep[u], fe_other<4>(a, q));
                        const double2 c0 = xy[2 * (int64_t)pq], c1 = xy[2 * (int64_t)pq + 1];
                        Y[u][q][0] = c0.x; Y[u][q][1] = c0.y; Y[u][q][2] = c1.x;
                        F[u][q] = c1.y;
                    }
                }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (p0 + u >= e) break;
                add_inc(km[u], kt[u], Y[u], F[u]);
            }
        }
    }
    // the load terms were summed in units of 6|t| without their constant factor
    // (1/24, or 1/120 for the nodal closed form): one division per row
    if (A.f.kind != FE_FN_ZERO)
        bsum /= (A.load_rule == FE_LOAD_DEFAULT && nodal_f) ? 120.0 : 24.0;
    // Boundary terms of the row (Neumann and Robin faces through its vertex, lifting
    // of Dirichlet neighbours): a second walk over the incidences that carry such a
    // bit, as in 2-D.
    if (bmask & BND) {
        for (int32_t p = s; p < e; ++p) {
            const int2 kmv = A.pincm[inc_at(sell, A.sptr, s, k, p - s)];
            const uint32_t meta = (uint32_t)kmv.y;
            if (!(meta & BND)) continue;
            const int32_t t = kmv.x >> 2;
            const int a = kmv.x & 3;
            const int4 epv = ep4[t];
            const double ktv = A.kappa ? A.kappa[t] : 1.0;
            int pqv[3];
            double Yv[3][3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                pqv[q] = sel4(epv, fe_other<4>(a, q));
                const double2 c0 = xy[2 * (int64_t)pqv[q]], c1 = xy[2 * (int64_t)pqv[q] + 1];
                Yv[q][0] = c0.x; Yv[q][1] = c0.y; Yv[q][2] = c1.x;
            }
            const double *Y1 = Yv[0], *Y2 = Yv[1], *Y3 = Yv[2];
            double d10[3], d20[3], d30[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d10[c] = Y1[c] - Y0[c];
                d20[c] = Y2[c] - Y0[c];
                d30[c] = Y3[c] - Y0[c];
            }
            double n1[3], n2[3], n3[3], n0[3];
            cross3(d20, d30, n1);
            cross3(d30, d10, n2);
            cross3(d10, d20, n3);
            for (int c = 0; c < 3; ++c) n0[c] = -(n1[c] + n2[c] + n3[c]);
            const double sc = ktv / (6.0 * dot3(n3, d30));
            const double kr[3] = {sc * dot3(n0, n1), sc * dot3(n0, n2), sc * dot3(n0, n3)};
            int off[3];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) off[jj] = (meta >> (Meta<4>::OFF + Meta<4>::OB * jj)) & Meta<4>::OMASK;
            // Neumann sides containing Y0: the sides opposite Y1, Y2, Y3
            const uint32_t nb = (meta >> Meta<4>::NBIT) & 7u;
            if (nb) {
                const double *nq[3] = {n1, n2, n3};
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    if (!((nb >> jj) & 1u)) continue;
                    const double *nf = nq[jj];
                    const double nn = sqrt(dot3(nf, nf));
                    const double area = 0.5 * nn;
                    double cen[3];
                    for (int c = 0; c < 3; ++c) cen[c] = (Y0[c] + Y1[c] + Y2[c] + Y3[c] - Yv[jj][c]) / 3.0;
                    double g;
                    if (A.gn.kind == FE_FN_DUDN_SINPROD) {
                        const double nrm[3] = {-nf[0] / nn, -nf[1] / nn, -nf[2] / nn};
                        g = fn_dudn<3>(A.gn, cen, nrm);
                    } else if (A.gn.kind == FE_FN_NODAL) {
                        double sg = A.gn.nodal[A.pi[k]];
                        for (int c = 0; c < 3; ++c)
                            if (c != jj) sg += A.gn.nodal[A.pi[pqv[c]]];
                        g = sg / 3.0;
                    } else {
                        g = fn_point<3>(A.gn, cen);
                    }
                    bsum += area * g / 3.0;
                }
            }
            const uint32_t db = (meta >> Meta<4>::DBIT) & 7u;
            // Robin faces containing Y0 (opposite Y1, Y2, Y3): face mass alpha |F| (1 +
            // delta) / 12, lifted at Dirichlet face vertices, and g_R at the centroid
            const uint32_t rb = (meta >> Meta<4>::RBIT) & 7u;
            if (rb) {
                const double *nq[3] = {n1, n2, n3};
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    if (!((rb >> jj) & 1u)) continue;
                    const double *nf = nq[jj];
                    const double nn = sqrt(dot3(nf, nf));
                    const double area = 0.5 * nn;
                    const double m1 = A.ralpha * area / 12.0;
                    acc[diag * BLOCK + tid] += A.ralpha * area / 6.0;
                    for (int r = 0; r < 3; ++r) {
                        if (r == jj) continue;
                        acc[off[r] * BLOCK + tid] += m1;
                        if (((db >> r) & 1u) && A.gd.kind != FE_FN_ZERO)
                            lift += m1 * dirichlet_value<3>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[pqv[r]] : 0,
                                                            Yv[r]);
                    }
                    if (A.gr.kind != FE_FN_ZERO) {
                        double cen[3];
                        for (int c = 0; c < 3; ++c) cen[c] = (Y0[c] + Y1[c] + Y2[c] + Y3[c] - Yv[jj][c]) / 3.0;
                        double g;
                        if (A.gr.kind == FE_FN_DUDN_SINPROD) {
                            const double nrm[3] = {-nf[0] / nn, -nf[1] / nn, -nf[2] / nn};
                            g = fn_dudn<3>(A.gr, cen, nrm);
                        } else if (A.gr.kind == FE_FN_NODAL) {
                            double sg = A.gr.nodal[A.pi[k]];
                            for (int c = 0; c < 3; ++c)
                                if (c != jj) sg += A.gr.nodal[A.pi[pqv[c]]];
                            g = sg / 3.0;
                        } else {
                            g = fn_point<3>(A.gr, cen);
                        }
                        bsum += area * g / 3.0;
                    }
                }
            }
            if (db && A.gd.kind != FE_FN_ZERO) {
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    if (!((db >> jj) & 1u)) continue;
                    lift += kr[jj] * dirichlet_value<3>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[pqv[jj]] : 0,
                                                        Yv[jj]);
                }
            }
        }
    }
    if (err) atomicOr(A.status + ST_ERR, err);
    if (rowd) gdi = dirichlet_value<3>(A.gd, A.gd.kind == FE_FN_NODAL ? A.pi[k] : 0, Y0);
    } while (false);
    if (COLS && A.direct) {
        // (the wavefront's own part of cols, which its walk above has finished reading)
        write_rows_direct<ROWCAP, BLOCK>(A, acc, mycols - (tid & 63), tid, k, live, len, diag, rowd, bsum, lift, gdi);
    } else if (live) {
        write_row<BLOCK>(A, acc, tid, k, len, rowd, bsum, lift, gdi);
    }
}

// ----------------------------------------------------------------------------- long rows
// Rows with more columns than the accumulators of the kernels above hold (INFO_LONG;
// a vertex with more than 31 / 63 neighbours): one workgroup per row.  The row's
// column set (labels, ascending) is formed again in LDS from its incidences, as the
// plan formed it.  Each chunk of LNB incidences is computed in parallel, one
// incidence per thread, with the same local matrix, load and side terms as above;
// thread 0 then adds the chunk's contributions in incidence (ascending element)
// order, so the sums have a fixed order.  The row goes straight to the label-order
// outputs.
constexpr int LNB = 256;

FE_DEV int lower_bound_i32(const int32_t *a, int n, int32_t x)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int NV>
__global__ __launch_bounds__(LNB) void k_assemble_long(AsmArgs A)
{
    constexpr int DIM = NV - 1;
    __shared__ int32_t cols[LCAND];
    __shared__ double acc[LCAND];
    __shared__ double cv[LNB][NV];       // chunk: contributions to the diagonal and the other columns
    __shared__ int32_t co[LNB][NV - 1];  // chunk: column offsets of the other vertices
    __shared__ double cb[LNB][2];        // chunk: contributions to b_load and to the lifting
    __shared__ int32_t sl[2 * (LNB / 64)];
    const int tid = threadIdx.x;
    const int32_t k = A.longk[blockIdx.x];
    const int32_t s = A.pincptr[k], d = A.pincptr[k + 1] - s;
    const int4 rec = A.precp[k];   // (start, info, length, diagonal offset)
    const int len = rec.z, diag = rec.w;
    const bool rowd = (rec.y >> 16) & 1;
    const int32_t i = A.pi[k];
    const int32_t nc = DIM * d + 1;
    const bool sell = NV == 4 && A.status[ST_SELL] != 0;
    if (nc > LCAND || len > nc) {
        if (tid == 0) atomicOr(A.status + ST_ERR, ERR_LIMIT);
        return;
    }
    // the column set: the other vertices of every incident element and i, sorted, unique
    int32_t M = 1;
    while (M < nc) M <<= 1;
    for (int32_t j = tid; j < d; j += LNB) {
        const int32_t key = A.pincm[inc_at(sell, A.sptr, s, k, j)].x;
        const int32_t t = key / NV;
        const int a = key - t * NV;
#pragma unroll
        for (int jj = 0; jj < NV - 1; ++jj) cols[DIM * j + jj] = A.elem[(int64_t)fe_other<NV>(a, jj) * A.NT + t];
    }
    for (int32_t j = DIM * d + tid; j < M; j += LNB) cols[j] = (j == DIM * d) ? i : INT32_MAX;
    __syncthreads();
    for (int32_t kk = 2; kk <= M; kk <<= 1)
        for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int32_t x = tid; x < M; x += LNB) {
                const int32_t l = x ^ jj;
                if (l > x) {
                    const int32_t p = cols[x], q = cols[l];
                    if (((x & kk) == 0) ? p > q : p < q) {
                        cols[x] = q;
                        cols[l] = p;
                    }
                }
            }
            __syncthreads();
        }
    int32_t u = 0;
    for (int32_t x0 = 0; x0 < M; x0 += LNB) {
        const int32_t x = x0 + tid;
        const int32_t c = x < M ? cols[x] : INT32_MAX;
        const bool first = c != INT32_MAX && (x == 0 || cols[x - 1] != c);
        int32_t tot;
        const int32_t ex = block_exclusive_i32<LNB>(first ? 1 : 0, sl, &tot);   // (reads before its barriers)
        if (first) cols[u + ex] = c;                                          // compaction: u + ex <= x
        u += tot;
        __syncthreads();
    }
    for (int c = tid; c < len; c += LNB) acc[c] = 0.0;
    // the row's own coordinates (and nodal f)
    double Y0[DIM], fi = 0.0;
    if (DIM == 2) {
        const double2 q = reinterpret_cast<const double2 *>(A.xyp)[k];
        Y0[0] = q.x; Y0[1] = q.y;
        if (A.f.kind == FE_FN_NODAL) fi = A.fp[k];
    } else {
        const double2 q0 = reinterpret_cast<const double2 *>(A.xyp)[2 * (int64_t)k];
        const double2 q1 = reinterpret_cast<const double2 *>(A.xyp)[2 * (int64_t)k + 1];
        Y0[0] = q0.x; Y0[1] = q0.y; Y0[DIM - 1] = q1.x;
        fi = q1.y;
    }
    const bool nodal_f = A.f.kind == FE_FN_NODAL;
    double fvert = 0.0;
    if (A.load_rule == FE_LOAD_TRAPEZOID && A.f.kind != FE_FN_ZERO) fvert = nodal_f ? fi : fn_point<DIM>(A.f, Y0);
    const int4 *ep4 = reinterpret_cast<const int4 *>(A.elemp);
    double bsum = 0.0, lift = 0.0;
    int32_t err = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < d; c0 += LNB) {
        const int32_t j = c0 + tid;
        if (j < d) {
            const int2 km = A.pincm[inc_at(sell, A.sptr, s, k, j)];
            const int32_t t = km.x / NV;
            const int a = km.x - t * NV;
            const uint32_t meta = (uint32_t)km.y;
            const int4 ep = ep4[t];
            const double kt = A.kappa ? A.kappa[t] : 1.0;
            int32_t pq[NV - 1], lab[NV - 1];
            double Y[NV - 1][DIM], F[NV - 1];
#pragma unroll
            for (int q = 0; q < NV - 1; ++q) {
                const int b = fe_other<NV>(a, q);
                pq[q] = (b == 0 ? ep.x : (b == 1 ? ep.y : (b == 2 ? ep.z : ep.w))) & EREC_POS;
                lab[q] = A.elem[(int64_t)b * A.NT + t];
                co[tid][q] = lower_bound_i32(cols, len, lab[q]);
                if (DIM == 2) {
                    const double2 c = reinterpret_cast<const double2 *>(A.xyp)[pq[q]];
                    Y[q][0] = c.x; Y[q][1] = c.y;
                    F[q] = nodal_f ? A.fp[pq[q]] : 0.0;
                } else {
                    const double2 c0v = reinterpret_cast<const double2 *>(A.xyp)[2 * (int64_t)pq[q]];
                    const double2 c1v = reinterpret_cast<const double2 *>(A.xyp)[2 * (int64_t)pq[q] + 1];
                    Y[q][0] = c0v.x; Y[q][1] = c0v.y; Y[q][DIM - 1] = c1v.x;
                    F[q] = c1v.y;
                }
            }
            if (!(kt > 0.0) || !isfinite(kt)) err |= ERR_KAPPA;
            double kv[NV];
            double bl = 0.0, lf = 0.0;
            const uint32_t nb = (meta >> Meta<NV>::NBIT) & ((1u << (NV - 1)) - 1);
            const uint32_t rb = (meta >> Meta<NV>::RBIT) & ((1u << (NV - 1)) - 1);
            const uint32_t db = (meta >> Meta<NV>::DBIT) & ((1u << (NV - 1)) - 1);
            if constexpr (DIM == 2) {
                const double *X1 = Y[0], *X2 = Y[1];
                const double E0x = X2[0] - X1[0], E0y = X2[1] - X1[1];
                const double E1x = Y0[0] - X2[0], E1y = Y0[1] - X2[1];
                const double E2x = X1[0] - Y0[0], E2y = X1[1] - Y0[1];
                const double area2 = E1x * E2y - E1y * E2x;
                if (!(area2 > 0.0) || !isfinite(area2)) err |= ERR_MEASURE;
                const double sc = kt / (2.0 * area2);
                const double k01 = sc * (E0x * E1x + E0y * E1y), k02 = sc * (E0x * E2x + E0y * E2y);
                kv[0] = sc * (E0x * E0x + E0y * E0y);
                kv[1] = k01;
                kv[2] = k02;
                if (A.f.kind != FE_FN_ZERO) {
                    if (A.load_rule == FE_LOAD_DEFAULT) {
                        double f1, f2;
                        if (nodal_f) {
                            f1 = 0.5 * (F[1] + fi);
                            f2 = 0.5 * (fi + F[0]);
                        } else {
                            const double m1[2] = {0.5 * (X2[0] + Y0[0]), 0.5 * (X2[1] + Y0[1])};
                            const double m2[2] = {0.5 * (Y0[0] + X1[0]), 0.5 * (Y0[1] + X1[1])};
                            f1 = fn_point<2>(A.f, m1);
                            f2 = fn_point<2>(A.f, m2);
                        }
                        bl += area2 * (f1 + f2) / 12.0;
                    } else if (A.load_rule == FE_LOAD_CENTROID) {
                        double fc;
                        if (nodal_f) {
                            fc = (fi + F[0] + F[1]) / 3.0;
                        } else {
                            const double c[2] = {(Y0[0] + X1[0] + X2[0]) / 3.0, (Y0[1] + X1[1] + X2[1]) / 3.0};
                            fc = fn_point<2>(A.f, c);
                        }
                        bl += area2 * fc / 6.0;
                    } else {
                        bl += area2 * fvert / 6.0;
                    }
                }
                // sides through the row's vertex: opposite X1 (to X2, edge E1) and
                // opposite X2 (to X1, edge E2)
                for (int jj = 0; jj < 2; ++jj) {
                    const bool nside = (nb >> jj) & 1u, rside = (rb >> jj) & 1u;
                    if (!nside && !rside) continue;
                    const double *Xo = jj == 0 ? X2 : X1;
                    const int32_t lo = jj == 0 ? lab[1] : lab[0];
                    const double ex = jj == 0 ? E1x : E2x, ey = jj == 0 ? E1y : E2y;
                    const double L = sqrt(ex * ex + ey * ey);
                    const double mid[2] = {0.5 * (Y0[0] + Xo[0]), 0.5 * (Y0[1] + Xo[1])};
                    const double nrm[2] = {ey / L, -ex / L};   // outward unit normal
                    auto side_value = [&](const DevFn &g) {
                        if (g.kind == FE_FN_DUDN_SINPROD) return fn_dudn<2>(g, mid, nrm);
                        if (g.kind == FE_FN_NODAL) return 0.5 * (g.nodal[i] + g.nodal[lo]);
                        return fn_point<2>(g, mid);
                    };
                    if (nside) bl += L * side_value(A.gn) / 2.0;
                    if (rside) {
                        const double m1 = A.ralpha * L / 6.0;
                        kv[0] += A.ralpha * L / 3.0;
                        kv[jj == 0 ? 2 : 1] += m1;
                        const bool other_d = jj == 0 ? ((db >> 1) & 1u) : (db & 1u);
                        if (other_d && A.gd.kind != FE_FN_ZERO) lf += m1 * dirichlet_value<2>(A.gd, lo, Xo);
                        if (A.gr.kind != FE_FN_ZERO) bl += L * side_value(A.gr) / 2.0;
                    }
                }
                if (db && A.gd.kind != FE_FN_ZERO) {
                    if (db & 1u) lf += k01 * dirichlet_value<2>(A.gd, lab[0], X1);
                    if (db & 2u) lf += k02 * dirichlet_value<2>(A.gd, lab[1], X2);
                }
            } else {
                const double *Y1 = Y[0], *Y2 = Y[1], *Y3 = Y[2];
                double d10[3], d20[3], d30[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    d10[c] = Y1[c] - Y0[c];
                    d20[c] = Y2[c] - Y0[c];
                    d30[c] = Y3[c] - Y0[c];
                }
                double n1[3], n2[3], n3[3], n0[3];
                cross3(d20, d30, n1);
                cross3(d30, d10, n2);
                cross3(d10, d20, n3);
                for (int c = 0; c < 3; ++c) n0[c] = -(n1[c] + n2[c] + n3[c]);
                const double vol6 = dot3(n3, d30);
                if (!(vol6 > 0.0) || !isfinite(vol6)) err |= ERR_MEASURE;
                const double sc = kt / (6.0 * vol6);
                const double kr[3] = {sc * dot3(n0, n1), sc * dot3(n0, n2), sc * dot3(n0, n3)};
                kv[0] = sc * dot3(n0, n0);
                kv[1] = kr[0]; kv[2] = kr[1]; kv[3] = kr[2];
                const double vol = vol6 / 6.0;
                const double alpha = 0.58541019662496845446;   // (5 + 3 sqrt 5) / 20
                const double beta = 0.13819660112501051518;    // (5 - sqrt 5) / 20
                if (A.load_rule == FE_LOAD_CENTROID && A.f.kind != FE_FN_ZERO) {
                    double fc;
                    if (nodal_f) {
                        fc = (fi + F[0] + F[1] + F[2]) / 4.0;
                    } else {
                        double c[3];
                        for (int q = 0; q < 3; ++q) c[q] = (Y0[q] + Y1[q] + Y2[q] + Y3[q]) / 4.0;
                        fc = fn_point<3>(A.f, c);
                    }
                    bl += vol * fc / 4.0;
                } else if (A.load_rule == FE_LOAD_TRAPEZOID && A.f.kind != FE_FN_ZERO) {
                    bl += vol * fvert / 4.0;
                } else if (nodal_f) {
                    const double sf = fi + F[0] + F[1] + F[2];
                    bl += vol * (fi + sf) / 20.0;
                } else if (A.f.kind != FE_FN_ZERO) {
                    double S[3];
                    for (int c = 0; c < 3; ++c) S[c] = Y0[c] + Y1[c] + Y2[c] + Y3[c];
                    double q = 0.0;
                    for (int kq = 0; kq < 4; ++kq) {
                        const double *Yk = kq == 0 ? Y0 : Y[kq - 1];
                        double pt[3];
                        for (int c = 0; c < 3; ++c) pt[c] = beta * S[c] + (alpha - beta) * Yk[c];
                        q += fn_point<3>(A.f, pt) * (kq == 0 ? alpha : beta);
                    }
                    bl += vol * q / 4.0;
                }
                // faces through the row's vertex: opposite Y1, Y2, Y3
                const double *nq[3] = {n1, n2, n3};
                for (int jj = 0; jj < 3; ++jj) {
                    const bool nside = (nb >> jj) & 1u, rside = (rb >> jj) & 1u;
                    if (!nside && !rside) continue;
                    const double *nf = nq[jj];
                    const double nn = sqrt(dot3(nf, nf));
                    const double area = 0.5 * nn;
                    double cen[3];
                    for (int c = 0; c < 3; ++c) cen[c] = (Y0[c] + Y1[c] + Y2[c] + Y3[c] - Y[jj][c]) / 3.0;
                    const double nrm[3] = {-nf[0] / nn, -nf[1] / nn, -nf[2] / nn};
                    auto face_value = [&](const DevFn &g) {
                        if (g.kind == FE_FN_DUDN_SINPROD) return fn_dudn<3>(g, cen, nrm);
                        if (g.kind == FE_FN_NODAL) {
                            double sg = g.nodal[i];
                            for (int c = 0; c < 3; ++c)
                                if (c != jj) sg += g.nodal[lab[c]];
                            return sg / 3.0;
                        }
                        return fn_point<3>(g, cen);
                    };
                    if (nside) bl += area * face_value(A.gn) / 3.0;
                    if (rside) {
                        const double m1 = A.ralpha * area / 12.0;
                        kv[0] += A.ralpha * area / 6.0;
                        for (int r = 0; r < 3; ++r) {
                            if (r == jj) continue;
                            kv[1 + r] += m1;
                            if (((db >> r) & 1u) && A.gd.kind != FE_FN_ZERO)
                                lf += m1 * dirichlet_value<3>(A.gd, lab[r], Y[r]);
                        }
                        if (A.gr.kind != FE_FN_ZERO) bl += area * face_value(A.gr) / 3.0;
                    }
                }
                if (db && A.gd.kind != FE_FN_ZERO)
                    for (int jj = 0; jj < 3; ++jj)
                        if ((db >> jj) & 1u) lf += kr[jj] * dirichlet_value<3>(A.gd, lab[jj], Y[jj]);
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) cv[tid][q] = kv[q];
            cb[tid][0] = bl;
            cb[tid][1] = lf;
        }
        __syncthreads();
        if (tid == 0) {
            const int32_t n = min(LNB, d - c0);
            for (int32_t jj = 0; jj < n; ++jj) {
                acc[diag] += cv[jj][0];
#pragma unroll
                for (int q = 0; q < NV - 1; ++q) acc[co[jj][q]] += cv[jj][1 + q];
                bsum += cb[jj][0];
                lift += cb[jj][1];
            }
        }
        __syncthreads();
    }
    if (err) atomicOr(A.status + ST_ERR, err);
    const int c0 = A.upper ? diag : 0;   // first column written
    const int64_t lstart = A.upper ? (int64_t)A.urowptr[i] - c0 : (int64_t)A.lrowptr[i];
    for (int c = c0 + tid; c < len; c += LNB) {
        const double x = acc[c];
        A.val[lstart + c] = x;
        if (A.val_bc) A.val_bc[lstart + c] = rowd ? (c == diag ? 1.0 : 0.0) : (A.isdl[cols[c]] ? 0.0 : x);
    }
    if (tid == 0) {
        const double gdi = rowd ? dirichlet_value<DIM>(A.gd, i, Y0) : 0.0;
        A.b[i] = rowd ? gdi : bsum - lift;
        if (A.b_load) A.b_load[i] = bsum;
        if (A.isd) A.isd[i] = (uint8_t)rowd;
    }
}

template <int ROWCAP, int BLOCK> int launch(int dim, const AsmArgs &A, hipStream_t s)
{
    const unsigned g = (unsigned)cdiv(A.N, BLOCK);
    if (dim == 2) {
        FE_TIMED("k_assemble_2d", s, hipLaunchKernelGGL((k_assemble_2d<ROWCAP, BLOCK, 4>), dim3(g), dim3(BLOCK), 0, s, A));
    } else if constexpr (ROWCAP >= 16) {   // (3-D rows have at least 15 columns in the interior)
        if (ROWCAP == 16 && A.rcols)
            FE_TIMED("k_assemble_3d", s,
                     hipLaunchKernelGGL((k_assemble_3d<ROWCAP, BLOCK, 2, ROWCAP == 16>), dim3(g), dim3(BLOCK), 0, s, A));
        else
            FE_TIMED("k_assemble_3d", s,
                     hipLaunchKernelGGL((k_assemble_3d<ROWCAP, BLOCK, 2, false>), dim3(g), dim3(BLOCK), 0, s, A));
    }
    return fe_launch_check();
}

}  // namespace

namespace {

int assemble_impl(fe_plan *plan, const int32_t *urowptr, const double *node, const double *kappa, const fe_fn *f,
                  const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r, double robin_alpha, int32_t load_rule,
                  double *val, double *val_bc, double *b, double *b_load, uint8_t *is_dirichlet, void *stream)
{
    if (!plan || !node || !val || !b) return FE_EINVAL;
    if (load_rule != FE_LOAD_DEFAULT && load_rule != FE_LOAD_CENTROID && load_rule != FE_LOAD_TRAPEZOID)
        return FE_EINVAL;
    if (!plan->pattern_done) return FE_EINVAL;
    if (!devfn_valid(f, false) || !devfn_valid(g_d, false) || !devfn_valid(g_n, true) || !devfn_valid(g_r, true))
        return FE_EINVAL;
    if (!(robin_alpha >= 0.0) || !std::isfinite(robin_alpha)) return FE_EINVAL;
    AsmArgs A{};
    A.N = (int32_t)plan->N;
    A.NT = (int32_t)plan->NT;
    A.kappa = kappa;
    A.pi = plan->pi;
    A.pincptr = plan->pincptr;
    A.prowptr = plan->prowptr;
    A.elemp = plan->elemp;
    A.pincm = plan->pincm;
    A.sptr = plan->sptr;
    A.prow_info = plan->prow_info;
    A.xyp = plan->xyp;
    A.fp = plan->fp;
    A.f = make_devfn(f);
    A.gd = make_devfn(g_d);
    A.gn = make_devfn(g_n);
    A.gr = make_devfn(g_r);
    A.ralpha = robin_alpha;
    A.load_rule = load_rule;
    A.valp = plan->valp;
    A.direct = plan->l1_agg;
    A.precp = plan->precp;
    A.rcols = (plan->dim == 3 && plan->l1_agg && plan->rows_reg) ? reinterpret_cast<const int32_t *>(plan->rslot) : nullptr;
    A.longk = plan->longk;
    A.elem = plan->elem;
    A.lrowptr = plan->l1_agg ? plan->prowptr : plan->rowlen;   // label-order row starts
    A.isdl = plan->isd;
    A.upper = urowptr != nullptr;
    A.urowptr = urowptr;
    A.val = val;
    A.val_bc = val_bc;
    A.b = b;
    A.b_load = b_load;
    A.isd = is_dirichlet;
    A.status = plan->status;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned gg = (unsigned)cdiv(A.N, 256);
    const double *fnodal = (A.f.kind == FE_FN_NODAL) ? A.f.nodal : nullptr;
    if (plan->dim == 2)
        FE_TIMED("k_scatter_coords", s,
                 hipLaunchKernelGGL(k_scatter_coords<2>, dim3(gg), dim3(256), 0, s, A.N, plan->piinv, node, plan->xyp, fnodal,
                               plan->fp));
    else
        FE_TIMED("k_scatter_coords", s,
                 hipLaunchKernelGGL(k_scatter_coords<3>, dim3(gg), dim3(256), 0, s, A.N, plan->piinv, node, plan->xyp, fnodal,
                               plan->fp));
    int rc = fe_launch_check();
    if (rc) return rc;
    // accumulator width (columns per row) by the plan's longest short row, and rows
    // per workgroup by the plan's launch setting (fe_plan_set_launch; 0: the widest
    // block whose accumulators take 32 KB of LDS)
    const int mr = plan->max_row;
    const int wb = plan->asm_block;
    if (plan->dim == 2 && mr <= 8) rc = (wb == 64)    ? launch<8, 64>(plan->dim, A, s)
                                        : (wb == 128) ? launch<8, 128>(plan->dim, A, s)
                                                      : launch<8, 256>(plan->dim, A, s);
    else if (mr <= 16) rc = (wb == 64) ? launch<16, 64>(plan->dim, A, s)
                       : (wb == 128) ? launch<16, 128>(plan->dim, A, s)
                                     : launch<16, 256>(plan->dim, A, s);
    else if (mr <= 32 || plan->dim == 2) rc = (wb == 64) ? launch<32, 64>(plan->dim, A, s)
                                                         : launch<32, 128>(plan->dim, A, s);
    else rc = launch<64, 64>(plan->dim, A, s);
    if (rc) return rc;
    if (plan->nlong > 0) {
        if (plan->dim == 2)
            FE_TIMED("k_assemble_long", s,
                     hipLaunchKernelGGL(k_assemble_long<3>, dim3((unsigned)plan->nlong), dim3(LNB), 0, s, A));
        else
            FE_TIMED("k_assemble_long", s,
                     hipLaunchKernelGGL(k_assemble_long<4>, dim3((unsigned)plan->nlong), dim3(LNB), 0, s, A));
        if ((rc = fe_launch_check())) return rc;
    }
    if (A.direct) return FE_OK;   // rows already in label order
    if (A.upper)
        FE_TIMED("k_values_to_label", s,
                 hipLaunchKernelGGL(k_values_to_label<true>, dim3((unsigned)cdiv(A.N, 256)), dim3(256), 0, s, A.N,
                                    urowptr, (const int4 *)plan->rowrec, (const int32_t *)plan->piinv,
                                    (const double *)plan->valp, val, val_bc, b, b_load, is_dirichlet));
    else
        FE_TIMED("k_values_to_label", s,
                 hipLaunchKernelGGL(k_values_to_label<false>, dim3((unsigned)cdiv(A.N, 256)), dim3(256), 0, s, A.N,
                                    (const int32_t *)plan->rowlen, (const int4 *)plan->rowrec,
                                    (const int32_t *)plan->piinv, (const double *)plan->valp, val, val_bc, b, b_load,
                                    is_dirichlet));
    return fe_launch_check();
}

}  // namespace

extern "C" int fe_assemble_quad(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                                const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r, double robin_alpha,
                                int32_t load_rule, double *val, double *val_bc, double *b, double *b_load,
                                uint8_t *is_dirichlet, void *stream)
{
    return assemble_impl(plan, nullptr, node, kappa, f, g_d, g_n, g_r, robin_alpha, load_rule, val, val_bc, b, b_load,
                         is_dirichlet, stream);
}

extern "C" int fe_assemble_upper(fe_plan *plan, const int32_t *rowptr_u, const double *node, const double *kappa,
                                 const fe_fn *f, const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r,
                                 double robin_alpha, int32_t load_rule, double *val_u, double *val_bc_u, double *b,
                                 double *b_load, uint8_t *is_dirichlet, void *stream)
{
    if (!rowptr_u) return FE_EINVAL;
    return assemble_impl(plan, rowptr_u, node, kappa, f, g_d, g_n, g_r, robin_alpha, load_rule, val_u, val_bc_u, b,
                         b_load, is_dirichlet, stream);
}

extern "C" int fe_assemble_robin(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                                 const fe_fn *g_d, const fe_fn *g_n, const fe_fn *g_r, double robin_alpha,
                                 double *val, double *val_bc, double *b, double *b_load, uint8_t *is_dirichlet,
                                 void *stream)
{
    return fe_assemble_quad(plan, node, kappa, f, g_d, g_n, g_r, robin_alpha, FE_LOAD_DEFAULT, val, val_bc, b, b_load,
                            is_dirichlet, stream);
}

extern "C" int fe_assemble(fe_plan *plan, const double *node, const double *kappa, const fe_fn *f,
                           const fe_fn *g_d, const fe_fn *g_n, double *val, double *val_bc, double *b,
                           double *b_load, uint8_t *is_dirichlet, void *stream)
{
    return fe_assemble_robin(plan, node, kappa, f, g_d, g_n, nullptr, 0.0, val, val_bc, b, b_load, is_dirichlet,
                             stream);
}
