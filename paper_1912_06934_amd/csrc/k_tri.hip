// Triangular smoothers of the two-stage preconditioner: ILU(0) (Sec. 3.2,
// Sec. 4.1), IC(0) (Sec. 4.1, Sec. 4.2) and symmetric Gauss-Seidel (Sec. 3.2,
// Sec. 4.2), each in a sweep order: the natural order, or a multicolour
// order (first-fit colouring in ascending row order on the symmetrised
// pattern, rows sorted by colour, ascending within a colour).
//
// Everything runs on A's own CSR pattern in its original numbering; the
// order only decides which stored entries count as "earlier" (lower) or
// "later" (upper).  Rows are grouped into dependency levels of the lower and
// of the upper triangle in that order.  A level with many rows is one launch
// across the whole GPU (thread per row); consecutive levels with few rows are
// walked by a single work-group with a barrier between levels.  In the
// multicolour order every colour is one level, so a sweep is a handful of
// wide launches; in the natural order a 2D grid has a few hundred narrow
// levels.  Either way every row sees its predecessors final, so the factors
// and solves equal the sequential algorithm in that order (up to the
// rounding of the sums).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace msrsb {
namespace {

constexpr int kNarrowThreads = 1024;
constexpr int kWideRows = 2048;  // a level with at least this many rows gets its own launch

// --- per-row device work ---

// position of column col in row i (columns ascending), or -1
__device__ __forceinline__ int find_col(const int *__restrict__ ci, int e0, int e1, int col)
{
    int lo = e0, hi = e1 - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int c = ci[mid];
        if (c == col) return mid;
        if (c < col) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

struct TriArgs {
    const int *rp, *ci, *dpos;
    const int8_t *side;  // -1 earlier column, 0 diagonal, +1 later
    const int *lord;     // earlier entries of each row, sorted by the column's rank
    const int *nlow;     // their count per row
};

// IKJ elimination of row i in the order (earlier neighbours k by rank)
__device__ void ilu_row(const TriArgs &t, int i, double *__restrict__ lu, int *__restrict__ flag)
{
    const int e0 = t.rp[i], e1 = t.rp[i + 1], nl = t.nlow[i];
    for (int u = 0; u < nl; ++u) {
        const int e = t.lord[e0 + u];
        const int k = t.ci[e];
        const double piv = lu[t.dpos[k]];
        if (piv == 0.0) flag[0] = 1;
        const double lik = lu[e] / piv;
        lu[e] = lik;
        for (int q = t.rp[k]; q < t.rp[k + 1]; ++q) {
            if (t.side[q] <= 0) continue;  // only entries later than k
            const int f = find_col(t.ci, e0, e1, t.ci[q]);
            if (f >= 0) lu[f] -= lik * lu[q];
        }
    }
}

// IC(0) row i: L_ij = (A_ij - sum_k L_ik L_jk) / L_jj over earlier j by rank,
// then L_ii = sqrt(A_ii - sum_k L_ik^2)
__device__ void ic_row(const TriArgs &t, int i, const double *__restrict__ a,
                       double *__restrict__ l, int *__restrict__ flag)
{
    const int e0 = t.rp[i], nl = t.nlow[i];
    for (int u = 0; u < nl; ++u) {
        const int e = t.lord[e0 + u];
        const int j = t.ci[e];
        double s = a[e];
        const int j0 = t.rp[j], j1 = t.rp[j + 1];
        for (int w = 0; w < u; ++w) {  // k earlier than j, stored in row i
            const int p = t.lord[e0 + w];
            const int f = find_col(t.ci, j0, j1, t.ci[p]);
            if (f >= 0) s -= l[p] * l[f];
        }
        l[e] = s / l[t.dpos[j]];
    }
    double s = a[t.dpos[i]];
    for (int u = 0; u < nl; ++u) {
        const double v = l[t.lord[e0 + u]];
        s -= v * v;
    }
    if (!(s > 0.0)) {
        flag[0] = 1;
        s = 1.0;
    }
    l[t.dpos[i]] = sqrt(s);
}

// x_i <- (x_i - sum over the stored entries on one side of vals x) / d_i
__device__ __forceinline__ void solve_row(const TriArgs &t, int i, int side, bool unit,
                                          const double *__restrict__ vals,
                                          double *__restrict__ x)
{
    double s = x[i];
    for (int e = t.rp[i]; e < t.rp[i + 1]; ++e)
        if (t.side[e] == side) s -= vals[e] * x[t.ci[e]];
    x[i] = unit ? s : s / vals[t.dpos[i]];
}

// --- kernels: wide (one level, thread per row) and narrow (levels walked by
// one work-group) ---

enum { OP_ILU = 0, OP_IC = 1, OP_LOWER = 2, OP_UPPER = 3 };

struct RowOp {
    int op = OP_LOWER;
    bool unit = false;
    const double *a = nullptr;  // IC(0): A's values
    double *f = nullptr;        // factor values (ILU, IC) or solve values
    double *x = nullptr;        // solve vector
    int *flag = nullptr;
};

__device__ __forceinline__ void do_row(const TriArgs &t, const RowOp &r, int i)
{
    switch (r.op) {
    case OP_ILU: ilu_row(t, i, r.f, r.flag); break;
    case OP_IC: ic_row(t, i, r.a, r.f, r.flag); break;
    case OP_LOWER: solve_row(t, i, -1, r.unit, r.f, r.x); break;
    default: solve_row(t, i, 1, r.unit, r.f, r.x); break;
    }
}

__global__ __launch_bounds__(256) void k_tri_wide(TriArgs t, RowOp r,
                                                  const int *__restrict__ rows, int count)
{
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u < count) do_row(t, r, rows[u]);
}

__global__ __launch_bounds__(kNarrowThreads) void k_tri_narrow(TriArgs t, RowOp r,
                                                               const int *__restrict__ lev_ptr,
                                                               const int *__restrict__ rows,
                                                               int lev0, int lev1)
{
    for (int l = lev0; l < lev1; ++l) {
        for (int u = lev_ptr[l] + threadIdx.x; u < lev_ptr[l + 1]; u += kNarrowThreads)
            do_row(t, r, rows[u]);
        __syncthreads();
    }
}

// The triangular solves of a run of narrow levels in the natural order, for
// systems of at most kNarrowLdsRows rows: x lives in LDS for the whole run,
// and a row's entries on the solved side (contiguous in the natural order:
// the columns before or after the diagonal) are loaded into registers while
// the previous level is still being solved, so a level costs LDS reads and
// one barrier instead of a chain of memory round trips.  The arithmetic and
// its order are those of solve_row.  A thread's first row of a level takes
// this path; further rows (levels wider than the work-group) and rows with
// more than kRowRegs entries on the side read their data from memory.
constexpr int kNarrowLdsRows = 16384;  // 128 KB of LDS
constexpr int kRowRegs = 8;

struct SolveRow {
    int i, ne;
    int c[kRowRegs];
    double v[kRowRegs];
    double d;
};

__global__ __launch_bounds__(kNarrowThreads) void k_tri_narrow_lds(TriArgs t, RowOp r,
                                                                   const int *__restrict__ lev_ptr,
                                                                   const int *__restrict__ rows,
                                                                   int lev0, int lev1, int n)
{
    extern __shared__ double sx[];
    const int tid = threadIdx.x;
    const bool lower = r.op == OP_LOWER;
    const int side = lower ? -1 : 1;
    for (int i = tid; i < n; i += kNarrowThreads) sx[i] = r.x[i];
    auto load = [&](int l, SolveRow &q) {
        q.i = -1;
        q.ne = 0;
        if (l >= lev1) return;
        const int u = lev_ptr[l] + tid;
        if (u >= lev_ptr[l + 1]) return;
        const int i = rows[u];
        const int dp = t.dpos[i];
        const int b = lower ? t.rp[i] : dp + 1, e = lower ? dp : t.rp[i + 1];
        q.i = i;
        q.ne = e - b;
#pragma unroll
        for (int k = 0; k < kRowRegs; ++k) {
            const int idx = b + k < e ? b + k : dp;
            q.c[k] = t.ci[idx];
            q.v[k] = r.f[idx];
        }
        q.d = r.unit ? 1.0 : r.f[dp];
    };
    auto slow = [&](int i) {
        double s = sx[i];
        for (int e = t.rp[i]; e < t.rp[i + 1]; ++e)
            if (t.side[e] == side) s -= r.f[e] * sx[t.ci[e]];
        sx[i] = r.unit ? s : s / r.f[t.dpos[i]];
    };
    SolveRow cur, nxt;
    load(lev0, cur);
    __syncthreads();
    for (int l = lev0; l < lev1; ++l) {
        load(l + 1, nxt);  // independent of x: in flight while this level is solved
        if (cur.i >= 0) {
            if (cur.ne <= kRowRegs) {
                double s = sx[cur.i];
#pragma unroll
                for (int k = 0; k < kRowRegs; ++k)
                    if (k < cur.ne) s -= cur.v[k] * sx[cur.c[k]];
                sx[cur.i] = r.unit ? s : s / cur.d;
            } else {
                slow(cur.i);
            }
        }
        for (int u = lev_ptr[l] + tid + kNarrowThreads; u < lev_ptr[l + 1]; u += kNarrowThreads)
            slow(rows[u]);
        __syncthreads();
        cur = nxt;
    }
    for (int i = tid; i < n; i += kNarrowThreads) r.x[i] = sx[i];
}

// A run of narrow levels in the natural order solved by one wavefront, with
// no barrier between levels: a wavefront's LDS operations complete in
// order, so a level reads the x values the previous levels wrote.  Each
// lane takes up to two rows of a level (levels of at most kTriWaveRows rows,
// rows of at most kTriWaveW entries on the solved side), whose entries are
// packed beforehand (k_tri_pack) and loaded kTriDepth levels ahead, so a
// level costs LDS reads, its products and one division.  The arithmetic and
// its order are those of solve_row.
// levels loaded ahead and steps per loop trip, by row width (the ring of
// loaded rows has to fit the registers); the solve takes rows of at most
// kTriWaveW entries on the solved side (2D 9-point stencils and narrower)
template <int W> constexpr int kTriDepth = W <= 4 ? 6 : 3;
template <int W> constexpr int kTriUnroll = W <= 4 ? 4 : 8;
constexpr int kTriWaveW = 4;
constexpr int kTriWaveRows = 128;       // rows per level (two per lane)
constexpr size_t kTriWaveLds = 160 * 1024;  // x, the spare slot and the level pointers

struct alignas(16) PackedRow {
    int i, ne, b, pad;     // row; its entries on the solved side: count, first
    int c[kRowRegs];       // their columns (at most kRowRegs kept)
    double v[kRowRegs];    // their values
    double d, pad2;        // the diagonal (1 for a unit diagonal)
};

__global__ __launch_bounds__(256) void k_tri_pack(TriArgs t, RowOp r,
                                                  const int *__restrict__ rows, int u0, int u1,
                                                  PackedRow *__restrict__ rec)
{
    const int u = u0 + static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
    if (u >= u1) return;
    const int i = rows[u];
    const int dp = t.dpos[i];
    const bool lower = r.op == OP_LOWER;
    const int b = lower ? t.rp[i] : dp + 1, e = lower ? dp : t.rp[i + 1];
    PackedRow q;
    q.i = i;
    q.ne = e - b;
    q.b = b;
    q.pad = 0;
#pragma unroll
    for (int k = 0; k < kRowRegs; ++k) {
        const int idx = b + k < e ? b + k : dp;
        q.c[k] = t.ci[idx];
        q.v[k] = r.f[idx];
    }
    q.d = r.unit ? 1.0 : r.f[dp];
    q.pad2 = 0.0;
    rec[u] = q;
}

// One packed row (at most kRowRegs entries): s = x_i - (its entries times
// x), x_i = s or s / d, in solve_row's order.  The slots past the row's
// count hold its own column (a valid index) and add zero, and a lane
// without a row (ok false) writes its duplicate's value to the spare slot
// sx[n]: no branch, so the loads kTriDepth levels ahead stay in flight.
template <int W>
__device__ __forceinline__ void tri_wave_solve(const RowOp &r, double *sx, int n,
                                               const PackedRow &q, bool ok)
{
    double s = sx[q.i];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const double xv = sx[q.c[k]];
        s -= (k < q.ne ? q.v[k] : 0.0) * xv;
    }
    sx[ok ? q.i : n] = r.unit ? s : s / q.d;
}

// W: the most entries of a row on the solved side (4 or kRowRegs); only
// those slots of the packed rows are loaded and used
template <int W>
__global__ __launch_bounds__(64) void k_tri_wave(RowOp r, const int *__restrict__ lev_ptr,
                                                 const PackedRow *__restrict__ rec, int lev0,
                                                 int lev1, int n)
{
    // n + 1 values: x and a spare slot; then the run's level pointers, kept
    // in LDS so that no other memory load sits between the rows' loads (a
    // wait for one would wait for all rows loaded before it)
    extern __shared__ double sx[];
    int *slev = reinterpret_cast<int *>(sx + n + 1);
    const int lane = threadIdx.x;
    for (int i = lane; i < n; i += 64) sx[i] = r.x[i];
    for (int l = lev0 + lane; l <= lev1; l += 64) slev[l - lev0] = lev_ptr[l];
    // the first kTriWaveRows rows of level l (positions clamped to the level,
    // and a level past the run to the last one: every load is in bounds)
    auto load = [&](int l, PackedRow (&q)[2], bool (&ok)[2]) {
        const int lc = min(l, lev1 - 1) - lev0;
        const int u0 = slev[lc], u1 = slev[lc + 1];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = u0 + lane + 64 * h;
            ok[h] = l < lev1 && u < u1;
            const PackedRow &g = rec[min(u, u1 - 1)];
            q[h].i = g.i;
            q[h].ne = g.ne;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                q[h].c[k] = g.c[k];
                q[h].v[k] = g.v[k];
            }
            q[h].d = g.d;
        }
    };
    PackedRow ring[kTriDepth<W>][2];
    bool rok[kTriDepth<W>][2];
#pragma unroll
    for (int k = 0; k < kTriDepth<W>; ++k) load(lev0 + k, ring[k], rok[k]);
    // kTriUnroll steps of kTriDepth levels per loop trip: the compiler waits
    // for every row in flight where the loop closes, so it closes rarely
    for (int l = lev0; l < lev1; l += kTriDepth<W> * kTriUnroll<W>) {
#pragma unroll
        for (int kk = 0; kk < kTriDepth<W> * kTriUnroll<W>; ++kk) {
            const int k = kk % kTriDepth<W>;
            // (levels past the run: their rows are marked, nothing is written;
            // the scheduling barriers keep a later level's arithmetic, and
            // with it the wait for its rows, below this level's)
            __builtin_amdgcn_sched_barrier(0);
            tri_wave_solve<W>(r, sx, n, ring[k][0], rok[k][0]);
            tri_wave_solve<W>(r, sx, n, ring[k][1], rok[k][1]);
            load(l + kk + kTriDepth<W>, ring[k], rok[k]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (int i = lane; i < n; i += 64) r.x[i] = sx[i];
}

// upper entries of the IC(0) array take the factor value of their transpose
__global__ __launch_bounds__(256) void k_ic_mirror(int64_t nnz, const int8_t *__restrict__ side,
                                                   const int *__restrict__ tpos,
                                                   double *__restrict__ l)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e < nnz && side[e] > 0) l[e] = l[tpos[e]];
}

__global__ __launch_bounds__(256) void k_copy_vals(int64_t m, const double *__restrict__ a,
                                                   double *__restrict__ b)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t < m) b[t] = a[t];
}

__global__ __launch_bounds__(256) void k_add(int n, const double *__restrict__ x,
                                             double *__restrict__ z)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) z[i] += x[i];
}

// --- host: colouring, levels, launch segments ---

// first fit in ascending row order on the symmetrised pattern
int first_fit_colours(int n, const std::vector<int> &rp, const std::vector<int> &ci,
                      std::vector<int> &colour)
{
    std::vector<int> trp(n + 1, 0), tci(ci.size());
    for (int c : ci) trp[c + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    {
        std::vector<int> pos(trp.begin(), trp.end() - 1);
        for (int i = 0; i < n; ++i)
            for (int e = rp[i]; e < rp[i + 1]; ++e) tci[pos[ci[e]]++] = i;
    }
    colour.assign(n, 0);
    std::vector<int> seen(n + 1, -1);
    int ncol = 0;
    for (int i = 0; i < n; ++i) {
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] < i) seen[colour[ci[e]]] = i;
        for (int e = trp[i]; e < trp[i + 1]; ++e)
            if (tci[e] < i) seen[colour[tci[e]]] = i;
        int c = 0;
        while (seen[c] == i) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// rows grouped by dependency level (lower: on earlier entries, visited in
// order; upper: on later entries, visited backwards); rows ascending within
// a level
void level_sets(int n, const std::vector<int> &rp, const std::vector<int> &ci,
                const std::vector<int> &order, const std::vector<int> &rank, bool lower,
                std::vector<int> &ptr, std::vector<int> &rows)
{
    std::vector<int> lev(n, 0);
    int maxl = 0;
    for (int t = 0; t < n; ++t) {
        const int i = order[lower ? t : n - 1 - t];
        int l = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (lower ? rank[j] < rank[i] : rank[j] > rank[i]) l = std::max(l, lev[j] + 1);
        }
        lev[i] = l;
        maxl = std::max(maxl, l);
    }
    ptr.assign(maxl + 2, 0);
    for (int i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int l = 0; l <= maxl; ++l) ptr[l + 1] += ptr[l];
    rows.resize(n);
    std::vector<int> pos(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[pos[lev[i]]++] = i;
}

void segments(const std::vector<int> &ptr, std::vector<TriSegment> &seg)
{
    seg.clear();
    const int nlev = static_cast<int>(ptr.size()) - 1;
    for (int l = 0; l < nlev; ++l) {
        const bool wide = ptr[l + 1] - ptr[l] >= kWideRows;
        if (!wide && !seg.empty() && !seg.back().wide && seg.back().lev1 == l) {
            seg.back().lev1 = l + 1;
            continue;
        }
        seg.push_back(TriSegment{l, l + 1, wide});
    }
}

template <typename T>
bool upload(T *&d, const std::vector<T> &h)
{
    if (hipMalloc(&d, std::max<size_t>(h.size(), 1) * sizeof(T)) != hipSuccess) return false;
    return hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

void run_levels(hipStream_t s, const TriOrder &t, bool lower, const RowOp &r)
{
    const TriArgs a{t.rp, t.ci, t.dpos, t.side, t.lord, t.nlow};
    const std::vector<int> &ptr = lower ? t.h_lev_l : t.h_lev_u;
    const std::vector<TriSegment> &seg = lower ? t.seg_l : t.seg_u;
    const int *rows = lower ? t.rows_l : t.rows_u;
    const int *dptr = lower ? t.ptr_l : t.ptr_u;
    for (const TriSegment &g : seg) {
        if (g.wide) {
            const int cnt = ptr[g.lev0 + 1] - ptr[g.lev0];
            k_tri_wide<<<(cnt + 255) / 256, 256, 0, s>>>(a, r, rows + ptr[g.lev0], cnt);
        } else if (t.ncolours == 0 && (r.op == OP_LOWER || r.op == OP_UPPER) &&
                   t.n <= kNarrowLdsRows && t.packed &&
                   (lower ? t.max_lo : t.max_up) <= kTriWaveW &&
                   (lower ? t.max_w_l : t.max_w_u) <= kTriWaveRows &&
                   static_cast<size_t>(t.n + 1) * sizeof(double) +
                           static_cast<size_t>(g.lev1 - g.lev0 + 1) * sizeof(int) <=
                       kTriWaveLds) {
            const size_t sh = static_cast<size_t>(t.n + 1) * sizeof(double) +
                              static_cast<size_t>(g.lev1 - g.lev0 + 1) * sizeof(int);
            auto *rec = static_cast<PackedRow *>(t.packed);
            const int u0 = ptr[g.lev0], u1 = ptr[g.lev1];
            k_tri_pack<<<(u1 - u0 + 255) / 256, 256, 0, s>>>(a, r, rows, u0, u1, rec);
            auto wave = [&](auto kern) {
                if (sh > 65536)
                    hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        static_cast<int>(sh));
                kern<<<1, 64, sh, s>>>(r, dptr, rec, g.lev0, g.lev1, t.n);
            };
            wave(k_tri_wave<kTriWaveW>);
        } else if (t.ncolours == 0 && (r.op == OP_LOWER || r.op == OP_UPPER) &&
                   t.n <= kNarrowLdsRows) {
            const size_t sh = static_cast<size_t>(t.n) * sizeof(double);
            if (sh > 65536)
                hipFuncSetAttribute(reinterpret_cast<const void *>(k_tri_narrow_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(sh));
            k_tri_narrow_lds<<<1, kNarrowThreads, sh, s>>>(a, r, dptr, rows, g.lev0, g.lev1, t.n);
        } else {
            k_tri_narrow<<<1, kNarrowThreads, 0, s>>>(a, r, dptr, rows, g.lev0, g.lev1);
        }
    }
}

}  // namespace

void free_tri_order(TriOrder &t)
{
    for (void *p : {static_cast<void *>(t.rank), static_cast<void *>(t.side),
                    static_cast<void *>(t.lord), static_cast<void *>(t.nlow),
                    static_cast<void *>(t.tpos), static_cast<void *>(t.rows_l),
                    static_cast<void *>(t.rows_u), static_cast<void *>(t.ptr_l),
                    static_cast<void *>(t.ptr_u), t.packed})
        if (p) hipFree(p);
    t = TriOrder();
}

msrsb_status tri_order_setup(msrsb_ctx *c, int ordering)
{
    TriOrder &t = c->tri[ordering];
    if (t.built) return MSRSB_OK;
    const int n = c->n;
    const std::vector<int> &rp = c->h_rp, &ci = c->h_ci;
    std::vector<int> order(n), rank(n);
    if (ordering == MSRSB_ORDER_MULTICOLOR) {
        std::vector<int> colour;
        const int ncol = first_fit_colours(n, rp, ci, colour);
        std::vector<int> start(ncol + 1, 0);
        for (int i = 0; i < n; ++i) start[colour[i] + 1]++;
        for (int k = 0; k < ncol; ++k) start[k + 1] += start[k];
        for (int i = 0; i < n; ++i) order[start[colour[i]]++] = i;
        t.ncolours = ncol;
    } else {
        std::iota(order.begin(), order.end(), 0);
        t.ncolours = 0;
    }
    t.n = n;
    for (int k = 0; k < n; ++k) rank[order[k]] = k;
    const int64_t nnz = c->nnz;
    std::vector<int8_t> side(nnz);
    std::vector<int> lord(nnz, 0), nlow(n, 0), tpos(nnz, -1);
    for (int i = 0; i < n; ++i) {
        std::vector<std::pair<int, int>> low;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            side[e] = j == i ? 0 : (rank[j] < rank[i] ? -1 : 1);
            if (side[e] < 0) low.emplace_back(rank[j], e);
            // the transposed entry (j, i), when stored
            const auto b = ci.begin() + rp[j], en = ci.begin() + rp[j + 1];
            const auto it = std::lower_bound(b, en, i);
            if (it != en && *it == i) tpos[e] = static_cast<int>(it - ci.begin());
        }
        std::sort(low.begin(), low.end());
        nlow[i] = static_cast<int>(low.size());
        for (size_t u = 0; u < low.size(); ++u) lord[rp[i] + u] = low[u].second;
    }
    t.sym_pattern = std::all_of(tpos.begin(), tpos.end(), [](int p) { return p >= 0; });
    std::vector<int> pl, rl, pu, ru;
    level_sets(n, rp, ci, order, rank, true, pl, rl);
    level_sets(n, rp, ci, order, rank, false, pu, ru);
    segments(pl, t.seg_l);
    segments(pu, t.seg_u);
    for (int i = 0; i < n; ++i) {
        int lo = 0, up = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            lo += side[e] < 0 ? 1 : 0;
            up += side[e] > 0 ? 1 : 0;
        }
        t.max_lo = std::max(t.max_lo, lo);
        t.max_up = std::max(t.max_up, up);
    }
    for (size_t l = 0; l + 1 < pl.size(); ++l) t.max_w_l = std::max(t.max_w_l, pl[l + 1] - pl[l]);
    for (size_t l = 0; l + 1 < pu.size(); ++l) t.max_w_u = std::max(t.max_w_u, pu[l + 1] - pu[l]);
    t.h_lev_l = pl;
    t.h_lev_u = pu;
    if (!upload(t.rank, rank) || !upload(t.side, side) || !upload(t.lord, lord) ||
        !upload(t.nlow, nlow) || !upload(t.tpos, tpos) || !upload(t.rows_l, rl) ||
        !upload(t.rows_u, ru) || !upload(t.ptr_l, pl) || !upload(t.ptr_u, pu)) {
        free_tri_order(t);
        return MSRSB_E_NOMEM;
    }
    // natural order on a system small enough for x in LDS: the solves' rows
    // packed by level position (one row per position of either triangle)
    if (t.ncolours == 0 && n <= kNarrowLdsRows &&
        hipMalloc(&t.packed, static_cast<size_t>(n) * sizeof(PackedRow)) != hipSuccess) {
        free_tri_order(t);
        return MSRSB_E_NOMEM;
    }
    t.rp = c->rp;
    t.ci = c->ci;
    t.dpos = c->diag_pos;
    t.built = true;
    return MSRSB_OK;
}

msrsb_status tri_factor(msrsb_ctx *c, int ordering, int kind)
{
    hipStream_t s = c->stream;
    TriOrder &t = c->tri[ordering];
    double *&f = kind == MSRSB_SMOOTH_ILU0 ? c->ilu_f[ordering] : c->ic_f[ordering];
    if (!f && hipMalloc(&f, c->nnz * sizeof(double)) != hipSuccess) return MSRSB_E_NOMEM;
    int *flag = c->dev_flag;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    RowOp r;
    r.f = f;
    r.flag = flag;
    const int nb = static_cast<int>((c->nnz + 255) / 256);
    if (kind == MSRSB_SMOOTH_ILU0) {
        k_copy_vals<<<nb, 256, 0, s>>>(c->nnz, c->a, f);
        r.op = OP_ILU;
        run_levels(s, t, true, r);
    } else {
        r.op = OP_IC;
        r.a = c->a;
        run_levels(s, t, true, r);
        k_ic_mirror<<<nb, 256, 0, s>>>(c->nnz, t.side, t.tpos, f);
    }
    int hflag = 0;
    hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSRSB_E_HIP;
    return hflag ? MSRSB_E_BREAKDOWN : MSRSB_OK;
}

// z += M^{-1} res for ILU(0) / IC(0) (res is overwritten); one half of a
// Gauss-Seidel sweep: (D + L)^{-1} (lower) or (D + U)^{-1} (upper) with A's
// own values
void tri_apply(msrsb_ctx *c, int ordering, int kind, double *res, double *z)
{
    hipStream_t s = c->stream;
    const TriOrder &t = c->tri[ordering];
    RowOp r;
    r.x = res;
    if (kind == MSRSB_SMOOTH_ILU0) {
        r.f = c->ilu_f[ordering];
        r.op = OP_LOWER;
        r.unit = true;
        run_levels(s, t, true, r);
        r.op = OP_UPPER;
        r.unit = false;
        run_levels(s, t, false, r);
    } else if (kind == MSRSB_SMOOTH_IC0) {
        r.f = c->ic_f[ordering];
        r.op = OP_LOWER;
        run_levels(s, t, true, r);
        r.op = OP_UPPER;
        run_levels(s, t, false, r);
    }
    k_add<<<(c->n + 255) / 256, 256, 0, s>>>(c->n, res, z);
}

void tri_gs_half(msrsb_ctx *c, int ordering, bool lower, double *res, double *z)
{
    hipStream_t s = c->stream;
    RowOp r;
    r.x = res;
    r.f = c->a;
    r.op = lower ? OP_LOWER : OP_UPPER;
    run_levels(s, c->tri[ordering], lower, r);
    k_add<<<(c->n + 255) / 256, 256, 0, s>>>(c->n, res, z);
}

}  // namespace msrsb
