// Coarse-level kernels: R = P^T values, the Galerkin operator A_c = R A P
// (eq. lin_system_coarse, Alg. 2), the exact coarse solver M_c^{-1} = A_c^{-1}
// and its application.
#include <utility>

#include "internal.h"

#include <type_traits>

namespace msrsb {
namespace {

inline int grid_for(int64_t m) { return static_cast<int>((m + kBlock - 1) / kBlock); }

// r[t] = p[src[t]], or 0 where src[t] < 0 (R's row padding)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int64_t m, const int *__restrict__ src,
                                                   const T *__restrict__ p, T *__restrict__ r)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t < m) {
        const int e = src[t];
        r[t] = e >= 0 ? p[e] : T(0);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t m, double *__restrict__ x, double v)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t < m) x[t] = v;
}

// A_c row j = sum over fine rows i in the support of j (R row j, ascending
// i) of P_ij * A_i* * P.  One work-group per coarse row.  The coarse columns
// reached by row j (its coarse neighbours) are found first and numbered in
// ascending order in an LDS map; each thread then accumulates its share of
// the fine rows into a private LDS column of per-neighbour partial sums, and
// the partial sums of every neighbour are added in thread order.  The column
// updates are LDS atomic adds: a thread's adds to one address land in
// program order (so the sums are reproducible), but unlike a load-add-store
// they do not have to wait for one another when two products may share a
// column.  No atomics touch A_c, so it is bitwise reproducible.  The lower and upper bandwidths
// of A_c are recorded for the coarse factorisation.
template <typename T, int NT, bool DIA>
__global__ __launch_bounds__(NT) void k_rap(int n, int nc, int maxnb, const int *__restrict__ rrp,
                                            const int *__restrict__ rci,
                                            const T *__restrict__ rv, const int *__restrict__ rp,
                                            const int *__restrict__ ci,
                                            const double *__restrict__ a, DiaOffsets d,
                                            const double *__restrict__ ad,
                                            const int *__restrict__ prp,
                                            const int *__restrict__ pci,
                                            const double *__restrict__ pv, double *__restrict__ ac,
                                            int *__restrict__ flag, int *__restrict__ band)
{
    extern __shared__ double smem[];
    __shared__ int wsum[NT / 64];
    double *acc = smem;                                         // maxnb * NT
    int *inv = reinterpret_cast<int *>(acc + maxnb * NT);       // maxnb
    short *map = reinterpret_cast<short *>(inv + maxnb);        // nc
    const int j = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ne = DIA ? d.n : 0;
    for (int t = tid; t < nc; t += NT) map[t] = 0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    for (int t = t0 + tid; t < t1; t += NT) {
        const int i = rci[t];
        const int e0 = DIA ? 0 : rp[i], e1 = DIA ? ne : rp[i + 1];
        for (int e = e0; e < e1; ++e) {
            const int k = DIA ? i + d.off[e] : ci[e];
            if (DIA && (k < 0 || k >= n || ad[static_cast<int64_t>(e) * n + i] == 0.0)) continue;
            for (int q = prp[k]; q < prp[k + 1]; ++q) map[pci[q]] = 1;
        }
    }
    __syncthreads();
    // number the marked coarse columns in ascending order (block scan)
    const int chunk = (nc + NT - 1) / NT;
    const int lo = tid * chunk, hi = min(nc, lo + chunk);
    int cnt = 0;
    for (int t = lo; t < hi; ++t) cnt += map[t];
    int pre = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(pre, off, 64);
        if (lane >= off) pre += o;
    }
    if (lane == 63) wsum[wid] = pre;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wid) base += wsum[w];
        total += wsum[w];
    }
    if (total > maxnb) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    int slot = base + pre - cnt;
    __syncthreads();
    for (int t = lo; t < hi; ++t) {
        if (map[t]) {
            inv[slot] = t;
            map[t] = static_cast<short>(slot++);
        } else {
            map[t] = -1;
        }
    }
    for (int s = 0; s < total; ++s) acc[s * NT + tid] = 0.0;
    __syncthreads();
    for (int t = t0 + tid; t < t1; t += NT) {
        const int i = rci[t];
        const double pij = static_cast<double>(rv[t]);
        const int e0 = DIA ? 0 : rp[i], e1 = DIA ? ne : rp[i + 1];
        for (int e = e0; e < e1; ++e) {
            const int k = DIA ? i + d.off[e] : ci[e];
            const double av = DIA ? ((k >= 0 && k < n) ? ad[static_cast<int64_t>(e) * n + i] : 0.0)
                                  : a[e];
            if (DIA && av == 0.0) continue;
            const double pa = pij * av;
            for (int q = prp[k]; q < prp[k + 1]; ++q)
                atomicAdd(&acc[map[pci[q]] * NT + tid], pa * pv[q]);
        }
    }
    __syncthreads();
    int bl = 0, bu = 0;
    for (int s = tid; s < total; s += NT) {
        double sum = 0.0;
        for (int l = 0; l < NT; ++l) sum += acc[s * NT + l];
        const int col = inv[s];
        ac[static_cast<int64_t>(j) * nc + col] = sum;
        if (sum != 0.0) {
            bl = max(bl, j - col);
            bu = max(bu, col - j);
        }
    }
    if (bl > 0) atomicMax(band, bl);
    if (bu > 0) atomicMax(band + 1, bu);
}

// The same product for a stencil A (ND diagonals, compile-time) and P in its
// row-major ELL form (PW slots, 16-bit columns, 0xFFFF = padding, values in
// T).  A fine row's ND coefficients and the ND neighbour rows of P (values
// and columns) are all loaded before they are used.  The order of the sums
// is that of k_rap (neighbours in offset order, slots in column order).
template <typename PT>
__device__ __forceinline__ void load_prow(const PT *__restrict__ p, const uint16_t *__restrict__ pc,
                                          int64_t row, PT (&v)[8], uint16_t (&c)[8])
{
    typedef uint16_t cvec __attribute__((ext_vector_type(8)));
    constexpr int L = 16 / sizeof(PT);
    typedef PT tvec __attribute__((ext_vector_type(L)));
    const cvec cc = *reinterpret_cast<const cvec *>(pc + row * 8);
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = cc[u];
    const tvec *vs = reinterpret_cast<const tvec *>(p + row * 8);
#pragma unroll
    for (int q = 0; q < 8 / L; ++q) {
        const tvec x = vs[q];
#pragma unroll
        for (int u = 0; u < L; ++u) v[L * q + u] = x[u];
    }
}

// The coarse columns of row j of R A P (stencil A with ND diagonals, ELL P):
// the columns of P's rows k = i + off that row i of R reaches through a
// nonzero A_ik, marked in map (nc entries of LDS) and numbered in ascending
// order, map[c] = slot or -1 and inv[slot] = c.  Returns their count (in
// every thread); the numbering is done only when the count fits cap.
// Called by all NT threads.
// Numbers the coarse columns marked in map (nc entries, 1 = marked) in
// ascending order: map[c] = slot or -1 and inv[slot] = c.  Returns their
// count (in every thread); the numbering is done only when the count fits
// cap.  Called by all NT threads after the marking.
template <int NT>
__device__ inline int number_columns(int nc, int cap, short *map, int *inv)
{
    __shared__ int wsum[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int chunk = (nc + NT - 1) / NT;
    const int lo = tid * chunk, hi = min(nc, lo + chunk);
    int cnt = 0;
    for (int t = lo; t < hi; ++t) cnt += map[t];
    int pre = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(pre, off, 64);
        if (lane >= off) pre += o;
    }
    if (lane == 63) wsum[wid] = pre;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wid) base += wsum[w];
        total += wsum[w];
    }
    if (total > cap) return total;
    int slot = base + pre - cnt;
    __syncthreads();
    for (int t = lo; t < hi; ++t) {
        if (map[t]) {
            inv[slot] = t;
            map[t] = static_cast<short>(slot++);
        } else {
            map[t] = -1;
        }
    }
    return total;
}

template <int NT, int ND>
__device__ inline int rap_columns(int n, int nc, int j, int cap, const int *__restrict__ rrp,
                                  const int *__restrict__ rci, const DiaOffsets &d,
                                  const double *__restrict__ ad,
                                  const uint16_t *__restrict__ pcol, short *map, int *inv)
{
    const int tid = threadIdx.x;
    for (int t = tid; t < nc; t += NT) map[t] = 0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    // entries t, t + NT, ... (UM of them) of a thread at once; a neighbour's
    // columns are read whether or not its coefficient is zero (the test comes
    // after), so every load of those entries is in flight together
    typedef uint16_t cvec __attribute__((ext_vector_type(8)));
    constexpr int UM = 4;
    for (int t = t0 + tid; t < t1; t += UM * NT) {
        int ii[UM];
        bool ok[UM];
#pragma unroll
        for (int q = 0; q < UM; ++q) {
            ok[q] = t + q * NT < t1;
            ii[q] = rci[ok[q] ? t + q * NT : t];
        }
        double av[UM][ND];
        cvec cc[UM][ND];
#pragma unroll
        for (int q = 0; q < UM; ++q)
#pragma unroll
            for (int o = 0; o < ND; ++o) {
                const int k = ii[q] + d.off[o];
                const bool in = k >= 0 && k < n;
                av[q][o] = in && ok[q] ? ad[static_cast<int64_t>(o) * n + ii[q]] : 0.0;
                cc[q][o] = *reinterpret_cast<const cvec *>(pcol + static_cast<int64_t>(in ? k : ii[q]) * 8);
            }
#pragma unroll
        for (int q = 0; q < UM; ++q)
#pragma unroll
            for (int o = 0; o < ND; ++o) {
                if (av[q][o] == 0.0) continue;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (cc[q][o][u] != 0xFFFFu) map[cc[q][o][u]] = 1;
            }
    }
    __syncthreads();
    return number_columns<NT>(nc, cap, map, inv);
}

// The column lists of R A P by coarse row, once per pattern (set-up of the
// coarse space): cols[j * kMaxCoarseNeighbours + s], s < ncol[j], ascending
// (a row with more columns stores its count only).
template <int ND>
__global__ __launch_bounds__(128) void k_rap_cols(int n, int nc, const int *__restrict__ rrp,
                                                  const int *__restrict__ rci, DiaOffsets d,
                                                  const double *__restrict__ ad,
                                                  const uint16_t *__restrict__ pcol,
                                                  int *__restrict__ cols, int *__restrict__ ncol)
{
    extern __shared__ double smem[];
    int *inv = reinterpret_cast<int *>(smem);                        // kMaxCoarseNeighbours
    short *map = reinterpret_cast<short *>(inv + kMaxCoarseNeighbours);  // nc
    const int j = blockIdx.x;
    const int total = rap_columns<128, ND>(n, nc, j, kMaxCoarseNeighbours, rrp, rci, d, ad, pcol,
                                           map, inv);
    __syncthreads();
    if (total <= kMaxCoarseNeighbours)
        for (int s = threadIdx.x; s < total; s += 128)
            cols[static_cast<int64_t>(j) * kMaxCoarseNeighbours + s] = inv[s];
    if (threadIdx.x == 0) ncol[j] = total;
}

// One product of R A P into the thread's LDS column of partial sums, with
// no branch: a padding slot of P (column 0xFFFF) and a column outside the
// row's list go to the spare column maxnb, which is never summed (a nonzero
// product there sets miss), and a zero coefficient adds +0.  The sums of
// the listed columns see the same nonzero terms in the same order as when
// those cases are skipped.  (For the node-block operators, whose rows of 81
// products per R entry made the per-slot branches' exec-mask work the
// largest instruction stream: 9.95 -> 8.46 ms at c3.)
__device__ __forceinline__ void rap_add(double *acc, const short *map, int maxnb, int tid, int nt,
                                        uint16_t c, double prod, bool &miss)
{
    const bool pad = c == 0xFFFFu;
    const int m = map[pad ? 0 : c];
    const bool hit = !pad && m >= 0;
    miss |= !pad && m < 0 && prod != 0.0;
    atomicAdd(&acc[(hit ? m : maxnb) * nt + tid], prod);
}

// The numeric product: with column lists (cols, ncol from k_rap_cols) the
// row's columns are installed in the LDS map directly; without, they are
// marked here as above.  A contribution to a column outside a list (A's
// values gained a nonzero since the lists were formed) sets flag[1], and
// the caller rebuilds the lists and repeats; more columns than maxnb set
// flag[0].
template <typename T, int NT, int ND, bool CSR>
__global__ __launch_bounds__(NT) void k_rap_ell(int n, int nc, int maxnb,
                                                const int *__restrict__ rrp,
                                                const int *__restrict__ rci,
                                                const T *__restrict__ rv, DiaOffsets d,
                                                const double *__restrict__ ad,
                                                const uint16_t *__restrict__ pcol,
                                                const T *__restrict__ pv, double *__restrict__ ac,
                                                int *__restrict__ flag, int *__restrict__ band,
                                                const int *__restrict__ cols,
                                                const int *__restrict__ ncol,
                                                const int *__restrict__ csr_rp,
                                                const int *__restrict__ order)
{
    extern __shared__ double smem[];
    double *acc = smem;                                         // (maxnb + 1) * NT
    int *inv = reinterpret_cast<int *>(acc + (maxnb + 1) * NT);  // maxnb
    short *map = reinterpret_cast<short *>(inv + maxnb);        // nc
    // with order, each XCD walks a contiguous run of the coarse rows listed
    // brick by brick, so that the rows it runs at once share their P rows
    // in its L2
    const int j = order ? order[xcd_group(blockIdx.x, gridDim.x)] : static_cast<int>(blockIdx.x);
    const int tid = threadIdx.x;
    int total;
    if (cols != nullptr) {
        total = ncol[j];
        if (total > maxnb) {
            if (tid == 0) flag[0] = 1;
            return;
        }
        for (int t = tid; t < nc; t += NT) map[t] = -1;
        __syncthreads();
        for (int s = tid; s < total; s += NT) {
            const int c = cols[static_cast<int64_t>(j) * kMaxCoarseNeighbours + s];
            inv[s] = c;
            map[c] = static_cast<short>(s);
        }
    } else {
        total = rap_columns<NT, ND>(n, nc, j, maxnb, rrp, rci, d, ad, pcol, map, inv);
        if (total > maxnb) {
            if (tid == 0) flag[0] = 1;
            return;
        }
    }
    for (int s = 0; s < total; ++s) acc[s * NT + tid] = 0.0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    bool miss = false;
    // UA entries of a thread per round (t, t + NT, ...), their loads all in
    // flight together; the sums are taken in the same entry order as one at
    // a time (UA = 1 for FP64 rows, which would not fit in registers twice)
    constexpr int UA = sizeof(T) == 4 ? 2 : 1;
    for (int t = t0 + tid; t < t1; t += UA * NT) {
        int ii[UA];
        double pij[UA];
#pragma unroll
        for (int q = 0; q < UA; ++q) {
            const bool ok = t + q * NT < t1;
            ii[q] = rci[ok ? t + q * NT : t];
            pij[q] = ok ? static_cast<double>(rv[t + q * NT]) : 0.0;
        }
        double av[UA][ND];
        T v[UA][ND][8];
        uint16_t cl[UA][ND][8];
#pragma unroll
        for (int q = 0; q < UA; ++q)
#pragma unroll
            for (int o = 0; o < ND; ++o) {
                const int k = ii[q] + d.off[o];
                const bool in = k >= 0 && k < n;
                const double a = ad[static_cast<int64_t>(o) * n + ii[q]];
                av[q][o] = in ? a : 0.0;
                load_prow<T>(pv, pcol, in ? k : ii[q], v[q][o], cl[q][o]);
            }
#pragma unroll
        for (int q = 0; q < UA; ++q)
#pragma unroll
            for (int o = 0; o < ND; ++o) {
                // (branches here: a third of the rows of P on box supports
                // are padded, so skipping pads and zero coefficients saves
                // more than the branch-free form of rap_add; measured 711
                // against 806 us at 128^3)
                if (av[q][o] == 0.0 || pij[q] == 0.0) continue;
                const double pa = pij[q] * av[q][o];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (cl[q][o][u] == 0xFFFFu) continue;
                    const int sl = map[cl[q][o][u]];
                    const double prod = pa * static_cast<double>(v[q][o][u]);
                    if (sl >= 0)
                        atomicAdd(&acc[sl * NT + tid], prod);
                    else if (prod != 0.0)
                        miss = true;
                }
            }
    }
    if (miss) flag[1] = 1;
    __syncthreads();
    int bl = 0, bu = 0;
    for (int s = tid; s < total; s += NT) {
        double sum = 0.0;
        for (int l = 0; l < NT; ++l) sum += acc[s * NT + l];
        const int col = inv[s];
        // dense row-major, or (CSR) the CSR whose row j lists the columns of
        // cols[j] in order
        if constexpr (CSR)
            ac[csr_rp[j] + s] = sum;
        else
            ac[static_cast<int64_t>(j) * nc + col] = sum;
        if (sum != 0.0) {
            bl = max(bl, j - col);
            bu = max(bu, col - j);
        }
    }
    if (bl > 0) atomicMax(band, bl);
    if (bu > 0) atomicMax(band + 1, bu);
}

// ---------------------------------------------------------------------------
// R A P for a node-block stencil A (NodeStencil: BS components per node,
// coefficient of row r at node offset o and column component l in
// v[(o BS + l) n + r], zero where the row has no such entry) and P in its
// row-major ELL form (8 slots, 16-bit columns).  Fine row i of R's row j
// reaches, through A, the P rows BS (node(i) + off[o]) + l; their columns
// are A_c's columns of row j.  Same structure as the DIA form above: the
// column lists once per pattern, then a numeric pass with per-thread LDS
// partial sums added in thread order (bitwise reproducible).
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(128) void k_rap_nbs_cols(int n, int nc, const int *__restrict__ rrp,
                                                      const int *__restrict__ rci, NodeStencil ns,
                                                      const double *__restrict__ av,
                                                      const uint16_t *__restrict__ pcol,
                                                      int *__restrict__ cols,
                                                      int *__restrict__ ncol)
{
    extern __shared__ double smem[];
    int *inv = reinterpret_cast<int *>(smem);                            // kMaxCoarseNeighbours
    short *map = reinterpret_cast<short *>(inv + kMaxCoarseNeighbours);  // nc
    typedef uint16_t cvec __attribute__((ext_vector_type(8)));
    const int j = blockIdx.x;
    for (int t = threadIdx.x; t < nc; t += 128) map[t] = 0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    for (int t = t0 + threadIdx.x; t < t1; t += 128) {
        const int i = rci[t];
        const int node = i / BS;
        for (int o = 0; o < ns.n; ++o) {
            const int nb = node + ns.off[o];
            const bool in = nb >= 0 && nb < ns.nn;
            double a[BS];
            cvec cc[BS];
#pragma unroll
            for (int l = 0; l < BS; ++l) {
                a[l] = in ? av[static_cast<int64_t>(o * BS + l) * n + i] : 0.0;
                cc[l] = *reinterpret_cast<const cvec *>(
                    pcol + static_cast<int64_t>(in ? nb * BS + l : i) * 8);
            }
#pragma unroll
            for (int l = 0; l < BS; ++l) {
                if (a[l] == 0.0) continue;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (cc[l][u] != 0xFFFFu) map[cc[l][u]] = 1;
            }
        }
    }
    __syncthreads();
    const int total = number_columns<128>(nc, kMaxCoarseNeighbours, map, inv);
    __syncthreads();
    if (total <= kMaxCoarseNeighbours)
        for (int q = threadIdx.x; q < total; q += 128)
            cols[static_cast<int64_t>(j) * kMaxCoarseNeighbours + q] = inv[q];
    if (threadIdx.x == 0) ncol[j] = total;
}

// The numeric product (one wavefront per coarse row): a thread takes R
// entries t, t + 64, ...; for each node offset it loads the BS coefficients
// and P rows, the next offset's loads issued before the current one's sums.
template <typename T, int BS>
__global__ __launch_bounds__(64) void k_rap_nbs(int n, int nc, int maxnb,
                                                const int *__restrict__ rrp,
                                                const int *__restrict__ rci,
                                                const T *__restrict__ rv, NodeStencil ns,
                                                const double *__restrict__ av,
                                                const uint16_t *__restrict__ pcol,
                                                const T *__restrict__ pv, double *__restrict__ ac,
                                                int *__restrict__ flag, int *__restrict__ band,
                                                const int *__restrict__ cols,
                                                const int *__restrict__ ncol)
{
    constexpr int NT = 64;
    extern __shared__ double smem[];
    double *acc = smem;                                          // (maxnb + 1) * NT
    int *inv = reinterpret_cast<int *>(acc + (maxnb + 1) * NT);  // maxnb
    short *map = reinterpret_cast<short *>(inv + maxnb);         // nc
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int total = ncol[j];
    if (total > maxnb) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    for (int t = tid; t < nc; t += NT) map[t] = -1;
    __syncthreads();
    for (int q = tid; q < total; q += NT) {
        const int c = cols[static_cast<int64_t>(j) * kMaxCoarseNeighbours + q];
        inv[q] = c;
        map[c] = static_cast<short>(q);
    }
    for (int q = 0; q < total; ++q) acc[q * NT + tid] = 0.0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    bool miss = false;
    // UE entries of a thread per step (t, t + NT, ...), each with the BS
    // coefficients and P rows of one node offset; the next offset's loads
    // are issued before the current one's sums
    constexpr int UE = 2;
    double a[2][UE][BS];
    T v[2][UE][BS][8];
    uint16_t cl[2][UE][BS][8];
    int ie[UE], ne[UE];
    double pe[UE];
    auto load = [&](int b, int o) {
#pragma unroll
        for (int e = 0; e < UE; ++e) {
            const int nb = ne[e] + ns.off[o];
            const bool in = nb >= 0 && nb < ns.nn && pe[e] != 0.0;
#pragma unroll
            for (int l = 0; l < BS; ++l) {
                a[b][e][l] = in ? av[static_cast<int64_t>(o * BS + l) * n + ie[e]] : 0.0;
                load_prow<T>(pv, pcol, in ? nb * BS + l : ie[e], v[b][e][l], cl[b][e][l]);
            }
        }
    };
    auto add = [&](int b) {
#pragma unroll
        for (int e = 0; e < UE; ++e)
#pragma unroll
            for (int l = 0; l < BS; ++l) {
                const double pa = pe[e] * a[b][e][l];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    rap_add(acc, map, maxnb, tid, NT, cl[b][e][l][u],
                            pa * static_cast<double>(v[b][e][l][u]), miss);
            }
    };
    for (int t = t0 + tid; t < t1; t += UE * NT) {
        // entries past the row, and R's padding (value 0), add nothing
#pragma unroll
        for (int e = 0; e < UE; ++e) {
            const bool ok = t + e * NT < t1;
            ie[e] = rci[ok ? t + e * NT : t];
            pe[e] = ok ? static_cast<double>(rv[t + e * NT]) : 0.0;
            ne[e] = ie[e] / BS;
        }
        load(0, 0);
        for (int o = 0; o < ns.n; o += 2) {
            if (o + 1 < ns.n) load(1, o + 1);
            add(0);
            if (o + 1 >= ns.n) break;
            if (o + 2 < ns.n) load(0, o + 2);
            add(1);
        }
    }
    if (miss) flag[1] = 1;
    __syncthreads();
    int bl = 0, bu = 0;
    for (int q = tid; q < total; q += NT) {
        double sum = 0.0;
        for (int l = 0; l < NT; ++l) sum += acc[q * NT + l];
        const int col = inv[q];
        ac[static_cast<int64_t>(j) * nc + col] = sum;
        if (sum != 0.0) {
            bl = max(bl, j - col);
            bu = max(bu, col - j);
        }
    }
    if (bl > 0) atomicMax(band, bl);
    if (bu > 0) atomicMax(band + 1, bu);
}

// ---------------------------------------------------------------------------
// Exact coarse inverse by blocked Gauss-Jordan elimination with partial
// pivoting, in place on a row-major n x n matrix X.
//
// Unblocked step k: pick the first row p >= k with the largest |x_pk|, swap
// rows k and p, scale row k by 1/x_kk (storing 1/x_kk at (k,k)), and for every
// other row r subtract x_rk times row k (storing -x_rk/x_kk at (r,k)).  After
// all n steps X holds A^{-1} with its columns permuted by the swaps, which are
// undone at the end.
//
// Blocking: columns are processed in panels of 64.  Within a panel, leaves of
// 8 columns are factored by one work-group with the leaf held in registers
// (every row of the matrix, 4 rows per thread); the leaf's transformation is
// then applied to the rest of the panel.  Once a panel is done its swaps are
// applied to the other columns, and its transformation, which is
// x <- x + (V - I_K) x_K with V the panel's final columns, is applied as a
// rank-64 update of the whole matrix.
// ---------------------------------------------------------------------------
constexpr int kLeaf = 8;
constexpr int kPanel = 64;
constexpr int kLeafThreads = 1024;

// Wavefront argmax of (v, r) pairs: the larger v wins, the lower r on a tie
// (a total order, so every lane ends with the same pair whatever the order
// of combination).  Quads by DPP quad permutes, rows of 16 by DPP rotates,
// then rows against rows by the 16- and 32-lane swaps: no LDS round trips.
__device__ __forceinline__ void argmax_take(double &v, int &r, double ov, int orow)
{
    if (ov > v || (ov == v && orow < r)) {
        v = ov;
        r = orow;
    }
}
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double &v, int &r)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u)), CTRL, 0xF, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        0, static_cast<int>(static_cast<uint32_t>(u >> 32)), CTRL, 0xF, 0xF, false));
    const int orow = __builtin_amdgcn_update_dpp(0, r, CTRL, 0xF, 0xF, false);
    argmax_take(v, r, __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo), orow);
}
template <bool HALVES>
__device__ __forceinline__ void argmax_swap(double &v, int &r)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(u), hi = static_cast<uint32_t>(u >> 32);
    const auto sl = HALVES ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                           : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto sh = HALVES ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                           : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const auto sr = HALVES ? __builtin_amdgcn_permlane32_swap(static_cast<uint32_t>(r),
                                                              static_cast<uint32_t>(r), false, false)
                           : __builtin_amdgcn_permlane16_swap(static_cast<uint32_t>(r),
                                                              static_cast<uint32_t>(r), false, false);
    // the two results are this lane's row (or half) and its partner's
    double a = __builtin_bit_cast(double, (static_cast<uint64_t>(sh[0]) << 32) | sl[0]);
    int ra = static_cast<int>(sr[0]);
    argmax_take(a, ra, __builtin_bit_cast(double, (static_cast<uint64_t>(sh[1]) << 32) | sl[1]),
                static_cast<int>(sr[1]));
    v = a;
    r = ra;
}
__device__ __forceinline__ void wave_argmax(double &v, int &r)
{
    argmax_dpp<0xB1>(v, r);   // quad_perm [1, 0, 3, 2]
    argmax_dpp<0x4E>(v, r);   // quad_perm [2, 3, 0, 1]
    argmax_dpp<0x124>(v, r);  // row_ror 4
    argmax_dpp<0x128>(v, r);  // row_ror 8
    argmax_swap<false>(v, r);
    argmax_swap<true>(v, r);
}

template <int R, int NT>
__global__ __launch_bounds__(NT) void k_gj_leaf(double *__restrict__ X, int n, int k0,
                                                          int nb, int kl, int lw,
                                                          int *__restrict__ piv,
                                                          double *__restrict__ bbuf,
                                                          int *__restrict__ flag)
{
    __shared__ double red_v[NT / 64];
    __shared__ int red_r[NT / 64];
    __shared__ double rowk[kLeaf], rowp[kLeaf];
    __shared__ int sh_piv[kLeaf];
    __shared__ double sw[2 * kLeaf][kPanel];  // the swap rows of each panel column
    const int tid = threadIdx.x;
    double v[R][kLeaf];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * NT;
#pragma unroll
        for (int c = 0; c < kLeaf; ++c)
            v[q][c] = (r < n && c < lw) ? X[static_cast<int64_t>(r) * n + kl + c] : 0.0;
    }
    // the steps unrolled, so that a step's column of the leaf is a register
    // known at compile time (lw < kLeaf only for the last leaf)
#pragma unroll
    for (int c = 0; c < kLeaf; ++c) {
        if (c >= lw) break;
        const int k = kl + c;
        // argmax |x_rk| over r >= k; ties go to the lowest row
        double best = -1.0;
        int brow = n;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * NT;
            double val = 0.0;
#pragma unroll
            for (int cc = 0; cc < kLeaf; ++cc)
                if (cc == c) val = fabs(v[q][cc]);
            if (r < n && r >= k && (val > best || (val == best && r < brow))) {
                best = val;
                brow = r;
            }
        }
        wave_argmax(best, brow);
        if ((tid & 63) == 0) {
            red_v[tid >> 6] = best;
            red_r[tid >> 6] = brow;
        }
        __syncthreads();
        // every thread combines the wavefronts' candidates in the same order
        // (no second barrier for a broadcast); red_v is written again only
        // after the next barrier, which every thread reaches after this read
        int p;
        {
            double b = red_v[0];
            int br = red_r[0];
            for (int w = 1; w < NT / 64; ++w)
                if (red_v[w] > b || (red_v[w] == b && red_r[w] < br)) {
                    b = red_v[w];
                    br = red_r[w];
                }
            if (br >= n) br = k;
            p = br;
            if (tid == 0) {
                if (!(b > 0.0)) flag[0] = 1;  // singular (or NaN) pivot column
                sh_piv[c] = br;
                piv[k] = br;
            }
        }
        // swap rows k and p of the leaf
        const int ok = k % NT, qk = k / NT;
        const int op = p % NT, qp = p / NT;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (tid == ok && q == qk)
#pragma unroll
                for (int cc = 0; cc < kLeaf; ++cc) rowk[cc] = v[q][cc];
            if (tid == op && q == qp)
#pragma unroll
                for (int cc = 0; cc < kLeaf; ++cc) rowp[cc] = v[q][cc];
        }
        __syncthreads();
        // the new row k is the old row p; pivot value d
        double prow[kLeaf];
#pragma unroll
        for (int cc = 0; cc < kLeaf; ++cc) prow[cc] = rowp[cc];
        double d = 0.0;
#pragma unroll
        for (int cc = 0; cc < kLeaf; ++cc)
            if (cc == c) d = prow[cc];
        const double dinv = 1.0 / d;
#pragma unroll
        for (int cc = 0; cc < kLeaf; ++cc) prow[cc] = (cc == c) ? dinv : prow[cc] * dinv;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * NT;
            if (r >= n) continue;
            if (r == k) {
#pragma unroll
                for (int cc = 0; cc < kLeaf; ++cc) v[q][cc] = prow[cc];
                continue;
            }
            if (r == p) {  // row p now holds the old row k
#pragma unroll
                for (int cc = 0; cc < kLeaf; ++cc) v[q][cc] = rowk[cc];
            }
            double f = 0.0;
#pragma unroll
            for (int cc = 0; cc < kLeaf; ++cc)
                if (cc == c) f = v[q][cc];
#pragma unroll
            for (int cc = 0; cc < kLeaf; ++cc)
                v[q][cc] = (cc == c) ? -f * prow[cc] : v[q][cc] - f * prow[cc];
        }
        // rowk / rowp are written again only after the next step's first
        // barrier, which every thread reaches after these reads
    }
    __syncthreads();  // sh_piv complete
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * NT;
        if (r < n)
#pragma unroll
            for (int c = 0; c < kLeaf; ++c)
                if (c < lw) X[static_cast<int64_t>(r) * n + kl + c] = v[q][c];
    }
    // the leaf's swaps on the other columns of the panel, then take the leaf
    // rows of those columns out (B) and zero them.  A column's swaps touch
    // the leaf rows kl + c and their pivot rows: slot c holds row kl + c and
    // slot kLeaf + c the pivot row of step c when that lies below the leaf
    // (a pivot row inside the leaf is that row's own slot).  All of them are
    // loaded at once, swapped in LDS in step order, and the rows below the
    // leaf are stored back; the same swaps in the same order as one at a
    // time in memory.
    if (tid < nb) {
        const int col = k0 + tid;
        if (col < kl || col >= kl + lw) {
            auto slot = [&](int c) { return sh_piv[c] < kl + lw ? sh_piv[c] - kl : kLeaf + c; };
            for (int c = 0; c < lw; ++c) {
                sw[c][tid] = X[static_cast<int64_t>(kl + c) * n + col];
                const int p = sh_piv[c];
                if (p >= kl + lw) sw[kLeaf + c][tid] = X[static_cast<int64_t>(p) * n + col];
            }
            // a pivot row below the leaf chosen at several steps is one row:
            // its slot at step c starts from its slot at the latest earlier
            // step that chose it
            for (int c = 0; c < lw; ++c) {
                const int p = sh_piv[c];
                if (p >= kl + lw)
                    for (int e = c - 1; e >= 0; --e)
                        if (sh_piv[e] == p) {
                            sw[kLeaf + c][tid] = sw[kLeaf + e][tid];
                            break;
                        }
                const int sp = slot(c);
                if (sp != c) {
                    const double t = sw[c][tid];
                    sw[c][tid] = sw[sp][tid];
                    sw[sp][tid] = t;
                }
            }
            for (int c = 0; c < lw; ++c) {
                const int p = sh_piv[c];
                bool last = p >= kl + lw;  // the last step with this pivot row stores it
                for (int e = c + 1; e < lw && last; ++e) last = sh_piv[e] != p;
                if (last) X[static_cast<int64_t>(p) * n + col] = sw[kLeaf + c][tid];
            }
            for (int c = 0; c < lw; ++c) {
                bbuf[c * kPanel + tid] = sw[c][tid];
                X[static_cast<int64_t>(kl + c) * n + col] = 0.0;
            }
        }
    }
}

// X[r, col] += sum_t V[r, t] B[t, col] over the panel columns outside the leaf
__global__ __launch_bounds__(kBlock) void k_gj_leaf_update(double *__restrict__ X, int n, int k0,
                                                           int nb, int kl, int lw,
                                                           const double *__restrict__ bbuf)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int r = static_cast<int>(t / kPanel), cc = static_cast<int>(t % kPanel);
    if (r >= n || cc >= nb) return;
    const int col = k0 + cc;
    if (col >= kl && col < kl + lw) return;
    const double *vr = X + static_cast<int64_t>(r) * n + kl;
    double s = X[static_cast<int64_t>(r) * n + col];
    for (int c = 0; c < lw; ++c) s += vr[c] * bbuf[c * kPanel + cc];
    X[static_cast<int64_t>(r) * n + col] = s;
}

// Apply the panel's swaps to every column outside the panel, then move the
// panel rows of those columns to B (nb x n, row-major) and zero them.
__global__ __launch_bounds__(kBlock) void k_gj_swap_extract(double *__restrict__ X, int n, int k0,
                                                            int nb, const int *__restrict__ piv,
                                                            double *__restrict__ B)
{
    const int col = blockIdx.x * kBlock + threadIdx.x;
    if (col >= n || (col >= k0 && col < k0 + nb)) return;
    for (int c = 0; c < nb; ++c) {
        const int k = k0 + c, p = piv[k];
        if (p != k) {
            const double t = X[static_cast<int64_t>(k) * n + col];
            X[static_cast<int64_t>(k) * n + col] = X[static_cast<int64_t>(p) * n + col];
            X[static_cast<int64_t>(p) * n + col] = t;
        }
    }
    for (int c = 0; c < nb; ++c) {
        B[static_cast<int64_t>(c) * n + col] = X[static_cast<int64_t>(k0 + c) * n + col];
        X[static_cast<int64_t>(k0 + c) * n + col] = 0.0;
    }
}

// Rank-nb update X[r, c] += sum_t X[r, k0+t] B[t, c] for every row r and every
// column c outside the panel.  64 x 64 output tiles, 4 x 4 per thread.
constexpr int kT = 64;
__global__ __launch_bounds__(256) void k_gj_gemm(double *__restrict__ X, int n, int k0, int nb,
                                                 const double *__restrict__ B)
{
    __shared__ double Vs[kT][kT + 1];
    __shared__ double Bs[kT][kT + 1];
    const int tile_r = blockIdx.y * kT;
    int tile_c = blockIdx.x * kT;
    // skip the panel's own column tile(s): tiles are enumerated over the
    // columns outside [k0, k0 + nb) packed left to right
    if (tile_c >= k0) tile_c += nb;
    if (tile_c >= n) return;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    for (int t = threadIdx.x; t < kT * kT; t += 256) {
        const int rr = t / kT, kk = t % kT;
        const int r = tile_r + rr;
        Vs[rr][kk] = (r < n && kk < nb) ? X[static_cast<int64_t>(r) * n + k0 + kk] : 0.0;
        const int cc = t % kT, k2 = t / kT;
        const int c = tile_c + cc;
        Bs[k2][cc] = (c < n && k2 < nb && !(c >= k0 && c < k0 + nb))
                         ? B[static_cast<int64_t>(k2) * n + c]
                         : 0.0;
    }
    __syncthreads();
    double acc[4][4] = {};
    for (int kk = 0; kk < nb; ++kk) {
        double va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            va[u] = Vs[ty * 4 + u][kk];
            vb[u] = Bs[kk][tx * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] += va[u] * vb[w];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = tile_r + ty * 4 + u;
        if (r >= n) continue;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int c = tile_c + tx * 4 + w;
            if (c < n && !(c >= k0 && c < k0 + nb)) X[static_cast<int64_t>(r) * n + c] += acc[u][w];
        }
    }
}

// Undo the column permutation: the swaps (k, piv[k]) applied to the columns
// in reverse order.  One thread composes the permutation.
__global__ void k_gj_colsrc(int n, const int *__restrict__ piv, int *__restrict__ colsrc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int j = 0; j < n; ++j) colsrc[j] = j;
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        const int t = colsrc[k];
        colsrc[k] = colsrc[p];
        colsrc[p] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_gj_permute(int n, const double *__restrict__ X,
                                                       const int *__restrict__ colsrc,
                                                       double *__restrict__ Y)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * n) return;
    const int r = static_cast<int>(t / n), j = static_cast<int>(t % n);
    Y[t] = X[static_cast<int64_t>(r) * n + colsrc[j]];
}

// ---------------------------------------------------------------------------
// Inverse of a symmetric positive definite A_c (the Galerkin operator of a
// symmetric positive definite A) through its Cholesky factor, A_c = L L^T:
//   1. band Cholesky by 64-wide panels K (k0 = 64 K): the diagonal block's
//      inverse factor Linv_K = L_KK^{-1}, then for the row tiles R1 >= R2
//      inside the band below K
//        L_R = X[R, K] Linv_K^T,   X[R1, R2] -= L_R1 L_R2^T,
//      with L_R^T kept in the (otherwise unused) upper triangle at X[K, R];
//      A_c's lower bandwidth bl bounds the band, which the factor keeps;
//   2. W = L^{-1} (lower triangular) by strips of 16 columns, each strip a
//      forward substitution down the row tiles I:
//        W[I, S] = Linv_I (E[I, S] - sum over band tiles K < I of L[I, K] W[K, S]);
//   3. A_c^{-1} = W^T W, lower tiles formed on the FP64 matrix cores and
//      mirrored, so the inverse is exactly symmetric.
// A non-positive (or non-finite) pivot sets the flag: A_c is not positive
// definite and the caller falls back to Gauss-Jordan with pivoting.
// ---------------------------------------------------------------------------
constexpr int kBP = 64;  // panel width

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// LDS row stride (doubles) of the MFMA operand tiles: a 16 x 16 x 4 operand
// read touches 16 rows x 4 k, which with a stride of 68 fall on 32 distinct
// bank pairs (two lanes each, the minimum for 64 double loads)
constexpr int kLds = kBP + 4;

// acc (a wavefront's 32 x 32 quadrant at (wr, wc)) += A B for 64 x 64
// operands in LDS on the FP64 matrix cores; A is stored by rows, A[row][k],
// and B by columns, Bt[col][k].  Operand lane l of the 16 x 16 x 4
// instruction holds A[l % 16][l / 16] and B[l / 16][l % 16]; result register
// q of lane l is D[4q + l / 16][l % 16].
__device__ inline void mfma_tile64(const double (*A)[kLds], const double (*Bt)[kLds],
                                   mfma_f64x4 (&acc)[2][2], int wr, int wc, int li, int lk)
{
#pragma unroll 4
    for (int kk = 0; kk < kBP; kk += 4) {
        const double a0 = A[wr + li][kk + lk], a1 = A[wr + 16 + li][kk + lk];
        const double b0 = Bt[wc + li][kk + lk], b1 = Bt[wc + 16 + li][kk + lk];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

__device__ inline void zero_acc(mfma_f64x4 (&acc)[2][2])
{
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
}

// acc (quadrant layout of mfma_tile64) into T[row][col] (or T[col][row])
__device__ inline void acc_to_lds(const mfma_f64x4 (&acc)[2][2], double (*T)[kLds], bool trans,
                                  int wr, int wc, int li, int lk)
{
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = wr + 16 * p + 4 * q + lk, c = wc + 16 * v + li;
                if (trans)
                    T[c][r] = acc[p][v][q];
                else
                    T[r][c] = acc[p][v][q];
            }
}

// lower-triangle pair (a, b), a >= b, of linear index t = a (a + 1) / 2 + b
__device__ inline void tri_pair(int t, int &a, int &b)
{
    int x = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (x * (x + 1) / 2 > t) --x;
    while ((x + 1) * (x + 2) / 2 <= t) ++x;
    a = x;
    b = t - x * (x + 1) / 2;
}

// Compile-time loop: f(std::integral_constant<int, K>) for K = B .. E - 1.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Within each row of 16 lanes, lane K's value to every lane of the row
// (DPP row_newbcast), for a double.
template <int K>
__device__ __forceinline__ double lane_to_row_d(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        0, static_cast<int>(static_cast<uint32_t>(u)), 0x150 + K, 0xF, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        0, static_cast<int>(static_cast<uint32_t>(u >> 32)), 0x150 + K, 0xF, 0xF, false));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Row G (lanes 16 G .. 16 G + 15) to every row, lane for lane: the 16-lane
// swap pairs rows (0, 1) and (2, 3), the 32-lane swap the two halves.
template <int G>
__device__ __forceinline__ uint32_t row_to_all(uint32_t v)
{
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const uint32_t y = (G & 1) ? a[1] : a[0];  // rows G & 1 and (G & 1) + 2, each twice
    const auto b = __builtin_amdgcn_permlane32_swap(y, y, false, false);
    return (G & 2) ? b[1] : b[0];
}
template <int G>
__device__ __forceinline__ double row_to_all_d(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = row_to_all<G>(static_cast<uint32_t>(u));
    const uint32_t hi = row_to_all<G>(static_cast<uint32_t>(u >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ inline double readlane_d(double v, int lane)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(u), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(u >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// ---- inverse Cholesky factor of a 64 x 64 diagonal block -----------------
// Linv = L^{-1} for a symmetric positive definite D = L L^T held in LDS,
// blocked by 16 x 16 blocks (i, j = 0 .. 3), right-looking:
//   for k = 0 .. 3:  Li_kk = L_kk^{-1} of the current D_kk (one wavefront);
//                    L_ik = D_ik Li_kk^T (i > k);
//                    D_ij -= L_ik L_jk^T (k < j <= i),
// then the blocks below the diagonal of L^{-1}, by distance from it,
//   Li_ij = -Li_ii (sum over j <= m < i of L_im Li_mj).
// The 16 x 16 products run on the FP64 matrix cores; the diagonal blocks are
// factored by Gaussian elimination on [D_kk | I] (below).

// Reciprocal by Newton-Raphson refinement of the hardware estimate: two
// steps r <- r + r (1 - p r) from v_rcp_f64 (about 2^-23 relative error)
// give the reciprocal to within about an ulp.
__device__ __forceinline__ double recip_nr(double p)
{
    double r = __builtin_amdgcn_rcp(p);
    double e = fma(-p, r, 1.0);
    r = fma(r, e, r);
    e = fma(-p, r, 1.0);
    return fma(r, e, r);
}

// One wavefront: Li block (kb, kb) = L_kk^{-1} of the 16 x 16 block (kb, kb)
// of D (lower triangle read).  Gaussian elimination without pivoting on
// [D_kk | I]: with D_kk = L_u diag(u) L_u^T (L_u unit lower triangular) the
// right half ends as L_u^{-1}, and L^{-1} = diag(u)^{-1/2} L_u^{-1}.  Column c
// of the left half is dead after step c and column c of the right half is
// born at step c, so both share one slot.  Lane r + 16 g holds row r, slots
// 4 g .. 4 g + 3.  Returns true on a non-positive or non-finite pivot.
__device__ __forceinline__ bool chol_inv16(const double (*D)[kLds], double (*Li)[kLds], int kb, int lane)
{
    const int r = lane & 15, g = lane >> 4, o = 16 * kb;
    double m[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = 4 * g + s;
        m[s] = c <= r ? D[o + r][o + c] : D[o + c][o + r];
    }
    double ur = 1.0;  // this lane's row's pivot
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value, gk = k >> 2, sk = k & 3;
        const double p = readlane_d(m[sk], k + 16 * gk);
        if (r == k) ur = p;
        const double rp = recip_nr(p);
        // x_rk of this lane's row (the same lane of row gk) and the pivot
        // row's entries of its slots (lane k of its own row), moved across
        // lanes by the VALU rather than through the LDS crossbar
        const double xrk = row_to_all_d<gk>(m[sk]);
        double pk[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) pk[s] = lane_to_row_d<k>(m[s]);
        const double mult = r > k ? xrk * rp : 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (s == sk && g == gk)
                m[s] = r > k ? -mult : (r == k ? 1.0 : m[s]);
            else
                m[s] = fma(-mult, pk[s], m[s]);
        }
    });
    const double rs = 1.0 / sqrt(ur);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = 4 * g + s;
        Li[o + r][o + c] = c <= r ? m[s] * rs : 0.0;
    }
    // every pivot is some lane's ur, so the check per lane covers them all
    return !(ur > 0.0) || !isfinite(ur);
}

// acc += (-)A B for 16 x 16 blocks in LDS: A at (ar, ac) by rows; B at
// (br, bc) by rows, or (bt) B^T at (br, bc) by rows.  Lane l supplies
// A[l % 16][kk + l / 16] and B[kk + l / 16][l % 16] at k-steps kk = 0, 4,
// 8, 12; result register q of lane l is row 4 q + l / 16, column l % 16.
__device__ inline mfma_f64x4 mfma16(const double (*A)[kLds], int ar, int ac, bool neg,
                                    const double (*B)[kLds], int br, int bc, bool bt,
                                    mfma_f64x4 acc, int li, int lk)
{
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
        const double av = A[ar + li][ac + kk + lk];
        const double b = bt ? B[br + li][bc + kk + lk] : B[br + kk + lk][bc + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(neg ? -av : av, b, acc, 0, 0, 0);
    }
    return acc;
}

// acc += (-)A B with B a 16 x 16 result held in registers (result register q
// of lane l is B's row 4 q + l / 16, column l % 16: B's k-step q operand)
__device__ inline mfma_f64x4 mfma16_breg(const double (*A)[kLds], int ar, int ac, bool neg,
                                         const mfma_f64x4 &B, mfma_f64x4 acc, int li, int lk)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double av = A[ar + li][ac + 4 * q + lk];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(neg ? -av : av, B[q], acc, 0, 0, 0);
    }
    return acc;
}

__device__ inline mfma_f64x4 load_blk(const double (*T)[kLds], int r0, int c0, int li, int lk)
{
    mfma_f64x4 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = T[r0 + 4 * q + lk][c0 + li];
    return v;
}

__device__ inline void store_blk(double (*T)[kLds], int r0, int c0, const mfma_f64x4 &v, int li,
                                 int lk)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) T[r0 + 4 * q + lk][c0 + li] = v[q];
}

// orders one wavefront's LDS writes before its own later LDS reads
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// D_ij -= L_ik L_jk^T (L's blocks stored in D's place)
__device__ inline void schur_blk(double (*D)[kLds], int i, int j, int k, int li, int lk)
{
    mfma_f64x4 acc = load_blk(D, 16 * i, 16 * j, li, lk);
    acc = mfma16(D, 16 * i, 16 * k, true, D, 16 * j, 16 * k, true, acc, li, lk);
    store_blk(D, 16 * i, 16 * j, acc, li, lk);
}

// Called by all 256 threads; D (64 x 64, symmetric positive definite, lower
// triangle read) is overwritten by L's blocks and Schur complements, Li
// receives L^{-1} on and below the diagonal (the blocks above it are not
// written).  Returns true in every thread when a pivot was not positive.
__device__ __forceinline__ bool chol_inv64(double (*D)[kLds], double (*Li)[kLds])
{
    __shared__ int bad_any;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    bool bad = false;
    if (threadIdx.x == 0) bad_any = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // wavefront 0 factors D_kk (already final: it updated it itself);
        // the others finish the previous step's Schur updates meanwhile
        if (w == 0) {
            bad |= chol_inv16(D, Li, k, lane);
        } else if (k > 0) {
            int t = 0;
#pragma unroll
            for (int i = k; i < 4; ++i)
#pragma unroll
                for (int j = k; j <= i; ++j) {
                    if (i == k && j == k) continue;
                    if (t++ % 3 == w - 1) schur_blk(D, i, j, k - 1, li, lk);
                }
        }
        __syncthreads();
        if (k == 3) break;
        // L_ik = D_ik Li_kk^T by wavefront i - k - 1; wavefront 0 goes on to
        // D_{k+1,k+1} -= L_{k+1,k} L_{k+1,k}^T, the next step's diagonal block
        const int i = k + 1 + w;
        if (i < 4) {
            mfma_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            acc = mfma16(D, 16 * i, 16 * k, false, Li, 16 * k, 16 * k, true, acc, li, lk);
            store_blk(D, 16 * i, 16 * k, acc, li, lk);
            if (w == 0) {
                wave_lds_sync();
                schur_blk(D, k + 1, k + 1, k, li, lk);
            }
        }
        __syncthreads();
    }
    // off-diagonal blocks of L^{-1}, one block per wavefront, by distance
#pragma unroll
    for (int d = 1; d < 4; ++d) {
        const int j = w, i = w + d;
        if (i < 4) {
            mfma_f64x4 sacc = {0.0, 0.0, 0.0, 0.0};
            for (int mm = j; mm < i; ++mm)
                sacc = mfma16(D, 16 * i, 16 * mm, false, Li, 16 * mm, 16 * j, false, sacc, li, lk);
            mfma_f64x4 res = {0.0, 0.0, 0.0, 0.0};
            res = mfma16_breg(Li, 16 * i, 16 * i, true, sacc, res, li, lk);
            store_blk(Li, 16 * i, 16 * j, res, li, lk);
        }
        __syncthreads();
    }
    if (bad) bad_any = 1;
    __syncthreads();
    return bad_any != 0;
}

// Linv (global, 64 x 64 row-major) from Li: the lower triangle, zeros above
__device__ inline void store_linv(const double (*Li)[kLds], double *__restrict__ Linv)
{
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int r = e / kBP, c = e % kBP;
        Linv[e] = c <= r ? Li[r][c] : 0.0;
    }
}

// Linv for the diagonal block X[K, K] (its lower triangle; rows and columns
// past nb padded with the identity)
__global__ __launch_bounds__(256) void k_chol_inv(const double *__restrict__ X, int n, int k0,
                                                  int nb, double *__restrict__ Linv,
                                                  int *__restrict__ flag)
{
    __shared__ double Dm[kBP][kLds];
    __shared__ double Li[kBP][kLds];
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int r = e / kBP, c = e % kBP;
        double v = r == c ? 1.0 : 0.0;
        if (r < nb && c < nb && c <= r) v = X[static_cast<int64_t>(k0 + r) * n + k0 + c];
        Dm[r][c] = v;
    }
    __syncthreads();
    const bool bad = chol_inv64(Dm, Li);
    store_linv(Li, Linv);
    if (bad && threadIdx.x == 0) flag[0] = 1;
}

// W = L^{-1} (row-major) by strips of 16 columns S = [c0, c0 + 16) and row
// tiles I from the strip's own panel down (a forward substitution).  Row
// tile I of a strip: wavefront w forms rows 16 w .. 16 w + 15 of
//   sum over K in [max(jp, I - tb), I) of L[I, K] W[K, S]
// (L[I, K] read transposed from the upper triangle of X, W[K, S] finished
// earlier; the operands of the next K tile are loaded while the current one
// is multiplied), subtracts it from the identity's block, and multiplies by
// Linv_I.  Entries of W above the diagonal come out as exact zeros (Linv_I is
// lower triangular).  Rs: 64 x 17 doubles of LDS.
__device__ __forceinline__ void w_row_tile(const double *__restrict__ X, int n, int tb,
                                  const double *__restrict__ LinvI, double *__restrict__ W, int c0,
                                  int I, double (*Rs)[17])
{
    const int jp = c0 / kBP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const bool cin = c0 + li < n;
    const int r0 = I * kBP;
    const int ra = r0 + 16 * w + li;  // this lane's A-operand row
    double lv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = LinvI[(16 * w + li) * kBP + 4 * u + lk];
    auto load = [&](int K, double (&av)[16], double (&bv)[16]) {
        const int q0 = K * kBP;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int row = q0 + 4 * u + lk;
            av[u] = (row < n && ra < n) ? X[static_cast<int64_t>(row) * n + ra] : 0.0;
            bv[u] = (row < n && cin) ? W[static_cast<int64_t>(row) * n + c0 + li] : 0.0;
        }
    };
    mfma_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    double a0[16], b0[16], a1[16], b1[16];
    const int kb = max(jp, I - tb);
    if (kb < I) load(kb, a0, b0);
    for (int K = kb; K < I; K += 2) {
        if (K + 1 < I) load(K + 1, a1, b1);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc, 0, 0, 0);
        if (K + 1 >= I) break;
        if (K + 2 < I) load(K + 2, a0, b0);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = 16 * w + 4 * q + lk;
        Rs[row][li] = (r0 + row == c0 + li ? 1.0 : 0.0) - acc[q];
    }
    __syncthreads();
    mfma_f64x4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 16; ++u)
        o = __builtin_amdgcn_mfma_f64_16x16x4f64(lv[u], Rs[4 * u + lk][li], o, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = r0 + 16 * w + 4 * q + lk;
        if (row < n && cin) W[static_cast<int64_t>(row) * n + c0 + li] = o[q];
    }
}

// Row tile I of W for every strip that reaches it (one work-group per strip,
// strips 0 .. gridDim.x - 1), when no panel update carries it
__global__ __launch_bounds__(256) void k_chol_w_row(const double *__restrict__ X, int n, int tb,
                                                    const double *__restrict__ LinvI,
                                                    double *__restrict__ W, int I)
{
    __shared__ double Rs[kBP][17];
    w_row_tile(X, n, tb, LinvI, W, 16 * blockIdx.x, I, Rs);
}

// Panel K of the band Cholesky for the lower tile pairs (R1, R2) of the band
// below it, R1 >= R2 >= rt0 = K + 1 (one work-group per pair):
//   L_R1 = X[R1, K] Linv^T, L_R2 = X[R2, K] Linv^T, X[R1, R2] -= L_R1 L_R2^T;
// the diagonal pairs store L_R^T at X[K, R] (upper triangle, read by the
// forward substitution).  X[R, K] itself is left as it was: other pairs of
// the same launch read it.  All operands and the output tile are fetched
// before the first product.  With Lnext set, the pair (K+1, K+1) (block 0,
// dispatched first) goes on to invert the freshly updated diagonal block of
// the next panel (nbn rows) into Lnext.
__global__ __launch_bounds__(256) void k_chol_update(double *__restrict__ X, int n, int k0, int nb,
                                                     int rt0, const double *__restrict__ Linv,
                                                     double *__restrict__ Lnext, int nbn,
                                                     int *__restrict__ flag, int npairs, int tb,
                                                     double *__restrict__ W)
{
    __shared__ double Ls[kBP][kLds];  // Linv by rows: the B operand of X[R, K] Linv^T
    __shared__ double A1[kBP][kLds];  // X[R1, K], then L_R1 (by rows)
    __shared__ double A2[kBP][kLds];  // X[R2, K], then L_R2 (by rows)
    if (static_cast<int>(blockIdx.x) >= npairs) {
        // the work-groups after the pairs: row tile K of W, one strip each
        // (W's earlier row tiles and L's band tiles left of panel K are
        // final; this launch writes neither)
        w_row_tile(X, n, tb, Linv, W, 16 * (blockIdx.x - npairs), rt0 - 1,
                   reinterpret_cast<double (*)[17]>(&A1[0][0]));
        return;
    }
    int a, b;
    tri_pair(blockIdx.x, a, b);
    const int r1 = (rt0 + a) * kBP, r2 = (rt0 + b) * kBP;
    const bool diag = a == b;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    {
        double gl[16], g1[16], g2[16];
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = t + 256 * it;
            const int r = e / kBP, c = e % kBP;
            gl[it] = Linv[e];
            g1[it] = (r1 + r < n && c < nb) ? X[static_cast<int64_t>(r1 + r) * n + k0 + c] : 0.0;
            g2[it] = (!diag && r2 + r < n && c < nb) ? X[static_cast<int64_t>(r2 + r) * n + k0 + c]
                                                     : 0.0;
        }
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = t + 256 * it;
            const int r = e / kBP, c = e % kBP;
            Ls[r][c] = gl[it];
            A1[r][c] = g1[it];
            if (!diag) A2[r][c] = g2[it];
        }
    }
    // the output tile, in the accumulator layout
    double xo[2][2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r1 + wr + 16 * p + 4 * q + lk, c = r2 + wc + 16 * v + li;
                xo[p][v][q] = (r < n && c < n) ? X[static_cast<int64_t>(r) * n + c] : 0.0;
            }
    __syncthreads();
    mfma_f64x4 acc1[2][2], acc2[2][2];
    zero_acc(acc1);
    mfma_tile64(A1, Ls, acc1, wr, wc, li, lk);
    if (!diag) {
        zero_acc(acc2);
        mfma_tile64(A2, Ls, acc2, wr, wc, li, lk);
    }
    __syncthreads();
    acc_to_lds(acc1, A1, false, wr, wc, li, lk);
    if (!diag) acc_to_lds(acc2, A2, false, wr, wc, li, lk);
    __syncthreads();
    zero_acc(acc1);
    mfma_tile64(A1, diag ? A1 : A2, acc1, wr, wc, li, lk);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                xo[p][v][q] -= acc1[p][v][q];
                const int r = r1 + wr + 16 * p + 4 * q + lk, c = r2 + wc + 16 * v + li;
                if (r < n && c < n) X[static_cast<int64_t>(r) * n + c] = xo[p][v][q];
            }
    if (!diag) return;
    // L_R^T at X[K, R]: row c of the tile holds column c of L_R
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = t + 256 * it;
        const int c = e / kBP, r = e % kBP;
        if (c < nb && r1 + r < n) X[static_cast<int64_t>(k0 + c) * n + r1 + r] = A1[r][c];
    }
    if (Lnext == nullptr || blockIdx.x != 0) return;
    // the next panel's diagonal block, now final: its inverse factor (rows
    // and columns past nbn padded with the identity; Ls is free again)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = wr + 16 * p + 4 * q + lk, c = wc + 16 * v + li;
                A2[r][c] = (r < nbn && c < nbn) ? xo[p][v][q] : (r == c ? 1.0 : 0.0);
            }
    __syncthreads();
    const bool bad = chol_inv64(A2, Ls);
    store_linv(Ls, Lnext);
    if (bad && t == 0) flag[0] = 1;
}

// A_c^{-1} = W^T W for the lower tile pairs (I, J), I >= J (one work-group
// per pair, the longest sums first): tile (I, J) = sum over K >= I of
// W[K, I]^T W[K, J] on the FP64 matrix cores, the next 64-deep chunk fetched
// into registers while the current one is multiplied.  The tile goes whole
// into the packed lower-tile array pk (zeros past n); a diagonal tile's
// upper triangle is its lower one transposed through LDS, so the inverse is
// exactly symmetric.
// LDS row stride of the WtW chunks, stored as loaded (row k of the chunk,
// 64 columns): the 16 x 4 transposed operand reads of a half-wavefront fall
// on distinct bank pairs, and so do the row-wise stores
constexpr int kLdsW = kBP + 16;

__global__ __launch_bounds__(256) void k_chol_wtw(const double *__restrict__ W, int n,
                                                  double *__restrict__ pk)
{
    __shared__ double As[kBP][kLdsW];  // As[k][r] = W[q0 + k][i0 + r]
    __shared__ double Bs[kBP][kLdsW];  // Bs[k][c] = W[q0 + k][j0 + c]
    int I, J;
    tri_pair(blockIdx.x, I, J);
    const int nt = (n + kBP - 1) / kBP;
    const int i0 = I * kBP, j0 = J * kBP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const int lr = threadIdx.x >> 6, lc = threadIdx.x & 63;
    double ra[16], rb[16];
    auto fetch = [&](int K) {
        const int q0 = K * kBP;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int row = q0 + lr + 4 * u;
            ra[u] = (row < n && i0 + lc < n) ? W[static_cast<int64_t>(row) * n + i0 + lc] : 0.0;
            rb[u] = (row < n && j0 + lc < n) ? W[static_cast<int64_t>(row) * n + j0 + lc] : 0.0;
        }
    };
    mfma_f64x4 acc[2][2];
    zero_acc(acc);
    fetch(I);
    for (int K = I; K < nt; ++K) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            As[lr + 4 * u][lc] = ra[u];
            Bs[lr + 4 * u][lc] = rb[u];
        }
        __syncthreads();
        if (K + 1 < nt) fetch(K + 1);
        // C[r][c] += sum_k As[k][r] Bs[k][c]: operand lane l supplies
        // A[l % 16][kk + l / 16] = As[kk + l / 16][row] and likewise for B
#pragma unroll 4
        for (int kk = 0; kk < kBP; kk += 4) {
            const double a0 = As[kk + lk][wr + li], a1 = As[kk + lk][wr + 16 + li];
            const double b0 = Bs[kk + lk][wc + li], b1 = Bs[kk + lk][wc + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    __syncthreads();
    // the tile through LDS (As, reused with its own stride)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                As[wr + 16 * p + 4 * q + lk][wc + 16 * v + li] = acc[p][v][q];
    __syncthreads();
    double *tile = pk + static_cast<int64_t>(blockIdx.x) * kBP * kBP;
#pragma unroll
    for (int it = 0; it < (kBP * kBP) / 256; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int r = e / kBP, c = e % kBP;
        double v = (I != J || r >= c) ? As[r][c] : As[c][r];
        if (i0 + r >= n || j0 + c >= n) v = 0.0;
        tile[e] = v;
    }
}

// y = S x for a symmetric S held as packed lower 64 x 64 tiles.  Tile t =
// (I, J) (one work-group each): thread (g, h) = (t / 16, t % 16) holds rows
// 4g .. 4g + 3 and columns 4h .. 4h + 3 of the tile; the row partials
// S_IJ x_J (16 lanes per row group) and, off the diagonal, the column
// partials S_IJ^T x_I (16 row groups per column group, across the four
// wavefronts through LDS) are reduced in a fixed order and written to
// part[t][0][.] and part[t][1][.].
__global__ __launch_bounds__(256) void k_symv_tiles(const double *__restrict__ pk, int n,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ part)
{
    __shared__ double sh[4][kBP];
    int I, J;
    tri_pair(blockIdx.x, I, J);
    const int t = threadIdx.x, g = t >> 4, h = t & 15;
    const int lane = t & 63, w = t >> 6;
    typedef double d4 __attribute__((ext_vector_type(4)));
    const d4 *tile = reinterpret_cast<const d4 *>(pk + static_cast<int64_t>(blockIdx.x) * kBP * kBP);
    d4 m[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) m[a] = tile[(4 * g + a) * (kBP / 4) + h];
    double xj[4], xi[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int cj = J * kBP + 4 * h + b, ri = I * kBP + 4 * g + b;
        xj[b] = cj < n ? x[cj] : 0.0;
        xi[b] = ri < n ? x[ri] : 0.0;
    }
    double* out = part + static_cast<int64_t>(blockIdx.x) * 2 * kBP;
    // rows: sum over the 16 lanes of a row group
    double rs[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = m[a][0] * xj[0];
        v += m[a][1] * xj[1];
        v += m[a][2] * xj[2];
        v += m[a][3] * xj[3];
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        rs[a] = v;
    }
    if (h == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) out[4 * g + a] = rs[a];
    }
    if (I == J) return;
    // columns: the four row groups of a wavefront by shuffles, then the
    // four wavefronts in order through LDS
    double cs[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double v = m[0][b] * xi[0];
        v += m[1][b] * xi[1];
        v += m[2][b] * xi[2];
        v += m[3][b] * xi[3];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        cs[b] = v;
    }
    if (lane < 16) {
#pragma unroll
        for (int b = 0; b < 4; ++b) sh[w][4 * h + b] = cs[b];
    }
    __syncthreads();
    if (t < kBP) out[kBP + t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
}

// y_I = sum over J <= I of the row partials of tile (I, J) and over J > I
// of the column partials of tile (J, I): four threads per row (one
// wavefront per quarter of J) each add their quarter in order of J, all its
// partials loaded first (nt <= kMaxCoarse / 64 = 64), then the quarters are
// added in order.
__global__ __launch_bounds__(256) void k_symv_final(const double *__restrict__ part, int n,
                                                   double *__restrict__ y)
{
    constexpr int kMaxTiles = kMaxCoarse / kBP;
    constexpr int kQ = kMaxTiles / 4;
    __shared__ double sh[4][kBP];
    const int I = blockIdx.x, nt = gridDim.x;
    const int r = threadIdx.x & 63, qd = threadIdx.x >> 6;
    double v[kQ];
#pragma unroll
    for (int u = 0; u < kQ; ++u) {
        const int J = qd * kQ + u;
        int64_t e = 0;
        if (J <= I)
            e = (static_cast<int64_t>(I) * (I + 1) / 2 + J) * 2 * kBP + r;
        else if (J < nt)
            e = (static_cast<int64_t>(J) * (J + 1) / 2 + I) * 2 * kBP + kBP + r;
        v[u] = J < nt ? part[e] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kQ; ++u) s += v[u];
    sh[qd][r] = s;
    __syncthreads();
    const int row = I * kBP + threadIdx.x;
    if (threadIdx.x < kBP && row < n)
        y[row] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

// y = M x, one wavefront per row; lanes stride over the columns (two per
// 16-byte load when n is even) and the 64 partial sums are added in a fixed
// butterfly order.
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double *__restrict__ M,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int row = (blockIdx.x * kBlock + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *mr = M + static_cast<int64_t>(row) * n;
    double s = 0.0;
    if ((n & 1) == 0) {
        const double2 *m2 = reinterpret_cast<const double2 *>(mr);
        const double2 *x2 = reinterpret_cast<const double2 *>(x);
        const int h = n >> 1;
#pragma unroll 8
        for (int c = lane; c < h; c += 64) {
            const double2 a = m2[c], b = x2[c];
            s += a.x * b.x + a.y * b.y;
        }
    } else {
        for (int c = lane; c < n; c += 64) s += mr[c] * x[c];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}

// y = M^T x in two stages: partials[seg][c] over row segments, then a fixed
// order sum over the segments.
constexpr int kGemvSeg = 64;
__global__ __launch_bounds__(kBlock) void k_gemv_t_partial(int n, const double *__restrict__ M,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ part)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const int seg = blockIdx.y;
    if (c >= n) return;
    const int rows = (n + kGemvSeg - 1) / kGemvSeg;
    const int r0 = seg * rows, r1 = min(n, r0 + rows);
    double s = 0.0;
    for (int r = r0; r < r1; ++r) s += M[static_cast<int64_t>(r) * n + c] * x[r];
    part[static_cast<int64_t>(seg) * n + c] = s;
}

__global__ __launch_bounds__(kBlock) void k_gemv_t_final(int n, const double *__restrict__ part,
                                                         double *__restrict__ y)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    double s = 0.0;
    for (int seg = 0; seg < kGemvSeg; ++seg) s += part[static_cast<int64_t>(seg) * n + c];
    y[c] = s;
}

}  // namespace

void launch_gather_r(hipStream_t s, int64_t m, const int *rsrc, bool fp32, const double *p64,
                     const float *p32, double *r64, float *r32)
{
    if (m <= 0) return;
    if (fp32)
        k_gather<float><<<grid_for(m), kBlock, 0, s>>>(m, rsrc, p32, r32);
    else
        k_gather<double><<<grid_for(m), kBlock, 0, s>>>(m, rsrc, p64, r64);
}

// R's values of the MsFV restriction on P^T's pattern: entry t of coarse
// row j (found by bisection of the row pointers) is 1 when its fine row lies
// in block j, else 0; pads (rsrc < 0) stay 0
template <typename T>
__global__ __launch_bounds__(kBlock) void k_r_indicator(int nc, int64_t m,
                                                        const int *__restrict__ rrp,
                                                        const int *__restrict__ rci,
                                                        const int *__restrict__ rsrc,
                                                        const int *__restrict__ part,
                                                        T *__restrict__ rv)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= m) return;
    int lo = 0, hi = nc - 1;  // the last row j with rrp[j] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rrp[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    rv[t] = (rsrc[t] >= 0 && part[rci[t]] == lo) ? T(1) : T(0);
}

void launch_r_indicator(hipStream_t s, int nc, int64_t m, const int *rrp, const int *rci,
                        const int *rsrc, const int *part, bool fp32, double *r64, float *r32)
{
    if (m <= 0) return;
    if (fp32)
        k_r_indicator<float><<<grid_for(m), kBlock, 0, s>>>(nc, m, rrp, rci, rsrc, part, r32);
    else
        k_r_indicator<double><<<grid_for(m), kBlock, 0, s>>>(nc, m, rrp, rci, rsrc, part, r64);
}

template <typename T, int NT>
void rap_t(hipStream_t s, size_t shmem, int n, int nc, int maxnb, const int *rrp, const int *rci,
           const T *rv, const int *rp, const int *ci, const double *a, const DiaOffsets &d,
           const double *ad, const int *prp, const int *pci, const double *pv, double *ac,
           int *flag, int *band)
{
    if (d.n > 0)
        k_rap<T, NT, true><<<nc, NT, shmem, s>>>(n, nc, maxnb, rrp, rci, rv, rp, ci, a, d, ad, prp,
                                                 pci, pv, ac, flag, band);
    else
        k_rap<T, NT, false><<<nc, NT, shmem, s>>>(n, nc, maxnb, rrp, rci, rv, rp, ci, a, d, ad, prp,
                                                  pci, pv, ac, flag, band);
}

// ---------------------------------------------------------------------------
// R A P for the 7-point stencil on a Cartesian grid whose supports are boxes
// and whose P rows reach the products of per-axis candidates (ProlongAxes):
// A_c[j, :] = sum over cells k of (R A)[j, k] P[k, :], with
// (R A)[j, k] = sum over the stencil neighbours i of k of R[j, i] A[i, k].
// R[j, :] lives on j's support box, so (R A)[j, :] lives on that box widened
// by one cell, D(j).  The candidates of a cell of D(j) lie within one coarse
// node of j on every axis (checked when the coarse space is set), so a row
// of A_c has at most the 27 columns of j's coarse neighbourhood.
//
// One work-group per coarse row, one thread per (x, y) column of D(j): the
// thread walks the column upward, forms (R A)[j, k] from the seven R entries
// and A coefficients around k, loads P's row k once, and adds its slots into
// 2 x 2 x 3 sums: its columns' x and y candidates are fixed (at most two
// each) and a plane's z candidates are the same for every thread.  The sums
// of each of the 27 columns are then added over the wavefront (a fixed
// butterfly) and over the wavefronts in order, so the result is reproducible.
// Each product term is formed once per coarse row, where the per-entry form
// of R A P re-reads a P row for every R entry next to it, and no LDS map or
// atomic is involved.
// ---------------------------------------------------------------------------
constexpr int kRapBoxMaxThreads = 512;

template <typename T, bool SYM>
__global__ __launch_bounds__(kRapBoxMaxThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_rap_box(
    int n, int nc, const int *__restrict__ rrp, RapBoxGeom g, const double *__restrict__ ad,
    const T *__restrict__ rv, const T *__restrict__ pv, double *__restrict__ ac,
    int *__restrict__ band, const int *__restrict__ order)
{
    constexpr int NW = kRapBoxMaxThreads / 64;
    __shared__ double part[27][NW];
    const int j = order ? order[xcd_group(blockIdx.x, gridDim.x)] : static_cast<int>(blockIdx.x);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nx = g.nx, nxy = g.nx * g.ny;
    const int org = g.box[4 * j], bx = g.box[4 * j + 1], bxy = g.box[4 * j + 2];
    const int by = bxy / bx, bz = g.box[4 * j + 3] / bxy;
    const int x0 = org % nx, y0 = (org / nx) % g.ny, z0 = org / nxy;
    // D(j): the support box and the cells next to it, inside the grid
    const int lx = max(x0 - 1, 0), ly = max(y0 - 1, 0), lz = max(z0 - 1, 0);
    const int ex = min(x0 + bx + 1, nx) - lx, ey = min(y0 + by + 1, g.ny) - ly;
    const int hz = min(z0 + bz + 1, g.nz);
    const int jx = j % g.ncx, jy = (j / g.ncx) % g.ncy, jz = j / (g.ncx * g.ncy);
    const T *__restrict__ rj = rv + rrp[j];
    // acc[ix][iy][dz]: column (ax + ix, ay + iy, jz - 1 + dz) of this
    // thread's cells
    double acc[2][2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[a][b][c] = 0.0;
    int tx0 = 0, ty0 = 0;  // first x / y candidate of the column, minus j's, plus 1
    if (tid < ex * ey) {
        const int py = tid / ex, x = lx + (tid - py * ex), y = ly + py;
        const int tx = g.tab[x], ty = g.tab[nx + y];
        const int cx = tx >> 16, cy = ty >> 16;
        tx0 = (tx & 0xFFFF) - jx + 1;
        ty0 = (ty & 0xFFFF) - jy + 1;
        // membership of the column and its x / y neighbours in the support
        const bool mxc = x >= x0 && x < x0 + bx, mxl = x - 1 >= x0 && x - 1 < x0 + bx,
                   mxr = x + 1 >= x0 && x + 1 < x0 + bx;
        const bool myc = y >= y0 && y < y0 + by, myl = y - 1 >= y0 && y - 1 < y0 + by,
                   myr = y + 1 >= y0 && y + 1 < y0 + by;
        // neighbour o of the stencil (-nxy, -nx, -1, 0, 1, nx, nxy): the
        // in-plane R offsets from the column's own box position
        const int qc = (x - x0) + bx * (y - y0);
        const int dq[7] = {-bxy, -bx, -1, 0, 1, bx, bxy};
        const int off[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
        const bool mxy[7] = {mxc && myc, mxc && myl, mxl && myc, mxc && myc,
                             mxr && myc, mxc && myr, mxc && myc};
        for (int z = lz; z < hz; ++z) {
            const int k = x + nx * y + nxy * z;
            const int zq = z - z0;  // the plane's position in the box
            const bool zin = zq >= 0 && zq < bz;
            const bool mz[7] = {zq - 1 >= 0 && zq - 1 < bz, zin, zin, zin, zin, zin,
                                zq + 1 >= 0 && zq + 1 < bz};
            const int q = qc + bxy * zq;
            // R[j, i] and A[i, k] for the neighbours i = k + off inside the
            // support (A[i, k] is row i's coefficient at -off; with SYM only
            // the offsets >= 0 are stored, and A[i, k] = A[k, i] above k)
            double rr[7], aa[7];
            bool m[7];
#pragma unroll
            for (int o = 0; o < 7; ++o) {
                m[o] = mxy[o] && mz[o];
                rr[o] = 0.0;
                aa[o] = 0.0;
                if (m[o]) {
                    rr[o] = static_cast<double>(rj[q + dq[o]]);
                    aa[o] = (SYM && o > 3) ? ad[static_cast<int64_t>(o) * n + k]
                                           : ad[static_cast<int64_t>(6 - o) * n + k + off[o]];
                }
            }
            T pr[8];
            {
                constexpr int L = 16 / sizeof(T);
                typedef T tvec __attribute__((ext_vector_type(L)));
                const tvec *vs = reinterpret_cast<const tvec *>(pv + static_cast<int64_t>(k) * 8);
#pragma unroll
                for (int u = 0; u < 8 / L; ++u) {
                    const tvec v = vs[u];
#pragma unroll
                    for (int l = 0; l < L; ++l) pr[L * u + l] = v[l];
                }
            }
            double ra = 0.0;
#pragma unroll
            for (int o = 0; o < 7; ++o)
                if (m[o]) ra += rr[o] * aa[o];
            // P's slots (ix fastest over cx, then iy over cy, then iz) in the
            // fixed 2 x 2 x 2 order, zero where the column has no such slot
            const bool x2 = cx == 2, y2 = cy == 2;
            double cv[2][2][2];
            const int sz = cx * cy;  // slots per z candidate: 1, 2 or 4
#pragma unroll
            for (int iz = 0; iz < 2; ++iz) {
                // slot iz * sz + ix + cx iy, picked without indexing by a
                // lane value: sz, cx in {1, 2, 4} and {1, 2}
                auto pick = [&](int u1, int u2, int u4) -> double {
                    return static_cast<double>(sz == 4 ? pr[u4] : (sz == 2 ? pr[u2] : pr[u1]));
                };
                cv[0][0][iz] = iz == 0 ? static_cast<double>(pr[0]) : pick(1, 2, 4);
                cv[1][0][iz] = x2 ? (iz == 0 ? static_cast<double>(pr[1]) : pick(2, 3, 5)) : 0.0;
                cv[0][1][iz] = y2 ? (iz == 0 ? static_cast<double>(x2 ? pr[2] : pr[1])
                                             : (x2 ? static_cast<double>(pr[6])
                                                   : static_cast<double>(pr[3])))
                                  : 0.0;
                cv[1][1][iz] = (x2 && y2) ? static_cast<double>(iz == 0 ? pr[3] : pr[7]) : 0.0;
            }
            const int tz = g.tab[nx + g.ny + z];
            const int dz0 = (tz & 0xFFFF) - jz + 1, cz = tz >> 16;
#pragma unroll
            for (int iz = 0; iz < 2; ++iz) {
                if (iz >= cz) break;
                const int dz = dz0 + iz;  // the same for every thread
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (d != dz) continue;
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) acc[a][b][d] += ra * cv[a][b][iz];
                }
            }
        }
    }
    // the 27 columns: each thread's share, then the wavefront, then the
    // wavefronts in order
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int ix = t % 3 - tx0, iy = (t / 3) % 3 - ty0;
        double v = 0.0;
        if (ix == 0 && iy == 0) v = acc[0][0][t / 9];
        if (ix == 1 && iy == 0) v = acc[1][0][t / 9];
        if (ix == 0 && iy == 1) v = acc[0][1][t / 9];
        if (ix == 1 && iy == 1) v = acc[1][1][t / 9];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) part[t][w] = v;
    }
    __syncthreads();
    if (tid < 27) {
        const int t = tid;
        const int cx = jx + t % 3 - 1, cy = jy + (t / 3) % 3 - 1, cz = jz + t / 9 - 1;
        if (cx >= 0 && cx < g.ncx && cy >= 0 && cy < g.ncy && cz >= 0 && cz < g.ncz) {
            double sum = 0.0;
            const int nw = (blockDim.x + 63) >> 6;
            for (int q = 0; q < nw; ++q) sum += part[t][q];
            const int col = cx + g.ncx * (cy + g.ncy * cz);
            ac[static_cast<int64_t>(j) * nc + col] = sum;
            if (sum != 0.0) {
                if (j > col) atomicMax(band, j - col);
                if (col > j) atomicMax(band + 1, col - j);
            }
        }
    }
}

// R A P for a node-block operator with 3 components per node and the 27
// node offsets (NodeStencil), on support boxes of nodes (RapBoxGeom over the
// node grid and the coarse node grid).  Coarse dof j = 3 J + c (coarse node
// J, component c): R's row j holds component c of the nodes of J's support
// box; P's row 3 k + c' reaches the dofs 3 K + c' of node k's candidate
// coarse nodes K.  So
//   A_c[j, 3 K + c'] = sum over the nodes k of J's box widened by one node
//                      of (R A)[j, 3 k + c'] P[3 k + c', 3 K + c'],
//   (R A)[j, 3 k + c'] = sum over the 27 neighbours i of k in the support of
//                        R[j, 3 i + c] A[3 i + c, 3 k + c'],
// and a row has at most 27 coarse nodes x 3 components of columns.  As in
// k_rap_box: one thread per (x, y) column of the widened box walks z, the
// products go into 3 x 2 x 2 x 3 register sums (component, x and y
// candidate, z offset), and the 81 sums are added over the wavefront and
// then over the wavefronts in a fixed order (reproducible).
template <typename T>
__global__ __launch_bounds__(kRapBoxMaxThreads) void k_rap_box_nbs(
    int n, int nc, const int *__restrict__ rrp, RapBoxGeom g, const double *__restrict__ av,
    const T *__restrict__ rv, const T *__restrict__ pv, double *__restrict__ ac,
    int *__restrict__ band)
{
    constexpr int NW = kRapBoxMaxThreads / 64;
    __shared__ double part[81][NW];
    const int j = static_cast<int>(blockIdx.x), J = j / 3, cj = j - 3 * J;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nx = g.nx, nxy = g.nx * g.ny;
    const int org = g.box[4 * J], bx = g.box[4 * J + 1], bxy = g.box[4 * J + 2];
    const int by = bxy / bx, bz = g.box[4 * J + 3] / bxy;
    const int x0 = org % nx, y0 = (org / nx) % g.ny, z0 = org / nxy;
    const int lx = max(x0 - 1, 0), ly = max(y0 - 1, 0), lz = max(z0 - 1, 0);
    const int ex = min(x0 + bx + 1, nx) - lx, ey = min(y0 + by + 1, g.ny) - ly;
    const int hz = min(z0 + bz + 1, g.nz);
    const int jx = J % g.ncx, jy = (J / g.ncx) % g.ncy, jz = J / (g.ncx * g.ncy);
    const T *__restrict__ rj = rv + rrp[j];
    double acc[3][2][2][3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[q][a][b][c] = 0.0;
    int tx0 = 0, ty0 = 0;
    if (tid < ex * ey) {
        const int py = tid / ex, x = lx + (tid - py * ex), y = ly + py;
        const int tx = g.tab[x], ty = g.tab[nx + y];
        const int cx = tx >> 16, cy = ty >> 16;
        tx0 = (tx & 0xFFFF) - jx + 1;
        ty0 = (ty & 0xFFFF) - jy + 1;
        const bool x2 = cx == 2, y2 = cy == 2;
        const int sz = cx * cy;
        for (int z = lz; z < hz; ++z) {
            const int k = x + nx * y + nxy * z;
            // (R A)[j, 3 k + c'] over the neighbours i = k - (ox, oy, oz) of
            // k inside the support (node offset o of row 3 i + cj is k - i)
            double ra[3] = {0.0, 0.0, 0.0};
            for (int o = 0; o < 27; ++o) {
                const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
                const int ix = x - ox, iy = y - oy, iz = z - oz;
                if (ix < x0 || ix >= x0 + bx || iy < y0 || iy >= y0 + by || iz < z0 ||
                    iz >= z0 + bz)
                    continue;
                const double r =
                    static_cast<double>(rj[(ix - x0) + bx * ((iy - y0) + by * (iz - z0))]);
                const int64_t row = 3 * static_cast<int64_t>(k - (ox + nx * oy + nxy * oz)) + cj;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    ra[q] += r * av[static_cast<int64_t>(o * 3 + q) * n + row];
            }
            const int tz = g.tab[nx + g.ny + z];
            const int dz0 = (tz & 0xFFFF) - jz + 1, czz = tz >> 16;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                T pr[8];
                {
                    constexpr int L = 16 / sizeof(T);
                    typedef T tvec __attribute__((ext_vector_type(L)));
                    const tvec *vs =
                        reinterpret_cast<const tvec *>(pv + (3 * static_cast<int64_t>(k) + q) * 8);
#pragma unroll
                    for (int u = 0; u < 8 / L; ++u) {
                        const tvec v = vs[u];
#pragma unroll
                        for (int l = 0; l < L; ++l) pr[L * u + l] = v[l];
                    }
                }
                // the row's slots (x fastest over cx, then y, then z) in the
                // fixed 2 x 2 x 2 order, zero where the node has no such slot
                double cv[2][2][2];
#pragma unroll
                for (int iz = 0; iz < 2; ++iz) {
                    auto pick = [&](int u1, int u2, int u4) -> double {
                        return static_cast<double>(sz == 4 ? pr[u4] : (sz == 2 ? pr[u2] : pr[u1]));
                    };
                    cv[0][0][iz] = iz == 0 ? static_cast<double>(pr[0]) : pick(1, 2, 4);
                    cv[1][0][iz] = x2 ? (iz == 0 ? static_cast<double>(pr[1]) : pick(2, 3, 5)) : 0.0;
                    cv[0][1][iz] = y2 ? (iz == 0 ? static_cast<double>(x2 ? pr[2] : pr[1])
                                                 : (x2 ? static_cast<double>(pr[6])
                                                       : static_cast<double>(pr[3])))
                                      : 0.0;
                    cv[1][1][iz] = (x2 && y2) ? static_cast<double>(iz == 0 ? pr[3] : pr[7]) : 0.0;
                }
#pragma unroll
                for (int iz = 0; iz < 2; ++iz) {
                    if (iz >= czz) break;
                    const int dz = dz0 + iz;  // the same for every thread
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (d != dz) continue;
#pragma unroll
                        for (int a = 0; a < 2; ++a)
#pragma unroll
                            for (int b = 0; b < 2; ++b) acc[q][a][b][d] += ra[q] * cv[a][b][iz];
                    }
                }
            }
        }
    }
    // the 81 columns (coarse node offset t / 3, x fastest; component t % 3)
#pragma unroll
    for (int t = 0; t < 81; ++t) {
        const int q = t % 3, tn = t / 3;
        const int ix = tn % 3 - tx0, iy = (tn / 3) % 3 - ty0;
        double v = 0.0;
        if (ix == 0 && iy == 0) v = acc[q][0][0][tn / 9];
        if (ix == 1 && iy == 0) v = acc[q][1][0][tn / 9];
        if (ix == 0 && iy == 1) v = acc[q][0][1][tn / 9];
        if (ix == 1 && iy == 1) v = acc[q][1][1][tn / 9];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) part[t][w] = v;
    }
    __syncthreads();
    for (int t = tid; t < 81; t += blockDim.x) {
        const int q = t % 3, tn = t / 3;
        const int kx = jx + tn % 3 - 1, ky = jy + (tn / 3) % 3 - 1, kz = jz + tn / 9 - 1;
        if (kx >= 0 && kx < g.ncx && ky >= 0 && ky < g.ncy && kz >= 0 && kz < g.ncz) {
            double sum = 0.0;
            const int nw = (blockDim.x + 63) >> 6;
            for (int u = 0; u < nw; ++u) sum += part[t][u];
            const int col = 3 * (kx + g.ncx * (ky + g.ncy * kz)) + q;
            ac[static_cast<int64_t>(j) * nc + col] = sum;
            if (sum != 0.0) {
                if (j > col) atomicMax(band, j - col);
                if (col > j) atomicMax(band + 1, col - j);
            }
        }
    }
}

// a kernel's dynamic LDS above the 64 KB default needs the function's limit
// raised first (the column map of the coarse grid grows with nc)
template <typename F>
void allow_lds(F *f, size_t shmem)
{
    if (shmem > 65536)
        hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem));
}

template <typename T, int ND>
void rap_ell_t(hipStream_t s, size_t shmem, int n, int nc, int maxnb, const int *rrp,
               const int *rci, const T *rv, const DiaOffsets &d, const double *ad,
               const uint16_t *pcol16, const T *pv, double *ac, int *flag, int *band,
               const int *cols, const int *ncol, const int *csr_rp, const int *order)
{
    if (csr_rp) {
        allow_lds(k_rap_ell<T, 128, ND, true>, shmem);
        k_rap_ell<T, 128, ND, true><<<nc, 128, shmem, s>>>(n, nc, maxnb, rrp, rci, rv, d, ad,
                                                           pcol16, pv, ac, flag, band, cols,
                                                           ncol, csr_rp, order);
    } else {
        allow_lds(k_rap_ell<T, 128, ND, false>, shmem);
        k_rap_ell<T, 128, ND, false><<<nc, 128, shmem, s>>>(n, nc, maxnb, rrp, rci, rv, d, ad,
                                                            pcol16, pv, ac, flag, band, cols,
                                                            ncol, nullptr, order);
    }
}

template <typename T>
bool rap_ell(hipStream_t s, size_t shmem, int n, int nc, int maxnb, const int *rrp,
             const int *rci, const T *rv, const DiaOffsets &d, const double *ad,
             const uint16_t *pcol16, const T *pv, double *ac, int *flag, int *band,
             const int *cols, const int *ncol, const int *csr_rp, const int *order)
{
    switch (d.n) {
    case 3: rap_ell_t<T, 3>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band,
                            cols, ncol, csr_rp, order);
        return true;
    case 5: rap_ell_t<T, 5>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band,
                            cols, ncol, csr_rp, order);
        return true;
    case 7: rap_ell_t<T, 7>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band,
                            cols, ncol, csr_rp, order);
        return true;
    case 9: rap_ell_t<T, 9>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band,
                            cols, ncol, csr_rp, order);
        return true;
    default: return false;
    }
}

bool rap_uses_ell(int maxnb, const DiaOffsets &d, int pw, const uint16_t *pcol16)
{
    return maxnb <= 32 && pw == 8 && pcol16 &&
           (d.n == 3 || d.n == 5 || d.n == 7 || d.n == 9);
}

bool rap_uses_nbs(const NodeStencil &ns, int pw, const uint16_t *pcol16)
{
    return ns.n > 0 && (ns.bs == 2 || ns.bs == 3) && pw == 8 && pcol16;
}

void launch_rap_cols(hipStream_t s, int n, int nc, const int *rrp, const int *rci,
                     const DiaOffsets &d, const double *ad, const uint16_t *pcol16, int *cols,
                     int *ncol, const NodeStencil *ns, const double *nsv)
{
    const size_t shmem = sizeof(int) * kMaxCoarseNeighbours + sizeof(short) * nc + 16;
    if (ns) {
        if (ns->bs == 3) {
            allow_lds(k_rap_nbs_cols<3>, shmem);
            k_rap_nbs_cols<3><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, *ns, nsv, pcol16, cols, ncol);
        } else if (ns->bs == 2) {
            allow_lds(k_rap_nbs_cols<2>, shmem);
            k_rap_nbs_cols<2><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, *ns, nsv, pcol16, cols, ncol);
        }
        return;
    }
    switch (d.n) {
    case 3:
        allow_lds(k_rap_cols<3>, shmem);
        k_rap_cols<3><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, d, ad, pcol16, cols, ncol);
        break;
    case 5:
        allow_lds(k_rap_cols<5>, shmem);
        k_rap_cols<5><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, d, ad, pcol16, cols, ncol);
        break;
    case 7:
        allow_lds(k_rap_cols<7>, shmem);
        k_rap_cols<7><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, d, ad, pcol16, cols, ncol);
        break;
    case 9:
        allow_lds(k_rap_cols<9>, shmem);
        k_rap_cols<9><<<nc, 128, shmem, s>>>(n, nc, rrp, rci, d, ad, pcol16, cols, ncol);
        break;
    default: break;
    }
}

bool rap_uses_box(const DiaOffsets &d, int pw, const RapBoxGeom *g)
{
    // 7-point stencil (offsets -nxy, -nx, -1, 0, 1, nx, nxy), P rows of 8
    // slots, geometry checked with the coarse space (threads > 0)
    if (!g || g->threads <= 0 || d.n != 7 || pw != 8) return false;
    const int nx = g->nx, nxy = g->nx * g->ny;
    const int want[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
    for (int o = 0; o < 7; ++o)
        if (d.off[o] != want[o]) return false;
    return true;
}

int rap_box_band(const RapBoxGeom &g)
{
    return (g.ncx > 1 ? 1 : 0) + (g.ncy > 1 ? g.ncx : 0) + (g.ncz > 1 ? g.ncx * g.ncy : 0);
}

void launch_rap(hipStream_t s, int n, int nc, int maxnb, const int *rrp, const int *rci,
                bool fp32, const double *r64, const float *r32, const int *rp, const int *ci,
                const double *a, const DiaOffsets &d, const double *ad, const int *prp,
                const int *pci, const double *pcsr, int pw, const uint16_t *pcol16,
                const double *pe64, const float *pe32, double *ac, int *flag, int *band,
                const int *cols, const int *ncol, const int *csr_rp, const NodeStencil *ns,
                const double *nsv, const int *order, const RapBoxGeom *boxg,
                const RapBoxGeom *nboxg)
{
    // the node-block box form: 3 components, 27 node offsets, dense A_c
    if (nboxg && nboxg->threads > 0 && ns && nsv && !csr_rp && ns->bs == 3 && ns->n == 27 &&
        pw == 8) {
        if (fp32)
            k_rap_box_nbs<float><<<nc, nboxg->threads, 0, s>>>(n, nc, rrp, *nboxg, nsv, r32, pe32,
                                                              ac, band);
        else
            k_rap_box_nbs<double><<<nc, nboxg->threads, 0, s>>>(n, nc, rrp, *nboxg, nsv, r64,
                                                               pe64, ac, band);
        return;
    }
    if (!csr_rp && rap_uses_box(d, pw, boxg)) {
        {
            auto go = [&](auto tag) {
                using T = decltype(tag);
                const T *rv = std::is_same<T, float>::value ? reinterpret_cast<const T *>(r32)
                                                            : reinterpret_cast<const T *>(r64);
                const T *pv = std::is_same<T, float>::value ? reinterpret_cast<const T *>(pe32)
                                                            : reinterpret_cast<const T *>(pe64);
                if (d.sym)
                    k_rap_box<T, true><<<nc, boxg->threads, 0, s>>>(n, nc, rrp, *boxg, ad, rv, pv,
                                                                    ac, band, order);
                else
                    k_rap_box<T, false><<<nc, boxg->threads, 0, s>>>(n, nc, rrp, *boxg, ad, rv,
                                                                     pv, ac, band, order);
            };
            if (fp32) go(0.0f);
            else go(0.0);
            return;
        }
    }
    // node-block stencil A with its column lists: one wavefront per coarse row
    if (ns && nsv && cols && !csr_rp && rap_uses_nbs(*ns, pw, pcol16)) {
        const size_t sh = sizeof(double) * (maxnb + 1) * 64 + sizeof(int) * maxnb +
                          sizeof(short) * static_cast<size_t>(nc) + 16;
        auto go = [&](auto tag, auto bsc) {
            using T = decltype(tag);
            constexpr int BS = decltype(bsc)::value;
            allow_lds(k_rap_nbs<T, BS>, sh);
            const T *rv = std::is_same<T, float>::value ? reinterpret_cast<const T *>(r32)
                                                        : reinterpret_cast<const T *>(r64);
            const T *pv = std::is_same<T, float>::value ? reinterpret_cast<const T *>(pe32)
                                                        : reinterpret_cast<const T *>(pe64);
            k_rap_nbs<T, BS><<<nc, 64, sh, s>>>(n, nc, maxnb, rrp, rci, rv, *ns, nsv, pcol16, pv,
                                                ac, flag, band, cols, ncol);
        };
        if (ns->bs == 3) {
            if (fp32) go(0.0f, std::integral_constant<int, 3>{});
            else go(0.0, std::integral_constant<int, 3>{});
        } else {
            if (fp32) go(0.0f, std::integral_constant<int, 2>{});
            else go(0.0, std::integral_constant<int, 2>{});
        }
        return;
    }
    // 128 threads while the per-thread partial sums fit in 32 KB of LDS
    const int nt = maxnb <= 32 ? 128 : 64;
    const size_t shmem = sizeof(double) * (maxnb + 1) * nt + sizeof(int) * maxnb +
                         sizeof(short) * static_cast<size_t>(nc) + 16;
    // stencil A and 8-wide ELL P: the batched form
    if (nt == 128 && d.n > 0 && pw == 8 && pcol16) {
        const bool done =
            fp32 ? rap_ell<float>(s, shmem, n, nc, maxnb, rrp, rci, r32, d, ad, pcol16, pe32, ac,
                                  flag, band, cols, ncol, csr_rp, order)
                 : rap_ell<double>(s, shmem, n, nc, maxnb, rrp, rci, r64, d, ad, pcol16, pe64, ac,
                                   flag, band, cols, ncol, csr_rp, order);
        if (done) return;
    }
    if (nt == 128) {
        if (fp32)
            rap_t<float, 128>(s, shmem, n, nc, maxnb, rrp, rci, r32, rp, ci, a, d, ad, prp, pci,
                              pcsr, ac, flag, band);
        else
            rap_t<double, 128>(s, shmem, n, nc, maxnb, rrp, rci, r64, rp, ci, a, d, ad, prp, pci,
                               pcsr, ac, flag, band);
    } else {
        if (fp32)
            rap_t<float, 64>(s, shmem, n, nc, maxnb, rrp, rci, r32, rp, ci, a, d, ad, prp, pci,
                             pcsr, ac, flag, band);
        else
            rap_t<double, 64>(s, shmem, n, nc, maxnb, rrp, rci, r64, rp, ci, a, d, ad, prp, pci,
                              pcsr, ac, flag, band);
    }
}

void launch_fill(hipStream_t s, int64_t m, double *x, double v)
{
    if (m > 0) k_fill<<<grid_for(m), kBlock, 0, s>>>(m, x, v);
}

msrsb_status coarse_inverse(hipStream_t s, int n, double *X, double *inv_out, double *bbuf,
                            int *piv, int *colsrc, int *flag, int *host_flag)
{
    if (n < 1 || n > kMaxCoarse) return MSRSB_E_ARG;
    // rows per thread and threads of the leaf kernel: one row per thread up
    // to 1,024 rows (the fewest threads that hold them), then 1,024 threads
    const int R = (n + kLeafThreads - 1) / kLeafThreads;
    const int lt = R > 1 ? kLeafThreads : n <= 64 ? 64 : n <= 128 ? 128 : n <= 256 ? 256
                                                                : n <= 512 ? 512 : 1024;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    double *bleaf = bbuf;                       // kLeaf x kPanel
    double *bpanel = bbuf + kLeaf * kPanel;     // kPanel x n
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int nb = min(kPanel, n - k0);
        for (int kl = k0; kl < k0 + nb; kl += kLeaf) {
            const int lw = min(kLeaf, k0 + nb - kl);
            auto leaf = [&](auto kern, int threads) {
                kern<<<1, threads, 0, s>>>(X, n, k0, nb, kl, lw, piv, bleaf, flag);
            };
            switch (R > 1 ? R + 3 : lt == 64 ? 0 : lt == 128 ? 1 : lt == 256 ? 2 : lt == 512 ? 3 : 4) {
            case 0: leaf(k_gj_leaf<1, 64>, 64); break;
            case 1: leaf(k_gj_leaf<1, 128>, 128); break;
            case 2: leaf(k_gj_leaf<1, 256>, 256); break;
            case 3: leaf(k_gj_leaf<1, 512>, 512); break;
            case 4: leaf(k_gj_leaf<1, kLeafThreads>, kLeafThreads); break;
            case 5: leaf(k_gj_leaf<2, kLeafThreads>, kLeafThreads); break;
            case 6: leaf(k_gj_leaf<3, kLeafThreads>, kLeafThreads); break;
            default: leaf(k_gj_leaf<4, kLeafThreads>, kLeafThreads); break;
            }
            if (nb > lw)
                k_gj_leaf_update<<<grid_for(static_cast<int64_t>(n) * kPanel), kBlock, 0, s>>>(
                    X, n, k0, nb, kl, lw, bleaf);
        }
        if (n > nb) {
            k_gj_swap_extract<<<grid_for(n), kBlock, 0, s>>>(X, n, k0, nb, piv, bpanel);
            const int other = n - nb;
            dim3 grid((other + kT - 1) / kT, (n + kT - 1) / kT);
            k_gj_gemm<<<grid, 256, 0, s>>>(X, n, k0, nb, bpanel);
        }
    }
    k_gj_colsrc<<<1, 64, 0, s>>>(n, piv, colsrc);
    k_gj_permute<<<grid_for(static_cast<int64_t>(n) * n), kBlock, 0, s>>>(n, X, colsrc, inv_out);
    hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSRSB_E_HIP;
    return *host_flag ? MSRSB_E_COARSE_SINGULAR : MSRSB_OK;
}

// X's tiles (I, J) with |I - J| <= tb from A: the band Cholesky below reads
// and writes no other tile of its workspace
__global__ __launch_bounds__(256) void k_copy_band_tiles(const double *__restrict__ A,
                                                        double *__restrict__ X, int n, int tb)
{
    const int nt = (n + kBP - 1) / kBP, w = 2 * tb + 1;
    const int I = static_cast<int>(blockIdx.x) / w, J = I - tb + static_cast<int>(blockIdx.x) % w;
    if (J < 0 || J >= nt) return;
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int r = I * kBP + e / kBP, c = J * kBP + e % kBP;
        if (r < n && c < n) X[static_cast<int64_t>(r) * n + c] = A[static_cast<int64_t>(r) * n + c];
    }
}

msrsb_status coarse_inverse_spd(hipStream_t s, int n, const double *A, double *X, int bl,
                                double *Linv, double *W, double *pk, int *flag, int *host_flag)
{
    if (n < 1 || n > kMaxCoarse) return MSRSB_E_ARG;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    const int nt = (n + kBP - 1) / kBP;
    // row tiles below a panel that the band reaches
    const int tb = min(nt - 1, (max(bl, 0) + kBP - 1) / kBP);
    k_copy_band_tiles<<<nt * (2 * tb + 1), 256, 0, s>>>(A, X, n, tb);
    // each panel's update also inverts the next panel's diagonal block, which
    // it finalises; a panel without band rows below it leaves the next block
    // untouched, and that block is inverted on its own.  Row tile K of W =
    // L^{-1} rides along with panel K's update (extra work-groups, which run
    // beside the diagonal inversion), or gets a launch of its own.
    bool have_inv = false;
    for (int K = 0; K < nt; ++K) {
        const int k0 = K * kBP, nb = min(kBP, n - k0);
        double *li = Linv + static_cast<int64_t>(K) * kBP * kBP;
        if (!have_inv) k_chol_inv<<<1, 256, 0, s>>>(X, n, k0, nb, li, flag);
        const int T = min(nt - 1, K + tb) - K;
        // strips of 16 columns left of the end of panel K
        const int nstrips = (min(n, k0 + kBP) + 15) / 16;
        have_inv = T > 0;
        if (T > 0) {
            const int nbn = min(kBP, n - k0 - kBP);
            const int npairs = T * (T + 1) / 2;
            k_chol_update<<<npairs + nstrips, 256, 0, s>>>(X, n, k0, nb, K + 1, li,
                                                           li + kBP * kBP, nbn, flag, npairs, tb,
                                                           W);
        } else {
            k_chol_w_row<<<nstrips, 256, 0, s>>>(X, n, tb, li, W, K);
        }
    }
    k_chol_wtw<<<nt * (nt + 1) / 2, 256, 0, s>>>(W, n, pk);
    hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSRSB_E_HIP;
    return *host_flag ? MSRSB_E_COARSE_SINGULAR : MSRSB_OK;
}

void launch_symv_packed(hipStream_t s, int n, const double *pk, const double *x, double *y,
                        double *part)
{
    const int nt = (n + kBP - 1) / kBP;
    k_symv_tiles<<<nt * (nt + 1) / 2, 256, 0, s>>>(pk, n, x, part);
    k_symv_final<<<nt, 256, 0, s>>>(part, n, y);
}

void launch_gemv(hipStream_t s, int n, const double *m, const double *x, double *y, bool trans,
                 double *partials)
{
    if (!trans) {
        k_gemv<<<grid_for(static_cast<int64_t>(n) * 64), kBlock, 0, s>>>(n, m, x, y);
    } else {
        dim3 grid((n + kBlock - 1) / kBlock, kGemvSeg);
        k_gemv_t_partial<<<grid, kBlock, 0, s>>>(n, m, x, partials);
        k_gemv_t_final<<<grid_for(n), kBlock, 0, s>>>(n, partials, y);
    }
}

}  // namespace msrsb
