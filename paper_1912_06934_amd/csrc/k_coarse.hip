// Coarse-level kernels: R = P^T values, the Galerkin operator A_c = R A P
// (eq. lin_system_coarse, Alg. 2), the exact coarse solver M_c^{-1} = A_c^{-1}
// and its application.
#include <utility>

#include "internal.h"

namespace msrsb {
namespace {

inline int grid_for(int64_t m) { return static_cast<int>((m + kBlock - 1) / kBlock); }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int64_t m, const int *__restrict__ src,
                                                   const T *__restrict__ p, T *__restrict__ r)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < m) r[t] = p[src[t]];
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t m, double *__restrict__ x, double v)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < m) x[t] = v;
}

// A_c row j = sum over fine rows i in the support of j (R row j, ascending
// i) of P_ij * A_i* * P.  One work-group per coarse row.  The coarse columns
// reached by row j (its coarse neighbours) are found first and numbered in
// ascending order in an LDS map; each thread then accumulates its share of
// the fine rows into a private LDS column of per-neighbour partial sums, and
// the partial sums of every neighbour are added in thread order.  No atomics
// touch A_c, so it is bitwise reproducible.  The lower and upper bandwidths
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
                acc[map[pci[q]] * NT + tid] += pa * pv[q];
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

template <typename T, int NT, int ND>
__global__ __launch_bounds__(NT) void k_rap_ell(int n, int nc, int maxnb,
                                                const int *__restrict__ rrp,
                                                const int *__restrict__ rci,
                                                const T *__restrict__ rv, DiaOffsets d,
                                                const double *__restrict__ ad,
                                                const uint16_t *__restrict__ pcol,
                                                const T *__restrict__ pv, double *__restrict__ ac,
                                                int *__restrict__ flag, int *__restrict__ band)
{
    extern __shared__ double smem[];
    __shared__ int wsum[NT / 64];
    double *acc = smem;                                         // maxnb * NT
    int *inv = reinterpret_cast<int *>(acc + maxnb * NT);       // maxnb
    short *map = reinterpret_cast<short *>(inv + maxnb);        // nc
    const int j = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int t = tid; t < nc; t += NT) map[t] = 0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    for (int t = t0 + tid; t < t1; t += NT) {
        const int i = rci[t];
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const int k = i + d.off[o];
            if (k < 0 || k >= n || ad[static_cast<int64_t>(o) * n + i] == 0.0) continue;
            typedef uint16_t cvec __attribute__((ext_vector_type(8)));
            const cvec cc = *reinterpret_cast<const cvec *>(pcol + static_cast<int64_t>(k) * 8);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (cc[u] != 0xFFFFu) map[cc[u]] = 1;
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
        double av[ND];
        T v[ND][8];
        uint16_t cl[ND][8];
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const int k = i + d.off[o];
            const bool in = k >= 0 && k < n;
            const double a = ad[static_cast<int64_t>(o) * n + i];
            av[o] = in ? a : 0.0;
            load_prow<T>(pv, pcol, in ? k : i, v[o], cl[o]);
        }
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            if (av[o] == 0.0) continue;
            const double pa = pij * av[o];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (cl[o][u] != 0xFFFFu)
                    acc[map[cl[o][u]] * NT + tid] += pa * static_cast<double>(v[o][u]);
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

template <int R>
__global__ __launch_bounds__(kLeafThreads) void k_gj_leaf(double *__restrict__ X, int n, int k0,
                                                          int nb, int kl, int lw,
                                                          int *__restrict__ piv,
                                                          double *__restrict__ bbuf,
                                                          int *__restrict__ flag)
{
    __shared__ double red_v[kLeafThreads / 64];
    __shared__ int red_r[kLeafThreads / 64];
    __shared__ double rowk[kLeaf], rowp[kLeaf];
    __shared__ int sh_p;
    __shared__ int sh_piv[kLeaf];
    const int tid = threadIdx.x;
    double v[R][kLeaf];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * kLeafThreads;
#pragma unroll
        for (int c = 0; c < kLeaf; ++c)
            v[q][c] = (r < n && c < lw) ? X[static_cast<int64_t>(r) * n + kl + c] : 0.0;
    }
    for (int c = 0; c < lw; ++c) {
        const int k = kl + c;
        // argmax |x_rk| over r >= k; ties go to the lowest row
        double best = -1.0;
        int brow = n;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * kLeafThreads;
            double val = 0.0;
#pragma unroll
            for (int cc = 0; cc < kLeaf; ++cc)
                if (cc == c) val = fabs(v[q][cc]);
            if (r < n && r >= k && (val > best || (val == best && r < brow))) {
                best = val;
                brow = r;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int orow = __shfl_xor(brow, off, 64);
            if (ob > best || (ob == best && orow < brow)) {
                best = ob;
                brow = orow;
            }
        }
        if ((tid & 63) == 0) {
            red_v[tid >> 6] = best;
            red_r[tid >> 6] = brow;
        }
        __syncthreads();
        if (tid == 0) {
            double b = red_v[0];
            int br = red_r[0];
            for (int w = 1; w < kLeafThreads / 64; ++w)
                if (red_v[w] > b || (red_v[w] == b && red_r[w] < br)) {
                    b = red_v[w];
                    br = red_r[w];
                }
            if (!(b > 0.0)) flag[0] = 1;  // singular (or NaN) pivot column
            if (br >= n) br = k;
            sh_p = br;
            sh_piv[c] = br;
            piv[k] = br;
        }
        __syncthreads();
        const int p = sh_p;
        // swap rows k and p of the leaf
        const int ok = k % kLeafThreads, qk = k / kLeafThreads;
        const int op = p % kLeafThreads, qp = p / kLeafThreads;
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
            const int r = tid + q * kLeafThreads;
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
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * kLeafThreads;
        if (r < n)
#pragma unroll
            for (int c = 0; c < kLeaf; ++c)
                if (c < lw) X[static_cast<int64_t>(r) * n + kl + c] = v[q][c];
    }
    // the leaf's swaps on the other columns of the panel, then take the leaf
    // rows of those columns out (B) and zero them
    if (tid < nb) {
        const int col = k0 + tid;
        if (col < kl || col >= kl + lw) {
            for (int c = 0; c < lw; ++c) {
                const int k = kl + c, p = sh_piv[c];
                if (p != k) {
                    const double t = X[static_cast<int64_t>(k) * n + col];
                    X[static_cast<int64_t>(k) * n + col] = X[static_cast<int64_t>(p) * n + col];
                    X[static_cast<int64_t>(p) * n + col] = t;
                }
            }
            for (int c = 0; c < lw; ++c) {
                bbuf[c * kPanel + tid] = X[static_cast<int64_t>(kl + c) * n + col];
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
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
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
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * n) return;
    const int r = static_cast<int>(t / n), j = static_cast<int>(t % n);
    Y[t] = X[static_cast<int64_t>(r) * n + colsrc[j]];
}

// ---------------------------------------------------------------------------
// Pivot-free block Gauss-Jordan, for a symmetric positive definite A_c (the
// Galerkin operator of a symmetric positive definite A), in place on X.
// For each 64-wide panel K (diagonal block D = X[K,K], G = D^{-1}):
//   X[K,C] <- G X[K,C]                         (block row, C != K)
//   X[R,C] <- X[R,C] - X[R,K] X[K,C]          (rank-64 update, R, C != K)
//   X[R,K] <- -X[R,K] G,  X[K,K] <- G          (block column)
// After the last panel X = A_c^{-1}.  Without pivoting the part of X not yet
// eliminated keeps A_c's band: at panel K rows below k0 + 64 + bl have a zero
// block column and columns right of k0 + 64 + bu a zero block row, so the
// updates stop there (bl, bu = lower and upper bandwidth of A_c).
// ---------------------------------------------------------------------------
constexpr int kBP = 64;
constexpr int kSuper = 128;  // columns per super-panel (a multiple of kBP)

// G = D^{-1} for the 64 x 64 diagonal block D by Gauss-Jordan without
// pivoting, blocked by 16 (the same elimination as the unblocked one, grouped
// in four sub-panels P of 16 pivots; Q = the other 48 indices):
//   M_PP <- G_P = M_PP^{-1}        (one wavefront, unblocked, below)
//   H = G_P M_PQ,  M_QQ <- M_QQ - M_QP H,  M_QP <- -M_QP G_P,  M_PQ <- H
// Rows and columns past nb are padded with the identity.  Non-positive pivots
// set the flag.
constexpr int kDS = kBP + 1;  // LDS row stride of the block

// Unblocked Gauss-Jordan on the 16 x 16 block at (o, o) of M in one
// wavefront: lane l keeps row l / 4, columns 4 (l % 4) .. + 3 in registers
// and takes the pivot row, the pivot and its own multiplier from the other
// lanes by shuffles.  Row c becomes x_cj / d (1 / d in column c) and every
// other row r becomes x_rj - (x_rc / d) x_cj (-x_rc / d in column c).
__device__ inline void gj16(double (*M)[kDS], int o, int lane, bool &bad)
{
    const int r = lane >> 2, q4 = lane & 3;
    double a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = M[o + r][o + 4 * q4 + j];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int cq = c >> 2, cj = c & 3;
        double pv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pv[j] = __shfl(a[j], 4 * c + q4, 64);
        const double d = __shfl(a[cj], 4 * c + cq, 64);
        const double f = __shfl(a[cj], 4 * r + cq, 64);
        bad |= !(d > 0.0);
        const double inv = 1.0 / d;
        const bool piv = r == c;
        const double g = piv ? -inv : f * inv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double base = piv ? 0.0 : a[j];
            a[j] = (4 * q4 + j == c) ? -g : base - g * pv[j];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) M[o + r][o + 4 * q4 + j] = a[j];
}

__global__ __launch_bounds__(256) void k_bgj_diag(const double *__restrict__ X, int n, int k0,
                                                  int nb, double *__restrict__ G,
                                                  int *__restrict__ flag)
{
    __shared__ double M[kBP][kDS];
    __shared__ double H[16][kDS];   // G_P M_PQ
    __shared__ double Cp[kBP][17];  // M_QP before the sub-panel (column block P)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    #pragma unroll
    for (int it_ = 0; it_ < (kBP * kBP) / 256; ++it_) {
        const int e = t + 256 * it_;
        const int r = e / kBP, c = e % kBP;
        M[r][c] = (r < nb && c < nb) ? X[static_cast<int64_t>(k0 + r) * n + k0 + c]
                                     : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    bool bad = false;
    for (int p = 0; p < 4; ++p) {
        const int o = 16 * p;
        if (w == 0) gj16(M, o, lane, bad);
        __syncthreads();
        // H = G_P M_PQ (columns outside P) and a copy of the column block P
        #pragma unroll
        for (int it_ = 0; it_ < (16 * kBP) / 256; ++it_) {
            const int e = t + 256 * it_;
            const int k = e / kBP, j = e % kBP;
            if (j >= o && j < o + 16) continue;
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < 16; ++m) s += M[o + k][o + m] * M[o + m][j];
            H[k][j] = s;
        }
        #pragma unroll
        for (int it_ = 0; it_ < (kBP * 16) / 256; ++it_) {
            const int e = t + 256 * it_;
            const int r = e / 16, k = e % 16;
            Cp[r][k] = M[r][o + k];
        }
        __syncthreads();
        // column j of the rows outside P: M_rj -= M_rP H_Pj, or -M_rP G_P in P;
        // the rows of P take H
        {
            const int j = lane;
            const bool inP = j >= o && j < o + 16;
            double hc[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) hc[k] = inP ? M[o + k][j] : H[k][j];
            for (int r = w; r < kBP; r += 4) {
                if (r >= o && r < o + 16) {
                    if (!inP) M[r][j] = H[r - o][j];
                    continue;
                }
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) s += Cp[r][k] * hc[k];
                M[r][j] = inP ? -s : M[r][j] - s;
            }
        }
        __syncthreads();
    }
    if (bad) flag[0] = 1;
    #pragma unroll
    for (int it_ = 0; it_ < (kBP * kBP) / 256; ++it_) {
        const int e = t + 256 * it_;
        const int r = e / kBP, c = e % kBP;
        if (r < nb && c < nb) G[r * kBP + c] = M[r][c];
    }
}

// X[K, tile] <- G X[K, tile] for the column tiles left of cu other than K
__global__ __launch_bounds__(256) void k_bgj_rowblock(double *__restrict__ X, int n, int k0,
                                                      int nb, const double *__restrict__ G,
                                                      int ct0)
{
    __shared__ double Gs[kBP][kBP + 1];
    __shared__ double Xs[kBP][kBP + 1];
    const int kt = k0 / kBP;
    if (blockIdx.x == gridDim.x - 1) {  // the diagonal block becomes G
        for (int e = threadIdx.x; e < nb * nb; e += 256)
            X[static_cast<int64_t>(k0 + e / nb) * n + k0 + e % nb] = G[(e / nb) * kBP + e % nb];
        return;
    }
    const int tile = ct0 + blockIdx.x < kt ? ct0 + blockIdx.x : ct0 + blockIdx.x + 1;
    const int c0 = tile * kBP;
    #pragma unroll
    for (int it_ = 0; it_ < (kBP * kBP) / 256; ++it_) {
        const int t = threadIdx.x + 256 * it_;
        const int r = t / kBP, c = t % kBP;
        Gs[r][c] = (r < nb && c < nb) ? G[r * kBP + c] : 0.0;
        Xs[r][c] = (r < nb && c0 + c < n) ? X[static_cast<int64_t>(k0 + r) * n + c0 + c] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int k = 0; k < nb; ++k) {
        double g[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            g[u] = Gs[ty * 4 + u][k];
            x[u] = Xs[k][tx * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] += g[u] * x[w];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = ty * 4 + u;
        if (r >= nb) continue;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int c = c0 + tx * 4 + w;
            if (c < n) X[static_cast<int64_t>(k0 + r) * n + c] = acc[u][w];
        }
    }
}

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

// One 64-wide panel K inside a super-panel, for one row tile R != K (one
// work-group per row tile below the band limit):
//   X[R, t] -= X[R, K] (G X[K, t])   for the other column tiles t of the
//                                    super-panel (G X[K, t] formed here from
//                                    the unmodified X[K, t])
//   X[R, K] <- -X[R, K] G
// The row block K itself is updated afterwards by k_bgj_rowblock.
__global__ __launch_bounds__(256) void k_bgj_inner(double *__restrict__ X, int n, int k0, int nb,
                                                   const double *__restrict__ G, int ct0, int nct)
{
    __shared__ double Gs[kBP][kLds];  // G by rows
    __shared__ double Gt[kBP][kLds];  // G by columns
    __shared__ double As[kBP][kLds];  // X[R, K] before this panel, by rows
    __shared__ double Kt[kBP][kLds];  // X[K, t] by columns, then (G X[K, t]) by columns
    const int kt = k0 / kBP;
    const int tr = blockIdx.x < kt ? blockIdx.x : blockIdx.x + 1;
    const int r0 = tr * kBP;
    #pragma unroll
    for (int it_ = 0; it_ < (kBP * kBP) / 256; ++it_) {
        const int e = threadIdx.x + 256 * it_;
        const int a = e / kBP, b = e % kBP;
        const double g = (a < nb && b < nb) ? G[a * kBP + b] : 0.0;
        Gs[a][b] = g;
        Gt[b][a] = g;
        As[a][b] = (r0 + a < n && b < nb) ? X[static_cast<int64_t>(r0 + a) * n + k0 + b] : 0.0;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    mfma_f64x4 acc[2][2];
    for (int u = 0; u < nct; ++u) {
        const int tc = ct0 + u < kt ? ct0 + u : ct0 + u + 1;
        const int c0 = tc * kBP;
        __syncthreads();
        #pragma unroll
        for (int it_ = 0; it_ < (kBP * kBP) / 256; ++it_) {
            const int e = threadIdx.x + 256 * it_;
            const int a = e / kBP, b = e % kBP;
            Kt[b][a] = (a < nb && c0 + b < n) ? X[static_cast<int64_t>(k0 + a) * n + c0 + b] : 0.0;
        }
        __syncthreads();
        zero_acc(acc);
        mfma_tile64(Gs, Kt, acc, wr, wc, li, lk);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    Kt[wc + 16 * v + li][wr + 16 * p + 4 * q + lk] = acc[p][v][q];
        __syncthreads();
        zero_acc(acc);
        mfma_tile64(As, Kt, acc, wr, wc, li, lk);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + wr + 16 * p + 4 * q + lk;
                    const int c = c0 + wc + 16 * v + li;
                    if (r < n && c < n) X[static_cast<int64_t>(r) * n + c] -= acc[p][v][q];
                }
    }
    __syncthreads();
    zero_acc(acc);
    mfma_tile64(As, Gt, acc, wr, wc, li, lk);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr + 16 * p + 4 * q + lk;
                const int c = wc + 16 * v + li;
                if (r < n && c < nb) X[static_cast<int64_t>(r) * n + k0 + c] = -acc[p][v][q];
            }
}

// Rows s0 .. s0+ns-1 of the columns outside the super-panel (up to c_hi) move
// to B (ns x n) and are zeroed.
__global__ __launch_bounds__(kBlock) void k_bgj_extract(double *__restrict__ X, int n, int s0,
                                                        int ns, int c_hi, double *__restrict__ B)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (c >= c_hi || (c >= s0 && c < s0 + ns)) return;
    const int64_t e = static_cast<int64_t>(s0 + t) * n + c;
    B[static_cast<int64_t>(t) * n + c] = X[e];
    X[e] = 0.0;
}

// X[R, C] += X[R, S] B[:, C] for row tiles below the band limit and column
// tiles outside the super-panel S = [s0, s0 + ns) (ns a multiple of 64); the
// super-panel's combined Gauss-Jordan transformation applied to the other
// columns, on the FP64 matrix cores (mfma_tile64).  The next 64-deep chunk of
// X[R, S] and B is loaded into registers while the current one is
// multiplied, and the X[R, C] tile is fetched at the start.
__global__ __launch_bounds__(256) void k_bgj_outer(double *__restrict__ X, int n, int s0, int ns,
                                                   const double *__restrict__ B)
{
    __shared__ double As[kBP][kLds];
    __shared__ double Bt[kBP][kLds];
    const int st0 = s0 / kBP, nst = (ns + kBP - 1) / kBP;
    const int tr = blockIdx.y;
    const int tc = blockIdx.x < st0 ? blockIdx.x : blockIdx.x + nst;
    const int r0 = tr * kBP, c0 = tc * kBP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    // the output tile, in the accumulator layout
    double xo[2][2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr + 16 * u + 4 * q + lk;
                const int c = c0 + wc + 16 * v + li;
                xo[u][v][q] = (r < n && c < n) ? X[static_cast<int64_t>(r) * n + c] : 0.0;
            }
    // thread t loads rows t / 64 + 4 k, column t % 64 of each 64 x 64 chunk
    const int lr = threadIdx.x >> 6, lc = threadIdx.x & 63;
    double ra[16], rb[16];
    auto fetch = [&](int kb) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int a = lr + 4 * k;
            ra[k] = (r0 + a < n && kb + lc < ns)
                        ? X[static_cast<int64_t>(r0 + a) * n + s0 + kb + lc] : 0.0;
            rb[k] = (kb + a < ns && c0 + lc < n) ? B[static_cast<int64_t>(kb + a) * n + c0 + lc]
                                                 : 0.0;
        }
    };
    mfma_f64x4 acc[2][2];
    zero_acc(acc);
    fetch(0);
    for (int kb = 0; kb < ns; kb += kBP) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            As[lr + 4 * k][lc] = ra[k];
            Bt[lc][lr + 4 * k] = rb[k];
        }
        __syncthreads();
        if (kb + kBP < ns) fetch(kb + kBP);
        mfma_tile64(As, Bt, acc, wr, wc, li, lk);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr + 16 * u + 4 * q + lk;
                const int c = c0 + wc + 16 * v + li;
                if (r < n && c < n) X[static_cast<int64_t>(r) * n + c] = xo[u][v][q] + acc[u][v][q];
            }
}

// y = M x, one wavefront per row; lanes stride over the columns (two per
// 16-byte load when n is even) and the 64 partial sums are added in a fixed
// butterfly order.
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double *__restrict__ M,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
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
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
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

template <typename T, int ND>
void rap_ell_t(hipStream_t s, size_t shmem, int n, int nc, int maxnb, const int *rrp,
               const int *rci, const T *rv, const DiaOffsets &d, const double *ad,
               const uint16_t *pcol16, const T *pv, double *ac, int *flag, int *band)
{
    k_rap_ell<T, 128, ND><<<nc, 128, shmem, s>>>(n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac,
                                                 flag, band);
}

template <typename T>
bool rap_ell(hipStream_t s, size_t shmem, int n, int nc, int maxnb, const int *rrp,
             const int *rci, const T *rv, const DiaOffsets &d, const double *ad,
             const uint16_t *pcol16, const T *pv, double *ac, int *flag, int *band)
{
    switch (d.n) {
    case 3: rap_ell_t<T, 3>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band); return true;
    case 5: rap_ell_t<T, 5>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band); return true;
    case 7: rap_ell_t<T, 7>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band); return true;
    case 9: rap_ell_t<T, 9>(s, shmem, n, nc, maxnb, rrp, rci, rv, d, ad, pcol16, pv, ac, flag, band); return true;
    default: return false;
    }
}

void launch_rap(hipStream_t s, int n, int nc, int maxnb, const int *rrp, const int *rci,
                bool fp32, const double *r64, const float *r32, const int *rp, const int *ci,
                const double *a, const DiaOffsets &d, const double *ad, const int *prp,
                const int *pci, const double *pcsr, int pw, const uint16_t *pcol16,
                const double *pe64, const float *pe32, double *ac, int *flag, int *band)
{
    // 128 threads while the per-thread partial sums fit in 32 KB of LDS
    const int nt = maxnb <= 32 ? 128 : 64;
    const size_t shmem = sizeof(double) * maxnb * nt + sizeof(int) * maxnb +
                         sizeof(short) * static_cast<size_t>(nc) + 16;
    // stencil A and 8-wide ELL P: the batched form
    if (nt == 128 && d.n > 0 && pw == 8 && pcol16) {
        const bool done = fp32 ? rap_ell<float>(s, shmem, n, nc, maxnb, rrp, rci, r32, d, ad,
                                                pcol16, pe32, ac, flag, band)
                               : rap_ell<double>(s, shmem, n, nc, maxnb, rrp, rci, r64, d, ad,
                                                 pcol16, pe64, ac, flag, band);
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
    const int R = (n + kLeafThreads - 1) / kLeafThreads;  // rows per thread
    hipMemsetAsync(flag, 0, sizeof(int), s);
    double *bleaf = bbuf;                       // kLeaf x kPanel
    double *bpanel = bbuf + kLeaf * kPanel;     // kPanel x n
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int nb = min(kPanel, n - k0);
        for (int kl = k0; kl < k0 + nb; kl += kLeaf) {
            const int lw = min(kLeaf, k0 + nb - kl);
            switch (R) {
            case 1:
                k_gj_leaf<1><<<1, kLeafThreads, 0, s>>>(X, n, k0, nb, kl, lw, piv, bleaf, flag);
                break;
            case 2:
                k_gj_leaf<2><<<1, kLeafThreads, 0, s>>>(X, n, k0, nb, kl, lw, piv, bleaf, flag);
                break;
            case 3:
                k_gj_leaf<3><<<1, kLeafThreads, 0, s>>>(X, n, k0, nb, kl, lw, piv, bleaf, flag);
                break;
            default:
                k_gj_leaf<4><<<1, kLeafThreads, 0, s>>>(X, n, k0, nb, kl, lw, piv, bleaf, flag);
                break;
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

msrsb_status coarse_inverse_spd(hipStream_t s, int n, double *X, int bl, int bu, double *G,
                                double *B, int *flag, int *host_flag)
{
    if (n < 1 || n > kMaxCoarse) return MSRSB_E_ARG;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    // super-panels of kSuper columns: their 64-wide panels are eliminated
    // within the super-panel, then one rank-kSuper update carries the
    // combined transformation to the other columns
    for (int s0 = 0; s0 < n; s0 += kSuper) {
        const int ns = min(kSuper, n - s0);
        const int st0 = s0 / kBP, st1 = (s0 + ns + kBP - 1) / kBP;
        for (int k0 = s0; k0 < s0 + ns; k0 += kBP) {
            const int nb = min(kBP, n - k0);
            const int rl = min(n, k0 + nb + bl);
            const int rtiles = (rl + kBP - 1) / kBP;
            k_bgj_diag<<<1, 256, 0, s>>>(X, n, k0, nb, G, flag);
            const int inner = st1 - st0 - 1;  // super-panel column tiles other than K
            if (rtiles > 1) k_bgj_inner<<<rtiles - 1, 256, 0, s>>>(X, n, k0, nb, G, st0, inner);
            k_bgj_rowblock<<<inner + 1, 256, 0, s>>>(X, n, k0, nb, G, st0);
        }
        const int rl = min(n, s0 + ns + bl), cu = min(n, s0 + ns + bu);
        const int rtiles = (rl + kBP - 1) / kBP, ctiles = (cu + kBP - 1) / kBP;
        const int outer = ctiles - (st1 - st0);
        if (outer > 0) {
            // whole column tiles are extracted: the GEMM reads B up to the tile edge
            const int c_hi = min(n, ctiles * kBP);
            k_bgj_extract<<<dim3((c_hi + kBlock - 1) / kBlock, ns), kBlock, 0, s>>>(X, n, s0, ns,
                                                                                   c_hi, B);
            k_bgj_outer<<<dim3(outer, rtiles), 256, 0, s>>>(X, n, s0, ns, B);
        }
    }
    hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSRSB_E_HIP;
    return *host_flag ? MSRSB_E_COARSE_SINGULAR : MSRSB_OK;
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
