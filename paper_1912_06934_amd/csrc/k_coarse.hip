// Coarse-level kernels: R = P^T values, the Galerkin operator A_c = R A P
// (eq. lin_system_coarse, Alg. 2), the exact coarse solver M_c^{-1} = A_c^{-1}
// and its application.
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
// i) of P_ij * A_i* * P.  One wavefront per coarse row.  The coarse columns
// reached by row j (its coarse neighbours) are found first and numbered in
// ascending order in an LDS map; each lane then accumulates its share of the
// fine rows into a private LDS column of per-neighbour partial sums, and the
// 64 partial sums of every neighbour are added in lane order.  The result does
// not depend on scheduling (no atomics), so it is bitwise reproducible.
template <typename T>
__global__ __launch_bounds__(64) void k_rap(int nc, int maxnb, const int *__restrict__ rrp,
                                            const int *__restrict__ rci, const T *__restrict__ rv,
                                            const int *__restrict__ rp,
                                            const int *__restrict__ ci,
                                            const double *__restrict__ a,
                                            const int *__restrict__ prp,
                                            const int *__restrict__ pci, const T *__restrict__ pv,
                                            double *__restrict__ ac, int *__restrict__ flag)
{
    extern __shared__ double smem[];
    double *acc = smem;                                         // maxnb * 64
    int *inv = reinterpret_cast<int *>(acc + maxnb * 64);       // maxnb
    short *map = reinterpret_cast<short *>(inv + maxnb);        // nc
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    for (int t = lane; t < nc; t += 64) map[t] = 0;
    __syncthreads();
    const int t0 = rrp[j], t1 = rrp[j + 1];
    for (int t = t0 + lane; t < t1; t += 64) {
        const int i = rci[t];
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int k = ci[e];
            for (int q = prp[k]; q < prp[k + 1]; ++q) map[pci[q]] = 1;
        }
    }
    __syncthreads();
    // number the marked coarse columns in ascending order (wavefront scan)
    const int chunk = (nc + 63) / 64;
    const int lo = lane * chunk, hi = min(nc, lo + chunk);
    int cnt = 0;
    for (int t = lo; t < hi; ++t) cnt += map[t];
    int pre = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(pre, off, 64);
        if (lane >= off) pre += o;
    }
    const int total = __shfl(pre, 63, 64);
    if (total > maxnb) {
        if (lane == 0) flag[0] = 1;
        return;
    }
    int slot = pre - cnt;
    __syncthreads();
    for (int t = lo; t < hi; ++t) {
        if (map[t]) {
            inv[slot] = t;
            map[t] = static_cast<short>(slot++);
        } else {
            map[t] = -1;
        }
    }
    for (int s = 0; s < total; ++s) acc[s * 64 + lane] = 0.0;
    __syncthreads();
    for (int t = t0 + lane; t < t1; t += 64) {
        const int i = rci[t];
        const double pij = static_cast<double>(rv[t]);
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int k = ci[e];
            const double pa = pij * a[e];
            for (int q = prp[k]; q < prp[k + 1]; ++q) {
                const int sl = map[pci[q]];
                acc[sl * 64 + lane] += pa * static_cast<double>(pv[q]);
            }
        }
    }
    __syncthreads();
    for (int s = lane; s < total; s += 64) {
        double sum = 0.0;
        for (int l = 0; l < 64; ++l) sum += acc[s * 64 + l];
        ac[static_cast<int64_t>(j) * nc + inv[s]] = sum;
    }
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

// y = M x, one wavefront per row; lanes stride over the columns and the 64
// partial sums are added in a fixed butterfly order.
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double *__restrict__ M,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *mr = M + static_cast<int64_t>(row) * n;
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s += mr[c] * x[c];
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

void launch_rap(hipStream_t s, int nc, int maxnb, const int *rrp, const int *rci, bool fp32,
                const double *r64, const float *r32, const int *rp, const int *ci,
                const double *a, const int *prp, const int *pci, const double *p64,
                const float *p32, double *ac, int *flag)
{
    const size_t shmem = sizeof(double) * maxnb * 64 + sizeof(int) * maxnb +
                         sizeof(short) * static_cast<size_t>(nc) + 16;
    if (fp32)
        k_rap<float><<<nc, 64, shmem, s>>>(nc, maxnb, rrp, rci, r32, rp, ci, a, prp, pci, p32,
                                           ac, flag);
    else
        k_rap<double><<<nc, 64, shmem, s>>>(nc, maxnb, rrp, rci, r64, rp, ci, a, prp, pci, p64,
                                            ac, flag);
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
