// Krylov-level kernels: SpMV, smoother sweeps, restriction / prolongation
// (Alg. 3), deterministic two-stage reductions and the fused vector updates
// of PCG and GMRES.
#include "internal.h"

#include <type_traits>

namespace msrsb {
namespace {

inline int grid_for(int64_t m) { return static_cast<int>((m + kBlock - 1) / kBlock); }

// block-wide sum in a fixed order (butterfly within wavefronts, then the
// wavefront sums in index order)
__device__ inline double block_sum(double v)
{
    __shared__ double sh[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
    __syncthreads();
    return s;  // valid in thread 0
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(int m, const double *__restrict__ part,
                                                         double *__restrict__ out)
{
    double s = 0.0;
    for (int t = threadIdx.x; t < m; t += kBlock) s += part[t];
    s = block_sum(s);
    if (threadIdx.x == 0) out[0] = s;
}

void finish(hipStream_t st, int m, const double *part, double *out)
{
    k_sum_partials<<<1, kBlock, 0, st>>>(m, part, out);
}

__device__ inline double row_dot(int i, const int *__restrict__ rp, const int *__restrict__ ci,
                                 const double *__restrict__ a, const double *__restrict__ x)
{
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += a[e] * x[ci[e]];
    return s;
}

__global__ __launch_bounds__(kBlock) void k_spmv(int n, const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int i = xcd_row();
    if (i < n) y[i] = row_dot(i, rp, ci, a, x);
}

__global__ __launch_bounds__(kBlock) void k_residual(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ f,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ r)
{
    const int i = xcd_row();
    if (i < n) r[i] = f[i] - row_dot(i, rp, ci, a, x);
}

// z_out = z_in + M^{-1} (v - A z_in), M diagonal (Jacobi or l1-Jacobi).
// With zero_start, z_in is taken as zero and A is not touched.
__global__ __launch_bounds__(kBlock) void k_sweep64(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const double *__restrict__ a,
                                                    const double *__restrict__ dinv,
                                                    const double *__restrict__ v,
                                                    const double *__restrict__ zin,
                                                    double *__restrict__ zout, int zero_start)
{
    const int i = xcd_row();
    if (i >= n) return;
    if (zero_start) {
        zout[i] = dinv[i] * v[i];
        return;
    }
    zout[i] = zin[i] + dinv[i] * (v[i] - row_dot(i, rp, ci, a, zin));
}

// FP32 smoother: matrix values, diagonal and the residual arithmetic in FP32
__global__ __launch_bounds__(kBlock) void k_sweep32(int n, const int *__restrict__ rp,
                                                    const int *__restrict__ ci,
                                                    const float *__restrict__ a,
                                                    const float *__restrict__ dinv,
                                                    const double *__restrict__ v,
                                                    const double *__restrict__ zin,
                                                    double *__restrict__ zout, int zero_start)
{
    const int i = xcd_row();
    if (i >= n) return;
    if (zero_start) {
        zout[i] = static_cast<double>(dinv[i] * static_cast<float>(v[i]));
        return;
    }
    float s = 0.0f;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += a[e] * static_cast<float>(zin[ci[e]]);
    zout[i] = zin[i] + static_cast<double>(dinv[i] * (static_cast<float>(v[i]) - s));
}

// v_c = R x with R = P^T stored by coarse rows (padded to 64-entry groups,
// pads of value 0): one work-group per coarse row (neighbouring coarse rows,
// which share fine rows, on one XCD).  With R16 the columns are read as
// 16-bit offsets from the group's base (a wavefront's 64 entries share one
// group).  A step takes U entries per lane, all of them loaded (positions
// beyond the row end re-read its last entry and are skipped) before their x
// values are gathered, so a coarse row of up to U kBlock entries costs two
// round trips; the launch takes the smallest U that covers the longest row.
// Each lane sums its entries (lane, lane + kBlock, ...) in ascending order
// whatever U is, then a fixed butterfly and wavefront order combine the
// lanes, so the result is reproducible and does not depend on U.
template <typename T, typename XT, bool R16, int U>
__global__ __launch_bounds__(kBlock) void k_restrict_b(int nc, const int *__restrict__ rrp,
                                                       const int *__restrict__ rci,
                                                       const uint16_t *__restrict__ roff,
                                                       const int *__restrict__ rbase,
                                                       const T *__restrict__ rv,
                                                       const XT *__restrict__ x,
                                                       double *__restrict__ xc)
{
    const int j = xcd_group(blockIdx.x, gridDim.x);
    if (j >= nc) return;
    double s = 0.0;
    const int t1 = rrp[j + 1];
    for (int t = rrp[j] + threadIdx.x; t < t1; t += U * kBlock) {
        int c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(t + u * kBlock, t1 - 1);
            c[u] = R16 ? rbase[e >> 6] + static_cast<int>(roff[e]) : rci[e];
            v[u] = rv[e];
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = static_cast<double>(x[c[u]]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t + u * kBlock < t1) s += static_cast<double>(v[u]) * xv[u];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) xc[j] = s;
}

// v_c = R x when every support is a box of the grid: entry q of coarse row j
// (fine rows ascending) is box cell (q mod bx, (q div bx) mod by, q div bx by),
// so the columns follow from the box and a step's values and gathers are
// loaded together (one memory round trip instead of two).  The entries per
// lane and the summation order are those of k_restrict_b; its pads (value 0)
// are not visited.  q < 2^16, so the float quotients below are exact.
template <typename T, typename XT, int U>
__global__ __launch_bounds__(kBlock) void k_restrict_box(int nc, const int *__restrict__ rrp,
                                                         const int *__restrict__ box, int nx,
                                                         int nxy, const T *__restrict__ rv,
                                                         const XT *__restrict__ x,
                                                         double *__restrict__ xc)
{
    const int j = xcd_group(blockIdx.x, gridDim.x);
    if (j >= nc) return;
    const int r0 = rrp[j];
    const int org = box[4 * j], bx = box[4 * j + 1], bxy = box[4 * j + 2];
    const int t1 = r0 + box[4 * j + 3];
    const float ibx = 1.0f / static_cast<float>(bx), ibxy = 1.0f / static_cast<float>(bxy);
    double s = 0.0;
    for (int t = r0 + threadIdx.x; t < t1; t += U * kBlock) {
        T v[U];
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(t + u * kBlock, t1 - 1);
            const int q = e - r0;
            const int qz = static_cast<int>((static_cast<float>(q) + 0.5f) * ibxy);
            const int rem = q - qz * bxy;
            const int qy = static_cast<int>((static_cast<float>(rem) + 0.5f) * ibx);
            v[u] = rv[e];
            xv[u] = x[org + (rem - qy * bx) + qy * nx + qz * nxy];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t + u * kBlock < t1) s += static_cast<double>(v[u]) * static_cast<double>(xv[u]);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) xc[j] = s;
}

__global__ __launch_bounds__(kBlock) void k_dot(int n, const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                double *__restrict__ part)
{
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        s += x[i] * y[i];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_copy(int n, const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ __launch_bounds__(kBlock) void k_axpy(int n, double alpha, const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] += alpha * x[i];
}

// Jacobi diagonal inverse 1/a_ii, l1-Jacobi 1/sum_j |a_ij|, their FP32 copies
// and the FP32 copy of A's values
__global__ __launch_bounds__(kBlock) void k_diag_inverses(int n, const int *__restrict__ rp,
                                                          const int *__restrict__ ci,
                                                          const double *__restrict__ a,
                                                          double *__restrict__ dj,
                                                          double *__restrict__ dl1,
                                                          float *__restrict__ dj32,
                                                          float *__restrict__ dl1_32,
                                                          float *__restrict__ a32,
                                                          int *__restrict__ flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double d = 0.0, l1 = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        if (ci[e] == i) d = a[e];
        l1 += fabs(a[e]);
        if (a32) a32[e] = static_cast<float>(a[e]);
    }
    if (d == 0.0 || l1 == 0.0) flag[0] = 1;
    dj[i] = 1.0 / d;
    dl1[i] = 1.0 / l1;
    if (dj32) {
        dj32[i] = static_cast<float>(1.0 / d);
        dl1_32[i] = static_cast<float>(1.0 / l1);
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_values(int64_t m, const int *__restrict__ src,
                                                          const double *__restrict__ a,
                                                          double *__restrict__ out)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t < m) out[t] = a[src[t]];
}

// out[t] = V_t . w for t < k (block (b, t) computes the partial over chunk b)
__global__ __launch_bounds__(kBlock) void k_multi_dot(int n, const double *__restrict__ V,
                                                      int64_t ldv, const double *__restrict__ w,
                                                      double *__restrict__ part)
{
    const int t = blockIdx.y;
    const double *vt = V + static_cast<int64_t>(t) * ldv;
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        s += vt[i] * w[i];
    s = block_sum(s);
    if (threadIdx.x == 0) part[static_cast<int64_t>(t) * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_multi_dot_final(int nb, int k,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ out)
{
    const int t = blockIdx.x;
    if (t >= k) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += part[static_cast<int64_t>(t) * nb + b];
    s = block_sum(s);
    if (threadIdx.x == 0) out[t] = s;
}

// w += sign * sum_t h[t] V_t
__global__ __launch_bounds__(kBlock) void k_multi_axpy(int n, int k, const double *__restrict__ V,
                                                       int64_t ldv, const double *__restrict__ h,
                                                       double *__restrict__ w, double sign)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += h[t] * V[static_cast<int64_t>(t) * ldv + i];
    w[i] += sign * s;
}

__global__ __launch_bounds__(kBlock) void k_scale_by_inv(int n, const double *__restrict__ w,
                                                         const double *__restrict__ nrm2,
                                                         double *__restrict__ v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double nr = sqrt(nrm2[0]);
    v[i] = nr > 0.0 ? w[i] / nr : 0.0;
}

// ---------------------------------------------------------------------------
// DIA kernels: A stored as [noff][n] values on fixed column offsets; entries
// a row does not have are zero.  The kernels are instantiated for the
// diagonal counts of common stencils (ND > 0, a compile-time constant) so
// that all loads of a row are issued before the first product; ND == 0 takes
// the count at run time.  A neighbour outside [0, n) reads row i instead and
// the value is then replaced by zero.
//
// SYM: A is symmetric with symmetric offsets (off[o] = -off[ND-1-o]); the
// coefficient of a lower offset is read from the mirrored upper diagonal at
// the neighbour's row, A(i, i+off) = A(i+off, i), so only the diagonal and
// the upper diagonals stream from memory (the mirrored reads are rows that
// the same work-group or its XCD neighbours just loaded).
// ---------------------------------------------------------------------------
template <int ND, bool SYM, typename MT>
__device__ __forceinline__ MT dia_coef(const MT *__restrict__ a, int o, int i, int kk, int n)
{
    if constexpr (SYM) {
        if (o < ND / 2) return a[static_cast<int64_t>(ND - 1 - o) * n + kk];
    }
    return a[static_cast<int64_t>(o) * n + i];
}

template <int ND, bool SYM, typename MT, typename XT>
__device__ __forceinline__ MT dia_dot(int i, int n, const DiaOffsets &d,
                                      const MT *__restrict__ a, const XT *__restrict__ x)
{
    MT s = MT(0);
    if constexpr (ND > 0) {
        MT av[ND];
        double xv[ND];
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const int k = i + d.off[o];
            const bool in = k >= 0 && k < n;
            const int kk = in ? k : i;
            av[o] = dia_coef<ND, SYM>(a, o, i, kk, n);
            const double t = static_cast<double>(x[kk]);
            xv[o] = in ? t : 0.0;
        }
#pragma unroll
        for (int o = 0; o < ND; ++o) s += av[o] * static_cast<MT>(xv[o]);
    } else {
        for (int o = 0; o < d.n; ++o) {
            const int k = i + d.off[o];
            const MT av = a[static_cast<int64_t>(o) * n + i];
            const double xv = (k >= 0 && k < n) ? static_cast<double>(x[k]) : 0.0;
            s += av * static_cast<MT>(xv);
        }
    }
    return s;
}

// The work-group's rows are contiguous (xcd_row), so a neighbour row inside
// its kBlock-row tile (the +-1 offsets, and half the rows' +-nx) was loaded
// by another thread of the same work-group.  The tiled forms below share
// those values through LDS and load from memory only the neighbours outside
// the tile, all before one barrier.  Every thread of the work-group must
// call them (rows past n read row n - 1 and contribute nothing).
constexpr int kTileMaxDiag = 9;

template <int ND>
struct TileRows {
    int kk[ND];
    bool in[ND], loc[ND];
    __device__ __forceinline__ TileRows(int i, int ic, int t, int n, const DiaOffsets &d)
    {
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const int k = i + d.off[o];
            in[o] = k >= 0 && k < n;
            kk[o] = in[o] ? k : ic;
            const int tl = t + d.off[o];
            loc[o] = tl >= 0 && tl < kBlock;
        }
    }
};

// Row i's coefficients: its own diagonals' entries, and for a symmetric
// operator the lower ones as the neighbours' upper entries (from LDS inside
// the tile).  load() before the barrier, finish() after it.
template <int ND, bool SYM, typename MT>
struct TileCoefs {
    static constexpr int MID = ND / 2;
    MT av[ND];
    __device__ __forceinline__ void load(const MT *__restrict__ a, int n, int ic, int t,
                                         const TileRows<ND> &r, MT (*sa)[kBlock])
    {
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            if (!SYM || o >= MID)
                av[o] = a[static_cast<int64_t>(o) * n + ic];
            else if (!r.loc[o])
                av[o] = a[static_cast<int64_t>(ND - 1 - o) * n + r.kk[o]];
        }
        if constexpr (SYM) {
#pragma unroll
            for (int o = MID + 1; o < ND; ++o) sa[o - MID - 1][t] = av[o];
        }
    }
    __device__ __forceinline__ void finish(int t, const DiaOffsets &d, const TileRows<ND> &r,
                                           MT (*sa)[kBlock])
    {
        if constexpr (SYM) {
#pragma unroll
            for (int o = 0; o < MID; ++o)
                if (r.loc[o]) av[o] = sa[ND - 1 - o - MID - 1][t + d.off[o]];
        }
    }
};

// (sum over the stencil of a_io x_k) with the arithmetic of dia_dot, tiled
template <int ND, bool SYM, typename MT, typename XT>
__device__ __forceinline__ MT tile_dia_dot(int i, int n, const DiaOffsets &d,
                                           const MT *__restrict__ a, const XT *__restrict__ x)
{
    __shared__ XT sx[kBlock];
    __shared__ MT sa[SYM ? ND / 2 : 1][kBlock];
    const int t = threadIdx.x;
    const int ic = i < n ? i : n - 1;
    const TileRows<ND> r(i, ic, t, n, d);
    TileCoefs<ND, SYM, MT> c;
    c.load(a, n, ic, t, r, sa);
    XT xk[ND];
#pragma unroll
    for (int o = 0; o < ND; ++o)
        if (!r.loc[o]) xk[o] = x[r.kk[o]];
    sx[t] = x[ic];
    __syncthreads();
    c.finish(t, d, r, sa);
#pragma unroll
    for (int o = 0; o < ND; ++o)
        if (r.loc[o]) xk[o] = sx[t + d.off[o]];
    MT s = MT(0);
#pragma unroll
    for (int o = 0; o < ND; ++o) {
        const double xv = r.in[o] ? static_cast<double>(xk[o]) : 0.0;
        s += c.av[o] * static_cast<MT>(xv);
    }
    return s;
}

// Whether a stencil kernel gathering vector type XT takes the tiled form:
// the diagonal count is known at compile time and the vector is FP64.
// Measured at 128^3: the tiled form takes FP64 sweeps from 30 to 25 us,
// while FP32 gathers are cheap enough that the barrier and second phase make
// FP32 sweeps slower (12 -> 15 us).
template <int ND, typename XT>
constexpr bool kTiled = ND > 0 && ND <= kTileMaxDiag && sizeof(XT) == 8;

// r - alpha q of the PCG update, one rounding, the same in every kernel that
// forms it
__device__ __forceinline__ double pcg_residual(double r, double q, double alpha)
{
    return fma(-alpha, q, r);
}

// Per-block partial sums of NV values, stored at part[q * gridDim.x + block];
// a one-block finishing kernel then adds them in block order, so the total
// does not depend on scheduling.
template <int NV>
__device__ inline void block_partials(double (&v)[NV], double *__restrict__ part)
{
    __shared__ double sh[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double t = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) t += sh[q][w];
            part[static_cast<int64_t>(q) * gridDim.x + blockIdx.x] = t;
        }
    }
}

// sums of the NV partial arrays (nb partials each) in a fixed order, then the
// scalar update of the Krylov method; one block of kFinThreads threads
constexpr int kFinThreads = 1024;

// The block's sums of NV partial arrays of nb entries: array q starts at
// part + q * nb, or, for q = NV - 1 when last is given, at last.
template <int NV>
__device__ inline void sum_partials_block(int nb, const double *__restrict__ part, double (&tot)[NV],
                                          const double *__restrict__ last = nullptr)
{
    __shared__ double sh[NV][kFinThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double *src = (q == NV - 1 && last) ? last : part + static_cast<int64_t>(q) * nb;
        double x = 0.0;
#pragma unroll 8
        for (int b = threadIdx.x; b < nb; b += kFinThreads) x += src[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[q][wid] = x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) t += sh[q][w];
        tot[q] = t;
    }
}

// alpha = (r.z)_old / (p.q), breakdown on p.q <= 0 or non-finite values
__global__ __launch_bounds__(kFinThreads) void k_fin_alpha(int nb, const double *__restrict__ part,
                                                           double *__restrict__ scal)
{
    // the scalar read first, so that its load overlaps the partials' loads
    const double rz = scal[S_RZ_OLD];
    double t[1];
    sum_partials_block<1>(nb, part, t);
    if (threadIdx.x != 0) return;
    const double pq = t[0];
    scal[S_PQ] = pq;
    const bool bad = !(pq > 0.0) || !isfinite(pq) || !isfinite(rz);
    if (bad) scal[S_BREAK] = 1.0;
    scal[S_ALPHA] = bad ? 0.0 : rz / pq;
}

// flexible (Polak-Ribiere) beta = r.(z - z_old) / (r.z)_old from the
// partials [0, nb) of r.z and [nb, 2 nb) of r.(z - z_old).  With host_out
// (inside PCG) also r.r of the step's residual update, from the partials
// part_rr: written with the breakdown flag to a host mailbox (coherent
// pinned memory), the values first and then, after a system-scope fence,
// the iteration tag the host waits for.
__global__ __launch_bounds__(kFinThreads) void k_fin_beta(int nb, const double *__restrict__ part,
                                                          double *__restrict__ scal,
                                                          const double *__restrict__ part_rr,
                                                          double *__restrict__ host_out,
                                                          double tag)
{
    // the scalars read first, so that their loads overlap the partials' loads
    const double rz_old = scal[S_RZ_OLD], brk = scal[S_BREAK];
    // r.z, r.(z - z_old) and (inside PCG) r.r in one pass
    double t[3];
    sum_partials_block<3>(nb, part, t, host_out != nullptr ? part_rr : part);
    if (threadIdx.x != 0) return;
    scal[S_RZ] = t[0];
    scal[S_RZDIFF] = t[1];
    const double b = t[1] / rz_old;
    const bool bad = !isfinite(b);
    if (bad) scal[S_BREAK] = 1.0;
    scal[S_BETA] = bad ? 0.0 : b;
    scal[S_RZ_OLD] = t[0];
    if (host_out == nullptr) return;
    scal[S_RR] = t[2];
    host_out[0] = t[2];
    host_out[1] = bad ? 1.0 : brk;
    __threadfence_system();
    host_out[2] = tag;
}

// ---------------------------------------------------------------------------
// Node-block stencil (NBS) kernels: thread per row r = bs * node + l, the
// row's entries visited by node offset, then component (ascending columns,
// the CSR order); an offset that leaves the node range, or reaches a node that
// is no neighbour (a wrap at a grid line), has zero values.
// ---------------------------------------------------------------------------
template <int BS, typename MT>
__device__ __forceinline__ MT nbs_dot(int r, int n, const NodeStencil &ns,
                                      const MT *__restrict__ v, const double *__restrict__ x)
{
    const int node = r / BS;
    MT s = MT(0);
#pragma unroll 3
    for (int o = 0; o < ns.n; ++o) {
        const int nb = node + ns.off[o];
        const bool in = nb >= 0 && nb < ns.nn;
        const int base = (in ? nb : node) * BS;
        MT a[BS];
        double xv[BS];
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            a[l] = v[static_cast<int64_t>(o * BS + l) * n + r];
            xv[l] = x[base + l];
        }
#pragma unroll
        for (int l = 0; l < BS; ++l) s += in ? a[l] * static_cast<MT>(xv[l]) : MT(0);
    }
    return s;
}

template <int BS>
__global__ __launch_bounds__(kBlock) void k_nbs_spmv(int n, NodeStencil ns,
                                                     const double *__restrict__ v,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < n) y[r] = nbs_dot<BS, double>(r, n, ns, v, x);
}

template <int BS, typename MT>
__global__ __launch_bounds__(kBlock) void k_nbs_residual(int n, NodeStencil ns,
                                                         const MT *__restrict__ v,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ x,
                                                         double *__restrict__ res)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < n)
        res[r] = static_cast<double>(static_cast<MT>(f[r]) - nbs_dot<BS, MT>(r, n, ns, v, x));
}

// z_out = z_in + D^{-1} (v - A z_in) (Jacobi-type sweep), or D^{-1} v from zero
template <int BS, typename MT>
__global__ __launch_bounds__(kBlock) void k_nbs_sweep(int n, NodeStencil ns,
                                                      const MT *__restrict__ a,
                                                      const MT *__restrict__ dinv,
                                                      const double *__restrict__ vin,
                                                      const double *__restrict__ zin,
                                                      double *__restrict__ zout, int zero_start)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    if (zero_start) {
        zout[r] = static_cast<double>(dinv[r] * static_cast<MT>(vin[r]));
        return;
    }
    const MT s = nbs_dot<BS, MT>(r, n, ns, a, zin);
    zout[r] = zin[r] + static_cast<double>(dinv[r] * (static_cast<MT>(vin[r]) - s));
}

// p = z + beta p_old (p = z when beta = 0), q = A p, and the p.q partials
template <int BS>
__global__ __launch_bounds__(kBlock) void k_nbs_pcg_p_spmv(
    int n, NodeStencil ns, const double *__restrict__ v, const double *__restrict__ z,
    const double *__restrict__ pold, double *__restrict__ pnew, double *__restrict__ q,
    double *__restrict__ part, const double *__restrict__ scal)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    const double beta = scal[S_BETA];
    const bool restart = beta == 0.0;
    double pq[1] = {0.0};
    if (r < n) {
        const int node = r / BS;
        double s = 0.0;
#pragma unroll 3
        for (int o = 0; o < ns.n; ++o) {
            const int nb = node + ns.off[o];
            const bool in = nb >= 0 && nb < ns.nn;
            const int base = (in ? nb : node) * BS;
            double a[BS], pk[BS];
#pragma unroll
            for (int l = 0; l < BS; ++l) {
                a[l] = v[static_cast<int64_t>(o * BS + l) * n + r];
                pk[l] = restart ? z[base + l] : z[base + l] + beta * pold[base + l];
            }
#pragma unroll
            for (int l = 0; l < BS; ++l) s += in ? a[l] * pk[l] : 0.0;
        }
        const double pr = restart ? z[r] : z[r] + beta * pold[r];
        pnew[r] = pr;
        q[r] = s;
        pq[0] = pr * s;
    }
    block_partials<1>(pq, part);
}

// The same in two passes, for operators whose rows gather many columns:
// p = z + beta p_old once per row, then q = A p with the p.q partials, so
// each of a row's columns is gathered from one vector instead of two (at
// 81 columns per row that halves the gathered bytes).  Same arithmetic and
// order as k_nbs_pcg_p_spmv.
__global__ __launch_bounds__(kBlock) void k_p_update(int n, const double *__restrict__ z,
                                                     const double *__restrict__ pold,
                                                     double *__restrict__ pnew,
                                                     const double *__restrict__ scal)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    const double beta = scal[S_BETA];
    pnew[r] = beta == 0.0 ? z[r] : z[r] + beta * pold[r];
}

template <int BS>
__global__ __launch_bounds__(kBlock) void k_nbs_spmv_dot(int n, NodeStencil ns,
                                                         const double *__restrict__ v,
                                                         const double *__restrict__ p,
                                                         double *__restrict__ q,
                                                         double *__restrict__ part)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    double pq[1] = {0.0};
    if (r < n) {
        const double s = nbs_dot<BS, double>(r, n, ns, v, p);
        q[r] = s;
        pq[0] = p[r] * s;
    }
    block_partials<1>(pq, part);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_to_nbs(int n, int nslot,
                                                       const int *__restrict__ rp,
                                                       const int8_t *__restrict__ slot,
                                                       const double *__restrict__ a,
                                                       T *__restrict__ v)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    for (int t = 0; t < nslot; ++t) v[static_cast<int64_t>(t) * n + r] = T(0);
    for (int e = rp[r]; e < rp[r + 1]; ++e)
        v[static_cast<int64_t>(slot[e]) * n + r] = static_cast<T>(a[e]);
}

template <int ND, bool SYM>
__global__ __launch_bounds__(kBlock) void k_dia_spmv(int n, DiaOffsets d,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y)
{
    const int i = xcd_row();
    if (i < n) y[i] = dia_dot<ND, SYM>(i, n, d, a, x);
}

// r = f - A x; with MT = float the matrix values and the products are FP32
// (the residual inside the preconditioner of the precision form)
template <int ND, bool SYM, typename MT, typename XT = double, typename RT = double>
__global__ __launch_bounds__(kBlock) void k_dia_residual(int n, DiaOffsets d,
                                                         const MT *__restrict__ a,
                                                         const double *__restrict__ f,
                                                         const XT *__restrict__ x,
                                                         RT *__restrict__ r)
{
    const int i = xcd_row();
    if (i < n) r[i] = static_cast<RT>(f[i] - static_cast<double>(dia_dot<ND, SYM>(i, n, d, a, x)));
}

// z_out = z_in + dinv (v - A z_in), smoother matrix and arithmetic in MT
template <int ND, bool SYM, typename MT, typename ZT = double>
__global__ __launch_bounds__(kBlock) void k_dia_sweep(int n, DiaOffsets d, const MT *__restrict__ a,
                                                      const MT *__restrict__ dinv,
                                                      const double *__restrict__ v,
                                                      const ZT *__restrict__ zin,
                                                      ZT *__restrict__ zout)
{
    const int i = xcd_row();
    if constexpr (kTiled<ND, ZT>) {
        const int ic = i < n ? i : n - 1;
        const double vi = v[ic];
        const MT di = dinv[ic];
        const ZT zi = zin[ic];
        const MT dot = tile_dia_dot<ND, SYM>(i, n, d, a, zin);
        if (i >= n) return;
        const MT res = static_cast<MT>(vi) - dot;
        zout[i] = static_cast<ZT>(static_cast<double>(zi) + static_cast<double>(di * res));
    } else {
        if (i >= n) return;
        const MT res = static_cast<MT>(v[i]) - dia_dot<ND, SYM>(i, n, d, a, zin);
        zout[i] = static_cast<ZT>(static_cast<double>(zin[i]) + static_cast<double>(dinv[i] * res));
    }
}

// two sweeps from z = 0: z1 = dinv v, z2 = z1 + dinv (v - A z1), with z1 of
// the neighbours recomputed on the fly
template <int ND, bool SYM, typename MT, typename ZT = double>
__global__ __launch_bounds__(kBlock) void k_dia_sweep2_zero(int n, DiaOffsets d,
                                                            const MT *__restrict__ a,
                                                            const MT *__restrict__ dinv,
                                                            const double *__restrict__ v,
                                                            ZT *__restrict__ zout)
{
    const int i = xcd_row();
    if constexpr (kTiled<ND, double>) {
        // tiled (see TileRows): the neighbours' z1 = dinv v from LDS inside
        // the tile, formed from memory outside it
        __shared__ MT sz1[kBlock];
        __shared__ MT sa[SYM ? ND / 2 : 1][kBlock];
        const int t = threadIdx.x;
        const int ic = i < n ? i : n - 1;
        const TileRows<ND> r(i, ic, t, n, d);
        TileCoefs<ND, SYM, MT> c;
        c.load(a, n, ic, t, r, sa);
        MT dk[ND];
        double vk[ND];
#pragma unroll
        for (int o = 0; o < ND; ++o)
            if (!r.loc[o]) {
                dk[o] = dinv[r.kk[o]];
                vk[o] = v[r.kk[o]];
            }
        const double vi = v[ic];
        const MT di = dinv[ic];
        sz1[t] = static_cast<MT>(static_cast<double>(di * static_cast<MT>(vi)));
        __syncthreads();
        c.finish(t, d, r, sa);
        MT s = MT(0);
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const MT z1 = r.loc[o] ? sz1[t + d.off[o]]
                                   : static_cast<MT>(static_cast<double>(dk[o] * static_cast<MT>(vk[o])));
            s += c.av[o] * (r.in[o] ? z1 : MT(0));
        }
        if (i >= n) return;
        const double z1i = static_cast<double>(di * static_cast<MT>(vi));
        zout[i] = static_cast<ZT>(z1i + static_cast<double>(di * (static_cast<MT>(vi) - s)));
        return;
    }
    if (i >= n) return;
    MT s = MT(0);
    if constexpr (ND > 0) {
        MT av[ND], dk[ND];
        double vk[ND];
        bool in[ND];
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const int k = i + d.off[o];
            in[o] = k >= 0 && k < n;
            const int kk = in[o] ? k : i;
            av[o] = dia_coef<ND, SYM>(a, o, i, kk, n);
            dk[o] = dinv[kk];
            vk[o] = v[kk];
        }
#pragma unroll
        for (int o = 0; o < ND; ++o) {
            const MT z1 = static_cast<MT>(static_cast<double>(dk[o] * static_cast<MT>(vk[o])));
            s += av[o] * (in[o] ? z1 : MT(0));
        }
    } else {
        for (int o = 0; o < d.n; ++o) {
            const int k = i + d.off[o];
            const MT av = a[static_cast<int64_t>(o) * n + i];
            MT z1 = MT(0);
            if (k >= 0 && k < n)
                z1 = static_cast<MT>(static_cast<double>(dinv[k] * static_cast<MT>(v[k])));
            s += av * z1;
        }
    }
    const double z1i = static_cast<double>(dinv[i] * static_cast<MT>(v[i]));
    zout[i] = static_cast<ZT>(z1i + static_cast<double>(dinv[i] * (static_cast<MT>(v[i]) - s)));
}

// The PCG update x += alpha p, r_out = r_in - alpha q with the r.r partials,
// fused with the two sweeps from zero above (tiled form) that read the
// updated residual: a row's own r_out goes through LDS as z1 = dinv r_out,
// and outside the tile r_in and q are read and the update formed on the spot.
// r_out must not alias r_in (other work-groups still read r_in).
template <int ND, bool SYM, typename MT, typename ZT>
__global__ __launch_bounds__(kBlock) void k_pcg_update_sweep2(int n, DiaOffsets d,
                                                              const MT *__restrict__ a,
                                                              const MT *__restrict__ dinv,
                                                              ZT *__restrict__ zout, UpdArgs u)
{
    __shared__ MT sz1[kBlock];
    __shared__ MT sa[SYM ? ND / 2 : 1][kBlock];
    const int i = xcd_row();
    const int t = threadIdx.x;
    const int ic = i < n ? i : n - 1;
    const double alpha = u.scal[S_ALPHA];
    const TileRows<ND> r(i, ic, t, n, d);
    TileCoefs<ND, SYM, MT> c;
    c.load(a, n, ic, t, r, sa);
    MT dk[ND];
    double vk[ND], qk[ND];
#pragma unroll
    for (int o = 0; o < ND; ++o)
        if (!r.loc[o]) {
            dk[o] = dinv[r.kk[o]];
            vk[o] = u.rin[r.kk[o]];
            qk[o] = u.q[r.kk[o]];
        }
    const double xi = u.x[ic], pi = u.p[ic];
    const double vi = pcg_residual(u.rin[ic], u.q[ic], alpha);
    const MT di = dinv[ic];
    sz1[t] = static_cast<MT>(static_cast<double>(di * static_cast<MT>(vi)));
    __syncthreads();
    c.finish(t, d, r, sa);
    MT s = MT(0);
#pragma unroll
    for (int o = 0; o < ND; ++o) {
        MT z1;
        if (r.loc[o]) {
            z1 = sz1[t + d.off[o]];
        } else {
            const double vo = pcg_residual(vk[o], qk[o], alpha);
            z1 = static_cast<MT>(static_cast<double>(dk[o] * static_cast<MT>(vo)));
        }
        s += c.av[o] * (r.in[o] ? z1 : MT(0));
    }
    double rr[1] = {0.0};
    if (i < n) {
        const double z1i = static_cast<double>(di * static_cast<MT>(vi));
        zout[i] = static_cast<ZT>(z1i + static_cast<double>(di * (static_cast<MT>(vi) - s)));
        u.x[i] = fma(alpha, pi, xi);
        u.rout[i] = vi;
        rr[0] = vi * vi;
    }
    block_partials<1>(rr, u.part);
}

// last smoothing sweep of the preconditioner inside PCG, fused with the dot
// products r.z and r.(z - z_old) and the flexible beta
template <int ND, bool SYM, typename MT, typename ZT = double>
__global__ __launch_bounds__(kBlock) void k_dia_sweep_dots(
    int n, DiaOffsets d, const MT *__restrict__ a, const MT *__restrict__ dinv,
    const double *__restrict__ r, const ZT *__restrict__ zin, double *__restrict__ zout,
    const double *__restrict__ zold, double *__restrict__ part)
{
    const int i = xcd_row();
    double v[2] = {0.0, 0.0};
    if constexpr (kTiled<ND, ZT>) {
        const int ic = i < n ? i : n - 1;
        const double ri = r[ic], zo = zold[ic];
        const MT di = dinv[ic];
        const ZT zi = zin[ic];
        const MT dot = tile_dia_dot<ND, SYM>(i, n, d, a, zin);
        if (i < n) {
            const MT res = static_cast<MT>(ri) - dot;
            const double z = static_cast<double>(zi) + static_cast<double>(di * res);
            zout[i] = z;
            v[0] = ri * z;
            v[1] = ri * (z - zo);
        }
    } else if (i < n) {
        const MT res = static_cast<MT>(r[i]) - dia_dot<ND, SYM>(i, n, d, a, zin);
        const double z = static_cast<double>(zin[i]) + static_cast<double>(dinv[i] * res);
        zout[i] = z;
        v[0] = r[i] * z;
        v[1] = r[i] * (z - zold[i]);
    }
    block_partials<2>(v, part);
}

// r.z and r.(z - z_old) with the flexible beta (when the last stage of the
// preconditioner is not a fused DIA sweep)
__global__ __launch_bounds__(kBlock) void k_dots_beta(int n, const double *__restrict__ r,
                                                      const double *__restrict__ z,
                                                      const double *__restrict__ zold,
                                                      double *__restrict__ part)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < n) {
        v[0] = r[i] * z[i];
        v[1] = r[i] * (z[i] - zold[i]);
    }
    block_partials<2>(v, part);
}

// p_new = z + beta p_old, q = A p_new, p_new.q and alpha = (r.z) / (p.q).
// DIA: ND and SYM as in dia_dot; ND < 0 is the CSR form.  beta == 0 (a
// restart) never reads p_old.
template <int ND, bool SYM>
__global__ __launch_bounds__(kBlock) void k_pcg_p_spmv(
    int n, DiaOffsets d, const double *__restrict__ ad, const int *__restrict__ rp,
    const int *__restrict__ ci, const double *__restrict__ a, const double *__restrict__ z,
    const double *__restrict__ pold, double *__restrict__ pnew, double *__restrict__ q,
    double *__restrict__ part, const double *__restrict__ scal)
{
    const int i = xcd_row();
    const double beta = scal[S_BETA];
    const bool restart = beta == 0.0;
    double v[1] = {0.0};
    if (i < n) {
        double s = 0.0;
        if constexpr (ND > 0) {
            double av[ND], pk[ND];
            bool in[ND];
            int kk[ND];
#pragma unroll
            for (int o = 0; o < ND; ++o) {
                const int k = i + d.off[o];
                in[o] = k >= 0 && k < n;
                kk[o] = in[o] ? k : i;
                av[o] = dia_coef<ND, SYM>(ad, o, i, kk[o], n);
            }
            if (restart) {
#pragma unroll
                for (int o = 0; o < ND; ++o) pk[o] = z[kk[o]];
            } else {
                double po[ND];
#pragma unroll
                for (int o = 0; o < ND; ++o) {
                    pk[o] = z[kk[o]];
                    po[o] = pold[kk[o]];
                }
                // keep all loads ahead of the arithmetic (one round trip)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int o = 0; o < ND; ++o) pk[o] += beta * po[o];
            }
#pragma unroll
            for (int o = 0; o < ND; ++o) s += av[o] * (in[o] ? pk[o] : 0.0);
            // p_new at row i is the zero offset's entry (no second round trip)
            double pc = pk[0];
#pragma unroll
            for (int o = 1; o < ND; ++o)
                if (d.off[o] == 0) pc = pk[o];
            pnew[i] = pc;
            q[i] = s;
            v[0] = pc * s;
        } else if constexpr (ND == 0) {
            for (int o = 0; o < d.n; ++o) {
                const int k = i + d.off[o];
                const double av = ad[static_cast<int64_t>(o) * n + i];
                double pk = 0.0;
                if (k >= 0 && k < n) pk = restart ? z[k] : z[k] + beta * pold[k];
                s += av * pk;
            }
        } else {
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const int k = ci[e];
                s += a[e] * (restart ? z[k] : z[k] + beta * pold[k]);
            }
        }
        if constexpr (ND <= 0) {
            const double pi = restart ? z[i] : z[i] + beta * pold[i];
            pnew[i] = pi;
            q[i] = s;
            v[0] = pi * s;
        }
    }
    block_partials<1>(v, part);
}

// The DIA form of the kernel above with the work-group's own rows shared
// through LDS: every thread loads z, p_old and (SYM) its upper coefficients
// at its own row, and a neighbour inside the work-group's kBlock rows (the
// +-1 offsets, and half the rows' +-nx) is read from LDS; only neighbours
// outside the tile (+-nx ny, the other half of +-nx, the tile-edge +-1) are
// loaded from memory, all before the barrier.  Rows of a work-group are
// contiguous (xcd_row).  Same arithmetic and order as the kernel above.
template <int ND, bool SYM>
__global__ __launch_bounds__(kBlock) void k_pcg_p_spmv_dia(
    int n, DiaOffsets d, const double *__restrict__ ad, const double *__restrict__ z,
    const double *__restrict__ pold, double *__restrict__ pnew, double *__restrict__ q,
    double *__restrict__ part, const double *__restrict__ scal)
{
    constexpr int MID = ND / 2;  // the zero offset of a symmetric offset set
    __shared__ double sz[kBlock], sp[kBlock];
    __shared__ double sa[SYM ? MID : 1][kBlock];
    const int t = threadIdx.x;
    const int i = xcd_row();
    const int ic = i < n ? i : n - 1;
    const double beta = scal[S_BETA];
    const bool restart = beta == 0.0;
    double av[ND], zk[ND], pk[ND];
    bool in[ND], loc[ND];
#pragma unroll
    for (int o = 0; o < ND; ++o) {
        const int k = i + d.off[o];
        in[o] = k >= 0 && k < n;
        const int kk = in[o] ? k : ic;
        const int tl = t + d.off[o];
        loc[o] = tl >= 0 && tl < kBlock;
        if (!SYM || o >= MID)
            av[o] = ad[static_cast<int64_t>(o) * n + ic];
        if (!loc[o]) {
            zk[o] = z[kk];
            pk[o] = restart ? 0.0 : pold[kk];
            if (SYM && o < MID) av[o] = ad[static_cast<int64_t>(ND - 1 - o) * n + kk];
        }
    }
    sz[t] = z[ic];
    sp[t] = restart ? 0.0 : pold[ic];
    if constexpr (SYM) {
#pragma unroll
        for (int o = MID + 1; o < ND; ++o) sa[o - MID - 1][t] = av[o];
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < ND; ++o) {
        if (loc[o]) {
            const int tl = t + d.off[o];
            zk[o] = sz[tl];
            pk[o] = sp[tl];
            if (SYM && o < MID) av[o] = sa[ND - 1 - o - MID - 1][tl];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int o = 0; o < ND; ++o) {
        const double pv = restart ? zk[o] : zk[o] + beta * pk[o];
        zk[o] = pv;
        s += av[o] * (in[o] ? pv : 0.0);
    }
    double v[1] = {0.0};
    if (i < n) {
        double pc = zk[0];
#pragma unroll
        for (int o = 1; o < ND; ++o)
            if (d.off[o] == 0) pc = zk[o];
        pnew[i] = pc;
        q[i] = s;
        v[0] = pc * s;
    }
    block_partials<1>(v, part);
}

// x += alpha p, r_out = r_in - alpha q, and r.r (out of place, as the fused
// form above)
__global__ __launch_bounds__(kBlock) void k_pcg_update(int n, double *__restrict__ x,
                                                       const double *__restrict__ rin,
                                                       double *__restrict__ rout,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ q,
                                                       double *__restrict__ part,
                                                       const double *__restrict__ scal)
{
    const double alpha = scal[S_ALPHA];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = pcg_residual(rin[i], q[i], alpha);
        rout[i] = ri;
        v[0] = ri * ri;
    }
    block_partials<1>(v, part);
}

// z (+)= P w_c with P in row-major ELL layout; a row's values are read with
// 16-byte loads and its coarse columns are 16-bit (0xFFFF marks padding)
template <typename T, int PW, typename ZT = double>
__global__ __launch_bounds__(kBlock) void k_prolong_ell(int n, const uint16_t *__restrict__ pcol,
                                                        const T *__restrict__ pv,
                                                        const double *__restrict__ wc,
                                                        ZT *__restrict__ z, int zero)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int col[PW];
    T val[PW];
    {
        typedef uint16_t cvec __attribute__((ext_vector_type(PW)));
        constexpr int L = 16 / sizeof(T);
        typedef T tvec __attribute__((ext_vector_type(L)));
        const cvec cs = *reinterpret_cast<const cvec *>(pcol + static_cast<int64_t>(i) * PW);
#pragma unroll
        for (int u = 0; u < PW; ++u) col[u] = cs[u] == 0xFFFFu ? -1 : static_cast<int>(cs[u]);
        const tvec *vs = reinterpret_cast<const tvec *>(pv + static_cast<int64_t>(i) * PW);
#pragma unroll
        for (int q = 0; q < PW / L; ++q) {
            const tvec v = vs[q];
#pragma unroll
            for (int u = 0; u < L; ++u) val[L * q + u] = v[u];
        }
    }
    // all gathers issued at once; padding slots read entry 0 and contribute
    // zero
    double g[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) g[q] = wc[col[q] >= 0 ? col[q] : 0];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < PW; ++q) s += col[q] >= 0 ? static_cast<double>(val[q]) * g[q] : 0.0;
    z[i] = static_cast<ZT>(zero ? s : static_cast<double>(z[i]) + s);
}

// The same product with the columns formed from the row's grid position
// (ProlongAxes) instead of loaded: the row's values are the only P data read.
// Slot u of the row is (ix, iy, iz) with ix fastest, as the ascending column
// order puts them; slots past cx cy cz are padding.
// SPLIT (PW 8): pv is P's split form (slots 0-3 of every row, then slots
// 4-7 of the 8-entry rows), located through ax.wtab.
template <typename T, int PW, typename ZT = double, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void k_prolong_axes(int n, ProlongAxes ax,
                                                         const T *__restrict__ pv,
                                                         const double *__restrict__ wc,
                                                         ZT *__restrict__ z, int zero)
{
    static_assert(!SPLIT || PW == 8, "the split form has 8-slot rows");
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const unsigned xy = static_cast<unsigned>(i) / static_cast<unsigned>(ax.nx);
    const int x = i - static_cast<int>(xy) * ax.nx;
    const unsigned zz = xy / static_cast<unsigned>(ax.ny);
    const int y = static_cast<int>(xy - zz * static_cast<unsigned>(ax.ny));
    int tx, ty, tz;
    T val[PW];
    constexpr int L = 16 / sizeof(T);
    typedef T tvec __attribute__((ext_vector_type(L)));
    if constexpr (SPLIT) {
        // the wavefront's entry of the per-64-row table (a scalar load): the
        // second-half index needs no per-row table load
        const int4 wt = ax.wtab[__builtin_amdgcn_readfirstlane(i >> 6)];
        const uint32_t lane = threadIdx.x & 63u;
        const uint64_t mask = static_cast<uint64_t>(static_cast<uint32_t>(wt.y)) |
                              (static_cast<uint64_t>(static_cast<uint32_t>(wt.z)) << 32);
        const bool f = (mask >> lane) & 1u;
        const int h = wt.x + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                 static_cast<uint32_t>(mask >> 32),
                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
        tx = ax.tab[x];
        ty = ax.tab[ax.nx + y];
        tz = ax.tab[ax.nx + ax.ny + zz];
        const tvec *lo = reinterpret_cast<const tvec *>(pv + static_cast<int64_t>(i) * 4);
#pragma unroll
        for (int q = 0; q < 4 / L; ++q) {
            const tvec v = lo[q];
#pragma unroll
            for (int u = 0; u < L; ++u) val[L * q + u] = v[u];
        }
        // a row with fewer than 8 entries uses slots 0-3 only: its buffer
        // load lies past the end and returns zeros without a memory access
        const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<T *>(pv + static_cast<int64_t>(n) * 4), 0,
            static_cast<int>(ax.n8 * 4 * static_cast<int64_t>(sizeof(T))), 0x00020000);
        const uint32_t off = f ? static_cast<uint32_t>(h) * (4 * sizeof(T)) : 0x80000000u;
#pragma unroll
        for (int q = 0; q < 4 / L; ++q) {
            const tvec v = __builtin_bit_cast(
                tvec, __builtin_amdgcn_raw_buffer_load_b128(rh, off + 16 * q, 0, 0));
#pragma unroll
            for (int u = 0; u < L; ++u) val[4 + L * q + u] = v[u];
        }
    } else {
        tx = ax.tab[x];
        ty = ax.tab[ax.nx + y];
        tz = ax.tab[ax.nx + ax.ny + zz];
        const tvec *vs = reinterpret_cast<const tvec *>(pv + static_cast<int64_t>(i) * PW);
#pragma unroll
        for (int q = 0; q < PW / L; ++q) {
            const tvec v = vs[q];
#pragma unroll
            for (int u = 0; u < L; ++u) val[L * q + u] = v[u];
        }
    }
    const int sx = (tx >> 16) - 1, sy = (ty >> 16) - 1;  // 0 or 1: shift of that axis
    const int cnt = (tx >> 16) * (ty >> 16) * (tz >> 16);
    const int base = (tx & 0xFFFF) + ax.ncx * (ty & 0xFFFF) + ax.ncxy * (tz & 0xFFFF);
    double g[PW];
#pragma unroll
    for (int u = 0; u < PW; ++u) {
        const int ix = u & sx, u1 = u >> sx;
        const int iy = u1 & sy, iz = u1 >> sy;
        g[u] = wc[u < cnt ? base + ix + ax.ncx * iy + ax.ncxy * iz : 0];
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < PW; ++u) s += u < cnt ? static_cast<double>(val[u]) * g[u] : 0.0;
    z[i] = static_cast<ZT>(zero ? s : static_cast<double>(z[i]) + s);
}

// generic width (rows wider than 8)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_ell_w(int n, int pw, const int *__restrict__ pcol,
                                                          const T *__restrict__ pv,
                                                          const double *__restrict__ wc,
                                                          double *__restrict__ z, int zero)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int q = 0; q < pw; ++q) {
        const int64_t e = static_cast<int64_t>(i) * pw + q;
        const int c = pcol[e];
        if (c < 0) break;
        s += static_cast<double>(pv[e]) * wc[c];
    }
    z[i] = zero ? s : z[i] + s;
}

// CSR -> DIA values (slot of every CSR entry precomputed), padding zeroed
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_to_dia(int n, int noff, const int *__restrict__ rp,
                                                       const int8_t *__restrict__ slot,
                                                       const double *__restrict__ a,
                                                       T *__restrict__ ad)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int o = 0; o < noff; ++o) ad[static_cast<int64_t>(o) * n + i] = T(0);
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        ad[static_cast<int64_t>(slot[e]) * n + i] = static_cast<T>(a[e]);
}

// flag[0] = 1 unless A_ij == A_ji for every stored entry (and the transposed
// entry exists)
__global__ __launch_bounds__(kBlock) void k_check_symmetric(int n, const int *__restrict__ rp,
                                                            const int *__restrict__ ci,
                                                            const double *__restrict__ a,
                                                            int *__restrict__ flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        int lo = rp[j], hi = rp[j + 1] - 1, found = -1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] == i) {
                found = mid;
                break;
            }
            if (ci[mid] < i) lo = mid + 1; else hi = mid - 1;
        }
        if (found < 0 || a[found] != a[e]) flag[0] = 1;
    }
}

}  // namespace

void launch_spmv(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                 const double *x, double *y)
{
    k_spmv<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a, x, y);
}

void launch_residual(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                     const double *f, const double *x, double *r)
{
    k_residual<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a, f, x, r);
}

void launch_sweep(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                  const float *a32, const double *dinv, const float *dinv32, bool fp32,
                  const double *v, const double *zin, double *zout, bool zero_start)
{
    if (fp32)
        k_sweep32<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a32, dinv32, v, zin, zout,
                                                 zero_start ? 1 : 0);
    else
        k_sweep64<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a, dinv, v, zin, zout,
                                                 zero_start ? 1 : 0);
}

// entries per lane and step of the restriction kernels: the smallest power
// of two (at most 16) whose step covers R's longest row (its pads included);
// an unknown length (0) takes 16
template <typename F>
static void with_restrict_unroll(int maxlen, F &&f)
{
    if (maxlen > 0 && maxlen <= kBlock)
        f(std::integral_constant<int, 1>{});
    else if (maxlen > 0 && maxlen <= 2 * kBlock)
        f(std::integral_constant<int, 2>{});
    else if (maxlen > 0 && maxlen <= 4 * kBlock)
        f(std::integral_constant<int, 4>{});
    else if (maxlen > 0 && maxlen <= 8 * kBlock)
        f(std::integral_constant<int, 8>{});
    else
        f(std::integral_constant<int, 16>{});
}

template <typename T, typename XT>
static void restrict_kernels(hipStream_t s, int nc, const int *rrp, const int *rci,
                             const uint16_t *roff16, const int *rbase, const T *rv, const XT *x,
                             double *xc, const RestrictBoxes &boxes)
{
    with_restrict_unroll(boxes.maxlen, [&](auto u) {
        constexpr int U = decltype(u)::value;
        if (boxes.box)
            k_restrict_box<T, XT, U><<<nc, kBlock, 0, s>>>(nc, rrp, boxes.box, boxes.nx, boxes.nxy,
                                                           rv, x, xc);
        else if (roff16)
            k_restrict_b<T, XT, true, U><<<nc, kBlock, 0, s>>>(nc, rrp, rci, roff16, rbase, rv, x,
                                                               xc);
        else
            k_restrict_b<T, XT, false, U><<<nc, kBlock, 0, s>>>(nc, rrp, rci, roff16, rbase, rv,
                                                                x, xc);
    });
}

void launch_restrict(hipStream_t s, int nc, const int *rrp, const int *rci,
                     const uint16_t *roff16, const int *rbase, bool fp32, const double *r64,
                     const float *r32, const double *x, double *xc, const RestrictBoxes &boxes)
{
    if (fp32)
        restrict_kernels<float, double>(s, nc, rrp, rci, roff16, rbase, r32, x, xc, boxes);
    else
        restrict_kernels<double, double>(s, nc, rrp, rci, roff16, rbase, r64, x, xc, boxes);
}

void launch_dot(hipStream_t s, int n, const double *x, const double *y, double *partials,
                double *out)
{
    const int nb = std::min(kReduceBlocks, std::max(1, grid_for(n)));
    k_dot<<<nb, kBlock, 0, s>>>(n, x, y, partials);
    finish(s, nb, partials, out);
}




void launch_copy(hipStream_t s, int n, const double *x, double *y)
{
    k_copy<<<grid_for(n), kBlock, 0, s>>>(n, x, y);
}

void launch_axpy(hipStream_t s, int n, double alpha, const double *x, double *y)
{
    k_axpy<<<grid_for(n), kBlock, 0, s>>>(n, alpha, x, y);
}

void launch_diag_inverses(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                          double *dj, double *dl1, float *dj32, float *dl1_32, float *a32,
                          int64_t nnz, int *flag)
{
    (void)nnz;
    k_diag_inverses<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a, dj, dl1, dj32, dl1_32, a32,
                                                   flag);
}

void launch_gather_values(hipStream_t s, int64_t m, const int *src, const double *a, double *out)
{
    if (m > 0) k_gather_values<<<grid_for(m), kBlock, 0, s>>>(m, src, a, out);
}

void launch_multi_dot(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                      const double *w, double *partials, double *out)
{
    const int nb = std::min(64, std::max(1, grid_for(n)));
    dim3 grid(nb, k);
    k_multi_dot<<<grid, kBlock, 0, s>>>(n, V, ldv, w, partials);
    k_multi_dot_final<<<k, kBlock, 0, s>>>(nb, k, partials, out);
}

void launch_multi_axpy(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                       const double *h, double *w, double sign)
{
    k_multi_axpy<<<grid_for(n), kBlock, 0, s>>>(n, k, V, ldv, h, w, sign);
}

void launch_norm_scale(hipStream_t s, int n, const double *w, double *vout, double *partials,
                       double *out_norm2)
{
    launch_dot(s, n, w, w, partials, out_norm2);
    k_scale_by_inv<<<grid_for(n), kBlock, 0, s>>>(n, w, out_norm2, vout);
}

// Calls f(std::integral_constant<int, ND>, std::bool_constant<SYM>): the
// diagonal counts of 1D, 2D and 3D point stencils and of the 9- and 27-point
// stencils get their own instantiation, anything else the run-time form
// (ND = 0, full storage).
template <int ND, typename F>
void with_sym(const DiaOffsets &d, F &&f)
{
    if (d.sym)
        f(std::integral_constant<int, ND>{}, std::true_type{});
    else
        f(std::integral_constant<int, ND>{}, std::false_type{});
}

template <typename F>
void with_ndiag(const DiaOffsets &d, F &&f)
{
    switch (d.n) {
    case 3: with_sym<3>(d, f); return;
    case 5: with_sym<5>(d, f); return;
    case 7: with_sym<7>(d, f); return;
    case 9: with_sym<9>(d, f); return;
    case 27: with_sym<27>(d, f); return;
    default: f(std::integral_constant<int, 0>{}, std::false_type{}); return;
    }
}

#define MSRSB_DIA_ARGS(nd, sym) decltype(nd)::value, decltype(sym)::value

void launch_dia_spmv(hipStream_t s, int n, const DiaOffsets &d, const double *a, const double *x,
                     double *y)
{
    with_ndiag(d, [&](auto nd, auto sym) {
        k_dia_spmv<MSRSB_DIA_ARGS(nd, sym)><<<grid_for(n), kBlock, 0, s>>>(n, d, a, x, y);
    });
}

void launch_dia_residual(hipStream_t s, int n, const DiaOffsets &d, const double *a,
                         const float *a32, const double *f, const double *x, double *r)
{
    with_ndiag(d, [&](auto nd, auto sym) {
        if (a32)
            k_dia_residual<MSRSB_DIA_ARGS(nd, sym), float><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a32, f, x, r);
        else
            k_dia_residual<MSRSB_DIA_ARGS(nd, sym), double><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a, f, x, r);
    });
}

void launch_dia_sweep(hipStream_t s, int n, const DiaOffsets &d, bool fp32, const double *a64,
                      const float *a32, const double *dinv64, const float *dinv32,
                      const double *v, const double *zin, double *zout, bool zero2,
                      const UpdArgs *upd)
{
    with_ndiag(d, [&](auto nd, auto sym) {
        constexpr int ND = decltype(nd)::value;
        if (zero2 && upd) {
            // v is upd->rout; the tiled stencils fuse the update, others
            // take it first on its own
            if constexpr (kTiled<ND, double>) {
                if (fp32)
                    k_pcg_update_sweep2<MSRSB_DIA_ARGS(nd, sym), float, double>
                        <<<grid_for(n), kBlock, 0, s>>>(n, d, a32, dinv32, zout, *upd);
                else
                    k_pcg_update_sweep2<MSRSB_DIA_ARGS(nd, sym), double, double>
                        <<<grid_for(n), kBlock, 0, s>>>(n, d, a64, dinv64, zout, *upd);
                return;
            }
            launch_pcg_update(s, n, *upd);
        }
        if (zero2) {
            if (fp32)
                k_dia_sweep2_zero<MSRSB_DIA_ARGS(nd, sym), float>
                    <<<grid_for(n), kBlock, 0, s>>>(n, d, a32, dinv32, v, zout);
            else
                k_dia_sweep2_zero<MSRSB_DIA_ARGS(nd, sym), double>
                    <<<grid_for(n), kBlock, 0, s>>>(n, d, a64, dinv64, v, zout);
        } else if (fp32) {
            k_dia_sweep<MSRSB_DIA_ARGS(nd, sym), float><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a32, dinv32, v, zin, zout);
        } else {
            k_dia_sweep<MSRSB_DIA_ARGS(nd, sym), double><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a64, dinv64, v, zin, zout);
        }
    });
}

void launch_dia_sweep_dots(hipStream_t s, int n, const DiaOffsets &d, bool fp32,
                           const double *a64, const float *a32, const double *dinv64,
                           const float *dinv32, const double *r, const double *zin, double *zout,
                           const double *zold, double *part, double *scal,
                           const double *part_rr, double *host_out, int tag)
{
    with_ndiag(d, [&](auto nd, auto sym) {
        if (fp32)
            k_dia_sweep_dots<MSRSB_DIA_ARGS(nd, sym), float><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a32, dinv32, r, zin, zout, zold, part);
        else
            k_dia_sweep_dots<MSRSB_DIA_ARGS(nd, sym), double><<<grid_for(n), kBlock, 0, s>>>(
                n, d, a64, dinv64, r, zin, zout, zold, part);
    });
    k_fin_beta<<<1, kFinThreads, 0, s>>>(grid_for(n), part, scal, part_rr, host_out, tag);
}

// The two-stage preconditioner of the precision form with FP32 intermediate
// vectors (stencil A, l1/point-Jacobi x2 pre and post, 4- or 8-wide P): the
// smoothing iterates, the residual fed to the restriction and the
// prolongation's output are FP32; the final sweep writes the FP64 z and the
// PCG dots.  _pre: z1 = two sweeps from zero, tmp = v - A z1, vc = R tmp.
void launch_prec_f32_pre(hipStream_t s, int n, const DiaOffsets &d, const float *a32,
                         const float *dinv32, const double *v, float *z1, float *tmp, int nc,
                         const int *rrp, const int *rci, const uint16_t *roff16,
                         const int *rbase, const float *r32, double *vc,
                         const RestrictBoxes &boxes, const UpdArgs *upd)
{
    with_ndiag(d, [&](auto nd, auto sym) {
        constexpr int ND = decltype(nd)::value;
        bool fused = false;
        if constexpr (kTiled<ND, double>) {
            if (upd) {
                k_pcg_update_sweep2<MSRSB_DIA_ARGS(nd, sym), float, float>
                    <<<grid_for(n), kBlock, 0, s>>>(n, d, a32, dinv32, z1, *upd);
                fused = true;
            }
        }
        if (!fused) {
            if (upd) launch_pcg_update(s, n, *upd);
            k_dia_sweep2_zero<MSRSB_DIA_ARGS(nd, sym), float, float>
                <<<grid_for(n), kBlock, 0, s>>>(n, d, a32, dinv32, v, z1);
        }
        k_dia_residual<MSRSB_DIA_ARGS(nd, sym), float, float, float>
            <<<grid_for(n), kBlock, 0, s>>>(n, d, a32, v, z1, tmp);
    });
    restrict_kernels<float, float>(s, nc, rrp, rci, roff16, rbase, r32, tmp, vc, boxes);
}

// _post: z1 += P wc, z2 = sweep(z1), z = sweep(z2) with r.z, r.(z - zold)
// and the flexible beta
void launch_prec_f32_post(hipStream_t s, int n, const DiaOffsets &d, const float *a32,
                          const float *dinv32, const double *v, float *z1, float *z2, int pw,
                          const uint16_t *pcol16, const float *p32, const double *wc,
                          double *zout, const double *zold, double *partials, double *scal,
                          const double *part_rr, double *host_out, int tag,
                          const ProlongAxes &axes)
{
    // (FP32 P is read in its padded rows: axes.wtab is not set for it)
    if (axes.tab && pw == 8)
        k_prolong_axes<float, 8, float><<<grid_for(n), kBlock, 0, s>>>(n, axes, p32, wc, z1, 0);
    else if (axes.tab)
        k_prolong_axes<float, 4, float><<<grid_for(n), kBlock, 0, s>>>(n, axes, p32, wc, z1, 0);
    else if (pw == 8)
        k_prolong_ell<float, 8, float><<<grid_for(n), kBlock, 0, s>>>(n, pcol16, p32, wc, z1, 0);
    else
        k_prolong_ell<float, 4, float><<<grid_for(n), kBlock, 0, s>>>(n, pcol16, p32, wc, z1, 0);
    with_ndiag(d, [&](auto nd, auto sym) {
        k_dia_sweep<MSRSB_DIA_ARGS(nd, sym), float, float><<<grid_for(n), kBlock, 0, s>>>(
            n, d, a32, dinv32, v, z1, z2);
        k_dia_sweep_dots<MSRSB_DIA_ARGS(nd, sym), float, float><<<grid_for(n), kBlock, 0, s>>>(
            n, d, a32, dinv32, v, z2, zout, zold, partials);
    });
    k_fin_beta<<<1, kFinThreads, 0, s>>>(grid_for(n), partials, scal, part_rr, host_out, tag);
}

void launch_dots_beta(hipStream_t s, int n, const double *r, const double *z, const double *zold,
                      double *part, double *scal, const double *part_rr, double *host_out,
                      int tag)
{
    k_dots_beta<<<grid_for(n), kBlock, 0, s>>>(n, r, z, zold, part);
    k_fin_beta<<<1, kFinThreads, 0, s>>>(grid_for(n), part, scal, part_rr, host_out, tag);
}

void launch_pcg_p_spmv(hipStream_t s, int n, const DiaOffsets &d, const double *ad,
                       const int *rp, const int *ci, const double *a, const double *z,
                       const double *pold, double *pnew, double *q, double *part, double *scal)
{
    if (d.n > 0)
        with_ndiag(d, [&](auto nd, auto sym) {
            constexpr int ND = decltype(nd)::value;
            if constexpr (ND > 0 && ND <= 9)
                k_pcg_p_spmv_dia<MSRSB_DIA_ARGS(nd, sym)><<<grid_for(n), kBlock, 0, s>>>(
                    n, d, ad, z, pold, pnew, q, part, scal);
            else
                k_pcg_p_spmv<MSRSB_DIA_ARGS(nd, sym)><<<grid_for(n), kBlock, 0, s>>>(
                    n, d, ad, rp, ci, a, z, pold, pnew, q, part, scal);
        });
    else
        k_pcg_p_spmv<-1, false><<<grid_for(n), kBlock, 0, s>>>(n, d, ad, rp, ci, a, z, pold, pnew,
                                                               q, part, scal);
    k_fin_alpha<<<1, kFinThreads, 0, s>>>(grid_for(n), part, scal);
}

void launch_pcg_update(hipStream_t s, int n, const UpdArgs &u)
{
    k_pcg_update<<<grid_for(n), kBlock, 0, s>>>(n, u.x, u.rin, u.rout, u.p, u.q, u.part, u.scal);
}

template <typename T>
void prolong_t(hipStream_t s, int n, int pw, const int *pcol, const uint16_t *pcol16, const T *pv,
               const double *wc, double *z, bool zero, const ProlongAxes &axes)
{
    if constexpr (std::is_same_v<T, double>) {
        // FP64 P in the split form
        if (axes.wtab && pw == 8) {
            k_prolong_axes<T, 8, double, true><<<grid_for(n), kBlock, 0, s>>>(n, axes, pv, wc, z,
                                                                              zero ? 1 : 0);
            return;
        }
    }
    if (axes.tab && pw == 4)
        k_prolong_axes<T, 4><<<grid_for(n), kBlock, 0, s>>>(n, axes, pv, wc, z, zero ? 1 : 0);
    else if (axes.tab && pw == 8)
        k_prolong_axes<T, 8><<<grid_for(n), kBlock, 0, s>>>(n, axes, pv, wc, z, zero ? 1 : 0);
    else if (pcol16 && pw == 4)
        k_prolong_ell<T, 4><<<grid_for(n), kBlock, 0, s>>>(n, pcol16, pv, wc, z, zero ? 1 : 0);
    else if (pcol16 && pw == 8)
        k_prolong_ell<T, 8><<<grid_for(n), kBlock, 0, s>>>(n, pcol16, pv, wc, z, zero ? 1 : 0);
    else
        k_prolong_ell_w<T><<<grid_for(n), kBlock, 0, s>>>(n, pw, pcol, pv, wc, z, zero ? 1 : 0);
}

void launch_prolong_ell(hipStream_t s, int n, int pw, const int *pcol, const uint16_t *pcol16,
                        bool fp32, const double *p64, const float *p32, const double *wc,
                        double *z, bool zero, const ProlongAxes &axes)
{
    if (fp32)
        prolong_t<float>(s, n, pw, pcol, pcol16, p32, wc, z, zero, axes);
    else
        prolong_t<double>(s, n, pw, pcol, pcol16, p64, wc, z, zero, axes);
}

void launch_csr_to_dia(hipStream_t s, int n, int noff, const int *rp, const int8_t *slot,
                       const double *a, double *ad64, float *ad32)
{
    if (ad32)
        k_csr_to_dia<float><<<grid_for(n), kBlock, 0, s>>>(n, noff, rp, slot, a, ad32);
    else
        k_csr_to_dia<double><<<grid_for(n), kBlock, 0, s>>>(n, noff, rp, slot, a, ad64);
}

void launch_check_symmetric(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                            int *flag)
{
    k_check_symmetric<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, a, flag);
}


// ---- node-block stencil launchers ----
template <typename F>
void with_bs(int bs, F &&f)
{
    if (bs == 2) f(std::integral_constant<int, 2>{});
    else f(std::integral_constant<int, 3>{});
}

void launch_csr_to_nbs(hipStream_t s, int n, int nslot, const int *rp, const int8_t *slot,
                       const double *a, double *v64, float *v32)
{
    if (v64) k_csr_to_nbs<double><<<grid_for(n), kBlock, 0, s>>>(n, nslot, rp, slot, a, v64);
    if (v32) k_csr_to_nbs<float><<<grid_for(n), kBlock, 0, s>>>(n, nslot, rp, slot, a, v32);
}

void launch_nbs_spmv(hipStream_t s, int n, const NodeStencil &ns, const double *v, const double *x,
                     double *y)
{
    with_bs(ns.bs, [&](auto b) {
        k_nbs_spmv<decltype(b)::value><<<grid_for(n), kBlock, 0, s>>>(n, ns, v, x, y);
    });
}

void launch_nbs_residual(hipStream_t s, int n, const NodeStencil &ns, const double *v,
                         const float *v32, const double *f, const double *x, double *r)
{
    with_bs(ns.bs, [&](auto b) {
        constexpr int BS = decltype(b)::value;
        if (v32)
            k_nbs_residual<BS, float><<<grid_for(n), kBlock, 0, s>>>(n, ns, v32, f, x, r);
        else
            k_nbs_residual<BS, double><<<grid_for(n), kBlock, 0, s>>>(n, ns, v, f, x, r);
    });
}

void launch_nbs_sweep(hipStream_t s, int n, const NodeStencil &ns, bool fp32, const double *v,
                      const float *v32, const double *dinv, const float *dinv32,
                      const double *vin, const double *zin, double *zout, bool zero_start)
{
    with_bs(ns.bs, [&](auto b) {
        constexpr int BS = decltype(b)::value;
        if (fp32)
            k_nbs_sweep<BS, float><<<grid_for(n), kBlock, 0, s>>>(n, ns, v32, dinv32, vin, zin,
                                                                  zout, zero_start ? 1 : 0);
        else
            k_nbs_sweep<BS, double><<<grid_for(n), kBlock, 0, s>>>(n, ns, v, dinv, vin, zin, zout,
                                                                   zero_start ? 1 : 0);
    });
}

void launch_nbs_pcg_p_spmv(hipStream_t s, int n, const NodeStencil &ns, const double *v,
                           const double *z, const double *pold, double *pnew, double *q,
                           double *part, double *scal)
{
    // two passes (k_p_update, k_nbs_spmv_dot): 157 -> 5 + 115 us per call on
    // the 3D Q1 operator at 824k rows
    k_p_update<<<grid_for(n), kBlock, 0, s>>>(n, z, pold, pnew, scal);
    with_bs(ns.bs, [&](auto b) {
        k_nbs_spmv_dot<decltype(b)::value><<<grid_for(n), kBlock, 0, s>>>(n, ns, v, pnew, q, part);
    });
    k_fin_alpha<<<1, kFinThreads, 0, s>>>(grid_for(n), part, scal);
}

}  // namespace msrsb
