// Krylov-level kernels: SpMV, smoother sweeps, restriction / prolongation
// (Alg. 3), deterministic two-stage reductions and the fused vector updates
// of PCG and GMRES.
#include "internal.h"

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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = row_dot(i, rp, ci, a, x);
}

__global__ __launch_bounds__(kBlock) void k_residual(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ f,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ r)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (zero_start) {
        zout[i] = static_cast<double>(dinv[i] * static_cast<float>(v[i]));
        return;
    }
    float s = 0.0f;
    for (int e = rp[i]; e < rp[i + 1]; ++e) s += a[e] * static_cast<float>(zin[ci[e]]);
    zout[i] = zin[i] + static_cast<double>(dinv[i] * (static_cast<float>(v[i]) - s));
}

// v_c = R x with R = P^T stored by coarse rows: one work-group per coarse row
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(int nc, const int *__restrict__ rrp,
                                                     const int *__restrict__ rci,
                                                     const T *__restrict__ rv,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ xc)
{
    const int j = blockIdx.x;
    double s = 0.0;
    for (int t = rrp[j] + threadIdx.x; t < rrp[j + 1]; t += kBlock)
        s += static_cast<double>(rv[t]) * x[rci[t]];
    s = block_sum(s);
    if (threadIdx.x == 0) xc[j] = s;
}

// z += P w_c
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int n, const int *__restrict__ prp,
                                                        const int *__restrict__ pci,
                                                        const T *__restrict__ pv,
                                                        const double *__restrict__ wc,
                                                        double *__restrict__ z)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = prp[i]; e < prp[i + 1]; ++e) s += static_cast<double>(pv[e]) * wc[pci[e]];
    z[i] += s;
}

__global__ __launch_bounds__(kBlock) void k_dot(int n, const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                double *__restrict__ part)
{
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += x[i] * y[i];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// r.z and r.(z - z_old) in one pass
__global__ __launch_bounds__(kBlock) void k_dot2(int n, const double *__restrict__ r,
                                                 const double *__restrict__ z,
                                                 const double *__restrict__ zo,
                                                 double *__restrict__ part)
{
    double s0 = 0.0, s1 = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        s0 += r[i] * z[i];
        s1 += r[i] * (z[i] - zo[i]);
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[kReduceBlocks + blockIdx.x] = s1;
    }
}

// q = A p and the partial sums of p.q
__global__ __launch_bounds__(kBlock) void k_spmv_dot(int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ p,
                                                     double *__restrict__ q,
                                                     double *__restrict__ part)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        const double qi = row_dot(i, rp, ci, a, p);
        q[i] = qi;
        s = p[i] * qi;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// alpha = r.z / p.q, with the breakdown flag for p.q <= 0 or non-finite values
__global__ void k_cg_alpha(double *scal)
{
    if (threadIdx.x != 0) return;
    const double pq = scal[S_PQ], rz = scal[S_RZ_OLD];
    const bool bad = !(pq > 0.0) || !isfinite(pq) || !isfinite(rz);
    if (bad) scal[S_BREAK] = 1.0;
    scal[S_ALPHA] = bad ? 0.0 : rz / pq;
}

// x += alpha p, r -= alpha q, partial sums of r.r
__global__ __launch_bounds__(kBlock) void k_cg_update(int n, double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ scal,
                                                      double *__restrict__ part)
{
    const double alpha = scal[S_ALPHA];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s = ri * ri;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// flexible (Polak-Ribiere) beta = r.(z - z_old) / (r.z)_old
__global__ void k_cg_beta(double *scal)
{
    if (threadIdx.x != 0) return;
    const double rzo = scal[S_RZ_OLD];
    const double b = scal[S_RZDIFF] / rzo;
    if (!isfinite(b)) scal[S_BREAK] = 1.0;
    scal[S_BETA] = isfinite(b) ? b : 0.0;
    scal[S_RZ_OLD] = scal[S_RZ];
}

__global__ __launch_bounds__(kBlock) void k_p_update(int n, double *__restrict__ p,
                                                     const double *__restrict__ z,
                                                     const double *__restrict__ scal)
{
    const double beta = scal[S_BETA];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(kBlock) void k_copy(int n, const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ __launch_bounds__(kBlock) void k_axpy(int n, double alpha, const double *__restrict__ x,
                                                 double *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
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
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
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
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += h[t] * V[static_cast<int64_t>(t) * ldv + i];
    w[i] += sign * s;
}

__global__ __launch_bounds__(kBlock) void k_scale_by_inv(int n, const double *__restrict__ w,
                                                         const double *__restrict__ nrm2,
                                                         double *__restrict__ v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nr = sqrt(nrm2[0]);
    v[i] = nr > 0.0 ? w[i] / nr : 0.0;
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

void launch_restrict(hipStream_t s, int nc, const int *rrp, const int *rci, bool fp32,
                     const double *r64, const float *r32, const double *x, double *xc)
{
    if (fp32)
        k_restrict<float><<<nc, kBlock, 0, s>>>(nc, rrp, rci, r32, x, xc);
    else
        k_restrict<double><<<nc, kBlock, 0, s>>>(nc, rrp, rci, r64, x, xc);
}

void launch_prolong_add(hipStream_t s, int n, const int *prp, const int *pci, bool fp32,
                        const double *p64, const float *p32, const double *wc, double *z)
{
    if (fp32)
        k_prolong_add<float><<<grid_for(n), kBlock, 0, s>>>(n, prp, pci, p32, wc, z);
    else
        k_prolong_add<double><<<grid_for(n), kBlock, 0, s>>>(n, prp, pci, p64, wc, z);
}

void launch_dot(hipStream_t s, int n, const double *x, const double *y, double *partials,
                double *out)
{
    const int nb = std::min(kReduceBlocks, std::max(1, grid_for(n)));
    k_dot<<<nb, kBlock, 0, s>>>(n, x, y, partials);
    finish(s, nb, partials, out);
}

void launch_dot2(hipStream_t s, int n, const double *r, const double *z, const double *zold,
                 double *partials, double *out_rz, double *out_rzdiff)
{
    const int nb = std::min(kReduceBlocks, std::max(1, grid_for(n)));
    k_dot2<<<nb, kBlock, 0, s>>>(n, r, z, zold, partials);
    finish(s, nb, partials, out_rz);
    finish(s, nb, partials + kReduceBlocks, out_rzdiff);
}

void launch_spmv_dot(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                     const double *p, double *q, double *partials, double *out_pq)
{
    const int nb = grid_for(n);
    k_spmv_dot<<<nb, kBlock, 0, s>>>(n, rp, ci, a, p, q, partials);
    finish(s, nb, partials, out_pq);
}

void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p,
                      const double *q, const double *scal, double *partials, double *out_rr)
{
    const int nb = grid_for(n);
    k_cg_update<<<nb, kBlock, 0, s>>>(n, x, r, p, q, scal, partials);
    finish(s, nb, partials, out_rr);
}

void launch_cg_alpha(hipStream_t s, double *scal) { k_cg_alpha<<<1, 64, 0, s>>>(scal); }
void launch_cg_beta(hipStream_t s, double *scal) { k_cg_beta<<<1, 64, 0, s>>>(scal); }

void launch_p_update(hipStream_t s, int n, double *p, const double *z, const double *scal)
{
    k_p_update<<<grid_for(n), kBlock, 0, s>>>(n, p, z, scal);
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

}  // namespace msrsb
