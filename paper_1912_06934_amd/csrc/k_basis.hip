// Basis construction kernels: filter + Jacobi operator, initial basis and the
// restricted smoothing iteration of enhanced MsRSB (Sec. 2.1, Sec. 3.1,
// Alg. 1).
#include "internal.h"

namespace msrsb {
namespace {

__device__ inline double wave_max(double v)
{
    // NaN-propagating max over the 64 lanes of a wavefront
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

// Filter (eq. negoffdiag) and zero-row-sum diagonal (eq. Dhat_zero_rowsum):
// per row, Dhat_ii = -sum_{j != i, same component} G_ij with
// G_ij = min(A_ij, 0) when filtering; then J = I - omega Dhat^{-1} Ghat, i.e.
// J_ii = 1 - omega, J_ij = -omega G_ij / Dhat_ii.  A row with Dhat_ii == 0 is
// frozen (J_i = e_i).  J's pattern is A's restricted to same-component
// entries (all of A's entries for scalar problems), in the same order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_filter_jacobi(
    int n, int bs, int filter, double omega, const int *__restrict__ rp,
    const int *__restrict__ ci, const double *__restrict__ a, const int *__restrict__ jrp,
    T *__restrict__ jv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e0 = rp[i], e1 = rp[i + 1];
    const int ic = i % bs;
    double d = 0.0;
    for (int e = e0; e < e1; ++e) {
        const int j = ci[e];
        if (j == i || j % bs != ic) continue;
        double g = a[e];
        if (filter && g > 0.0) g = 0.0;
        d -= g;
    }
    int out = jrp[i];
    for (int e = e0; e < e1; ++e) {
        const int j = ci[e];
        if (j % bs != ic) continue;
        double v;
        if (d == 0.0) {
            v = (j == i) ? 1.0 : 0.0;
        } else if (j == i) {
            v = 1.0 - omega;
        } else {
            double g = a[e];
            if (filter && g > 0.0) g = 0.0;
            v = -omega * g / d;
        }
        jv[out++] = static_cast<T>(v);
    }
}

// Initial basis (Sec. 2.1): characteristic function of the coarse block.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_basis(int n, const int *__restrict__ prp,
                                                       const int *__restrict__ pci,
                                                       const int *__restrict__ part,
                                                       T *__restrict__ p)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int pi = part[i];
    for (int e = prp[i]; e < prp[i + 1]; ++e) p[e] = (pci[e] == pi) ? T(1) : T(0);
}

// One restricted smoothing iteration (eq. smoother, Alg. 1).  One thread per
// fine row i holds row i's pattern (at most W coarse columns) in registers and
// accumulates T_ij = sum_k J_ik P_kj over the J-neighbours k in ascending
// order; entries of P_k* outside row i's pattern are dropped, which keeps
// every basis function inside its support.  The row is then rescaled by its
// FP64 sum so P stays a partition of unity, and |T - P_old| on interior rows
// feeds e_it (wavefront max, then one 64-bit atomic max per wavefront).
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_smooth(
    int n, const int *__restrict__ jrp, const int *__restrict__ jci, const T *__restrict__ jv,
    const int *__restrict__ prp, const int *__restrict__ pci, const T *__restrict__ pin,
    T *__restrict__ pout, const uint8_t *__restrict__ interior,
    unsigned long long *__restrict__ eit_bits)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double emax = 0.0;
    if (i < n) {
        const int p0 = prp[i];
        const int np = prp[i + 1] - p0;
        int col[W];
        T acc[W];
#pragma unroll
        for (int s = 0; s < W; ++s) {
            col[s] = (s < np) ? pci[p0 + s] : -1;
            acc[s] = T(0);
        }
        const int e1 = jrp[i + 1];
        for (int e = jrp[i]; e < e1; ++e) {
            const int k = jci[e];
            const T w = jv[e];
            const int q1 = prp[k + 1];
            for (int q = prp[k]; q < q1; ++q) {
                const int c = pci[q];
                const T wv = w * pin[q];
#pragma unroll
                for (int s = 0; s < W; ++s) acc[s] += (col[s] == c) ? wv : T(0);
            }
        }
        double rs = 0.0;
#pragma unroll
        for (int s = 0; s < W; ++s)
            if (s < np) rs += static_cast<double>(acc[s]);
        const bool inner = eit_bits != nullptr && interior[i] != 0;
#pragma unroll
        for (int s = 0; s < W; ++s) {
            if (s < np) {
                if (inner) {
                    const double dlt = fabs(static_cast<double>(acc[s]) -
                                            static_cast<double>(pin[p0 + s]));
                    emax = (dlt > emax || dlt != dlt) ? dlt : emax;
                }
                pout[p0 + s] = static_cast<T>(static_cast<double>(acc[s]) / rs);
            }
        }
    }
    if (eit_bits != nullptr) {
        emax = wave_max(emax);
        if ((threadIdx.x & 63) == 0 && emax != 0.0)
            atomicMax(eit_bits, static_cast<unsigned long long>(__double_as_longlong(emax)));
    }
}

// Partial statistics of P: max |row sum - 1|, min and max entry.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_basis_stats(int n, const int *__restrict__ prp,
                                                        const T *__restrict__ p,
                                                        double *__restrict__ partials)
{
    __shared__ double sh[3][kBlock];
    double err = 0.0, lo = 1e300, hi = -1e300;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int e = prp[i]; e < prp[i + 1]; ++e) {
            const double v = static_cast<double>(p[e]);
            s += v;
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
        const double d = fabs(s - 1.0);
        err = (d > err || d != d) ? d : err;
    }
    sh[0][threadIdx.x] = err;
    sh[1][threadIdx.x] = lo;
    sh[2][threadIdx.x] = hi;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = sh[0][threadIdx.x + st];
            sh[0][threadIdx.x] = (o > sh[0][threadIdx.x] || o != o) ? o : sh[0][threadIdx.x];
            sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + st]);
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = sh[0][0];
        partials[3 * blockIdx.x + 1] = sh[1][0];
        partials[3 * blockIdx.x + 2] = sh[2][0];
    }
}

__global__ void k_basis_stats_final(int nb, const double *__restrict__ partials,
                                    double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double err = 0.0, lo = 1e300, hi = -1e300;
    for (int b = 0; b < nb; ++b) {
        const double o = partials[3 * b];
        err = (o > err || o != o) ? o : err;
        lo = fmin(lo, partials[3 * b + 1]);
        hi = fmax(hi, partials[3 * b + 2]);
    }
    out[0] = err;
    out[1] = lo;
    out[2] = hi;
}

__global__ __launch_bounds__(kBlock) void k_f32_to_f64(int64_t m, const float *__restrict__ s,
                                                       double *__restrict__ d)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < m) d[t] = static_cast<double>(s[t]);
}

__global__ __launch_bounds__(kBlock) void k_f64_to_f32(int64_t m, const double *__restrict__ s,
                                                       float *__restrict__ d)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < m) d[t] = static_cast<float>(s[t]);
}

inline int grid_for(int64_t m) { return static_cast<int>((m + kBlock - 1) / kBlock); }

template <typename T, int W>
void smooth_w(hipStream_t s, int n, const int *jrp, const int *jci, const T *jv, const int *prp,
              const int *pci, const T *pin, T *pout, const uint8_t *interior,
              unsigned long long *eit)
{
    k_smooth<T, W><<<grid_for(n), kBlock, 0, s>>>(n, jrp, jci, jv, prp, pci, pin, pout, interior,
                                                   eit);
}

template <typename T>
void smooth_t(hipStream_t s, int n, int maxw, const int *jrp, const int *jci, const T *jv,
              const int *prp, const int *pci, const T *pin, T *pout, const uint8_t *interior,
              unsigned long long *eit)
{
    if (maxw <= 4)
        smooth_w<T, 4>(s, n, jrp, jci, jv, prp, pci, pin, pout, interior, eit);
    else if (maxw <= 8)
        smooth_w<T, 8>(s, n, jrp, jci, jv, prp, pci, pin, pout, interior, eit);
    else if (maxw <= 16)
        smooth_w<T, 16>(s, n, jrp, jci, jv, prp, pci, pin, pout, interior, eit);
    else
        smooth_w<T, 32>(s, n, jrp, jci, jv, prp, pci, pin, pout, interior, eit);
}

}  // namespace

void launch_filter_jacobi(hipStream_t s, int n, int bs, int filter, double omega, const int *rp,
                          const int *ci, const double *a, const int *jrp, double *jv64,
                          float *jv32)
{
    if (jv32)
        k_filter_jacobi<float><<<grid_for(n), kBlock, 0, s>>>(n, bs, filter, omega, rp, ci, a, jrp,
                                                              jv32);
    else
        k_filter_jacobi<double><<<grid_for(n), kBlock, 0, s>>>(n, bs, filter, omega, rp, ci, a,
                                                               jrp, jv64);
}

void launch_init_basis(hipStream_t s, int n, const int *prp, const int *pci, const int *part,
                       double *p64, float *p32)
{
    if (p32)
        k_init_basis<float><<<grid_for(n), kBlock, 0, s>>>(n, prp, pci, part, p32);
    else
        k_init_basis<double><<<grid_for(n), kBlock, 0, s>>>(n, prp, pci, part, p64);
}

void launch_smooth(hipStream_t s, int n, int maxw, bool fp32, const int *jrp, const int *jci,
                   const double *jv64, const float *jv32, const int *prp, const int *pci,
                   const double *pin64, double *pout64, const float *pin32, float *pout32,
                   const uint8_t *interior, unsigned long long *eit_bits)
{
    if (fp32)
        smooth_t<float>(s, n, maxw, jrp, jci, jv32, prp, pci, pin32, pout32, interior, eit_bits);
    else
        smooth_t<double>(s, n, maxw, jrp, jci, jv64, prp, pci, pin64, pout64, interior,
                         eit_bits);
}

void launch_basis_stats(hipStream_t s, int n, const int *prp, bool fp32, const double *p64,
                        const float *p32, double *partials, double *out3)
{
    const int nb = 256;
    if (fp32)
        k_basis_stats<float><<<nb, kBlock, 0, s>>>(n, prp, p32, partials);
    else
        k_basis_stats<double><<<nb, kBlock, 0, s>>>(n, prp, p64, partials);
    k_basis_stats_final<<<1, 64, 0, s>>>(nb, partials, out3);
}

void launch_p_convert(hipStream_t s, int64_t m, const float *src, double *dst)
{
    if (m > 0) k_f32_to_f64<<<grid_for(m), kBlock, 0, s>>>(m, src, dst);
}

void launch_p_convert_down(hipStream_t s, int64_t m, const double *src, float *dst)
{
    if (m > 0) k_f64_to_f32<<<grid_for(m), kBlock, 0, s>>>(m, src, dst);
}

}  // namespace msrsb
