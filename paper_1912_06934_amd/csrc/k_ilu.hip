// ILU(0) smoother: incomplete LU on A's own pattern in natural order
// (the no-fill factorisation used as the second stage of the preconditioner,
// Sec. 3.2).  Rows are grouped into dependency levels of the lower (and upper)
// triangle; one work-group walks the levels in order with a barrier between
// them, so every row sees its finished predecessors and the result equals the
// sequential natural-order factorisation and substitutions.
#include <algorithm>

#include "internal.h"

namespace msrsb {
namespace {

constexpr int kIluThreads = 1024;

// IKJ elimination of the rows of one level after another
__global__ __launch_bounds__(kIluThreads) void k_ilu0_factor(
    int nlev, const int *__restrict__ lev_ptr, const int *__restrict__ lev_rows,
    const int *__restrict__ rp, const int *__restrict__ ci, const int *__restrict__ dpos,
    double *__restrict__ lu, int *__restrict__ flag)
{
    for (int l = 0; l < nlev; ++l) {
        for (int t = lev_ptr[l] + threadIdx.x; t < lev_ptr[l + 1]; t += kIluThreads) {
            const int i = lev_rows[t];
            const int e0 = rp[i], e1 = rp[i + 1];
            for (int e = e0; e < e1; ++e) {
                const int k = ci[e];
                if (k >= i) break;
                const double piv = lu[dpos[k]];
                if (piv == 0.0) flag[0] = 1;
                const double lik = lu[e] / piv;
                lu[e] = lik;
                // subtract lik * U_k* on row i's pattern (columns > k)
                int f = e + 1;
                for (int q = dpos[k] + 1; q < rp[k + 1]; ++q) {
                    const int col = ci[q];
                    while (f < e1 && ci[f] < col) ++f;
                    if (f < e1 && ci[f] == col) lu[f] -= lik * lu[q];
                }
            }
        }
        __syncthreads();
    }
}

// x <- L^{-1} x (unit lower), levels in order
__global__ __launch_bounds__(kIluThreads) void k_ilu0_lower(
    int nlev, const int *__restrict__ lev_ptr, const int *__restrict__ lev_rows,
    const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ lu,
    double *__restrict__ x)
{
    for (int l = 0; l < nlev; ++l) {
        for (int t = lev_ptr[l] + threadIdx.x; t < lev_ptr[l + 1]; t += kIluThreads) {
            const int i = lev_rows[t];
            double s = x[i];
            for (int e = rp[i]; e < rp[i + 1] && ci[e] < i; ++e) s -= lu[e] * x[ci[e]];
            x[i] = s;
        }
        __syncthreads();
    }
}

// x <- U^{-1} x, levels of the upper triangle (from the last row up)
__global__ __launch_bounds__(kIluThreads) void k_ilu0_upper(
    int nlev, const int *__restrict__ lev_ptr, const int *__restrict__ lev_rows,
    const int *__restrict__ rp, const int *__restrict__ ci, const int *__restrict__ dpos,
    const double *__restrict__ lu, double *__restrict__ x)
{
    for (int l = 0; l < nlev; ++l) {
        for (int t = lev_ptr[l] + threadIdx.x; t < lev_ptr[l + 1]; t += kIluThreads) {
            const int i = lev_rows[t];
            double s = x[i];
            for (int e = dpos[i] + 1; e < rp[i + 1]; ++e) s -= lu[e] * x[ci[e]];
            x[i] = s / lu[dpos[i]];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_copy_vals(int64_t m, const double *__restrict__ a,
                                                   double *__restrict__ b)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < m) b[t] = a[t];
}

__global__ __launch_bounds__(256) void k_add(int n, const double *__restrict__ x,
                                             double *__restrict__ z)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] += x[i];
}

// levels of the lower triangle: lev(i) = 1 + max lev(j) over j < i in row i
void levels(int n, const std::vector<int> &rp, const std::vector<int> &ci, bool lower,
            std::vector<int> &ptr, std::vector<int> &rows)
{
    std::vector<int> lev(n, 0);
    int maxl = 0;
    if (lower) {
        for (int i = 0; i < n; ++i) {
            int l = 0;
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (ci[e] < i) l = std::max(l, lev[ci[e]] + 1);
            lev[i] = l;
            maxl = std::max(maxl, l);
        }
    } else {
        for (int i = n - 1; i >= 0; --i) {
            int l = 0;
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (ci[e] > i) l = std::max(l, lev[ci[e]] + 1);
            lev[i] = l;
            maxl = std::max(maxl, l);
        }
    }
    ptr.assign(maxl + 2, 0);
    for (int i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int l = 0; l <= maxl; ++l) ptr[l + 1] += ptr[l];
    rows.resize(n);
    std::vector<int> pos(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[pos[lev[i]]++] = i;
}

}  // namespace

msrsb_status ilu0_setup(msrsb_ctx *c)
{
    hipStream_t s = c->stream;
    if (!c->ilu_lev_ptr) {
        std::vector<int> pl, rl, pu, ru;
        levels(c->n, c->h_rp, c->h_ci, true, pl, rl);
        levels(c->n, c->h_rp, c->h_ci, false, pu, ru);
        c->ilu_nlev_l = static_cast<int>(pl.size()) - 1;
        c->ilu_nlev_u = static_cast<int>(pu.size()) - 1;
        if (hipMalloc(&c->ilu_lev_ptr, pl.size() * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->ilu_lev_rows, rl.size() * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->ilu_lev_ptr_u, pu.size() * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->ilu_lev_rows_u, ru.size() * sizeof(int)) != hipSuccess)
            return MSRSB_E_NOMEM;
        hipMemcpy(c->ilu_lev_ptr, pl.data(), pl.size() * sizeof(int), hipMemcpyHostToDevice);
        hipMemcpy(c->ilu_lev_rows, rl.data(), rl.size() * sizeof(int), hipMemcpyHostToDevice);
        hipMemcpy(c->ilu_lev_ptr_u, pu.data(), pu.size() * sizeof(int), hipMemcpyHostToDevice);
        hipMemcpy(c->ilu_lev_rows_u, ru.data(), ru.size() * sizeof(int), hipMemcpyHostToDevice);
    }
    if (!c->ilu && hipMalloc(&c->ilu, c->nnz * sizeof(double)) != hipSuccess) return MSRSB_E_NOMEM;
    k_copy_vals<<<static_cast<int>((c->nnz + 255) / 256), 256, 0, s>>>(c->nnz, c->a, c->ilu);
    int *flag = c->dev_flag;
    hipMemsetAsync(flag, 0, sizeof(int), s);
    k_ilu0_factor<<<1, kIluThreads, 0, s>>>(c->ilu_nlev_l, c->ilu_lev_ptr, c->ilu_lev_rows, c->rp,
                                            c->ci, c->diag_pos, c->ilu, flag);
    int hflag = 0;
    hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return MSRSB_E_HIP;
    if (hflag) return MSRSB_E_COARSE_SINGULAR;
    c->ilu_valid = true;
    return MSRSB_OK;
}

// z += U^{-1} L^{-1} res   (res is overwritten)
void launch_ilu0_apply(msrsb_ctx *c, const double *res, double *z, double *tmp)
{
    hipStream_t s = c->stream;
    (void)tmp;
    double *x = const_cast<double *>(res);
    k_ilu0_lower<<<1, kIluThreads, 0, s>>>(c->ilu_nlev_l, c->ilu_lev_ptr, c->ilu_lev_rows, c->rp,
                                           c->ci, c->ilu, x);
    k_ilu0_upper<<<1, kIluThreads, 0, s>>>(c->ilu_nlev_u, c->ilu_lev_ptr_u, c->ilu_lev_rows_u,
                                           c->rp, c->ci, c->diag_pos, c->ilu, x);
    k_add<<<(c->n + 255) / 256, 256, 0, s>>>(c->n, x, z);
}

}  // namespace msrsb
