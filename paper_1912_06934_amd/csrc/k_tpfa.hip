// Two-point flux approximation assembly on Cartesian grids (App. B.1) and the
// adjoint gradient with respect to log-permeability.
#include "internal.h"

namespace msrsb {
namespace {

struct Grid {
    int dim, nx, ny, nz;
    double h[3], area[3], bc[6];
};

__device__ inline double half_t(double k, const Grid &g, int d)
{
    return 2.0 * k * g.area[d] / g.h[d];
}

// One thread per cell: the row in ascending column order (z-, y-, x-,
// diagonal, x+, y+, z+ where the neighbour exists).  Interior faces use the
// series combination T = t_K t_L / (t_K + t_L) of the half-cell
// transmissibilities t = 2 k area / h; a Dirichlet face adds t_K to the
// diagonal and t_K g to the right-hand side.
__global__ __launch_bounds__(kBlock) void k_tpfa_values(Grid g, const double *__restrict__ logk,
                                                        const int *__restrict__ rp,
                                                        double *__restrict__ val,
                                                        double *__restrict__ rhs)
{
    const int n = g.nx * g.ny * g.nz;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int xyz[3] = {c % g.nx, (c / g.nx) % g.ny, c / (g.nx * g.ny)};
    const int nd[3] = {g.nx, g.ny, g.nz};
    const int stride[3] = {1, g.nx, g.nx * g.ny};
    const double kk = exp(logk[c]);
    double diag = 0.0, f = 0.0;
    int e = rp[c], dpos = -1;
    const int order_d[7] = {2, 1, 0, -1, 0, 1, 2};
    const int order_s[7] = {-1, -1, -1, 0, 1, 1, 1};
    for (int t = 0; t < 7; ++t) {
        const int d = order_d[t], s = order_s[t];
        if (d < 0) {
            dpos = e++;
            continue;
        }
        if (d >= g.dim) continue;
        const int nb = xyz[d] + s;
        if (nb < 0 || nb >= nd[d]) {
            const double gb = g.bc[2 * d + (s > 0 ? 1 : 0)];
            if (gb == gb) {
                const double tb = half_t(kk, g, d);
                diag += tb;
                f += tb * gb;
            }
            continue;
        }
        const int L = c + s * stride[d];
        const double tK = half_t(kk, g, d), tL = half_t(exp(logk[L]), g, d);
        const double T = tK * tL / (tK + tL);
        diag += T;
        val[e++] = -T;
    }
    val[dpos] = diag;
    if (rhs) rhs[c] = f;
}

// grad_K = -[ sum_faces T k_L/(k_K+k_L) (p_K-p_L)(lam_K-lam_L)
//             + sum_Dirichlet T_b (p_K - g_b) lam_K ]
__global__ __launch_bounds__(kBlock) void k_tpfa_grad(Grid g, const double *__restrict__ logk,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ lam,
                                                      double *__restrict__ grad)
{
    const int n = g.nx * g.ny * g.nz;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int xyz[3] = {c % g.nx, (c / g.nx) % g.ny, c / (g.nx * g.ny)};
    const int nd[3] = {g.nx, g.ny, g.nz};
    const int stride[3] = {1, g.nx, g.nx * g.ny};
    const double kk = exp(logk[c]);
    const double pc = p[c], lc = lam[c];
    double s = 0.0;
    for (int d = 0; d < g.dim; ++d) {
        for (int sg = -1; sg <= 1; sg += 2) {
            const int nb = xyz[d] + sg;
            if (nb < 0 || nb >= nd[d]) {
                const double gb = g.bc[2 * d + (sg > 0 ? 1 : 0)];
                if (gb == gb) s += half_t(kk, g, d) * (pc - gb) * lc;
                continue;
            }
            const int L = c + sg * stride[d];
            const double kl = exp(logk[L]);
            const double tK = half_t(kk, g, d), tL = half_t(kl, g, d);
            const double T = tK * tL / (tK + tL);
            s += T * kl / (kk + kl) * (pc - p[L]) * (lc - lam[L]);
        }
    }
    grad[c] = -s;
}

Grid make_grid(int dim, const int *dims, const double *h, const double *bc)
{
    Grid g;
    g.dim = dim;
    g.nx = dims[0];
    g.ny = dims[1];
    g.nz = dim == 3 ? dims[2] : 1;
    g.h[0] = h[0];
    g.h[1] = h[1];
    g.h[2] = dim == 3 ? h[2] : 1.0;
    if (dim == 3) {
        g.area[0] = g.h[1] * g.h[2];
        g.area[1] = g.h[0] * g.h[2];
        g.area[2] = g.h[0] * g.h[1];
    } else {
        g.area[0] = g.h[1];
        g.area[1] = g.h[0];
        g.area[2] = 1.0;
    }
    for (int t = 0; t < 6; ++t) g.bc[t] = bc[t];
    return g;
}

}  // namespace

void launch_tpfa_values(hipStream_t s, int dim, const int *dims, const double *h,
                        const double *bc, const double *logk, const int *rp, double *val,
                        double *rhs)
{
    const Grid g = make_grid(dim, dims, h, bc);
    const int n = g.nx * g.ny * g.nz;
    k_tpfa_values<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(g, logk, rp, val, rhs);
}

void launch_tpfa_grad(hipStream_t s, int dim, const int *dims, const double *h, const double *bc,
                      const double *logk, const double *p, const double *lam, double *grad)
{
    const Grid g = make_grid(dim, dims, h, bc);
    const int n = g.nx * g.ny * g.nz;
    k_tpfa_grad<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(g, logk, p, lam, grad);
}

}  // namespace msrsb
