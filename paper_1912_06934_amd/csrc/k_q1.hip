// Q1 (bi/trilinear) linear elasticity on a Cartesian grid of equal elements
// (App. "Linear elastostatics: Galerkin finite element formulation", eq.
// model_elastostatics_bilin_FE): the element stiffness, the matrix values as
// a function of log E (one Young's modulus per element), and the adjoint
// gradient with respect to log E, the vector-problem counterpart of the
// TPFA derivative (the paper itself has no adjoint).
//
// Numbering: nodes x + (nx+1) (y + (ny+1) z), dof = dim * node + l; local
// node q of an element has corner bits (q >> k) & 1 per axis k.  The matrix
// row of (node, l) lists the 3^dim neighbouring nodes in ascending index,
// dim components each (zeros kept).  Homogeneous Dirichlet dofs are handled
// by symmetric diagonalisation (Remark "FEM_Dir_BC"): their row and column
// are zero except for the diagonal.
#include <cmath>

#include "internal.h"

namespace msrsb {

void q1_element_stiffness(int dim, const double *h, double nu, double *K)
{
    const int nloc = 1 << dim, nd = dim * nloc;
    const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = 1.0 / (2.0 * (1.0 + nu));
    // stress-strain matrix in Voigt order (normal components, then shears)
    const int nv = dim == 2 ? 3 : 6;
    double D[6][6] = {};
    for (int a = 0; a < dim; ++a) {
        for (int b = 0; b < dim; ++b) D[a][b] = lam;
        D[a][a] += 2.0 * mu;
    }
    for (int a = dim; a < nv; ++a) D[a][a] = mu;
    const int sh2[1][2] = {{0, 1}};
    const int sh3[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    for (int t = 0; t < nd * nd; ++t) K[t] = 0.0;
    const double g = 1.0 / std::sqrt(3.0);
    double detJ = 1.0;
    for (int k = 0; k < dim; ++k) detJ *= h[k] / 2.0;
    for (int p = 0; p < nloc; ++p) {  // Gauss points: one per corner sign pattern
        double xi[3];
        for (int k = 0; k < dim; ++k) xi[k] = ((p >> k) & 1) ? g : -g;
        double G[8][3];
        for (int q = 0; q < nloc; ++q)
            for (int k = 0; k < dim; ++k) {
                double v = (((q >> k) & 1) ? 1.0 : -1.0) / 2.0;
                for (int m = 0; m < dim; ++m)
                    if (m != k) v *= (1.0 + (((q >> m) & 1) ? 1.0 : -1.0) * xi[m]) / 2.0;
                G[q][k] = v * 2.0 / h[k];
            }
        double B[6][24] = {};
        for (int q = 0; q < nloc; ++q) {
            for (int k = 0; k < dim; ++k) B[k][dim * q + k] = G[q][k];
            for (int r = 0; r < nv - dim; ++r) {
                const int a = dim == 2 ? sh2[r][0] : sh3[r][0];
                const int b = dim == 2 ? sh2[r][1] : sh3[r][1];
                B[dim + r][dim * q + a] = G[q][b];
                B[dim + r][dim * q + b] = G[q][a];
            }
        }
        for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nd; ++j) {
                double s = 0.0;
                for (int a = 0; a < nv; ++a)
                    for (int b = 0; b < nv; ++b) s += B[a][i] * D[a][b] * B[b][j];
                K[i * nd + j] += s * detJ;
            }
    }
    // exact symmetry, so that A_ij and A_ji come out equal to the bit
    for (int i = 0; i < nd; ++i)
        for (int j = i + 1; j < nd; ++j) {
            const double s = 0.5 * (K[i * nd + j] + K[j * nd + i]);
            K[i * nd + j] = K[j * nd + i] = s;
        }
}

namespace {

constexpr int kQ1MaxK = 24 * 24;

struct Q1Grid {
    int dim;
    int ne[3];  // elements per axis (1 for the unused axis in 2D)
    int nn[3];  // nodes per axis
};

// one thread per matrix row; the sum over the elements shared by the row's
// node and a neighbour runs in increasing element index, the same order for
// A_ij and A_ji
__global__ __launch_bounds__(kBlock) void k_q1_values(Q1Grid g, const double *__restrict__ k0,
                                                      const double *__restrict__ logE,
                                                      const uint8_t *__restrict__ fixed,
                                                      const int *__restrict__ rp,
                                                      double *__restrict__ val)
{
    __shared__ double K[kQ1MaxK];
    const int dim = g.dim, nd = dim << dim;
    for (int t = threadIdx.x; t < nd * nd; t += blockDim.x) K[t] = k0[t];
    __syncthreads();
    const int nrow = dim * g.nn[0] * g.nn[1] * g.nn[2];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrow) return;
    const int node = r / dim, l = r % dim;
    const int x[3] = {node % g.nn[0], (node / g.nn[0]) % g.nn[1], node / (g.nn[0] * g.nn[1])};
    const bool fr = fixed && fixed[r];
    int pos = rp[r];
    const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int d[3] = {dx, dy, dz};
                int y[3];
                bool ok = true;
                for (int k = 0; k < 3; ++k) {
                    y[k] = x[k] + d[k];
                    ok = ok && y[k] >= 0 && y[k] < g.nn[k];
                }
                if (!ok) continue;
                const int nb = y[0] + g.nn[0] * (y[1] + g.nn[1] * y[2]);
                // element origins shared by both nodes, per axis
                int lo[3], hi[3];
                for (int k = 0; k < 3; ++k) {
                    lo[k] = max(max(x[k], y[k]) - 1, 0);
                    hi[k] = min(min(x[k], y[k]), g.ne[k] - 1);
                }
                double acc[3] = {0.0, 0.0, 0.0};
                for (int oz = lo[2]; oz <= hi[2]; ++oz)
                    for (int oy = lo[1]; oy <= hi[1]; ++oy)
                        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                            const int e = ox + g.ne[0] * (oy + g.ne[1] * oz);
                            const double E = exp(logE[e]);
                            const int qi = (x[0] - ox) + 2 * (x[1] - oy) + 4 * (x[2] - oz);
                            const int qj = (y[0] - ox) + 2 * (y[1] - oy) + 4 * (y[2] - oz);
                            const double *kr = K + (dim * qi + l) * nd + dim * qj;
                            for (int m = 0; m < dim; ++m) acc[m] += E * kr[m];
                        }
                for (int m = 0; m < dim; ++m) {
                    const int col = dim * nb + m;
                    const bool kill = col != r && (fr || (fixed && fixed[col]));
                    val[pos++] = kill ? 0.0 : acc[m];
                }
            }
}

// grad_e = -E_e lambda_e^T K0 u_e over the element's dofs, with fixed dofs
// taken as zero (they do not depend on E)
__global__ __launch_bounds__(kBlock) void k_q1_grad(Q1Grid g, const double *__restrict__ k0,
                                                    const double *__restrict__ logE,
                                                    const uint8_t *__restrict__ fixed,
                                                    const double *__restrict__ u,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ grad)
{
    __shared__ double K[kQ1MaxK];
    const int dim = g.dim, nloc = 1 << dim, nd = dim * nloc;
    for (int t = threadIdx.x; t < nd * nd; t += blockDim.x) K[t] = k0[t];
    __syncthreads();
    const int nel = g.ne[0] * g.ne[1] * g.ne[2];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nel) return;
    const int o[3] = {e % g.ne[0], (e / g.ne[0]) % g.ne[1], e / (g.ne[0] * g.ne[1])};
    double ue[24], le[24];
    for (int q = 0; q < nloc; ++q) {
        const int node = (o[0] + (q & 1)) +
                         g.nn[0] * ((o[1] + ((q >> 1) & 1)) + g.nn[1] * (o[2] + ((q >> 2) & 1)));
        for (int l = 0; l < dim; ++l) {
            const int dof = dim * node + l;
            const bool f = fixed && fixed[dof];
            ue[dim * q + l] = f ? 0.0 : u[dof];
            le[dim * q + l] = f ? 0.0 : lam[dof];
        }
    }
    double s = 0.0;
    for (int a = 0; a < nd; ++a) {
        double t = 0.0;
        for (int b = 0; b < nd; ++b) t += K[a * nd + b] * ue[b];
        s += le[a] * t;
    }
    grad[e] = -exp(logE[e]) * s;
}

Q1Grid make_grid(int dim, const int *elems)
{
    Q1Grid g;
    g.dim = dim;
    for (int k = 0; k < 3; ++k) {
        g.ne[k] = k < dim ? elems[k] : 1;
        g.nn[k] = k < dim ? elems[k] + 1 : 1;
    }
    if (dim == 2) g.ne[2] = 1;
    return g;
}

}  // namespace

void launch_q1_values(hipStream_t s, int dim, const int *elems, const double *k0,
                      const double *logE, const uint8_t *fixed, const int *rp, double *val)
{
    const Q1Grid g = make_grid(dim, elems);
    const int64_t nrow = static_cast<int64_t>(dim) * g.nn[0] * g.nn[1] * g.nn[2];
    k_q1_values<<<static_cast<int>((nrow + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, k0, logE,
                                                                                  fixed, rp, val);
}

void launch_q1_grad(hipStream_t s, int dim, const int *elems, const double *k0,
                    const double *logE, const uint8_t *fixed, const double *u, const double *lam,
                    double *grad)
{
    const Q1Grid g = make_grid(dim, elems);
    const int64_t nel = static_cast<int64_t>(g.ne[0]) * g.ne[1] * g.ne[2];
    k_q1_grad<<<static_cast<int>((nel + kBlock - 1) / kBlock), kBlock, 0, s>>>(g, k0, logE, fixed,
                                                                               u, lam, grad);
}

}  // namespace msrsb
