// Internal declarations of the MsRSB HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "msrsb.h"

namespace msrsb {

constexpr int kBlock = 256;           // default work-group size
constexpr int kMaxPatternWidth = 32;  // max support entries per fine row
constexpr int kMaxCoarse = 4096;      // dense coarse inverse limit
constexpr int kReduceBlocks = 1024;   // partial-sum slots of two-stage reductions
constexpr int kMaxCoarseNeighbours = 96;  // LDS slots per coarse row in R A P

// Device scalars of the Krylov drivers (one FP64 array on the device).
enum Scalar {
    S_RR = 0,      // r.r
    S_PQ,          // p.A p
    S_RZ,          // r.z (current)
    S_RZ_OLD,      // r.z of the previous iteration
    S_RZDIFF,      // r.(z - z_old)
    S_ALPHA,
    S_BETA,
    S_FF,          // f.f
    S_BREAK,       // breakdown flag (non-zero = breakdown)
    S_TMP0,
    S_TMP1,
    S_TMP2,
    S_TMP3,
    S_COUNT = 32   // allocation size of the scalar array
};

struct Status {
    msrsb_status code = MSRSB_OK;
    std::string msg;
};

}  // namespace msrsb

struct msrsb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // state machine
    bool has_matrix = false, has_coarse = false, has_basis = false, has_coarse_op = false;

    // fine operator A (CSR)
    int n = 0;
    int64_t nnz = 0;
    int bs = 1;
    int *rp = nullptr, *ci = nullptr, *diag_pos = nullptr;
    double *a = nullptr;
    float *a32 = nullptr;
    std::vector<int> h_rp, h_ci;
    bool smoother_valid = false;

    // transpose of A (for msrsb_solve_transpose), values gathered from A
    int *at_rp = nullptr, *at_ci = nullptr, *at_src = nullptr, *at_diag = nullptr;
    double *at = nullptr;
    bool at_pattern = false;
    bool a_symmetric_pattern_checked = false;

    // Jacobi operator J (filtered), CSR; aliases rp/ci when bs == 1
    int *jrp = nullptr, *jci = nullptr;
    int64_t jnnz = 0;
    bool j_own_pattern = false;
    double *jv = nullptr;
    float *jv32 = nullptr;

    // coarse partition and P (frozen pattern)
    int nc = 0;
    int *part = nullptr, *prp = nullptr, *pci = nullptr;
    uint8_t *interior = nullptr;
    int64_t pnnz = 0;
    int pmaxw = 0;
    std::vector<int> h_prp, h_pci;
    double *p64[2] = {nullptr, nullptr};
    float *p32[2] = {nullptr, nullptr};
    int pcur = 0;          // which buffer holds the current P
    bool p_is32 = false;   // current P lives in p32[pcur]

    // R = P^T (CSR over coarse rows) with the source index into P
    int *rrp = nullptr, *rci = nullptr, *rsrc = nullptr;
    double *r64 = nullptr;
    float *r32 = nullptr;
    int rmaxnb = 0;  // max coarse neighbours of a coarse row (RAP)

    // coarse operator and its inverse
    double *ac = nullptr, *acinv = nullptr, *gj_b = nullptr;
    int *piv = nullptr, *colsrc = nullptr, *dev_flag = nullptr;

    // smoothers (diagonal inverses of A, and of A^T for the transposed solve)
    double *dinv_jac = nullptr, *dinv_l1 = nullptr;
    float *dinv_jac32 = nullptr, *dinv_l1_32 = nullptr;
    double *dinv_jac_t = nullptr, *dinv_l1_t = nullptr;
    float *dinv_jac32_t = nullptr, *dinv_l1_32_t = nullptr;
    float *at32 = nullptr;
    bool smoother32_valid = false, smoother_t_valid = false, smoother32_t_valid = false;
    double *ilu = nullptr;
    int *ilu_lev_ptr = nullptr, *ilu_lev_rows = nullptr;
    int ilu_nlev_l = 0, ilu_nlev_u = 0;
    int *ilu_lev_ptr_u = nullptr, *ilu_lev_rows_u = nullptr;
    std::vector<int> h_lev_ptr_l, h_lev_ptr_u;
    bool ilu_valid = false;

    // Krylov workspace
    double *w[12] = {};
    double *vc = nullptr, *wc = nullptr;
    double *partials = nullptr, *scal = nullptr;
    double *gm_v = nullptr, *gm_h = nullptr;  // GMRES basis and small arrays
    int gm_cap = 0;
    double *h_pinned = nullptr;
    unsigned long long *eit_bits = nullptr;

    // TPFA assembly description (set by msrsb_assemble_tpfa)
    bool tpfa = false;
    int tdim = 0, tdims[3] = {1, 1, 1};
    double th[3] = {1, 1, 1}, tbc[6] = {0, 0, 0, 0, 0, 0};
    double *tlogk = nullptr;

    // timings
    hipEvent_t ev_start[MSRSB_N_PHASES] = {}, ev_stop[MSRSB_N_PHASES] = {};
    bool ev_used[MSRSB_N_PHASES] = {};
};

namespace msrsb {

// ---- basis kernels (k_basis.hip) ----
void launch_filter_jacobi(hipStream_t s, int n, int bs, int filter, double omega,
                          const int *rp, const int *ci, const double *a,
                          const int *jrp, double *jv64, float *jv32);
void launch_init_basis(hipStream_t s, int n, const int *prp, const int *pci, const int *part,
                       double *p64, float *p32);
void launch_smooth(hipStream_t s, int n, int maxw, bool fp32, const int *jrp, const int *jci,
                   const double *jv64, const float *jv32, const int *prp, const int *pci,
                   const double *pin64, double *pout64, const float *pin32, float *pout32,
                   const uint8_t *interior, unsigned long long *eit_bits);
void launch_basis_stats(hipStream_t s, int n, const int *prp, bool fp32, const double *p64,
                        const float *p32, double *partials, double *out3);
void launch_p_convert(hipStream_t s, int64_t m, const float *src, double *dst);
void launch_p_convert_down(hipStream_t s, int64_t m, const double *src, float *dst);

// ---- coarse kernels (k_coarse.hip) ----
void launch_gather_r(hipStream_t s, int64_t m, const int *rsrc, bool fp32, const double *p64,
                     const float *p32, double *r64, float *r32);
void launch_rap(hipStream_t s, int nc, int maxnb, const int *rrp, const int *rci, bool fp32,
                const double *r64, const float *r32, const int *rp, const int *ci,
                const double *a, const int *prp, const int *pci, const double *p64,
                const float *p32, double *ac, int *flag);
void launch_fill(hipStream_t s, int64_t m, double *x, double v);
msrsb_status coarse_inverse(hipStream_t s, int nc, double *ac_work, double *inv_out,
                            double *bbuf, int *piv, int *colsrc, int *flag, int *host_flag);
void launch_gemv(hipStream_t s, int nc, const double *m, const double *x, double *y, bool trans,
                 double *partials);

// ---- Krylov kernels (k_krylov.hip) ----
void launch_spmv(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                 const double *x, double *y);
void launch_residual(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                     const double *f, const double *x, double *r);
void launch_sweep(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                  const float *a32, const double *dinv, const float *dinv32, bool fp32,
                  const double *v, const double *zin, double *zout, bool zero_start);
void launch_restrict(hipStream_t s, int nc, const int *rrp, const int *rci, bool fp32,
                     const double *r64, const float *r32, const double *x, double *xc);
void launch_prolong_add(hipStream_t s, int n, const int *prp, const int *pci, bool fp32,
                        const double *p64, const float *p32, const double *wc, double *z);
void launch_dot(hipStream_t s, int n, const double *x, const double *y, double *partials,
                double *out);
void launch_dot2(hipStream_t s, int n, const double *r, const double *z, const double *zold,
                 double *partials, double *out_rz, double *out_rzdiff);
void launch_spmv_dot(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                     const double *p, double *q, double *partials, double *out_pq);
void launch_cg_update(hipStream_t s, int n, double *x, double *r, const double *p,
                      const double *q, const double *scal, double *partials, double *out_rr);
void launch_cg_alpha(hipStream_t s, double *scal);
void launch_cg_beta(hipStream_t s, double *scal);
void launch_p_update(hipStream_t s, int n, double *p, const double *z, const double *scal);
void launch_copy(hipStream_t s, int n, const double *x, double *y);
void launch_axpy(hipStream_t s, int n, double alpha_host, const double *x, double *y);
void launch_diag_inverses(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                          double *dj, double *dl1, float *dj32, float *dl1_32, float *a32,
                          int64_t nnz, int *flag);
void launch_gather_values(hipStream_t s, int64_t m, const int *src, const double *a, double *out);

// ---- GMRES helpers (k_krylov.hip) ----
void launch_multi_dot(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                      const double *w, double *partials, double *out);
void launch_multi_axpy(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                       const double *h, double *w, double sign);
void launch_norm_scale(hipStream_t s, int n, const double *w, double *vout, double *partials,
                       double *out_norm);

// ---- ILU(0) (k_ilu.hip) ----
msrsb_status ilu0_setup(msrsb_ctx *c);
void launch_ilu0_apply(msrsb_ctx *c, const double *res, double *zinout, double *tmp);

// ---- TPFA (k_tpfa.hip) ----
void launch_tpfa_values(hipStream_t s, int dim, const int *dims, const double *h,
                        const double *bc, const double *logk, const int *rp, double *val,
                        double *rhs);
void launch_tpfa_grad(hipStream_t s, int dim, const int *dims, const double *h, const double *bc,
                      const double *logk, const double *p, const double *lam, double *grad);

}  // namespace msrsb
