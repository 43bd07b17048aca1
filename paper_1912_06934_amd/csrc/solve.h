// Preconditioner and Krylov drivers shared by the C ABI.
#pragma once

#include "internal.h"

namespace msrsb {

// Buffers for the r.z dot products and flexible beta computed at the end of
// a preconditioner application inside PCG.
struct PcgDots {
    const double *zold;
    double *part;
    double *scal;
    const double *part_rr;  // r.r partials of the step's update
    double *host_out;       // r.r mailbox of the step (null: beta only)
    int tag;           // the step's iteration number
};

// Temporaries of one preconditioner application: three FP64 and three FP32
// fine vectors, the coarse vectors and the partial sums of the coarse
// product.  By default they are the context's workspace.
struct ApplyBufs {
    double *z = nullptr, *spare = nullptr, *tmp = nullptr;  // n each
    float *f[3] = {nullptr, nullptr, nullptr};              // n each
    double *vc = nullptr, *wc = nullptr;                    // nc each
    double *part = nullptr;                                 // 64 nc + 64
};
ApplyBufs ctx_apply_bufs(msrsb_ctx *c);

msrsb_status ensure_workspace(msrsb_ctx *c);
bool is_tri(int kind);
msrsb_status ensure_smoother(msrsb_ctx *c, const msrsb_solve_opts *o, bool trans);
// With upd, v is first produced by the PCG update upd (upd->rout == v).
// bufs: the temporaries (null: the context's workspace).
void apply_two_stage(msrsb_ctx *c, const msrsb_solve_opts *o, const double *v, double *zout,
                     bool trans, const PcgDots *dots, const UpdArgs *upd = nullptr,
                     const ApplyBufs *bufs = nullptr);
msrsb_status pcg(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                 msrsb_solve_info *info, bool trans);
msrsb_status gmres(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                   msrsb_solve_info *info, bool trans);
msrsb_status richardson(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                        msrsb_solve_info *info, bool trans);
msrsb_status bicgstab(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                      msrsb_solve_info *info, bool trans);

}  // namespace msrsb
