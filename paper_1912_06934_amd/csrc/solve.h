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

msrsb_status ensure_workspace(msrsb_ctx *c);
msrsb_status ensure_smoother(msrsb_ctx *c, const msrsb_solve_opts *o, bool trans);
// With upd, v is first produced by the PCG update upd (upd->rout == v).
void apply_two_stage(msrsb_ctx *c, const msrsb_solve_opts *o, const double *v, double *zout,
                     bool trans, const PcgDots *dots, const UpdArgs *upd = nullptr);
msrsb_status pcg(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                 msrsb_solve_info *info, bool trans);
msrsb_status gmres(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                   msrsb_solve_info *info, bool trans);

}  // namespace msrsb
