// Two-stage preconditioner (Alg. 3, Alg. 4) and the Krylov drivers (PCG with
// the flexible Polak-Ribiere beta, right-preconditioned restarted GMRES).
// All vector arithmetic runs in device kernels; the host only queues work and
// reads the residual norm to decide when to stop.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "solve.h"

namespace msrsb {
namespace {

// --- GMRES small dense algebra (single thread; m <= 64) ---
// Apply the previous Givens rotations to the new Hessenberg column (h[0..j]
// from the Gram-Schmidt, ||w||^2 in nrm2), form the new rotation, update g
// and write |g[j+1]| and the rotated diagonal to res.
// With host_out (coherent pinned memory) the residual estimate and the
// denominator also go to the host mailbox: the values, a system-scope fence,
// then the step's tag the host waits for.
__global__ void k_gmres_givens(int j, int m, double *__restrict__ H, const double *__restrict__ h,
                               const double *__restrict__ nrm2, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g,
                               double *__restrict__ res, double *__restrict__ host_out,
                               double tag)
{
    if (threadIdx.x != 0) return;
    double col[65];
    for (int i = 0; i <= j; ++i) col[i] = h[i];
    col[j + 1] = sqrt(nrm2[0]);
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = sqrt(a * a + b * b);
    double c = 1.0, s = 0.0;
    if (den > 0.0) {
        c = a / den;
        s = b / den;
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = den;
    col[j + 1] = 0.0;
    for (int i = 0; i <= j; ++i) H[static_cast<int64_t>(i) * m + j] = col[i];
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    res[0] = fabs(g[j + 1]);
    res[1] = den;
    if (host_out == nullptr) return;
    host_out[0] = res[0];
    host_out[1] = den;
    __threadfence_system();
    host_out[2] = tag;
}

// y = H(0:k,0:k)^{-1} g(0:k) (upper triangular back substitution)
__global__ void k_gmres_solve(int k, int m, const double *__restrict__ H,
                              const double *__restrict__ g, double *__restrict__ y)
{
    if (threadIdx.x != 0) return;
    for (int r = k - 1; r >= 0; --r) {
        double s = g[r];
        for (int c = r + 1; c < k; ++c) s -= H[static_cast<int64_t>(r) * m + c] * y[c];
        y[r] = s / H[static_cast<int64_t>(r) * m + r];
    }
}

__global__ void k_gmres_init_g(int m, double *__restrict__ g, const double *__restrict__ nrm2)
{
    if (threadIdx.x != 0) return;
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = sqrt(nrm2[0]);
}

__global__ void k_vec_add(int k, double *__restrict__ a, const double *__restrict__ b)
{
    const int t = threadIdx.x;
    if (t < k) a[t] += b[t];
}

// out = a x + b y + c w (w may be null); out may alias x, y or w
__global__ __launch_bounds__(kBlock) void k_lincomb(int n, double a, const double *x, double b,
                                                    const double *y, double c, const double *w,
                                                    double *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double v = a * x[i] + b * y[i];
    if (w) v += c * w[i];
    out[i] = v;
}

void lincomb(hipStream_t s, int n, double a, const double *x, double b, const double *y,
             double c, const double *w, double *out)
{
    k_lincomb<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, a, x, b, y, c, w, out);
}

// The fine operator (A, or A^T for the transposed solve) in its CSR and,
// when available, DIA forms, with the diagonal inverses of its smoothers.
struct Op {
    const int *rp, *ci;
    const double *a;
    const float *a32;
    DiaOffsets d;
    const double *ad;
    const float *ad32;
    const double *dj, *dl1;
    const float *dj32, *dl132;
    NodeStencil ns;            // NBS form (ns.n == 0: none)
    const double *nv;
    const float *nv32;
};

Op fine_op(msrsb_ctx *c, bool trans)
{
    Op o;
    if (!trans || c->a_symmetric) {  // A^T = A: share A's data
        o.rp = c->rp;
        o.ci = c->ci;
        o.a = c->a;
        o.a32 = c->a32;
        o.d = c->a_off;
        o.ad = c->a_dia;
        o.ad32 = c->a_dia32;
        o.dj = c->dinv_jac;
        o.dl1 = c->dinv_l1;
        o.dj32 = c->dinv_jac32;
        o.dl132 = c->dinv_l1_32;
        o.ns = c->a_ns;
        o.nv = c->a_ns_val;
        o.nv32 = c->a_ns_val32;
    } else {
        o.rp = c->at_rp;
        o.ci = c->at_ci;
        o.a = c->at;
        o.a32 = c->at32;
        o.d = c->at_off;
        o.ad = c->at_dia;
        o.ad32 = c->at_dia32;
        o.dj = c->dinv_jac_t;
        o.dl1 = c->dinv_l1_t;
        o.dj32 = c->dinv_jac32_t;
        o.dl132 = c->dinv_l1_32_t;
        o.ns = NodeStencil();
        o.nv = nullptr;
        o.nv32 = nullptr;
    }
    return o;
}

// r = f - A x; fp32 (inside the preconditioner of the precision form) uses
// the FP32 copy of A's stencil values when there is one
void op_residual(hipStream_t s, int n, const Op &o, const double *f, const double *x, double *r,
                 bool fp32 = false)
{
    if (o.d.n > 0)
        launch_dia_residual(s, n, o.d, o.ad, fp32 ? o.ad32 : nullptr, f, x, r);
    else if (o.ns.n > 0)
        launch_nbs_residual(s, n, o.ns, o.nv, fp32 ? o.nv32 : nullptr, f, x, r);
    else
        launch_residual(s, n, o.rp, o.ci, o.a, f, x, r);
}

void op_spmv(hipStream_t s, int n, const Op &o, const double *x, double *y)
{
    if (o.d.n > 0)
        launch_dia_spmv(s, n, o.d, o.ad, x, y);
    else if (o.ns.n > 0)
        launch_nbs_spmv(s, n, o.ns, o.nv, x, y);
    else
        launch_spmv(s, n, o.rp, o.ci, o.a, x, y);
}

// p = z + beta p_old, q = A p, p.q and alpha (PCG)
void p_spmv(hipStream_t s, int n, const Op &o, const double *z, const double *pold, double *pnew,
            double *q, double *part, double *sc)
{
    if (o.d.n == 0 && o.ns.n > 0)
        launch_nbs_pcg_p_spmv(s, n, o.ns, o.nv, z, pold, pnew, q, part, sc);
    else
        launch_pcg_p_spmv(s, n, o.d, o.ad, o.rp, o.ci, o.a, z, pold, pnew, q, part, sc);
}

template <typename T>
msrsb_status dev_alloc(T **p, size_t count)
{
    if (*p) return MSRSB_OK;
    if (hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T)) !=
        hipSuccess)
        return MSRSB_E_NOMEM;
    return MSRSB_OK;
}

bool is_diag(int kind) { return kind == MSRSB_SMOOTH_JACOBI || kind == MSRSB_SMOOTH_L1JACOBI; }

// one smoothing sweep z += M^{-1} (v - A z); with zero, z is known to be zero
// and is not read.  The result may land in *spare, in which case the two
// pointers are exchanged.  ord: sweep order of the triangular smoothers.
void sweep(msrsb_ctx *c, const Op &o, int kind, bool fp32, const double *v, double **z,
           double **spare, bool zero, double *tmp, int ord)
{
    hipStream_t s = c->stream;
    const int n = c->n;
    if (is_diag(kind)) {
        const bool l1 = kind == MSRSB_SMOOTH_L1JACOBI;
        const double *d64 = l1 ? o.dl1 : o.dj;
        const float *d32 = l1 ? o.dl132 : o.dj32;
        if (o.d.n > 0 && !zero)
            launch_dia_sweep(s, n, o.d, fp32, o.ad, o.ad32, d64, d32, v, *z, *spare, false);
        else if (o.ns.n > 0)
            launch_nbs_sweep(s, n, o.ns, fp32, o.nv, o.nv32, d64, d32, v, *z, *spare, zero);
        else
            launch_sweep(s, n, o.rp, o.ci, o.a, o.a32, d64, d32, fp32, v, *z, *spare, zero);
        std::swap(*z, *spare);
    } else if (is_tri(kind)) {
        // residual, then the triangular solves in the order; SGS is a forward
        // sweep (D + L)^{-1} and a backward one (D + U)^{-1}, each on the
        // residual of the current iterate
        if (zero) {
            launch_copy(s, n, v, tmp);
            launch_fill(s, n, *z, 0.0);
        } else {
            op_residual(s, n, o, v, *z, tmp);
        }
        if (kind == MSRSB_SMOOTH_SGS) {
            tri_gs_half(c, ord, true, tmp, *z);
            op_residual(s, n, o, v, *z, tmp);
            tri_gs_half(c, ord, false, tmp, *z);
        } else {
            tri_apply(c, ord, kind, tmp, *z);
        }
    }
}

}  // namespace

bool is_tri(int kind)
{
    return kind == MSRSB_SMOOTH_ILU0 || kind == MSRSB_SMOOTH_IC0 || kind == MSRSB_SMOOTH_SGS;
}

msrsb_status ensure_workspace(msrsb_ctx *c)
{
    const size_t n = static_cast<size_t>(c->n);
    for (auto &p : c->w)
        if (dev_alloc(&p, n)) return MSRSB_E_NOMEM;
    for (auto &p : c->wf)
        if (dev_alloc(&p, n)) return MSRSB_E_NOMEM;
    const size_t np = std::max<size_t>({2 * (n / kBlock + 2), 2 * static_cast<size_t>(kReduceBlocks),
                                        64 * static_cast<size_t>(std::max(c->nc, 1)) + 64,
                                        static_cast<size_t>(64 * 66),
                                        static_cast<size_t>(3 * 2048)});
    if (dev_alloc(&c->partials, np) || dev_alloc(&c->partials_rr, n / kBlock + 2) ||
        dev_alloc(&c->scal, S_COUNT) ||
        dev_alloc(&c->vc, std::max(c->nc, 1)) || dev_alloc(&c->wc, std::max(c->nc, 1)) ||
        dev_alloc(&c->eit_val, 1) || dev_alloc(&c->dev_flag, 4))
        return MSRSB_E_NOMEM;
    if (!c->h_pinned && hipHostMalloc(reinterpret_cast<void **>(&c->h_pinned), 64 * sizeof(double),
                                      hipHostMallocCoherent) != hipSuccess)
        return MSRSB_E_NOMEM;
    return MSRSB_OK;
}

msrsb_status ensure_smoother(msrsb_ctx *c, const msrsb_solve_opts *o, bool trans)
{
    const int kinds[2] = {o->pre_sweeps > 0 ? o->pre_smoother : MSRSB_SMOOTH_NONE,
                          o->post_sweeps > 0 ? o->post_smoother : MSRSB_SMOOTH_NONE};
    const bool need_tri = is_tri(kinds[0]) || is_tri(kinds[1]);
    if (need_tri && trans) {
        c->err = "ILU(0), IC(0) and SGS are not available for the transposed solve";
        return MSRSB_E_ARG;
    }
    const bool fp32 = o->fp32_smoother != 0;
    const size_t n = static_cast<size_t>(c->n);
    hipStream_t s = c->stream;
    if (c->a_symmetric) trans = false;  // the smoothers of A^T are those of A
    const int noff = trans ? c->at_off.n : c->a_off.n;
    if (!trans) {
        if (!c->smoother_valid || (fp32 && !c->smoother32_valid)) {
            if (dev_alloc(&c->dinv_jac, n) || dev_alloc(&c->dinv_l1, n)) return MSRSB_E_NOMEM;
            if (fp32 && (dev_alloc(&c->dinv_jac32, n) || dev_alloc(&c->dinv_l1_32, n) ||
                         dev_alloc(&c->a32, static_cast<size_t>(c->nnz))))
                return MSRSB_E_NOMEM;
            if (fp32 && noff > 0 && dev_alloc(&c->a_dia32, n * noff)) return MSRSB_E_NOMEM;
            const size_t nslot = static_cast<size_t>(c->a_ns.n) * c->a_ns.bs;
            if (fp32 && nslot > 0 && dev_alloc(&c->a_ns_val32, n * nslot)) return MSRSB_E_NOMEM;
            launch_diag_inverses(s, c->n, c->rp, c->ci, c->a, c->dinv_jac, c->dinv_l1,
                                 fp32 ? c->dinv_jac32 : nullptr, fp32 ? c->dinv_l1_32 : nullptr,
                                 fp32 ? c->a32 : nullptr, c->nnz, c->dev_flag);
            if (fp32 && noff > 0)
                launch_csr_to_dia(s, c->n, noff, c->rp, c->a_slot, c->a, nullptr, c->a_dia32);
            if (fp32 && nslot > 0)
                launch_csr_to_nbs(s, c->n, static_cast<int>(nslot), c->rp, c->ns_slot, c->a,
                                  nullptr, c->a_ns_val32);
            c->smoother_valid = true;
            c->smoother32_valid = fp32;
        }
    } else {
        if (!c->smoother_t_valid || (fp32 && !c->smoother32_t_valid)) {
            if (dev_alloc(&c->dinv_jac_t, n) || dev_alloc(&c->dinv_l1_t, n)) return MSRSB_E_NOMEM;
            if (fp32 && (dev_alloc(&c->dinv_jac32_t, n) || dev_alloc(&c->dinv_l1_32_t, n) ||
                         dev_alloc(&c->at32, static_cast<size_t>(c->nnz))))
                return MSRSB_E_NOMEM;
            if (fp32 && noff > 0 && dev_alloc(&c->at_dia32, n * noff)) return MSRSB_E_NOMEM;
            launch_diag_inverses(s, c->n, c->at_rp, c->at_ci, c->at, c->dinv_jac_t, c->dinv_l1_t,
                                 fp32 ? c->dinv_jac32_t : nullptr,
                                 fp32 ? c->dinv_l1_32_t : nullptr, fp32 ? c->at32 : nullptr,
                                 c->nnz, c->dev_flag);
            if (fp32 && noff > 0)
                launch_csr_to_dia(s, c->n, noff, c->at_rp, c->at_slot, c->at, nullptr,
                                  c->at_dia32);
            c->smoother_t_valid = true;
            c->smoother32_t_valid = fp32;
        }
    }
    if (need_tri) {
        const int ord = o->ordering;
        msrsb_status st = tri_order_setup(c, ord);
        if (st) {
            c->err = "sweep order set-up failed";
            return st;
        }
        for (int k : kinds) {
            if (k == MSRSB_SMOOTH_IC0 && (!c->a_symmetric || !c->tri[ord].sym_pattern)) {
                c->err = "IC(0) needs a symmetric matrix";
                return MSRSB_E_ARG;
            }
            bool &ok = k == MSRSB_SMOOTH_ILU0 ? c->ilu_ok[ord] : c->ic_ok[ord];
            if ((k != MSRSB_SMOOTH_ILU0 && k != MSRSB_SMOOTH_IC0) || ok) continue;
            st = tri_factor(c, ord, k);
            if (st) {
                c->err = st == MSRSB_E_BREAKDOWN
                             ? (k == MSRSB_SMOOTH_ILU0 ? "zero pivot in ILU(0)"
                                                       : "non-positive pivot in IC(0)")
                             : "smoother factorisation failed";
                return st;
            }
            ok = true;
        }
    }
    return MSRSB_OK;
}

// z = B v (Alg. 4): z = 0; pre-smoothing; z += P M_c^{-1} R (v - A z);
// post-smoothing.  With trans the preconditioner of A^T is applied: A^T, the
// smoothers of A^T, pre and post exchanged, and A_c^{-T}.  With dots (inside
// PCG) the products r.z and r.(z - zold) and the flexible beta are formed as
// well, fused into the last sweep when possible.
// wc = A_c^{-1} vc (A_c^{-T} for trans): the SPD path's symmetric inverse
// from its packed lower tiles, otherwise the dense product
static void coarse_apply(msrsb_ctx *c, bool trans, const ApplyBufs &b)
{
    if (c->child) {  // multilevel: w_c = B_next v_c (the next level's workspace)
        apply_two_stage(c->child, &c->child_opts, b.vc, b.wc, trans, nullptr);
        return;
    }
    if (c->acinv_sym)
        launch_symv_packed(c->stream, c->nc, c->acinv_pk, b.vc, b.wc, c->symv_part);
    else
        launch_gemv(c->stream, c->nc, c->acinv, b.vc, b.wc, trans, b.part);
}

ApplyBufs ctx_apply_bufs(msrsb_ctx *c)
{
    ApplyBufs b;
    b.z = c->w[8];
    b.spare = c->w[9];
    b.tmp = c->w[10];
    for (int k = 0; k < 3; ++k) b.f[k] = c->wf[k];
    b.vc = c->vc;
    b.wc = c->wc;
    b.part = c->partials;
    return b;
}

// The FP64 prolongation reads P's split form while it holds the current P
// (fewer bytes: the zero slots of rows with fewer than 8 entries are not
// stored).  The FP32 one keeps the padded rows, which it reads as fast.
// prolong_p64 / prolong_p32 return the matching values.
static bool prolong_split(const msrsb_ctx *c)
{
    return c->paxes && c->ps_valid && c->pw == 8 && !c->p_is32;
}
static ProlongAxes prolong_axes(const msrsb_ctx *c)
{
    ProlongAxes a;
    if (c->paxes) {
        a.tab = c->paxes;
        a.nx = c->tdims[0];
        a.ny = c->tdims[1];
        a.ncx = c->pax_ncx;
        a.ncxy = c->pax_ncxy;
        if (prolong_split(c)) {
            a.wtab = c->psplit_wtab;
            a.n8 = c->psplit.n8;
        }
    }
    return a;
}
static const double *prolong_p64(const msrsb_ctx *c)
{
    return prolong_split(c) ? c->ps64[c->pcur] : c->p64[c->pcur];
}
static const float *prolong_p32(const msrsb_ctx *c)
{
    return c->p32[c->pcur];
}

static RestrictBoxes restrict_boxes(const msrsb_ctx *c)
{
    RestrictBoxes b;
    b.maxlen = c->rmaxlen;
    if (c->rbox) {
        b.box = c->rbox;
        b.nx = c->tdims[0];
        b.nxy = c->tdims[0] * c->tdims[1];
    }
    return b;
}

void apply_two_stage(msrsb_ctx *c, const msrsb_solve_opts *o, const double *v, double *zout,
                     bool trans, const PcgDots *dots, const UpdArgs *upd, const ApplyBufs *bufs)
{
    const ApplyBufs b = bufs ? *bufs : ctx_apply_bufs(c);
    hipStream_t s = c->stream;
    const int n = c->n;
    const Op op = fine_op(c, trans);
    const bool fp32 = o->fp32_smoother != 0;
    int pre_k = o->pre_smoother, pre_n = o->pre_sweeps;
    int post_k = o->post_smoother, post_n = o->post_sweeps;
    if (trans) {
        std::swap(pre_k, post_k);
        std::swap(pre_n, post_n);
    }
    if (pre_k == MSRSB_SMOOTH_NONE) pre_n = 0;
    if (post_k == MSRSB_SMOOTH_NONE) post_n = 0;
    double *z = b.z, *spare = b.spare, *tmp = b.tmp;
    // precision form inside PCG with two Jacobi-type sweeps on each side of a
    // stencil operator: FP32 intermediate vectors (launch_prec_f32_*)
    const bool f32_path = fp32 && dots && o->use_multiscale && op.d.n > 0 && c->pcol16 &&
                          c->p_is32 && (c->pw == 4 || c->pw == 8) && is_diag(pre_k) &&
                          pre_n == 2 && pre_k == post_k && post_n == 2;
    const bool sweep2 = pre_n >= 2 && is_diag(pre_k) && op.d.n > 0;
    // the PCG update that produces v: inside the first two-sweep kernel, or
    // on its own where the application starts otherwise
    if (upd && !f32_path && !sweep2) launch_pcg_update(s, n, *upd);
    if (f32_path) {
        const float *dinv = pre_k == MSRSB_SMOOTH_L1JACOBI ? op.dl132 : op.dj32;
        float *z1 = b.f[0], *z2 = b.f[1], *tf = b.f[2];
        launch_prec_f32_pre(s, n, op.d, op.ad32, dinv, v, z1, tf, c->nc, c->rrp, c->rci,
                            c->roff16, c->rbase, c->r32, b.vc, restrict_boxes(c), upd);
        coarse_apply(c, trans, b);
        launch_prec_f32_post(s, n, op.d, op.ad32, dinv, v, z1, z2, c->pw, c->pcol16,
                             prolong_p32(c), b.wc, zout, dots->zold, dots->part, dots->scal,
                             dots->part_rr, dots->host_out, dots->tag, prolong_axes(c));
        return;
    }
    bool zero = true;
    int t = 0;
    if (sweep2) {
        const bool l1 = pre_k == MSRSB_SMOOTH_L1JACOBI;
        launch_dia_sweep(s, n, op.d, fp32, op.ad, op.ad32, l1 ? op.dl1 : op.dj,
                         l1 ? op.dl132 : op.dj32, v, nullptr, z, true, upd);
        zero = false;
        t = 2;
    }
    for (; t < pre_n; ++t) {
        sweep(c, op, pre_k, fp32, v, &z, &spare, zero, tmp, o->ordering);
        zero = false;
    }
    if (o->use_multiscale) {
        const double *res = v;
        if (!zero) {
            op_residual(s, n, op, v, z, tmp, fp32);
            res = tmp;
        }
        launch_restrict(s, c->nc, c->rrp, c->rci, c->roff16, c->rbase, c->p_is32, c->r64, c->r32,
                        res, b.vc, restrict_boxes(c));
        coarse_apply(c, trans, b);
        launch_prolong_ell(s, n, c->pw, c->pcol_ell, c->pcol16, c->p_is32, prolong_p64(c),
                           prolong_p32(c),
                           b.wc, z, zero, prolong_axes(c));
        zero = false;
    }
    for (t = 0; t < post_n; ++t) {
        const bool last = t == post_n - 1;
        if (last && dots && is_diag(post_k) && op.d.n > 0 && !zero) {
            const bool l1 = post_k == MSRSB_SMOOTH_L1JACOBI;
            launch_dia_sweep_dots(s, n, op.d, fp32, op.ad, op.ad32, l1 ? op.dl1 : op.dj,
                                  l1 ? op.dl132 : op.dj32, v, z, zout, dots->zold,
                                  dots->part, dots->scal, dots->part_rr, dots->host_out,
                                  dots->tag);
            return;
        }
        sweep(c, op, post_k, fp32, v, &z, &spare, zero, tmp, o->ordering);
        zero = false;
    }
    if (zero)
        launch_fill(s, n, zout, 0.0);
    else
        launch_copy(s, n, z, zout);
    if (dots)
        launch_dots_beta(s, n, v, zout, dots->zold, dots->part, dots->scal, dots->part_rr,
                         dots->host_out, dots->tag);
}

// Wait until the device has tagged the r.r mailbox mb with iteration tag
// (mb[2]).  Only plain reads of pinned memory while the device works: a
// stream query puts a marker into the stream, and the barrier behind it
// leaves the device idle for several microseconds.  After a second without
// the tag the stream is queried, and if it has finished or failed without
// the tag arriving the wait reports failure instead of spinning on.  One
// Krylov step takes milliseconds at most, so a tag still missing after
// kMailboxDeadline means the device is stuck: the wait gives up with an
// error rather than holding the host forever.
constexpr auto kMailboxDeadline = std::chrono::seconds(120);

static bool wait_mailbox(hipStream_t s, volatile double *mb, int tag)
{
    const double want = tag;
    const auto start = std::chrono::steady_clock::now();
    auto t0 = start;
    for (unsigned spin = 1;; ++spin) {
        if (mb[2] == want) break;
        if ((spin & 0xFFFFu) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
            if (hipStreamQuery(s) != hipErrorNotReady) {
                if (mb[2] == want) break;
                return false;
            }
            t0 = std::chrono::steady_clock::now();
            if (t0 - start > kMailboxDeadline) return false;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return true;
}

static msrsb_status read_scalars(msrsb_ctx *c, int first, int count)
{
    hipMemcpyAsync(c->h_pinned, c->scal + first, count * sizeof(double), hipMemcpyDeviceToHost,
                   c->stream);
    return hipStreamSynchronize(c->stream) == hipSuccess ? MSRSB_OK : MSRSB_E_HIP;
}

// Preconditioned CG with flexible beta.  f, x device pointers (x = x0 on entry).
// Convergence of iteration k is read on the host while iteration k+1's
// preconditioner is already queued, so the device never waits for the host.
msrsb_status pcg(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                 msrsb_solve_info *info, bool trans)
{
    hipStream_t s = c->stream;
    const int n = c->n;
    const Op op = fine_op(c, trans);
    // r and p each alternate between two buffers: the kernels that update
    // them read the old values at neighbouring rows
    double *r = c->w[0], *z = c->w[1], *zold = c->w[2], *p = c->w[3], *q = c->w[4],
           *p2 = c->w[7], *r2 = c->w[12];
    double *sc = c->scal;
    launch_fill(s, S_COUNT, sc, 0.0);
    launch_dot(s, n, f, f, c->partials, sc + S_FF);
    if (read_scalars(c, S_FF, 1)) return MSRSB_E_HIP;
    double fn = std::sqrt(c->h_pinned[0]);
    if (fn == 0.0) fn = 1.0;
    const double thr2 = (o->rtol * fn) * (o->rtol * fn);
    int it = 0;
    msrsb_status rc = MSRSB_E_NOT_CONVERGED;
    bool restart = true, queued = false;
    double *hist = info ? info->history : nullptr;
    const int hcap = info ? info->history_cap : 0;
    PcgDots dots{zold, c->partials, sc, c->partials_rr, c->h_pinned + 8, 0};
    // r.r, the breakdown flag and the iteration tag, written by the device
    volatile double *hmon = c->h_pinned + 8;
    hmon[2] = -1.0;
    while (it <= o->max_iter) {
        if (restart) {
            op_residual(s, n, op, f, x, r);
            launch_dot(s, n, r, r, c->partials, sc + S_RR);
            if (read_scalars(c, S_RR, 1)) { rc = MSRSB_E_HIP; break; }
            const double rr = c->h_pinned[0];
            if (hist && it < hcap) hist[it] = std::sqrt(rr) / fn;
            if (!std::isfinite(rr)) { rc = MSRSB_E_BREAKDOWN; break; }
            if (rr <= thr2) { rc = MSRSB_OK; break; }
            if (it == o->max_iter) break;
            apply_two_stage(c, o, r, z, trans, nullptr);
            launch_dot(s, n, r, z, c->partials, sc + S_RZ_OLD);
            launch_fill(s, 1, sc + S_BETA, 0.0);   // p = z
            launch_fill(s, 1, sc + S_BREAK, 0.0);  // a queued-ahead step may have set it
            restart = false;
            queued = false;
        }
        if (!queued) {
            p_spmv(s, n, op, z, p, p2, q, c->partials, sc);
            std::swap(p, p2);
        }
        ++it;
        // x += alpha p and r2 = r - alpha q (inside the preconditioner's first
        // kernel where it can be), the next preconditioner application and
        // the next step's p = z + beta p, q = A p, all queued while the host
        // waits for r.r (the last two touch neither x nor r, so their work is
        // merely dropped if this step turns out to be the last)
        const UpdArgs upd{x, r, p, q, r2, c->partials_rr, sc};
        std::swap(r, r2);
        std::swap(z, zold);
        dots.zold = zold;
        dots.tag = it;
        apply_two_stage(c, o, r, z, trans, &dots, &upd);
        queued = it < o->max_iter;
        if (queued) {
            p_spmv(s, n, op, z, p, p2, q, c->partials, sc);
            std::swap(p, p2);
        }
        if (!wait_mailbox(s, hmon, it)) {
            c->err = "the device did not report the residual of a Krylov step";
            return MSRSB_E_HIP;
        }
        const double rr = hmon[0], brk = hmon[1];
        if (hist && it < hcap) hist[it] = std::sqrt(rr) / fn;
        if (brk != 0.0 || !std::isfinite(rr)) { rc = MSRSB_E_BREAKDOWN; break; }
        if (rr <= thr2) { restart = true; continue; }
        if (it >= o->max_iter) break;
    }
    // true residual at exit
    op_residual(s, n, op, f, x, r);
    launch_dot(s, n, r, r, c->partials, sc + S_TMP0);
    if (read_scalars(c, S_TMP0, 1)) return MSRSB_E_HIP;
    if (info) {
        info->iters = it;
        info->true_rel_res = std::sqrt(c->h_pinned[0]) / fn;
    }
    return rc;
}

// Right-preconditioned GMRES(m) with classical Gram-Schmidt applied twice.
msrsb_status gmres(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                   msrsb_solve_info *info, bool trans)
{
    hipStream_t s = c->stream;
    const int n = c->n;
    const int m = std::max(1, std::min(o->restart, 64));
    const Op op = fine_op(c, trans);
    if (c->gm_cap < m) {
        if (c->gm_v) hipFree(c->gm_v);
        if (c->gm_h) hipFree(c->gm_h);
        c->gm_v = c->gm_h = nullptr;
        if (dev_alloc(&c->gm_v, static_cast<size_t>(m + 1) * n) ||
            dev_alloc(&c->gm_h, static_cast<size_t>(m + 1) * m + 8 * (m + 2)))
            return MSRSB_E_NOMEM;
        c->gm_cap = m;
    }
    double *V = c->gm_v;
    double *H = c->gm_h;                        // (m+1) x m
    double *cs = H + (m + 1) * m, *sn = cs + (m + 2), *g = sn + (m + 2), *y = g + (m + 2);
    double *hc = y + (m + 2), *h2 = hc + (m + 2), *gsc = h2 + (m + 2);  // gsc: 2 scalars
    double *w = c->w[0], *zt = c->w[1], *r = c->w[2];
    double *sc = c->scal;
    // two mailbox slots in coherent pinned memory (steps alternate)
    volatile double *mbox[2] = {c->h_pinned + 16, c->h_pinned + 24};
    mbox[0][2] = mbox[1][2] = -1.0;
    launch_dot(s, n, f, f, c->partials, sc + S_FF);
    if (read_scalars(c, S_FF, 1)) return MSRSB_E_HIP;
    double fn = std::sqrt(c->h_pinned[0]);
    if (fn == 0.0) fn = 1.0;
    int it = 0;
    msrsb_status rc = MSRSB_E_NOT_CONVERGED;
    double *hist = info ? info->history : nullptr;
    const int hcap = info ? info->history_cap : 0;
    for (;;) {
        op_residual(s, n, op, f, x, r);
        launch_dot(s, n, r, r, c->partials, sc + S_RR);
        if (read_scalars(c, S_RR, 1)) return MSRSB_E_HIP;
        const double beta = std::sqrt(c->h_pinned[0]);
        if (hist && it < hcap) hist[it] = beta / fn;
        if (!std::isfinite(beta)) { rc = MSRSB_E_BREAKDOWN; break; }
        if (beta <= o->rtol * fn) { rc = MSRSB_OK; break; }
        if (it >= o->max_iter) break;
        launch_norm_scale(s, n, r, V, c->partials, sc + S_RR);
        k_gmres_init_g<<<1, 64, 0, s>>>(m, g, sc + S_RR);
        // one Arnoldi step: v_{j+1} and column j of H, its Givens rotation,
        // and the residual estimate posted to mailbox slot j mod 2 with tag
        auto step = [&](int jj, int tag) {
            const double *vj = V + static_cast<int64_t>(jj) * n;
            double *vn = V + static_cast<int64_t>(jj + 1) * n;
            apply_two_stage(c, o, vj, zt, trans, nullptr);
            op_spmv(s, n, op, zt, w);
            // CGS2: h = V^T w; w -= V h; h2 = V^T w; w -= V h2; h += h2
            launch_multi_dot(s, n, jj + 1, V, n, w, c->partials, hc);
            launch_multi_axpy(s, n, jj + 1, V, n, hc, w, -1.0);
            launch_multi_dot(s, n, jj + 1, V, n, w, c->partials, h2);
            launch_multi_axpy(s, n, jj + 1, V, n, h2, w, -1.0);
            k_vec_add<<<1, 64, 0, s>>>(jj + 1, hc, h2);
            launch_norm_scale(s, n, w, vn, c->partials, sc + S_TMP1);
            k_gmres_givens<<<1, 64, 0, s>>>(jj, m, H, hc, sc + S_TMP1, cs, sn, g, gsc,
                                            const_cast<double *>(mbox[jj & 1]), tag);
        };
        int j = 0;
        bool brk = false;
        if (it < o->max_iter) step(0, it + 1);
        for (j = 0; j < m && it < o->max_iter; ++j) {
            // step j + 1 goes into the queue before step j's residual is read,
            // so the device does not wait for the host; it writes only column
            // j + 1 of H, g[j + 1 ..] and v_{j + 2}, none of which the solution
            // after step j uses
            if (j + 1 < m && it + 1 < o->max_iter) step(j + 1, it + 2);
            if (!wait_mailbox(s, mbox[j & 1], it + 1)) {
                c->err = "the device did not report the residual of a Krylov step";
                return MSRSB_E_HIP;
            }
            ++it;
            const double res = mbox[j & 1][0], den = mbox[j & 1][1];
            if (hist && it < hcap) hist[it] = res / fn;
            if (!std::isfinite(res) || !(den > 0.0)) { brk = true; break; }
            if (res <= o->rtol * fn) { ++j; break; }
        }
        if (j > 0) {
            k_gmres_solve<<<1, 64, 0, s>>>(j, m, H, g, y);
            launch_fill(s, n, w, 0.0);
            launch_multi_axpy(s, n, j, V, n, y, w, 1.0);
            apply_two_stage(c, o, w, zt, trans, nullptr);
            launch_axpy(s, n, 1.0, zt, x);
        }
        if (brk) { rc = MSRSB_E_BREAKDOWN; break; }
    }
    op_residual(s, n, op, f, x, r);
    launch_dot(s, n, r, r, c->partials, sc + S_TMP0);
    if (read_scalars(c, S_TMP0, 1)) return MSRSB_E_HIP;
    const double tr = std::sqrt(c->h_pinned[0]) / fn;
    if (info) {
        info->iters = it;
        info->true_rel_res = tr;
    }
    if (rc == MSRSB_OK && !(tr <= o->rtol)) rc = MSRSB_E_NOT_CONVERGED;
    return rc;
}

// The stand-alone iteration of Sec. 3.2 (Richardson): x += B (f - A x) until
// the true residual meets the tolerance; iterations count applications of B.
msrsb_status richardson(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                        msrsb_solve_info *info, bool trans)
{
    hipStream_t s = c->stream;
    const int n = c->n;
    const Op op = fine_op(c, trans);
    double *r = c->w[0], *z = c->w[1];
    double *sc = c->scal;
    launch_dot(s, n, f, f, c->partials, sc + S_FF);
    if (read_scalars(c, S_FF, 1)) return MSRSB_E_HIP;
    double fn = std::sqrt(c->h_pinned[0]);
    if (fn == 0.0) fn = 1.0;
    double *hist = info ? info->history : nullptr;
    const int hcap = info ? info->history_cap : 0;
    int it = 0;
    double rel = 0.0;
    msrsb_status rc = MSRSB_E_NOT_CONVERGED;
    for (;;) {
        op_residual(s, n, op, f, x, r);
        launch_dot(s, n, r, r, c->partials, sc + S_RR);
        if (read_scalars(c, S_RR, 1)) return MSRSB_E_HIP;
        rel = std::sqrt(c->h_pinned[0]) / fn;
        if (hist && it < hcap) hist[it] = rel;
        if (!std::isfinite(rel)) { rc = MSRSB_E_BREAKDOWN; break; }
        if (rel <= o->rtol) { rc = MSRSB_OK; break; }
        if (it >= o->max_iter) break;
        apply_two_stage(c, o, r, z, trans, nullptr);
        launch_axpy(s, n, 1.0, z, x);
        ++it;
    }
    if (info) {
        info->iters = it;
        info->true_rel_res = rel;
    }
    return rc;
}

// Right-preconditioned BiCGStab (two applications of B per iteration,
// Sec. 4.1).  Scalars are read back on the host after each product; a pass
// that meets the tolerance after its first half ends there.  Convergence of
// the recursive residual is confirmed on the true residual, and the method
// starts again from x if that is still above the tolerance.  Breakdown:
// |rhat^T r| <= 1e-14 ||rhat|| ||r|| (an exact zero is hidden by rounding),
// or rhat^T v or t^T t zero.
msrsb_status bicgstab(msrsb_ctx *c, const double *f, double *x, const msrsb_solve_opts *o,
                      msrsb_solve_info *info, bool trans)
{
    hipStream_t s = c->stream;
    const int n = c->n;
    const Op op = fine_op(c, trans);
    // (w[5] and w[6] hold f and x of a host-staged solve)
    double *r = c->w[0], *rh = c->w[1], *p = c->w[2], *v = c->w[3], *y = c->w[4],
           *sv = c->w[7], *z = c->w[12], *t = c->w[13];
    double *sc = c->scal;
    auto dot = [&](const double *a, const double *b, double &out) {
        launch_dot(s, n, a, b, c->partials, sc + S_TMP0);
        if (read_scalars(c, S_TMP0, 1)) return false;
        out = c->h_pinned[0];
        return true;
    };
    double ff = 0.0;
    if (!dot(f, f, ff)) return MSRSB_E_HIP;
    double fn = std::sqrt(ff);
    if (fn == 0.0) fn = 1.0;
    double *hist = info ? info->history : nullptr;
    const int hcap = info ? info->history_cap : 0;
    int it = 0;
    msrsb_status rc = MSRSB_E_NOT_CONVERGED;
    bool restart = true;
    double rho = 1.0, alpha = 1.0, omega = 1.0, rhn = 0.0, rn = 0.0;
    while (it <= o->max_iter) {
        if (restart) {
            op_residual(s, n, op, f, x, r);
            double rr = 0.0;
            if (!dot(r, r, rr)) return MSRSB_E_HIP;
            const double rel = std::sqrt(rr) / fn;
            if (hist && it < hcap) hist[it] = rel;
            if (!std::isfinite(rel)) { rc = MSRSB_E_BREAKDOWN; break; }
            if (rel <= o->rtol) { rc = MSRSB_OK; break; }
            if (it >= o->max_iter) break;
            launch_copy(s, n, r, rh);
            launch_copy(s, n, r, p);
            rho = rr;
            rhn = std::sqrt(rr);
            restart = false;
        } else {
            double rho_new = 0.0;
            if (!dot(rh, r, rho_new)) return MSRSB_E_HIP;
            if (!(std::fabs(rho_new) > 1e-14 * rhn * rn)) { rc = MSRSB_E_BREAKDOWN; break; }
            const double beta = (rho_new / rho) * (alpha / omega);
            lincomb(s, n, 1.0, r, beta, p, -beta * omega, v, p);  // p = r + beta (p - omega v)
            rho = rho_new;
        }
        apply_two_stage(c, o, p, y, trans, nullptr);
        op_spmv(s, n, op, y, v);
        double sig = 0.0;
        if (!dot(rh, v, sig)) return MSRSB_E_HIP;
        if (sig == 0.0 || !std::isfinite(sig)) { rc = MSRSB_E_BREAKDOWN; break; }
        alpha = rho / sig;
        lincomb(s, n, 1.0, r, -alpha, v, 0.0, nullptr, sv);  // s = r - alpha v
        ++it;
        double ss = 0.0;
        if (!dot(sv, sv, ss)) return MSRSB_E_HIP;
        if (std::sqrt(ss) <= o->rtol * fn) {
            lincomb(s, n, 1.0, x, alpha, y, 0.0, nullptr, x);
            if (hist && it < hcap) hist[it] = std::sqrt(ss) / fn;
            restart = true;
            continue;
        }
        apply_two_stage(c, o, sv, z, trans, nullptr);
        op_spmv(s, n, op, z, t);
        double tt = 0.0, ts = 0.0;
        if (!dot(t, t, tt) || !dot(t, sv, ts)) return MSRSB_E_HIP;
        if (tt == 0.0 || !std::isfinite(tt)) { rc = MSRSB_E_BREAKDOWN; break; }
        omega = ts / tt;
        lincomb(s, n, 1.0, x, alpha, y, omega, z, x);        // x += alpha y + omega z
        lincomb(s, n, 1.0, sv, -omega, t, 0.0, nullptr, r);  // r = s - omega t
        double rr = 0.0;
        if (!dot(r, r, rr)) return MSRSB_E_HIP;
        rn = std::sqrt(rr);
        const double rel = rn / fn;
        if (hist && it < hcap) hist[it] = rel;
        if (!std::isfinite(rel)) { rc = MSRSB_E_BREAKDOWN; break; }
        if (rel <= o->rtol) { restart = true; continue; }
        if (omega == 0.0) { rc = MSRSB_E_BREAKDOWN; break; }
        if (it >= o->max_iter) break;
    }
    op_residual(s, n, op, f, x, r);
    double rr = 0.0;
    if (!dot(r, r, rr)) return MSRSB_E_HIP;
    if (info) {
        info->iters = it;
        info->true_rel_res = std::sqrt(rr) / fn;
    }
    return rc;
}

}  // namespace msrsb
