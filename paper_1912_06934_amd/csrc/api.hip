// C ABI of the enhanced MsRSB library: argument checking, the state machine,
// symbolic set-up on the host (patterns, transposes, level sets) and the
// sequencing of device kernels.  Numerical work runs in the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>

#include "internal.h"
#include "solve.h"

using namespace msrsb;

namespace {

msrsb_status fail(msrsb_ctx *c, msrsb_status code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) hipSetDevice(d);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) hipSetDevice(prev);
    }
};

template <typename T>
void dfree(T *&p)
{
    if (p) hipFree(p);
    p = nullptr;
}

template <typename T>
bool dalloc(T *&p, size_t count)
{
    dfree(p);
    return hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T)) ==
           hipSuccess;
}

template <typename T>
bool dalloc_keep(T *&p, size_t count)
{
    if (p) return true;
    return hipMalloc(reinterpret_cast<void **>(&p), std::max<size_t>(count, 1) * sizeof(T)) ==
           hipSuccess;
}

hipMemcpyKind kind_in(int where)
{
    return where == MSRSB_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_out(int where)
{
    return where == MSRSB_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

bool valid_where(int where) { return where == MSRSB_HOST || where == MSRSB_DEVICE; }

// copy a caller buffer to a host vector (for checks and symbolic work)
template <typename T>
bool to_host(msrsb_ctx *c, std::vector<T> &out, const T *src, size_t count, int where)
{
    out.resize(count);
    if (count == 0) return true;
    if (where == MSRSB_HOST) {
        std::memcpy(out.data(), src, count * sizeof(T));
        return true;
    }
    if (hipMemcpyAsync(out.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return false;
    return hipStreamSynchronize(c->stream) == hipSuccess;
}

void phase_begin(msrsb_ctx *c, int ph)
{
    if (!c->ev_start[ph]) {
        hipEventCreate(&c->ev_start[ph]);
        hipEventCreate(&c->ev_stop[ph]);
    }
    hipEventRecord(c->ev_start[ph], c->stream);
}

void phase_end(msrsb_ctx *c, int ph)
{
    hipEventRecord(c->ev_stop[ph], c->stream);
    c->ev_used[ph] = true;
}

void free_matrix(msrsb_ctx *c)
{
    dfree(c->rp);
    dfree(c->ci);
    dfree(c->diag_pos);
    dfree(c->a);
    dfree(c->a32);
    dfree(c->at_rp);
    dfree(c->at_ci);
    dfree(c->at_src);
    dfree(c->at);
    dfree(c->at32);
    if (c->j_own_pattern) {
        dfree(c->jrp);
        dfree(c->jci);
    }
    c->jrp = c->jci = nullptr;
    c->j_own_pattern = false;
    dfree(c->jv);
    dfree(c->jv32);
    for (int o = 0; o < 2; ++o) {
        free_tri_order(c->tri[o]);
        dfree(c->ilu_f[o]);
        dfree(c->ic_f[o]);
        c->ilu_ok[o] = c->ic_ok[o] = false;
    }
    dfree(c->dinv_jac);
    dfree(c->dinv_l1);
    dfree(c->dinv_jac32);
    dfree(c->dinv_l1_32);
    dfree(c->dinv_jac_t);
    dfree(c->dinv_l1_t);
    dfree(c->dinv_jac32_t);
    dfree(c->dinv_l1_32_t);
    for (auto &p : c->w) dfree(p);
    for (auto &p : c->wf) dfree(p);
    dfree(c->gm_v);
    dfree(c->gm_h);
    c->gm_cap = 0;
    dfree(c->partials);
    dfree(c->partials_rr);
    dfree(c->tlogk);
    dfree(c->qk0);
    dfree(c->qlogE);
    dfree(c->qfixed);
    c->q1 = false;
    dfree(c->a_slot);
    dfree(c->a_dia);
    dfree(c->a_dia32);
    dfree(c->at_slot);
    dfree(c->at_dia);
    dfree(c->at_dia32);
    dfree(c->jcol_ell);
    dfree(c->ns_slot);
    dfree(c->a_ns_val);
    dfree(c->a_ns_val32);
    c->a_ns = NodeStencil();
    c->a_off = DiaOffsets();
    c->at_off = DiaOffsets();
    c->j_off = DiaOffsets();
    c->j_dia = false;
    c->jw = 0;
    c->a_symmetric = false;
    c->at_pattern = false;
    c->smoother_valid = c->smoother32_valid = false;
    c->smoother_t_valid = c->smoother32_t_valid = false;
    c->tpfa = false;
}

void free_coarse(msrsb_ctx *c)
{
    dfree(c->part);
    dfree(c->prp);
    dfree(c->pci);
    dfree(c->interior);
    for (int t = 0; t < 2; ++t) {
        dfree(c->p64[t]);
        dfree(c->p32[t]);
    }
    dfree(c->rrp);
    dfree(c->rci);
    dfree(c->rsrc);
    dfree(c->roff16);
    dfree(c->rbase);
    dfree(c->rbox);
    dfree(c->paxes);
    dfree(c->psplit_tab);
    dfree(c->psplit_wtab);
    c->psplit = SplitRows{};
    c->ps_valid = false;
    for (int t = 0; t < 2; ++t) {
        dfree(c->ps64[t]);
        dfree(c->ps32[t]);
    }
    dfree(c->r64);
    dfree(c->r32);
    dfree(c->ac);
    dfree(c->acinv);
    dfree(c->acinv_pk);
    dfree(c->symv_part);
    dfree(c->gj_b);
    dfree(c->spd_buf);
    dfree(c->piv);
    dfree(c->colsrc);
    dfree(c->vc);
    dfree(c->wc);
    dfree(c->partials);
    dfree(c->partials_rr);
    dfree(c->pcol_ell);
    dfree(c->pcol16);
    dfree(c->p_csr_tmp);
    dfree(c->band);
    dfree(c->rap_cols);
    dfree(c->rap_ncol);
    dfree(c->rap_order);
    c->rap_box_threads = 0;
    dfree(c->nrbox);
    dfree(c->npaxes);
    c->rap_nbox_threads = 0;
    c->ac_outside_zero = false;
    c->rap_cols_valid = false;
    if (c->jmap_idx) hipFree(c->jmap_idx);
    c->jmap_idx = nullptr;
    dfree(c->jmap_tab);
    c->jmap_kind = 0;
    c->jmap_ntab = 0;
    c->pw = 0;
    c->has_coarse = c->has_basis = c->has_coarse_op = false;
}

// Validate a CSR pattern: monotone row pointers, sorted in-range columns,
// diagonal present.  Fills diag positions.
bool check_csr(const std::vector<int> &rp, const std::vector<int> &ci, int n,
               std::vector<int> &dpos, std::string &why)
{
    if (rp[0] != 0) {
        why = "rowptr[0] must be 0";
        return false;
    }
    dpos.assign(n, -1);
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) {
            why = "rowptr not monotone at row " + std::to_string(i);
            return false;
        }
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int j = ci[e];
            if (j < 0 || j >= n) {
                why = "column out of range in row " + std::to_string(i);
                return false;
            }
            if (e > rp[i] && ci[e - 1] >= j) {
                why = "columns not strictly ascending in row " + std::to_string(i);
                return false;
            }
            if (j == i) dpos[i] = e;
        }
        if (dpos[i] < 0) {
            why = "missing diagonal in row " + std::to_string(i);
            return false;
        }
    }
    return true;
}

// The distinct column offsets j - i of a CSR pattern, ascending, if there are
// at most kMaxDiag of them (the operator is stored as diagonals then).
bool dia_offsets(const std::vector<int> &rp, const std::vector<int> &ci, int n,
                 std::vector<int> &offs)
{
    offs.clear();
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int d = ci[e] - i;
            if (std::find(offs.begin(), offs.end(), d) == offs.end()) {
                offs.push_back(d);
                if (static_cast<int>(offs.size()) > kMaxDiag) return false;
            }
        }
    std::sort(offs.begin(), offs.end());
    return !offs.empty();
}

// After A's values change: its DIA copy, the symmetry flag, A^T's values and
// the smoother data (rebuilt lazily).
msrsb_status refresh_values(msrsb_ctx *c)
{
    hipStream_t s = c->stream;
    if (c->a_off.n > 0) launch_csr_to_dia(s, c->n, c->a_off.n, c->rp, c->a_slot, c->a, c->a_dia, nullptr);
    if (c->a_ns.n > 0)
        launch_csr_to_nbs(s, c->n, c->a_ns.n * c->a_ns.bs, c->rp, c->ns_slot, c->a, c->a_ns_val,
                          nullptr);
    hipMemsetAsync(c->dev_flag, 0, sizeof(int), s);
    launch_check_symmetric(s, c->n, c->rp, c->ci, c->a, c->dev_flag);
    int flag = 1;
    hipMemcpyAsync(&flag, c->dev_flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (c->at_pattern) {
        launch_gather_values(s, c->nnz, c->at_src, c->a, c->at);
        if (c->at_off.n > 0)
            launch_csr_to_dia(s, c->n, c->at_off.n, c->at_rp, c->at_slot, c->at, c->at_dia, nullptr);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(c, MSRSB_E_HIP, "value update failed");
    c->a_symmetric = flag == 0;
    // symmetric stencil storage: the lower diagonals mirror the upper ones
    {
        const DiaOffsets &d = c->a_off;
        bool pairs = d.n > 0 && (d.n & 1) && d.off[d.n / 2] == 0;
        for (int o = 0; pairs && o < d.n; ++o) pairs = d.off[o] == -d.off[d.n - 1 - o];
        c->a_off.sym = c->a_symmetric && pairs ? 1 : 0;
    }
    c->smoother_valid = c->smoother32_valid = false;
    c->smoother_t_valid = c->smoother32_t_valid = false;
    c->ilu_ok[0] = c->ilu_ok[1] = c->ic_ok[0] = c->ic_ok[1] = false;
    return MSRSB_OK;
}

msrsb_status install_pattern(msrsb_ctx *c, int n, int64_t nnz, std::vector<int> &&hrp,
                             std::vector<int> &&hci, const std::vector<int> &dpos, int bs)
{
    free_matrix(c);
    c->n = n;
    c->nnz = nnz;
    c->bs = bs;
    c->h_rp = std::move(hrp);
    c->h_ci = std::move(hci);
    if (!dalloc(c->rp, n + 1) || !dalloc(c->ci, nnz) || !dalloc(c->diag_pos, n) ||
        !dalloc(c->a, nnz))
        return fail(c, MSRSB_E_NOMEM, "device allocation of A failed");
    hipMemcpyAsync(c->rp, c->h_rp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->ci, c->h_ci.data(), nnz * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->diag_pos, dpos.data(), n * sizeof(int), hipMemcpyHostToDevice, c->stream);
    // DIA form of A when its rows use at most kMaxDiag distinct offsets
    {
        std::vector<int> offs;
        if (dia_offsets(c->h_rp, c->h_ci, n, offs)) {
            c->a_off.n = static_cast<int>(offs.size());
            for (size_t t = 0; t < offs.size(); ++t) c->a_off.off[t] = offs[t];
            std::vector<int8_t> slot(nnz);
            for (int i = 0; i < n; ++i)
                for (int e = c->h_rp[i]; e < c->h_rp[i + 1]; ++e)
                    slot[e] = static_cast<int8_t>(
                        std::lower_bound(offs.begin(), offs.end(), c->h_ci[e] - i) - offs.begin());
            if (!dalloc(c->a_slot, nnz) || !dalloc(c->a_dia, static_cast<size_t>(n) * offs.size()))
                return fail(c, MSRSB_E_NOMEM, "device allocation of A (DIA) failed");
            hipMemcpy(c->a_slot, slot.data(), nnz, hipMemcpyHostToDevice);
        }
    }
    // NBS form of a vector operator that is no DIA stencil: every entry's node
    // offset from one set of at most 27, and each row's columns distinct slots
    if (bs > 1 && c->a_off.n == 0 && n % bs == 0) {
        std::vector<int> offs;
        bool ok = true;
        for (int i = 0; i < n && ok; ++i)
            for (int e = c->h_rp[i]; e < c->h_rp[i + 1] && ok; ++e) {
                const int d = c->h_ci[e] / bs - i / bs;
                if (std::find(offs.begin(), offs.end(), d) == offs.end()) {
                    offs.push_back(d);
                    ok = static_cast<int>(offs.size()) <= kMaxNodeOffsets;
                }
            }
        if (ok && !offs.empty()) {
            std::sort(offs.begin(), offs.end());
            std::vector<int8_t> slot(nnz);
            for (int i = 0; i < n; ++i)
                for (int e = c->h_rp[i]; e < c->h_rp[i + 1]; ++e) {
                    const int o = static_cast<int>(
                        std::lower_bound(offs.begin(), offs.end(), c->h_ci[e] / bs - i / bs) -
                        offs.begin());
                    slot[e] = static_cast<int8_t>(o * bs + c->h_ci[e] % bs);
                }
            c->a_ns.n = static_cast<int>(offs.size());
            c->a_ns.bs = bs;
            c->a_ns.nn = n / bs;
            for (size_t t = 0; t < offs.size(); ++t) c->a_ns.off[t] = offs[t];
            if (!dalloc(c->ns_slot, nnz) ||
                !dalloc(c->a_ns_val, static_cast<size_t>(n) * offs.size() * bs))
                return fail(c, MSRSB_E_NOMEM, "device allocation of A (node stencil) failed");
            hipMemcpy(c->ns_slot, slot.data(), nnz, hipMemcpyHostToDevice);
        }
    }
    // J's pattern: A's own for scalar problems, same-component entries otherwise
    std::vector<int> jrp, jci;
    const std::vector<int> *pjrp = &c->h_rp, *pjci = &c->h_ci;
    if (bs == 1) {
        c->jrp = c->rp;
        c->jci = c->ci;
        c->jnnz = nnz;
        c->j_own_pattern = false;
    } else {
        jrp.assign(n + 1, 0);
        jci.reserve(nnz / bs + n);
        for (int i = 0; i < n; ++i) {
            for (int e = c->h_rp[i]; e < c->h_rp[i + 1]; ++e)
                if (c->h_ci[e] % bs == i % bs) jci.push_back(c->h_ci[e]);
            jrp[i + 1] = static_cast<int>(jci.size());
        }
        c->jnnz = static_cast<int64_t>(jci.size());
        if (!dalloc(c->jrp, n + 1) || !dalloc(c->jci, c->jnnz))
            return fail(c, MSRSB_E_NOMEM, "device allocation of J failed");
        c->j_own_pattern = true;
        hipMemcpy(c->jrp, jrp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice);
        hipMemcpy(c->jci, jci.data(), c->jnnz * sizeof(int), hipMemcpyHostToDevice);
        pjrp = &jrp;
        pjci = &jci;
    }
    // J's values are stored [jw][n]: DIA order when its offsets are few, else
    // ELL with explicit columns
    {
        std::vector<int> offs;
        if (dia_offsets(*pjrp, *pjci, n, offs)) {
            c->j_dia = true;
            c->jw = static_cast<int>(offs.size());
            c->j_off.n = c->jw;
            for (int t = 0; t < c->jw; ++t) c->j_off.off[t] = offs[t];
        } else {
            int w = 0;
            for (int i = 0; i < n; ++i) w = std::max(w, (*pjrp)[i + 1] - (*pjrp)[i]);
            c->j_dia = false;
            c->jw = w;
            std::vector<int> jcol(static_cast<size_t>(w) * n, -1);
            for (int i = 0; i < n; ++i)
                for (int e = (*pjrp)[i]; e < (*pjrp)[i + 1]; ++e)
                    jcol[static_cast<size_t>(e - (*pjrp)[i]) * n + i] = (*pjci)[e];
            if (!dalloc(c->jcol_ell, jcol.size()))
                return fail(c, MSRSB_E_NOMEM, "device allocation of J failed");
            hipMemcpy(c->jcol_ell, jcol.data(), jcol.size() * sizeof(int), hipMemcpyHostToDevice);
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "copying the pattern failed");
    c->has_matrix = true;
    return MSRSB_OK;
}

// explicit transpose pattern of A with a source map for the values
msrsb_status ensure_transpose(msrsb_ctx *c)
{
    if (c->at_pattern) return MSRSB_OK;  // values are kept current by refresh_values
    const int n = c->n;
    std::vector<int> trp(n + 1, 0), tci(c->nnz), src(c->nnz);
    for (int64_t e = 0; e < c->nnz; ++e) trp[c->h_ci[e] + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    std::vector<int> pos(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int e = c->h_rp[i]; e < c->h_rp[i + 1]; ++e) {
            const int j = c->h_ci[e];
            tci[pos[j]] = i;
            src[pos[j]] = e;
            pos[j]++;
        }
    if (!dalloc(c->at_rp, n + 1) || !dalloc(c->at_ci, c->nnz) || !dalloc(c->at_src, c->nnz) ||
        !dalloc(c->at, c->nnz))
        return fail(c, MSRSB_E_NOMEM, "device allocation of A^T failed");
    hipMemcpyAsync(c->at_rp, trp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->at_ci, tci.data(), c->nnz * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->at_src, src.data(), c->nnz * sizeof(int), hipMemcpyHostToDevice,
                   c->stream);
    launch_gather_values(c->stream, c->nnz, c->at_src, c->a, c->at);
    std::vector<int> offs;
    if (dia_offsets(trp, tci, n, offs)) {
        c->at_off.n = static_cast<int>(offs.size());
        for (size_t t = 0; t < offs.size(); ++t) c->at_off.off[t] = offs[t];
        std::vector<int8_t> slot(c->nnz);
        for (int i = 0; i < n; ++i)
            for (int e = trp[i]; e < trp[i + 1]; ++e)
                slot[e] = static_cast<int8_t>(
                    std::lower_bound(offs.begin(), offs.end(), tci[e] - i) - offs.begin());
        if (!dalloc(c->at_slot, c->nnz) || !dalloc(c->at_dia, static_cast<size_t>(n) * offs.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of A^T (DIA) failed");
        hipMemcpyAsync(c->at_slot, slot.data(), c->nnz, hipMemcpyHostToDevice, c->stream);
        launch_csr_to_dia(c->stream, n, c->at_off.n, c->at_rp, c->at_slot, c->at, c->at_dia,
                          nullptr);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "building A^T failed");
    c->at_pattern = true;
    return MSRSB_OK;
}

msrsb_status solve_opts_check(msrsb_ctx *c, const msrsb_solve_opts *o)
{
    if (!o) return fail(c, MSRSB_E_ARG, "solve options are NULL");
    auto sm_ok = [](int k) { return k >= MSRSB_SMOOTH_NONE && k <= MSRSB_SMOOTH_IC0; };
    if (!sm_ok(o->pre_smoother) || !sm_ok(o->post_smoother) || o->pre_sweeps < 0 ||
        o->post_sweeps < 0 || o->pre_sweeps > 64 || o->post_sweeps > 64)
        return fail(c, MSRSB_E_ARG, "invalid smoother options");
    if (o->ordering != MSRSB_ORDER_NATURAL && o->ordering != MSRSB_ORDER_MULTICOLOR)
        return fail(c, MSRSB_E_ARG, "invalid sweep order");
    if (o->krylov < MSRSB_KRYLOV_PCG || o->krylov > MSRSB_KRYLOV_BICGSTAB)
        return fail(c, MSRSB_E_ARG, "invalid Krylov method");
    if (!(o->rtol > 0.0) || o->max_iter < 0)
        return fail(c, MSRSB_E_ARG, "rtol must be > 0 and max_iter >= 0");
    if (o->krylov == MSRSB_KRYLOV_GMRES && (o->restart < 1 || o->restart > 64))
        return fail(c, MSRSB_E_ARG, "GMRES restart must be in [1, 64]");
    if (o->use_multiscale && !c->has_coarse_op)
        return fail(c, MSRSB_E_STATE, "build_coarse must run before a multiscale apply");
    return MSRSB_OK;
}

// The levels below this one (multilevel): their apply options (the same
// smoothers, in FP64, with their own coarse stage), workspaces, smoother data
// and, for a transposed solve of a non-symmetric level, A_c^T.
msrsb_status ensure_levels(msrsb_ctx *c, const msrsb_solve_opts *o, bool trans)
{
    for (msrsb_ctx *l = c; l->child; l = l->child) {
        if (is_tri(o->pre_smoother) || is_tri(o->post_smoother))
            return fail(c, MSRSB_E_ARG, "the coarse levels take Jacobi-type smoothers only");
        msrsb_ctx *ch = l->child;
        l->child_opts = *o;
        l->child_opts.fp32_smoother = 0;
        l->child_opts.use_multiscale = 1;
        msrsb_status st = ensure_workspace(ch);
        if (st) return fail(c, st, "workspace allocation of a coarse level failed");
        if (trans && !ch->a_symmetric && (st = ensure_transpose(ch)))
            return fail(c, st, "next level: " + ch->err);
        if ((st = ensure_smoother(ch, &l->child_opts, trans)))
            return fail(c, st, "next level: " + ch->err);
    }
    return MSRSB_OK;
}

msrsb_status do_solve(msrsb_ctx *c, const double *f, double *u, const msrsb_solve_opts *o,
                      msrsb_solve_info *info, int where, bool trans)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_matrix) return fail(c, MSRSB_E_STATE, "no matrix set");
    if (!f || !u || !valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid vector arguments");
    msrsb_status st = solve_opts_check(c, o);
    if (st) return st;
    st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    if (trans && o->use_multiscale && c->restriction != MSRSB_RESTRICT_GALERKIN)
        return fail(c, MSRSB_E_ARG, "the transposed solve needs the Galerkin restriction");
    if (trans && !c->a_symmetric && (st = ensure_transpose(c))) return st;
    if ((st = ensure_smoother(c, o, trans))) return fail(c, st, c->err.empty() ? "smoother set-up failed" : c->err);
    if (o->use_multiscale && (st = ensure_levels(c, o, trans))) return st;
    const size_t bytes = static_cast<size_t>(c->n) * sizeof(double);
    // device buffers are used in place; host buffers are staged
    const double *df = f;
    double *dx = u;
    if (where == MSRSB_HOST) {
        hipMemcpyAsync(c->w[5], f, bytes, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(c->w[6], u, bytes, hipMemcpyHostToDevice, c->stream);
        df = c->w[5];
        dx = c->w[6];
    }
    const int ph = trans ? MSRSB_PHASE_SOLVE_T : MSRSB_PHASE_SOLVE;
    phase_begin(c, ph);
    switch (o->krylov) {
    case MSRSB_KRYLOV_PCG: st = pcg(c, df, dx, o, info, trans); break;
    case MSRSB_KRYLOV_GMRES: st = gmres(c, df, dx, o, info, trans); break;
    case MSRSB_KRYLOV_RICHARDSON: st = richardson(c, df, dx, o, info, trans); break;
    default: st = bicgstab(c, df, dx, o, info, trans); break;
    }
    phase_end(c, ph);
    // a device that stopped reporting (see wait_mailbox) is not waited for
    if (st == MSRSB_E_HIP) {
        const std::string why = c->err.empty() ? "solve failed on the device" : c->err;
        return fail(c, st, why);
    }
    if (where == MSRSB_HOST) hipMemcpyAsync(u, dx, bytes, hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "solve failed on the device");
    if (st == MSRSB_E_BREAKDOWN) return fail(c, st, "Krylov breakdown (non-finite value or p^T A p <= 0)");
    if (st == MSRSB_E_NOT_CONVERGED) return fail(c, st, "iteration limit reached");
    if (st) return fail(c, st, "solve failed");
    return MSRSB_OK;
}

}  // namespace

extern "C" {

msrsb_status msrsb_create(msrsb_ctx **out, int device, void *hip_stream)
{
    if (!out) return MSRSB_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return MSRSB_E_ARG;
    msrsb_ctx *c = new (std::nothrow) msrsb_ctx();
    if (!c) return MSRSB_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard g(device);
    if (!dalloc(c->dev_flag, 4) || !dalloc(c->eit_val, 1) || !dalloc(c->scal, S_COUNT)) {
        delete c;
        return MSRSB_E_NOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_pinned), 64 * sizeof(double),
                      hipHostMallocCoherent) != hipSuccess) {
        delete c;
        return MSRSB_E_NOMEM;
    }
    // the device address of the allocation-free apply's scratch array (once
    // per device; a failure only disables that entry point)
    c->scratch = static_scratch_init(device);
    *out = c;
    return MSRSB_OK;
}

void msrsb_destroy(msrsb_ctx *c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    hipStreamSynchronize(c->stream);
    if (c->child) msrsb_destroy(c->child);
    free_coarse(c);
    free_matrix(c);
    dfree(c->dev_flag);
    dfree(c->eit_val);
    dfree(c->scal);
    if (c->h_pinned) hipHostFree(c->h_pinned);
    for (int p = 0; p < MSRSB_N_PHASES; ++p)
        if (c->ev_start[p]) {
            hipEventDestroy(c->ev_start[p]);
            hipEventDestroy(c->ev_stop[p]);
        }
    delete c;
}

const char *msrsb_last_error(const msrsb_ctx *c) { return c ? c->err.c_str() : ""; }

msrsb_status msrsb_set_stream(msrsb_ctx *c, void *hip_stream)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    hipStreamSynchronize(c->stream);
    if (c->child) msrsb_set_stream(c->child, hip_stream);
    c->stream = static_cast<hipStream_t>(hip_stream);
    return MSRSB_OK;
}

msrsb_status msrsb_set_matrix(msrsb_ctx *c, int32_t n, int64_t nnz, const int32_t *rowptr,
                              const int32_t *col, const double *val, int32_t block_size,
                              int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (n < 1 || nnz < n || !rowptr || !col || !val || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid matrix arguments");
    if (block_size < 1 || block_size > 3 || n % block_size)
        return fail(c, MSRSB_E_ARG, "block_size must be 1..3 and divide n");
    if (nnz > INT32_MAX) return fail(c, MSRSB_E_ARG, "nnz exceeds int32 indexing");
    std::vector<int> hrp, hci, dpos;
    if (!to_host(c, hrp, rowptr, static_cast<size_t>(n) + 1, where) ||
        !to_host(c, hci, col, static_cast<size_t>(nnz), where))
        return fail(c, MSRSB_E_HIP, "reading the pattern failed");
    if (hrp[n] != nnz) return fail(c, MSRSB_E_ARG, "rowptr[n] != nnz");
    std::string why;
    if (!check_csr(hrp, hci, n, dpos, why)) return fail(c, MSRSB_E_ARG, why);
    free_coarse(c);
    msrsb_status st = install_pattern(c, n, nnz, std::move(hrp), std::move(hci), dpos, block_size);
    if (st) return st;
    hipMemcpyAsync(c->a, val, nnz * sizeof(double), kind_in(where), c->stream);
    return refresh_values(c);
}

msrsb_status msrsb_update_values(msrsb_ctx *c, const double *val, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_matrix) return fail(c, MSRSB_E_STATE, "no matrix set");
    if (!val || !valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid values");
    hipMemcpyAsync(c->a, val, c->nnz * sizeof(double), kind_in(where), c->stream);
    return refresh_values(c);
}

msrsb_status msrsb_get_matrix(msrsb_ctx *c, int32_t *rowptr, int32_t *col, double *val, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_matrix) return fail(c, MSRSB_E_STATE, "no matrix set");
    if (!valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid where");
    if (rowptr)
        hipMemcpyAsync(rowptr, c->rp, (c->n + 1) * sizeof(int), kind_out(where), c->stream);
    if (col) hipMemcpyAsync(col, c->ci, c->nnz * sizeof(int), kind_out(where), c->stream);
    if (val) hipMemcpyAsync(val, c->a, c->nnz * sizeof(double), kind_out(where), c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "copy failed");
    return MSRSB_OK;
}

msrsb_status msrsb_assemble_tpfa(msrsb_ctx *c, int32_t dim, const int32_t dims[3],
                                 const double h[3], const double *log_k, const double bc[6],
                                 double *rhs_out, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if ((dim != 2 && dim != 3) || !dims || !h || !log_k || !bc || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid TPFA arguments");
    const int nx = dims[0], ny = dims[1], nz = dim == 3 ? dims[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1 || static_cast<int64_t>(nx) * ny * nz > (1 << 28))
        return fail(c, MSRSB_E_ARG, "invalid grid size");
    for (int d = 0; d < dim; ++d)
        if (!(h[d] > 0.0)) return fail(c, MSRSB_E_ARG, "cell sizes must be positive");
    const int n = nx * ny * nz;
    const bool same = c->tpfa && c->has_matrix && c->tdim == dim && c->tdims[0] == nx &&
                      c->tdims[1] == ny && c->tdims[2] == nz;
    if (!same) {
        // symbolic pattern: neighbours in ascending index order
        std::vector<int> hrp(n + 1, 0), hci, dpos(n);
        hci.reserve(static_cast<size_t>(n) * (2 * dim + 1));
        const int stride[3] = {1, nx, nx * ny};
        const int nd[3] = {nx, ny, nz};
        for (int cidx = 0; cidx < n; ++cidx) {
            const int xyz[3] = {cidx % nx, (cidx / nx) % ny, cidx / (nx * ny)};
            for (int d = dim - 1; d >= 0; --d)
                if (xyz[d] > 0) hci.push_back(cidx - stride[d]);
            dpos[cidx] = static_cast<int>(hci.size());
            hci.push_back(cidx);
            for (int d = 0; d < dim; ++d)
                if (xyz[d] + 1 < nd[d]) hci.push_back(cidx + stride[d]);
            hrp[cidx + 1] = static_cast<int>(hci.size());
        }
        const int64_t nnz = static_cast<int64_t>(hci.size());
        free_coarse(c);
        msrsb_status st = install_pattern(c, n, nnz, std::move(hrp), std::move(hci), dpos, 1);
        if (st) return st;
        c->tpfa = true;
        c->tdim = dim;
        c->tdims[0] = nx;
        c->tdims[1] = ny;
        c->tdims[2] = nz;
    }
    for (int d = 0; d < 3; ++d) c->th[d] = d < dim ? h[d] : 1.0;
    for (int t = 0; t < 6; ++t) c->tbc[t] = bc[t];
    if (!dalloc_keep(c->tlogk, n)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
    double *drhs = nullptr;
    if (rhs_out) {
        if (!dalloc_keep(c->w[11], n)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
        drhs = c->w[11];
    }
    hipMemcpyAsync(c->tlogk, log_k, n * sizeof(double), kind_in(where), c->stream);
    phase_begin(c, MSRSB_PHASE_ASSEMBLE);
    launch_tpfa_values(c->stream, dim, c->tdims, c->th, c->tbc, c->tlogk, c->rp, c->a, drhs);
    phase_end(c, MSRSB_PHASE_ASSEMBLE);
    if (rhs_out) hipMemcpyAsync(rhs_out, drhs, n * sizeof(double), kind_out(where), c->stream);
    return refresh_values(c);
}

msrsb_status msrsb_set_coarse(msrsb_ctx *c, int32_t nc, const int32_t *part,
                              const int32_t *sup_rowptr, const int32_t *sup_col,
                              const uint8_t *interior, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->has_matrix) return fail(c, MSRSB_E_STATE, "set_matrix must come first");
    if (nc < 1 || nc > kMaxCoarseLevel)
        return fail(c, MSRSB_E_ARG, "nc must be in [1, " + std::to_string(kMaxCoarseLevel) + "]");
    if (!part || !sup_rowptr || !sup_col || !interior || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid coarse arguments");
    const int n = c->n;
    std::vector<int> hpart, hprp, hpci;
    std::vector<uint8_t> hint;
    if (!to_host(c, hpart, part, n, where) || !to_host(c, hprp, sup_rowptr, n + 1, where))
        return fail(c, MSRSB_E_HIP, "reading the partition failed");
    if (hprp[0] != 0 || hprp[n] < n) return fail(c, MSRSB_E_ARG, "invalid support rowptr");
    const int64_t pnnz = hprp[n];
    if (!to_host(c, hpci, sup_col, pnnz, where) || !to_host(c, hint, interior, n, where))
        return fail(c, MSRSB_E_HIP, "reading the supports failed");
    int maxw = 0;
    for (int i = 0; i < n; ++i) {
        const int w = hprp[i + 1] - hprp[i];
        if (w < 1 || w > kMaxPatternWidth)
            return fail(c, MSRSB_E_ARG, "support row " + std::to_string(i) +
                                            " must have 1.." + std::to_string(kMaxPatternWidth) +
                                            " entries");
        maxw = std::max(maxw, w);
        bool found = false;
        for (int e = hprp[i]; e < hprp[i + 1]; ++e) {
            if (hpci[e] < 0 || hpci[e] >= nc)
                return fail(c, MSRSB_E_ARG, "support column out of range in row " +
                                                std::to_string(i));
            if (e > hprp[i] && hpci[e - 1] >= hpci[e])
                return fail(c, MSRSB_E_ARG, "support columns not ascending in row " +
                                                std::to_string(i));
            if (hpci[e] == hpart[i]) found = true;
        }
        if (!found)
            return fail(c, MSRSB_E_ARG, "part[" + std::to_string(i) + "] not in its support row");
    }
    {
        // every coarse block holds a row (its basis function starts there)
        std::vector<uint8_t> owned(nc, 0);
        for (int i = 0; i < n; ++i) owned[hpart[i]] = 1;
        for (int j = 0; j < nc; ++j)
            if (!owned[j])
                return fail(c, MSRSB_E_ARG, "coarse block " + std::to_string(j) + " has no row");
    }
    free_coarse(c);
    if (c->child) {  // a new coarse space replaces every level below it
        msrsb_destroy(c->child);
        c->child = nullptr;
    }
    c->nc = nc;
    c->pnnz = pnnz;
    c->pmaxw = maxw;
    c->pw = maxw <= 4 ? 4 : (maxw <= kMapWidth ? kMapWidth : maxw);
    const int pw = c->pw;
    c->h_prp = hprp;
    c->h_pci = hpci;
    if (static_cast<int64_t>(pw) * n >= INT32_MAX)
        return fail(c, MSRSB_E_ARG, "support pattern too large for int32 ELL indexing");
    // P's ELL columns, and R = P^T (coarse rows, fine rows ascending) with the
    // ELL index of every entry
    std::vector<int> pcol(static_cast<size_t>(pw) * n, -1);
    for (int i = 0; i < n; ++i)
        for (int e = hprp[i]; e < hprp[i + 1]; ++e)
            pcol[static_cast<size_t>(i) * pw + (e - hprp[i])] = hpci[e];
    // rows padded to multiples of 64 entries: a pad repeats the row's last
    // column with value 0 (rsrc = -1)
    std::vector<int> rlen(nc, 0);
    for (int64_t e = 0; e < pnnz; ++e) rlen[hpci[e]]++;
    std::vector<int> rrp(nc + 1, 0);
    for (int jj = 0; jj < nc; ++jj) rrp[jj + 1] = rrp[jj] + (rlen[jj] + 63) / 64 * 64;
    const int64_t rnnz = rrp[nc];
    int rmaxlen = 0;
    for (int jj = 0; jj < nc; ++jj) rmaxlen = std::max(rmaxlen, rrp[jj + 1] - rrp[jj]);
    std::vector<int> rci(rnnz), rsrc(rnnz, -1);
    {
        std::vector<int> pos(rrp.begin(), rrp.end() - 1);
        for (int i = 0; i < n; ++i)
            for (int e = hprp[i]; e < hprp[i + 1]; ++e) {
                const int jj = hpci[e];
                rci[pos[jj]] = i;
                rsrc[pos[jj]] = i * pw + (e - hprp[i]);
                pos[jj]++;
            }
        for (int jj = 0; jj < nc; ++jj)
            for (int t = pos[jj]; t < rrp[jj + 1]; ++t) rci[t] = rci[t - 1];
    }
    // supports that are boxes of the assembled grid: the restriction then
    // forms its columns instead of loading them.  Every entry is checked
    // against the box formula, so the fast path is exact whenever it is taken.
    std::vector<int> rbox;
    if (c->tpfa && c->bs == 1) {
        const int nx = c->tdims[0], ny = c->tdims[1];
        const int64_t nxy = static_cast<int64_t>(nx) * ny;
        rbox.resize(static_cast<size_t>(nc) * 4);
        for (int jj = 0; jj < nc && !rbox.empty(); ++jj) {
            const int len = rlen[jj], r0 = rrp[jj];
            if (len == 0) {
                rbox.clear();
                break;
            }
            const int f = rci[r0], l = rci[r0 + len - 1];
            const int x0 = f % nx, y0 = (f / nx) % ny, z0 = static_cast<int>(f / nxy);
            const int bx = l % nx - x0 + 1, by = (l / nx) % ny - y0 + 1;
            const int bz = static_cast<int>(l / nxy) - z0 + 1;
            bool ok = len <= 65536 && bx > 0 && by > 0 && bz > 0 &&
                      static_cast<int64_t>(bx) * by * bz == len;
            for (int q = 0; q < len && ok; ++q) {
                const int qx = q % bx, qy = (q / bx) % by, qz = q / (bx * by);
                ok = rci[r0 + q] == f + qx + qy * nx + qz * nxy;
            }
            if (!ok) {
                rbox.clear();
                break;
            }
            rbox[4 * jj] = f;
            rbox[4 * jj + 1] = bx;
            rbox[4 * jj + 2] = bx * by;
            rbox[4 * jj + 3] = len;
        }
    }
    // P's columns as products of per-axis candidates (box supports on a grid):
    // the coarse grid's extent from the boxes' origins, one table per axis,
    // then every row of the pattern checked against the product it implies
    std::vector<int> paxes;
    int ncx = 0, ncxy = 0;
    if (!rbox.empty() && (pw == 4 || pw == 8)) {
        const int nx = c->tdims[0], ny = c->tdims[1], nz = c->tdims[2];
        const int nxy = nx * ny;
        auto ox = [&](int j) { return rbox[4 * j] % nx; };
        auto oy = [&](int j) { return (rbox[4 * j] / nx) % ny; };
        auto oz = [&](int j) { return rbox[4 * j] / nxy; };
        int cx = 1, cy = 1;
        while (cx < nc && oy(cx) == oy(0) && oz(cx) == oz(0)) ++cx;
        while (cy * cx < nc && oz(cy * cx) == oz(0)) ++cy;
        bool ok = nc % (cx * cy) == 0;
        const int cz = ok ? nc / (cx * cy) : 0;
        // tab entries: first candidate | count << 16, counts 1 or 2
        auto axis = [&](int len, int nn, auto lo, auto ext) {
            for (int x = 0; x < len && ok; ++x) {
                int first = -1, cnt = 0;
                for (int a = 0; a < nn; ++a)
                    if (x >= lo(a) && x < lo(a) + ext(a)) {
                        if (first < 0) first = a;
                        ok = ok && a == first + cnt;
                        ++cnt;
                    }
                ok = ok && cnt >= 1 && cnt <= 2 && first <= 0xFFFF;
                if (ok) paxes.push_back(first | cnt << 16);
            }
        };
        axis(nx, cx, [&](int a) { return ox(a); }, [&](int a) { return rbox[4 * a + 1]; });
        axis(ny, cy, [&](int a) { return oy(a * cx); },
             [&](int a) { return rbox[4 * a * cx + 2] / rbox[4 * a * cx + 1]; });
        axis(nz, cz, [&](int a) { return oz(a * cx * cy); },
             [&](int a) { return rbox[4 * a * cx * cy + 3] / rbox[4 * a * cx * cy + 2]; });
        for (int i = 0; i < n && ok; ++i) {
            const int x = i % nx, y = (i / nx) % ny, z = i / nxy;
            const int tx = paxes[x], ty = paxes[nx + y], tz = paxes[nx + ny + z];
            const int kx = tx >> 16, ky = ty >> 16, kz = tz >> 16;
            ok = hprp[i + 1] - hprp[i] == kx * ky * kz;
            int e = hprp[i];
            for (int iz = 0; iz < kz && ok; ++iz)
                for (int iy = 0; iy < ky && ok; ++iy)
                    for (int ix = 0; ix < kx && ok; ++ix, ++e)
                        ok = hpci[e] == (tx & 0xFFFF) + ix + cx * ((ty & 0xFFFF) + iy) +
                                            cx * cy * ((tz & 0xFFFF) + iz);
        }
        if (ok) {
            ncx = cx;
            ncxy = cx * cy;
        } else {
            paxes.clear();
        }
    }
    // the box form of R A P: the cells next to a coarse node's support have
    // their candidates within one node of it on every axis, and the support
    // box widened by one cell has at most 512 (x, y) columns
    int rap_box_threads = 0;
    if (!paxes.empty() && pw == 8) {
        const int nx = c->tdims[0], ny = c->tdims[1], nz = c->tdims[2];
        const int cdim[3] = {ncx, ncxy / ncx, nc / ncxy};
        const int alen[3] = {nx, ny, nz}, abase[3] = {0, nx, nx + ny};
        bool ok = true;
        for (int ax = 0; ax < 3 && ok; ++ax) {
            std::vector<int> first(cdim[ax], -1), last(cdim[ax], -1);
            for (int x = 0; x < alen[ax]; ++x) {
                const int t = paxes[abase[ax] + x], c0 = t & 0xFFFF, cn = t >> 16;
                for (int q = c0; q < c0 + cn && q < cdim[ax]; ++q) {
                    if (first[q] < 0) first[q] = x;
                    last[q] = x;
                }
            }
            for (int q = 0; q < cdim[ax] && ok; ++q) {
                ok = first[q] >= 0;
                const int x1 = std::min(last[q] + 1, alen[ax] - 1);
                for (int x = std::max(first[q] - 1, 0); ok && x <= x1; ++x) {
                    const int t = paxes[abase[ax] + x], c0 = t & 0xFFFF, cn = t >> 16;
                    ok = c0 >= q - 1 && c0 + cn - 1 <= q + 1;
                }
            }
        }
        int maxcols = 0;
        for (int jj = 0; jj < nc && ok; ++jj) {
            const int f = rbox[4 * jj], bx = rbox[4 * jj + 1], by = rbox[4 * jj + 2] / bx;
            const int x0 = f % nx, y0 = (f / nx) % ny;
            const int ex = std::min(x0 + bx + 1, nx) - std::max(x0 - 1, 0);
            const int ey = std::min(y0 + by + 1, ny) - std::max(y0 - 1, 0);
            maxcols = std::max(maxcols, ex * ey);
        }
        if (ok && maxcols <= 512) rap_box_threads = (maxcols + 63) / 64 * 64;
    }
    // the box form of R A P for a node-block operator (3 components per node,
    // 27 node offsets): the node grid from the stencil's offsets, each coarse
    // node's support as a box of nodes (the same for its three dofs, checked
    // on R's rows), P's per-axis candidate coarse nodes (checked on every P
    // row), then the same window and size conditions as the scalar form
    std::vector<int> nrbox, npaxes;
    int ndims[3] = {0, 0, 0}, ncdims[3] = {0, 0, 0}, rap_nbox_threads = 0;
    if (c->bs == 3 && c->a_ns.n == 27 && pw == 8 && nc % 3 == 0) {
        const int nn = n / 3, ncn = nc / 3;
        const int nxn = c->a_ns.off[16], nxyn = c->a_ns.off[22];
        bool ok = nxn >= 3 && nxyn >= 3 * nxn && nxyn % nxn == 0 && nn % nxyn == 0;
        for (int o = 0; o < 27 && ok; ++o) {
            const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            ok = c->a_ns.off[o] == dx + nxn * dy + nxyn * dz;
        }
        const int nyn = ok ? nxyn / nxn : 0, nzn = ok ? nn / nxyn : 0;
        // support boxes of the coarse nodes, from R's rows of their dofs
        if (ok) nrbox.resize(static_cast<size_t>(ncn) * 4);
        for (int J = 0; J < ncn && ok; ++J) {
            const int len = rlen[3 * J];
            ok = len > 0 && rlen[3 * J + 1] == len && rlen[3 * J + 2] == len;
            if (!ok) break;
            const int r0 = rrp[3 * J];
            const int f = rci[r0] / 3, l = rci[r0 + len - 1] / 3;
            const int x0 = f % nxn, y0 = (f / nxn) % nyn, z0 = f / nxyn;
            const int bx = l % nxn - x0 + 1, by = (l / nxn) % nyn - y0 + 1, bz = l / nxyn - z0 + 1;
            ok = bx > 0 && by > 0 && bz > 0 && static_cast<int64_t>(bx) * by * bz == len &&
                 len <= 65536;
            for (int q = 0; q < len && ok; ++q) {
                const int node = f + q % bx + ((q / bx) % by) * nxn + (q / (bx * by)) * nxyn;
                for (int cmp = 0; cmp < 3 && ok; ++cmp)
                    ok = rci[rrp[3 * J + cmp] + q] == 3 * node + cmp;
            }
            nrbox[4 * J] = f;
            nrbox[4 * J + 1] = bx;
            nrbox[4 * J + 2] = bx * by;
            nrbox[4 * J + 3] = len;
        }
        // the coarse node grid from the boxes' origins, then per-axis tables
        int cx = 1, cy = 1;
        if (ok) {
            auto oy = [&](int J) { return (nrbox[4 * J] / nxn) % nyn; };
            auto oz = [&](int J) { return nrbox[4 * J] / nxyn; };
            while (cx < ncn && oy(cx) == oy(0) && oz(cx) == oz(0)) ++cx;
            while (cy * cx < ncn && oz(cy * cx) == oz(0)) ++cy;
            ok = ncn % (cx * cy) == 0;
        }
        const int cz = ok ? ncn / (cx * cy) : 0;
        auto axis = [&](int len, int cnt_axis, auto lo, auto ext) {
            for (int x = 0; x < len && ok; ++x) {
                int first = -1, cnt = 0;
                for (int a = 0; a < cnt_axis; ++a)
                    if (x >= lo(a) && x < lo(a) + ext(a)) {
                        if (first < 0) first = a;
                        ok = ok && a == first + cnt;
                        ++cnt;
                    }
                ok = ok && cnt >= 1 && cnt <= 2 && first <= 0xFFFF;
                if (ok) npaxes.push_back(first | cnt << 16);
            }
        };
        if (ok) {
            axis(nxn, cx, [&](int a) { return nrbox[4 * a] % nxn; },
                 [&](int a) { return nrbox[4 * a + 1]; });
            axis(nyn, cy, [&](int a) { return (nrbox[4 * a * cx] / nxn) % nyn; },
                 [&](int a) { return nrbox[4 * a * cx + 2] / nrbox[4 * a * cx + 1]; });
            axis(nzn, cz, [&](int a) { return nrbox[4 * a * cx * cy] / nxyn; },
                 [&](int a) { return nrbox[4 * a * cx * cy + 3] / nrbox[4 * a * cx * cy + 2]; });
        }
        // every P row: dof 3 i + l reaches the dofs 3 K + l of the product of
        // node i's candidates, ascending
        for (int i = 0; i < nn && ok; ++i) {
            const int x = i % nxn, y = (i / nxn) % nyn, z = i / nxyn;
            const int tx = npaxes[x], ty = npaxes[nxn + y], tz = npaxes[nxn + nyn + z];
            const int kx = tx >> 16, ky = ty >> 16, kz = tz >> 16;
            for (int cmp = 0; cmp < 3 && ok; ++cmp) {
                const int row = 3 * i + cmp;
                ok = hprp[row + 1] - hprp[row] == kx * ky * kz;
                int e = hprp[row];
                for (int iz = 0; iz < kz && ok; ++iz)
                    for (int iy = 0; iy < ky && ok; ++iy)
                        for (int ix = 0; ix < kx && ok; ++ix, ++e)
                            ok = hpci[e] == 3 * ((tx & 0xFFFF) + ix + cx * ((ty & 0xFFFF) + iy) +
                                                 cx * cy * ((tz & 0xFFFF) + iz)) + cmp;
            }
        }
        // nodes next to a support have their candidates within one coarse
        // node of it on every axis; the widened boxes fit a work-group
        const int cdim[3] = {cx, cy, cz}, alen[3] = {nxn, nyn, nzn}, abase[3] = {0, nxn, nxn + nyn};
        for (int ax = 0; ax < 3 && ok; ++ax) {
            std::vector<int> first(cdim[ax], -1), last(cdim[ax], -1);
            for (int x = 0; x < alen[ax]; ++x) {
                const int t = npaxes[abase[ax] + x], c0 = t & 0xFFFF, cn = t >> 16;
                for (int q = c0; q < c0 + cn && q < cdim[ax]; ++q) {
                    if (first[q] < 0) first[q] = x;
                    last[q] = x;
                }
            }
            for (int q = 0; q < cdim[ax] && ok; ++q) {
                ok = first[q] >= 0;
                const int x1 = std::min(last[q] + 1, alen[ax] - 1);
                for (int x = std::max(first[q] - 1, 0); ok && x <= x1; ++x) {
                    const int t = npaxes[abase[ax] + x], c0 = t & 0xFFFF, cn = t >> 16;
                    ok = c0 >= q - 1 && c0 + cn - 1 <= q + 1;
                }
            }
        }
        int maxcols = 0;
        for (int J = 0; J < ncn && ok; ++J) {
            const int f = nrbox[4 * J], bx = nrbox[4 * J + 1], by = nrbox[4 * J + 2] / bx;
            const int x0 = f % nxn, y0 = (f / nxn) % nyn;
            const int ex = std::min(x0 + bx + 1, nxn) - std::max(x0 - 1, 0);
            const int ey = std::min(y0 + by + 1, nyn) - std::max(y0 - 1, 0);
            maxcols = std::max(maxcols, ex * ey);
        }
        if (ok && maxcols <= 512) {
            rap_nbox_threads = (maxcols + 63) / 64 * 64;
            ndims[0] = nxn;
            ndims[1] = nyn;
            ndims[2] = nzn;
            ncdims[0] = cx;
            ncdims[1] = cy;
            ncdims[2] = cz;
        } else {
            nrbox.clear();
            npaxes.clear();
        }
    }
    // 16-bit column offsets when every 64-entry group spans fewer than 2^16 rows
    bool r16 = true;
    std::vector<int> rbase(rnnz / 64);
    std::vector<uint16_t> roff(rnnz);
    for (int64_t g = 0; g < rnnz / 64 && r16; ++g) {
        rbase[g] = rci[64 * g];
        for (int u = 0; u < 64; ++u) {
            const int d = rci[64 * g + u] - rbase[g];
            if (d < 0 || d > 0xFFFF) { r16 = false; break; }
            roff[64 * g + u] = static_cast<uint16_t>(d);
        }
    }
    c->rnnz = rnnz;
    c->rmaxlen = rmaxlen;
    c->rap_box_threads = rap_box_threads;
    c->rap_nbox_threads = rap_nbox_threads;
    for (int a = 0; a < 3; ++a) {
        c->ndims[a] = ndims[a];
        c->ncdims[a] = ncdims[a];
    }
    if (!dalloc(c->part, n) || !dalloc(c->prp, n + 1) || !dalloc(c->pci, pnnz) ||
        !dalloc(c->interior, n) || !dalloc(c->rrp, nc + 1) || !dalloc(c->rci, rnnz) ||
        !dalloc(c->rsrc, rnnz) ||
        (r16 && (!dalloc(c->roff16, rnnz) || !dalloc(c->rbase, rnnz / 64))) ||
        !dalloc(c->pcol_ell, pcol.size()) || !dalloc(c->band, 2))
        return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
    // the dense coarse operator and its inverse: only for a coarse space small
    // enough to be the last level (a larger one needs a further level, whose
    // matrix is the sparse A_c)
    c->dense_coarse = nc <= kMaxCoarse;
    if (c->dense_coarse) {
        const size_t nn = static_cast<size_t>(nc) * nc;
        const int ntc = (nc + 63) / 64, ntri = ntc * (ntc + 1) / 2;
        if (!dalloc(c->ac, nn) || !dalloc(c->acinv, nn) ||
            !dalloc(c->acinv_pk, static_cast<size_t>(ntri) * 64 * 64) ||
            !dalloc(c->symv_part, static_cast<size_t>(ntri) * 128) ||
            !dalloc(c->gj_b, 8 * 64 + 64 * static_cast<size_t>(nc) + nn) ||
            !dalloc(c->piv, nc) || !dalloc(c->colsrc, nc) ||
            !dalloc(c->spd_buf, static_cast<size_t>((nc + 63) / 64) * 64 * 64))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
    }
    hipMemcpyAsync(c->part, hpart.data(), n * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->prp, hprp.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->pci, hpci.data(), pnnz * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->interior, hint.data(), n, hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->rrp, rrp.data(), (nc + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->rci, rci.data(), rnnz * sizeof(int), hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->rsrc, rsrc.data(), rnnz * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (r16) {
        hipMemcpyAsync(c->roff16, roff.data(), rnnz * sizeof(uint16_t), hipMemcpyHostToDevice,
                       c->stream);
        hipMemcpyAsync(c->rbase, rbase.data(), rnnz / 64 * sizeof(int), hipMemcpyHostToDevice,
                       c->stream);
    }
    if (!paxes.empty()) {
        // the product's row order: 4 x 4 x 4 bricks of coarse nodes (ragged
        // at the far faces), bricks and the nodes in a brick lexicographic
        const int cx = ncx, cy = ncxy / ncx, cz = nc / ncxy;
        std::vector<int> order;
        order.reserve(nc);
        for (int bz = 0; bz < cz; bz += 4)
            for (int by = 0; by < cy; by += 4)
                for (int bx = 0; bx < cx; bx += 4)
                    for (int z = bz; z < std::min(bz + 4, cz); ++z)
                        for (int y = by; y < std::min(by + 4, cy); ++y)
                            for (int x = bx; x < std::min(bx + 4, cx); ++x)
                                order.push_back(x + cx * (y + cy * z));
        if (!dalloc(c->rap_order, order.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        hipMemcpyAsync(c->rap_order, order.data(), order.size() * sizeof(int),
                       hipMemcpyHostToDevice, c->stream);
        if (!dalloc(c->paxes, paxes.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        hipMemcpyAsync(c->paxes, paxes.data(), paxes.size() * sizeof(int), hipMemcpyHostToDevice,
                       c->stream);
        c->pax_ncx = ncx;
        c->pax_ncxy = ncxy;
        // P's split form for the smoothing iteration (8-slot rows on a 3D
        // grid): per axis, the two-candidate positions before each position
        // times the counts of the faster axes, bit 31 for two candidates
        const int gdim[3] = {c->tdims[0], c->tdims[1], c->tdims[2]};
        if (pw == 8 && gdim[0] > 1 && gdim[1] > 1 && gdim[2] > 1) {
            std::vector<int> st(static_cast<size_t>(gdim[0]) + gdim[1] + gdim[2]);
            int64_t scale = 1;
            bool ok = true;
            for (int ax = 0, base = 0; ax < 3; base += gdim[ax], ++ax) {
                int64_t cnt2 = 0;
                for (int x = 0; x < gdim[ax]; ++x) {
                    const bool two = (paxes[base + x] >> 16) == 2;
                    const int64_t v = cnt2 * scale;
                    ok = ok && v < (int64_t{1} << 29);
                    st[base + x] = static_cast<int>(v & 0x7FFFFFFF) |
                                   (two ? static_cast<int>(0x80000000u) : 0);
                    cnt2 += two ? 1 : 0;
                }
                scale *= cnt2;
            }
            // the three parts of an index (and of a neighbour's) sum below
            // 2^31, and the second halves' bytes (FP64) stay below 2^31 (one
            // buffer resource covers them)
            if (ok && scale * 32 <= INT32_MAX) {
                // per 64 rows: first second-half index and the 8-entry mask
                std::vector<int4> wt((n + 63) / 64, make_int4(0, 0, 0, 0));
                int h8 = 0;
                for (int i = 0; i < n; ++i) {
                    const int x = i % gdim[0], y = (i / gdim[0]) % gdim[1],
                              z = i / (gdim[0] * gdim[1]);
                    const bool f8 = (st[x] & st[gdim[0] + y] & st[gdim[0] + gdim[1] + z]) < 0;
                    int4 &e = wt[i / 64];
                    if (i % 64 == 0) e.x = h8;
                    if (f8) {
                        const int b = i % 64;
                        if (b < 32)
                            e.y = static_cast<int>(static_cast<uint32_t>(e.y) | (1u << b));
                        else
                            e.z = static_cast<int>(static_cast<uint32_t>(e.z) | (1u << (b - 32)));
                        ++h8;
                    }
                }
                if (!dalloc(c->psplit_tab, st.size()) || !dalloc(c->psplit_wtab, wt.size()))
                    return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
                hipMemcpyAsync(c->psplit_wtab, wt.data(), wt.size() * sizeof(int4),
                               hipMemcpyHostToDevice, c->stream);
                hipMemcpyAsync(c->psplit_tab, st.data(), st.size() * sizeof(int),
                               hipMemcpyHostToDevice, c->stream);
                c->psplit.tab = c->psplit_tab;
                c->psplit.nx = gdim[0];
                c->psplit.ny = gdim[1];
                c->psplit.nz = gdim[2];
                c->psplit.rnx = 1.0 / gdim[0];
                c->psplit.rny = 1.0 / gdim[1];
                c->psplit.n8 = scale;
            }
        }
    }
    if (rap_nbox_threads > 0) {
        if (!dalloc(c->nrbox, nrbox.size()) || !dalloc(c->npaxes, npaxes.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        hipMemcpyAsync(c->nrbox, nrbox.data(), nrbox.size() * sizeof(int), hipMemcpyHostToDevice,
                       c->stream);
        hipMemcpyAsync(c->npaxes, npaxes.data(), npaxes.size() * sizeof(int),
                       hipMemcpyHostToDevice, c->stream);
    }
    if (!rbox.empty()) {
        if (!dalloc(c->rbox, rbox.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        hipMemcpyAsync(c->rbox, rbox.data(), rbox.size() * sizeof(int), hipMemcpyHostToDevice,
                       c->stream);
    }
    hipMemcpyAsync(c->pcol_ell, pcol.data(), pcol.size() * sizeof(int), hipMemcpyHostToDevice,
                   c->stream);
    std::vector<uint16_t> pcol16;
    if ((pw == 4 || pw == 8) && nc < 0xFFFF) {
        pcol16.resize(pcol.size());
        for (size_t t = 0; t < pcol.size(); ++t)
            pcol16[t] = pcol[t] < 0 ? 0xFFFFu : static_cast<uint16_t>(pcol[t]);
        if (!dalloc(c->pcol16, pcol16.size()))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        hipMemcpyAsync(c->pcol16, pcol16.data(), pcol16.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice, c->stream);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "copying the coarse data failed");
    // slot maps of the smoothing product, stored as indices into a table of
    // the distinct maps (one byte per J entry when there are at most 256)
    if (maxw <= kMapWidth) {
        const size_t m = static_cast<size_t>(c->jw) * n;
        uint32_t *dmaps = nullptr;
        if (!dalloc(dmaps, m)) return fail(c, MSRSB_E_NOMEM, "allocation of the slot maps failed");
        launch_build_maps(c->stream, n, pw, c->jw, c->j_off, c->j_dia ? nullptr : c->jcol_ell,
                          c->jrp, c->jci, c->pcol_ell, dmaps);
        std::vector<uint32_t> hm(m);
        hipMemcpyAsync(hm.data(), dmaps, m * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            dfree(dmaps);
            return fail(c, MSRSB_E_HIP, "building the slot maps failed");
        }
        std::unordered_map<uint32_t, uint32_t> dict;
        std::vector<uint32_t> table;
        std::vector<uint16_t> idx(m);
        bool small = true;
        for (size_t t = 0; t < m && small; ++t) {
            auto it = dict.find(hm[t]);
            if (it == dict.end()) {
                if (table.size() >= 65536) {
                    small = false;
                    break;
                }
                it = dict.emplace(hm[t], static_cast<uint32_t>(table.size())).first;
                table.push_back(hm[t]);
            }
            idx[t] = static_cast<uint16_t>(it->second);
        }
        if (!small) {
            c->jmap_kind = 3;
            c->jmap_idx = dmaps;
        } else {
            dfree(dmaps);
            if (!dalloc(c->jmap_tab, table.size()))
                return fail(c, MSRSB_E_NOMEM, "allocation of the slot maps failed");
            hipMemcpy(c->jmap_tab, table.data(), table.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice);
            c->jmap_ntab = static_cast<int>(table.size());
            if (table.size() <= 256) {
                std::vector<uint8_t> i8(idx.begin(), idx.end());
                uint8_t *d = nullptr;
                if (!dalloc(d, m)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
                hipMemcpy(d, i8.data(), m, hipMemcpyHostToDevice);
                c->jmap_idx = d;
                c->jmap_kind = 1;
            } else {
                uint16_t *d = nullptr;
                if (!dalloc(d, m)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
                hipMemcpy(d, idx.data(), m * sizeof(uint16_t), hipMemcpyHostToDevice);
                c->jmap_idx = d;
                c->jmap_kind = 2;
            }
        }
    }
    c->rmaxnb = c->bs == 1 ? 32 : kMaxCoarseNeighbours;
    // the column pattern of R A P (symbolic part of the Galerkin product):
    // it depends on the patterns of A and P only, both fixed from here on
    // (build_coarse checks it against A's current values)
    c->rap_cols_valid = false;
    if (rap_uses_ell(c->rmaxnb, c->a_off, c->pw, c->pcol16) && c->a_dia) {
        if (!dalloc(c->rap_cols, static_cast<size_t>(nc) * kMaxCoarseNeighbours) ||
            !dalloc(c->rap_ncol, nc))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        launch_rap_cols(c->stream, c->n, nc, c->rrp, c->rci, c->a_off, c->a_dia, c->pcol16,
                        c->rap_cols, c->rap_ncol);
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
            return fail(c, MSRSB_E_HIP, "coarse pattern failed on the device");
        c->rap_cols_valid = true;
    } else if (rap_uses_nbs(c->a_ns, c->pw, c->pcol16) && c->a_ns_val) {
        // node-block stencil A: the same lists through its node offsets; the
        // product then reserves LDS for the longest list only
        if (!dalloc(c->rap_cols, static_cast<size_t>(nc) * kMaxCoarseNeighbours) ||
            !dalloc(c->rap_ncol, nc))
            return fail(c, MSRSB_E_NOMEM, "device allocation of the coarse data failed");
        launch_rap_cols(c->stream, c->n, nc, c->rrp, c->rci, c->a_off, nullptr, c->pcol16,
                        c->rap_cols, c->rap_ncol, &c->a_ns, c->a_ns_val);
        std::vector<int> hn(nc);
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess ||
            hipMemcpyAsync(hn.data(), c->rap_ncol, nc * sizeof(int), hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return fail(c, MSRSB_E_HIP, "coarse pattern failed on the device");
        const int mx = *std::max_element(hn.begin(), hn.end());
        if (mx <= kMaxCoarseNeighbours) {
            c->rmaxnb = std::max(mx, 1);
            c->rap_cols_valid = true;
        }
    }
    c->has_coarse = true;
    c->has_basis = c->has_coarse_op = false;
    return MSRSB_OK;
}

msrsb_status msrsb_set_coarse_level(msrsb_ctx *c, int32_t level, int32_t nc, const int32_t *part,
                                    const int32_t *sup_rowptr, const int32_t *sup_col,
                                    const uint8_t *interior, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (level < 1) return fail(c, MSRSB_E_ARG, "level must be >= 1");
    if (!c->has_coarse) return fail(c, MSRSB_E_STATE, "set_coarse must come first");
    if (level > 1) {
        if (!c->child) return fail(c, MSRSB_E_STATE, "set level " + std::to_string(level - 1) +
                                                         " first");
        const msrsb_status st = msrsb_set_coarse_level(c->child, level - 1, nc, part, sup_rowptr,
                                                       sup_col, interior, where);
        if (st) return fail(c, st, c->child->err);
        return MSRSB_OK;
    }
    // A_c's CSR pattern: the column lists of R A P (formed with the coarse
    // space, ascending), which the product writes into directly
    if (!c->rap_cols_valid || c->rmaxnb > 32)
        return fail(c, MSRSB_E_ARG, "a further level needs a stencil operator (3, 5, 7 or 9 "
                                    "diagonals) and supports of at most 8 coarse nodes per row");
    const int n1 = c->nc;
    std::vector<int> ncol(n1), cols(static_cast<size_t>(n1) * kMaxCoarseNeighbours);
    hipMemcpyAsync(ncol.data(), c->rap_ncol, n1 * sizeof(int), hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(cols.data(), c->rap_cols, cols.size() * sizeof(int), hipMemcpyDeviceToHost,
                   c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "reading the coarse pattern failed");
    std::vector<int> rp(n1 + 1, 0), ci;
    for (int j = 0; j < n1; ++j) {
        if (ncol[j] > 32)
            return fail(c, MSRSB_E_ARG, "a coarse row has more than 32 coarse neighbours");
        rp[j + 1] = rp[j] + ncol[j];
    }
    ci.reserve(rp[n1]);
    for (int j = 0; j < n1; ++j)
        for (int t = 0; t < ncol[j]; ++t) ci.push_back(cols[static_cast<size_t>(j) * kMaxCoarseNeighbours + t]);
    if (!c->child) {
        msrsb_status st = msrsb_create(&c->child, c->device, c->stream);
        if (st) return fail(c, st, "creating the next level failed");
    }
    // zero values until the first build_coarse writes A_c (a missing
    // diagonal in the pattern is refused here)
    std::vector<double> zeros(ci.size(), 0.0);
    msrsb_status st = msrsb_set_matrix(c->child, n1, static_cast<int64_t>(ci.size()), rp.data(),
                                       ci.data(), zeros.data(), 1, MSRSB_HOST);
    if (!st) st = msrsb_set_coarse(c->child, nc, part, sup_rowptr, sup_col, interior, where);
    if (st) return fail(c, st, "next level: " + c->child->err);
    c->has_coarse_op = false;
    return MSRSB_OK;
}

msrsb_status msrsb_get_level(msrsb_ctx *c, int32_t level, msrsb_ctx **out)
{
    if (!c || !out) return MSRSB_E_ARG;
    *out = nullptr;
    msrsb_ctx *l = c;
    for (int k = 0; k < level && l; ++k) l = l->child;
    if (level < 0 || !l) return fail(c, MSRSB_E_ARG, "no such level");
    *out = l;
    return MSRSB_OK;
}

msrsb_status msrsb_setup_basis(msrsb_ctx *c, const msrsb_basis_opts *o, msrsb_basis_info *info)
{
    if (!c) return MSRSB_E_ARG;
    if (o) c->basis_opts = *o;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->has_coarse) return fail(c, MSRSB_E_STATE, "set_coarse must come first");
    if (!o || !(o->omega > 0.0) || o->max_iter < 0 || o->check_every < 1)
        return fail(c, MSRSB_E_ARG, "invalid basis options");
    hipStream_t s = c->stream;
    const bool fp32 = o->fp32_basis != 0;
    msrsb_status st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    const size_t jm = static_cast<size_t>(c->jw) * c->n, pm = static_cast<size_t>(c->pw) * c->n;
    if (fp32) {
        if (!dalloc_keep(c->jv32, jm) || !dalloc_keep(c->p32[0], pm) ||
            !dalloc_keep(c->p32[1], pm) || !dalloc_keep(c->r32, c->rnnz))
            return fail(c, MSRSB_E_NOMEM, "allocation of the FP32 basis failed");
    } else {
        if (!dalloc_keep(c->jv, jm) || !dalloc_keep(c->p64[0], pm) ||
            !dalloc_keep(c->p64[1], pm) || !dalloc_keep(c->r64, c->rnnz))
            return fail(c, MSRSB_E_NOMEM, "allocation of the FP64 basis failed");
    }
    // factored J (s_i and the upper diagonals of the filtered A) for a
    // symmetric stencil with the slot counts the smoothing kernel specialises
    const bool jsym = c->j_dia && c->bs == 1 && c->a_off.sym && c->jmap_kind == 1 &&
                      (c->jw == 3 || c->jw == 5 || c->jw == 7 || c->jw == 9 || c->jw == 27);
    phase_begin(c, MSRSB_PHASE_FILTER);
    launch_filter_jacobi(s, c->n, c->bs, o->filter, o->omega, c->rp, c->ci, c->a, c->jw, c->j_off,
                         c->j_dia, jsym, fp32 ? nullptr : c->jv, fp32 ? c->jv32 : nullptr,
                         // A's DIA copy when it has J's offsets (scalar A: J's pattern is A's)
                         c->bs == 1 && c->a_off.n == c->jw && c->a_off.n > 0 ? c->a_dia
                                                                            : nullptr,
                         // the node-block copy of A (vector problems)
                         c->a_ns.n > 0 ? &c->a_ns : nullptr, c->a_ns.n > 0 ? c->a_ns_val : nullptr);
    phase_end(c, MSRSB_PHASE_FILTER);
    c->ps_valid = false;  // P changes from here on
    phase_begin(c, MSRSB_PHASE_INIT);
    const bool warm = o->warm_start && c->has_basis;
    if (!warm) {
        c->pcur = 0;
        launch_init_basis(s, c->n, c->pw, c->pcol_ell, c->part, fp32 ? nullptr : c->p64[0],
                          fp32 ? c->p32[0] : nullptr);
    } else if (fp32 != c->p_is32) {
        if (fp32) {
            launch_p_convert_down(s, pm, c->p64[c->pcur], c->p32[c->pcur]);
        } else {
            if (!dalloc_keep(c->p64[c->pcur], pm)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
            launch_p_convert(s, pm, c->p32[c->pcur], c->p64[c->pcur]);
        }
    }
    c->p_is32 = fp32;
    phase_end(c, MSRSB_PHASE_INIT);
    SmoothArgs sa;
    sa.n = c->n;
    sa.pw = c->pw;
    sa.jw = c->jw;
    sa.joff = c->j_off;
    sa.jcol = c->j_dia ? nullptr : c->jcol_ell;
    sa.pcol = c->pcol_ell;
    sa.jmap_kind = c->jmap_kind;
    sa.jmap_idx = c->jmap_idx;
    sa.jmap_tab = c->jmap_tab;
    sa.jmap_ntab = c->jmap_ntab;
    sa.interior = c->interior;
    sa.sym = jsym;
    sa.omega = o->omega;
    // FP64 rows overflow an XCD's L2 between a row's two z-neighbour reads
    // in the plain order; FP32 rows fit, and measure no faster tiled
    if (c->j_dia && !fp32) sa.go = grid_order_for(c->n, c->j_off);
    // P split in halves during the iteration (box supports on a 3D grid,
    // 8-slot rows, the factored 7-point J in the grid's offsets): the zero
    // slots of rows with fewer than 8 entries are neither read nor written
    const SplitRows &pg = c->psplit;
    const int gx = pg.nx, gxy = pg.nx * pg.ny;
    phase_begin(c, MSRSB_PHASE_SMOOTH);
    const bool split = pg.tab && o->max_iter > 0 && jsym && c->jw == 7 && c->pw == 8 &&
                       c->jmap_kind == 1 && static_cast<int64_t>(gxy) * pg.nz == c->n &&
                       c->j_off.off[0] == -gxy && c->j_off.off[1] == -gx &&
                       c->j_off.off[2] == -1 && c->j_off.off[3] == 0 && c->j_off.off[4] == 1 &&
                       c->j_off.off[5] == gx && c->j_off.off[6] == gxy;
    if (split) {
        const size_t sm = static_cast<size_t>(c->n + pg.n8) * 4;
        const bool okb = fp32 ? dalloc_keep(c->ps32[0], sm) && dalloc_keep(c->ps32[1], sm)
                              : dalloc_keep(c->ps64[0], sm) && dalloc_keep(c->ps64[1], sm);
        if (!okb) return fail(c, MSRSB_E_NOMEM, "allocation of the split basis failed");
        launch_p_split(s, c->n, pg, fp32, c->p64[c->pcur], c->p32[c->pcur], c->ps64[c->pcur],
                       c->ps32[c->pcur]);
        sa.split = pg;
    }
    double *const *q64 = split ? c->ps64 : c->p64;
    float *const *q32 = split ? c->ps32 : c->p32;
    int it = 0;
    double e_last = -1.0;
    for (it = 0; it < o->max_iter; ++it) {
        const bool check = (it % o->check_every) == 0;
        sa.eit_part = check ? c->partials : nullptr;
        sa.eit_out = c->eit_val;
        const int src = c->pcur, dst = 1 - c->pcur;
        launch_smooth(s, sa, fp32, c->jv, c->jv32, q64[src], q64[dst], q32[src], q32[dst]);
        c->pcur = dst;
        if (check && o->tol >= 0.0) {
            hipMemcpyAsync(c->h_pinned, c->eit_val, sizeof(double), hipMemcpyDeviceToHost, s);
            if (hipStreamSynchronize(s) != hipSuccess)
                return fail(c, MSRSB_E_HIP, "smoothing failed on the device");
            e_last = c->h_pinned[0];
            if (!std::isfinite(e_last) || e_last <= o->tol) {
                ++it;
                break;
            }
        }
    }
    if (split) {
        launch_p_merge(s, c->n, pg, fp32, c->ps64[c->pcur], c->ps32[c->pcur], c->p64[c->pcur],
                       c->p32[c->pcur]);
        c->ps_valid = true;
    }
    phase_end(c, MSRSB_PHASE_SMOOTH);
    // last computed e_it, and P's statistics
    hipMemcpyAsync(c->h_pinned, c->eit_val, sizeof(double), hipMemcpyDeviceToHost, s);
    launch_basis_stats(s, c->n, c->pw, c->pcol_ell, fp32, c->p64[c->pcur], c->p32[c->pcur],
                       c->partials, c->scal + S_TMP0);
    hipMemcpyAsync(c->h_pinned + 1, c->scal + S_TMP0, 3 * sizeof(double), hipMemcpyDeviceToHost,
                   s);
    if (hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "smoothing failed on the device");
    if (o->max_iter > 0) e_last = c->h_pinned[0];
    c->has_basis = true;
    c->has_coarse_op = false;
    if (info) {
        info->iters = it;
        info->e_it = e_last;
        info->max_rowsum_err = c->h_pinned[1];
        info->p_min = c->h_pinned[2];
        info->p_max = c->h_pinned[3];
    }
    if (!std::isfinite(e_last) || !std::isfinite(c->h_pinned[1]))
        return fail(c, MSRSB_E_BASIS_DIVERGED, "basis smoothing diverged (e_it not finite)");
    return MSRSB_OK;
}

msrsb_status msrsb_set_prolongation(msrsb_ctx *c, const double *val, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_coarse) return fail(c, MSRSB_E_STATE, "set_coarse must come first");
    if (!val || !valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid values");
    const size_t pm = static_cast<size_t>(c->pw) * c->n;
    if (!dalloc_keep(c->p64[0], pm) || !dalloc_keep(c->p64[1], pm) ||
        !dalloc_keep(c->r64, c->rnnz) || !dalloc_keep(c->p_csr_tmp, c->pnnz))
        return fail(c, MSRSB_E_NOMEM, "allocation failed");
    c->pcur = 0;
    c->p_is32 = false;
    c->ps_valid = false;
    hipMemcpyAsync(c->p_csr_tmp, val, c->pnnz * sizeof(double), kind_in(where), c->stream);
    launch_csr_to_ell(c->stream, c->n, c->pw, c->prp, c->p_csr_tmp, c->p64[0]);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MSRSB_E_HIP, "copy failed");
    c->has_basis = true;
    c->has_coarse_op = false;
    return MSRSB_OK;
}

msrsb_status msrsb_get_prolongation(msrsb_ctx *c, int32_t *rowptr, int32_t *col, double *val,
                                    int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_coarse) return fail(c, MSRSB_E_STATE, "set_coarse must come first");
    if (!valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid where");
    const hipMemcpyKind hk = where == MSRSB_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    if (rowptr) hipMemcpy(rowptr, c->h_prp.data(), (c->n + 1) * sizeof(int), hk);
    if (col) hipMemcpy(col, c->h_pci.data(), c->pnnz * sizeof(int), hk);
    if (val) {
        if (!c->has_basis) return fail(c, MSRSB_E_STATE, "no basis yet");
        if (!dalloc_keep(c->p_csr_tmp, c->pnnz)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
        launch_ell_to_csr(c->stream, c->n, c->pw, c->prp, c->p_is32, c->p64[c->pcur],
                          c->p32[c->pcur], c->p_csr_tmp);
        hipMemcpyAsync(val, c->p_csr_tmp, c->pnnz * sizeof(double), kind_out(where), c->stream);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MSRSB_E_HIP, "copy failed");
    return MSRSB_OK;
}

msrsb_status msrsb_build_coarse(msrsb_ctx *c, const msrsb_coarse_opts *o)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->has_basis) return fail(c, MSRSB_E_STATE, "setup_basis must come first");
    const int restriction = o ? o->restriction : MSRSB_RESTRICT_GALERKIN;
    const int factor = o ? o->factor : MSRSB_FACTOR_AUTO;
    if (restriction != MSRSB_RESTRICT_GALERKIN && restriction != MSRSB_RESTRICT_MSFV)
        return fail(c, MSRSB_E_ARG, "unknown restriction");
    if (factor != MSRSB_FACTOR_AUTO && factor != MSRSB_FACTOR_PIVOTED &&
        factor != MSRSB_FACTOR_CHOLESKY)
        return fail(c, MSRSB_E_ARG, "unknown factor");
    if (factor == MSRSB_FACTOR_CHOLESKY && !c->child &&
        !(c->a_symmetric && restriction == MSRSB_RESTRICT_GALERKIN))
        return fail(c, MSRSB_E_ARG, "the Cholesky form needs a symmetric A and the Galerkin "
                                    "restriction");
    c->has_coarse_op = false;
    c->restriction = restriction;
    hipStream_t s = c->stream;
    msrsb_status st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    const bool fp32 = c->p_is32;
    if (fp32 ? !dalloc_keep(c->r32, c->rnnz) : !dalloc_keep(c->r64, c->rnnz))
        return fail(c, MSRSB_E_NOMEM, "allocation failed");
    const int nc = c->nc;
    const int64_t nn = static_cast<int64_t>(nc) * nc;
    if (!c->child && !c->dense_coarse)
        return fail(c, MSRSB_E_ARG, "a coarse space of more than " + std::to_string(kMaxCoarse) +
                                        " unknowns needs a further level "
                                        "(msrsb_set_coarse_level)");
    if (!dalloc_keep(c->p_csr_tmp, c->pnnz)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
    // with a further level the product is written as that level's CSR matrix
    double *acout = c->child ? c->child->a : c->ac;
    const int *csr_rp = c->child ? c->child->rp : nullptr;
    phase_begin(c, MSRSB_PHASE_RAP);
    if (restriction == MSRSB_RESTRICT_GALERKIN)
        launch_gather_r(s, c->rnnz, c->rsrc, fp32, c->p64[c->pcur], c->p32[c->pcur], c->r64,
                        c->r32);
    else  // the block indicator, on the pattern of P^T (which contains it)
        launch_r_indicator(s, nc, c->rnnz, c->rrp, c->rci, c->rsrc, c->part, fp32, c->r64,
                           c->r32);
    RapBoxGeom boxg;  // the box form's geometry (threads 0: not applicable)
    if (c->rap_box_threads > 0 && c->rbox && c->paxes) {
        boxg.box = c->rbox;
        boxg.tab = c->paxes;
        boxg.nx = c->tdims[0];
        boxg.ny = c->tdims[1];
        boxg.nz = c->tdims[2];
        boxg.ncx = c->pax_ncx;
        boxg.ncy = c->pax_ncxy / c->pax_ncx;
        boxg.ncz = nc / c->pax_ncxy;
        boxg.threads = c->rap_box_threads;
    }
    RapBoxGeom nboxg;  // the node-block box form's geometry (threads 0: not applicable)
    if (c->rap_nbox_threads > 0 && c->nrbox && c->npaxes) {
        nboxg.box = c->nrbox;
        nboxg.tab = c->npaxes;
        nboxg.nx = c->ndims[0];
        nboxg.ny = c->ndims[1];
        nboxg.nz = c->ndims[2];
        nboxg.ncx = c->ncdims[0];
        nboxg.ncy = c->ncdims[1];
        nboxg.ncz = c->ncdims[2];
        nboxg.threads = c->rap_nbox_threads;
    }
    bool have_csr = false;  // the CSR copy of P, for the general RAP only
    bool lists_rebuilt = false;
    // the node-block stencil form runs on its column lists (no CSR copy of P)
    const bool nbs = rap_uses_nbs(c->a_ns, c->pw, c->pcol16) && c->a_ns_val && !csr_rp;
    const bool boxr = !c->child && !nbs && c->a_dia && rap_uses_box(c->a_off, c->pw, &boxg);
    for (;;) {
        if (!boxr && !have_csr && !rap_uses_ell(c->rmaxnb, c->a_off, c->pw, c->pcol16) &&
            !(nbs && c->rap_cols_valid)) {
            launch_ell_to_csr(s, c->n, c->pw, c->prp, fp32, c->p64[c->pcur], c->p32[c->pcur],
                              c->p_csr_tmp);
            have_csr = true;
        }
        hipMemsetAsync(c->dev_flag, 0, 2 * sizeof(int), s);
        hipMemsetAsync(c->band, 0, 2 * sizeof(int), s);
        if (!c->child && !(boxr && c->ac_outside_zero)) launch_fill(s, nn, c->ac, 0.0);
        c->ac_outside_zero = false;
        launch_rap(s, c->n, nc, c->rmaxnb, c->rrp, c->rci, fp32, c->r64, c->r32, c->rp, c->ci,
                   c->a, c->a_off, c->a_dia, c->prp, c->pci, c->p_csr_tmp, c->pw, c->pcol16,
                   c->p64[c->pcur], c->p32[c->pcur], acout, c->dev_flag, c->band,
                   c->rap_cols_valid ? c->rap_cols : nullptr, c->rap_ncol, csr_rp,
                   nbs ? &c->a_ns : nullptr, nbs ? c->a_ns_val : nullptr, c->rap_order,
                   boxr ? &boxg : nullptr, nbs ? &nboxg : nullptr);
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess)
            return fail(c, MSRSB_E_HIP, std::string("coarse product launch failed: ") +
                                            hipGetErrorString(le));
        if (boxr) {
            // every column of a row lies in its 27-column neighbourhood: no
            // list can be missed, and the band follows from the coarse grid
            // (an upper bound of the nonzeros' band), so the factorisation is
            // queued without waiting for the product
            c->h_band[0] = c->h_band[1] = rap_box_band(boxg);
            c->ac_outside_zero = true;
            break;
        }
        int hflag[2] = {0, 0};
        hipMemcpyAsync(hflag, c->dev_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(c->h_band, c->band, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess)
            return fail(c, MSRSB_E_HIP, "coarse operator failed on the device");
        if (hflag[1] && c->child)
            return fail(c, MSRSB_E_ARG, "A's values opened a coarse coupling outside the next "
                                        "level's pattern: set the coarse levels again");
        if (hflag[0] && c->child)
            return fail(c, MSRSB_E_ARG, "a coarse row has more columns than the next level holds");
        if (hflag[1]) {
            // A gained a nonzero outside the column lists: form them again
            // from A's current values and repeat the product
            if (lists_rebuilt)
                return fail(c, MSRSB_E_HIP, "coarse operator pattern is inconsistent");
            if (nbs)
                launch_rap_cols(s, c->n, nc, c->rrp, c->rci, c->a_off, nullptr, c->pcol16,
                                c->rap_cols, c->rap_ncol, &c->a_ns, c->a_ns_val);
            else
                launch_rap_cols(s, c->n, nc, c->rrp, c->rci, c->a_off, c->a_dia, c->pcol16,
                                c->rap_cols, c->rap_ncol);
            lists_rebuilt = true;
            continue;
        }
        if (!hflag[0]) break;
        if (c->rmaxnb >= kMaxCoarseNeighbours)
            return fail(c, MSRSB_E_ARG, "a coarse row has more than " +
                                            std::to_string(kMaxCoarseNeighbours) +
                                            " coarse neighbours");
        c->rmaxnb = std::min(kMaxCoarseNeighbours, 2 * c->rmaxnb);
    }
    phase_end(c, MSRSB_PHASE_RAP);
    phase_begin(c, MSRSB_PHASE_FACTOR);
    if (c->child) {
        // the coarse solver of this level is the next level's preconditioner
        // (Alg. 2 "set up coarse system solver"): its matrix A_c was written
        // above; filter, basis and coarse operator of that level follow
        msrsb_ctx *ch = c->child;
        st = refresh_values(ch);
        if (!st) st = msrsb_setup_basis(ch, &c->basis_opts, nullptr);
        msrsb_coarse_opts co{MSRSB_RESTRICT_GALERKIN, factor};
        if (!st) st = msrsb_build_coarse(ch, &co);
        phase_end(c, MSRSB_PHASE_FACTOR);
        if (st) return fail(c, st, "next level: " + ch->err);
        c->has_coarse_op = true;
        return MSRSB_OK;
    }
    int hflag = 0;
    st = MSRSB_E_COARSE_SINGULAR;
    c->acinv_sym = false;
    double *work = c->gj_b + 8 * 64 + 64 * static_cast<size_t>(nc);
    if (c->a_symmetric && restriction == MSRSB_RESTRICT_GALERKIN &&
        factor != MSRSB_FACTOR_PIVOTED) {
        // symmetric positive definite A_c: band Cholesky, W = L^{-1} and
        // W^T W; a non-positive pivot falls back to partial pivoting (unless
        // the Cholesky form was asked for)
        st = coarse_inverse_spd(s, nc, c->ac, c->acinv, std::max(c->h_band[0], c->h_band[1]),
                                c->spd_buf, work, c->acinv_pk, c->dev_flag, &hflag);
        c->acinv_sym = st == MSRSB_OK;
        if (st == MSRSB_E_COARSE_SINGULAR && factor == MSRSB_FACTOR_CHOLESKY) {
            phase_end(c, MSRSB_PHASE_FACTOR);
            return fail(c, st, "non-positive pivot: the coarse operator is not positive definite");
        }
    }
    if (st == MSRSB_E_COARSE_SINGULAR) {
        hipMemcpyAsync(work, c->ac, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
        st = coarse_inverse(s, nc, work, c->acinv, c->gj_b, c->piv, c->colsrc, c->dev_flag,
                            &hflag);
    }
    phase_end(c, MSRSB_PHASE_FACTOR);
    if (st == MSRSB_E_COARSE_SINGULAR)
        return fail(c, st, "zero pivot: the coarse operator is singular");
    if (st) return fail(c, st, "coarse factorisation failed");
    c->has_coarse_op = true;
    return MSRSB_OK;
}

msrsb_status msrsb_get_coarse_matrix(msrsb_ctx *c, double *dense, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (!c->has_coarse_op) return fail(c, MSRSB_E_STATE, "build_coarse must come first");
    if (c->child)
        return fail(c, MSRSB_E_STATE, "with a further level A_c is that level's (sparse) matrix: "
                                      "read it with msrsb_get_matrix on msrsb_get_level");
    if (!dense || !valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid buffer");
    hipMemcpyAsync(dense, c->ac, static_cast<size_t>(c->nc) * c->nc * sizeof(double),
                   kind_out(where), c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MSRSB_E_HIP, "copy failed");
    return MSRSB_OK;
}

msrsb_status msrsb_apply_preconditioner(msrsb_ctx *c, const msrsb_solve_opts *o,
                                        const double *v, double *z, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->has_matrix) return fail(c, MSRSB_E_STATE, "no matrix set");
    if (!v || !z || !valid_where(where)) return fail(c, MSRSB_E_ARG, "invalid vectors");
    msrsb_status st = solve_opts_check(c, o);
    if (st) return st;
    st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    if ((st = ensure_smoother(c, o, false))) return st;
    if (o->use_multiscale && (st = ensure_levels(c, o, false))) return st;
    const size_t bytes = static_cast<size_t>(c->n) * sizeof(double);
    hipMemcpyAsync(c->w[5], v, bytes, kind_in(where), c->stream);
    apply_two_stage(c, o, c->w[5], c->w[6], false, nullptr);
    hipMemcpyAsync(z, c->w[6], bytes, kind_out(where), c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MSRSB_E_HIP, "apply failed");
    return MSRSB_OK;
}

msrsb_status msrsb_solve(msrsb_ctx *c, const double *f, double *u, const msrsb_solve_opts *o,
                         msrsb_solve_info *info, int where)
{
    if (c) c->err.clear();
    return do_solve(c, f, u, o, info, where, false);
}

msrsb_status msrsb_solve_transpose(msrsb_ctx *c, const double *g, double *lambda,
                                   const msrsb_solve_opts *o, msrsb_solve_info *info, int where)
{
    if (c) c->err.clear();
    return do_solve(c, g, lambda, o, info, where, true);
}

msrsb_status msrsb_tpfa_adjoint_grad(msrsb_ctx *c, const double *log_k, const double *p,
                                     const double *lambda, double *grad, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->tpfa) return fail(c, MSRSB_E_STATE, "A was not assembled by msrsb_assemble_tpfa");
    if (!log_k || !p || !lambda || !grad || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid vectors");
    msrsb_status st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    const size_t bytes = static_cast<size_t>(c->n) * sizeof(double);
    const double *dk = log_k, *dp = p, *dl = lambda;
    double *dg = grad;
    if (where == MSRSB_HOST) {
        hipMemcpyAsync(c->w[7], log_k, bytes, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(c->w[8], p, bytes, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(c->w[9], lambda, bytes, hipMemcpyHostToDevice, c->stream);
        dk = c->w[7];
        dp = c->w[8];
        dl = c->w[9];
        dg = c->w[10];
    }
    phase_begin(c, MSRSB_PHASE_GRAD);
    launch_tpfa_grad(c->stream, c->tdim, c->tdims, c->th, c->tbc, dk, dp, dl, dg);
    phase_end(c, MSRSB_PHASE_GRAD);
    if (where == MSRSB_HOST)
        hipMemcpyAsync(grad, dg, bytes, hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "gradient failed on the device");
    return MSRSB_OK;
}

msrsb_status msrsb_assemble_q1(msrsb_ctx *c, int32_t dim, const int32_t elems[3],
                               const double h[3], double nu, const double *log_E,
                               const uint8_t *fixed, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if ((dim != 2 && dim != 3) || !elems || !h || !log_E || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid Q1 arguments");
    if (!(nu > -1.0 && nu < 0.5)) return fail(c, MSRSB_E_ARG, "Poisson ratio out of range");
    int64_t nn = 1, nel = 1;
    for (int k = 0; k < dim; ++k) {
        if (elems[k] < 1 || !(h[k] > 0.0)) return fail(c, MSRSB_E_ARG, "invalid grid");
        nn *= elems[k] + 1;
        nel *= elems[k];
    }
    if (nn * dim > (1 << 27)) return fail(c, MSRSB_E_ARG, "grid too large");
    const int n = static_cast<int>(nn * dim);
    int ne[3] = {1, 1, 1}, nnd[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) {
        ne[k] = elems[k];
        nnd[k] = elems[k] + 1;
    }
    bool same = c->q1 && c->has_matrix && c->qdim == dim;
    for (int k = 0; k < 3; ++k) same = same && c->qelems[k] == ne[k];
    if (!same) {
        // symbolic pattern: per row the 3^dim neighbouring nodes in ascending
        // index, dim components each
        std::vector<int> hrp(n + 1, 0), hci, dpos(n);
        hci.reserve(static_cast<size_t>(n) * (dim == 3 ? 81 : 18));
        const int zr = dim == 3 ? 1 : 0;
        for (int node = 0; node < static_cast<int>(nn); ++node) {
            const int x = node % nnd[0], y = (node / nnd[0]) % nnd[1], z = node / (nnd[0] * nnd[1]);
            for (int l = 0; l < dim; ++l) {
                const int r = dim * node + l;
                for (int dz = -zr; dz <= zr; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int X = x + dx, Y = y + dy, Z = z + dz;
                            if (X < 0 || Y < 0 || Z < 0 || X >= nnd[0] || Y >= nnd[1] || Z >= nnd[2])
                                continue;
                            const int nb = X + nnd[0] * (Y + nnd[1] * Z);
                            for (int m = 0; m < dim; ++m) {
                                if (dim * nb + m == r) dpos[r] = static_cast<int>(hci.size());
                                hci.push_back(dim * nb + m);
                            }
                        }
                hrp[r + 1] = static_cast<int>(hci.size());
            }
        }
        const int64_t nnz = static_cast<int64_t>(hci.size());
        free_coarse(c);
        msrsb_status st = install_pattern(c, n, nnz, std::move(hrp), std::move(hci), dpos, dim);
        if (st) return st;
        c->q1 = true;
        c->qdim = dim;
        for (int k = 0; k < 3; ++k) c->qelems[k] = ne[k];
    }
    for (int k = 0; k < 3; ++k) c->qh[k] = k < dim ? h[k] : 1.0;
    c->qnu = nu;
    const int nd = dim << dim;
    std::vector<double> k0(static_cast<size_t>(nd) * nd);
    q1_element_stiffness(dim, c->qh, nu, k0.data());
    if (!dalloc_keep(c->qk0, 24 * 24) || !dalloc_keep(c->qlogE, nel))
        return fail(c, MSRSB_E_NOMEM, "allocation failed");
    hipMemcpyAsync(c->qk0, k0.data(), k0.size() * sizeof(double), hipMemcpyHostToDevice,
                   c->stream);
    hipMemcpyAsync(c->qlogE, log_E, nel * sizeof(double), kind_in(where), c->stream);
    if (fixed) {
        if (!dalloc_keep(c->qfixed, n)) return fail(c, MSRSB_E_NOMEM, "allocation failed");
        hipMemcpyAsync(c->qfixed, fixed, n, kind_in(where), c->stream);
    } else {
        dfree(c->qfixed);
    }
    phase_begin(c, MSRSB_PHASE_ASSEMBLE);
    launch_q1_values(c->stream, dim, c->qelems, c->qk0, c->qlogE, c->qfixed, c->rp, c->a);
    phase_end(c, MSRSB_PHASE_ASSEMBLE);
    return refresh_values(c);
}

msrsb_status msrsb_q1_adjoint_grad(msrsb_ctx *c, const double *u, const double *lambda,
                                   double *grad, int where)
{
    if (!c) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    c->err.clear();
    if (!c->q1) return fail(c, MSRSB_E_STATE, "A was not assembled by msrsb_assemble_q1");
    if (!u || !lambda || !grad || !valid_where(where))
        return fail(c, MSRSB_E_ARG, "invalid vectors");
    msrsb_status st = ensure_workspace(c);
    if (st) return fail(c, st, "workspace allocation failed");
    int64_t nel = 1;
    for (int k = 0; k < c->qdim; ++k) nel *= c->qelems[k];
    const size_t bytes = static_cast<size_t>(c->n) * sizeof(double);
    const double *du = u, *dl = lambda;
    double *dg = grad;
    if (where == MSRSB_HOST) {
        if (!dalloc_keep(c->w[11], std::max<int64_t>(c->n, nel)))
            return fail(c, MSRSB_E_NOMEM, "allocation failed");
        hipMemcpyAsync(c->w[8], u, bytes, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(c->w[9], lambda, bytes, hipMemcpyHostToDevice, c->stream);
        du = c->w[8];
        dl = c->w[9];
        dg = c->w[11];
    }
    phase_begin(c, MSRSB_PHASE_GRAD);
    launch_q1_grad(c->stream, c->qdim, c->qelems, c->qk0, c->qlogE, c->qfixed, du, dl, dg);
    phase_end(c, MSRSB_PHASE_GRAD);
    if (where == MSRSB_HOST)
        hipMemcpyAsync(grad, dg, nel * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, MSRSB_E_HIP, "gradient failed on the device");
    return MSRSB_OK;
}

msrsb_status msrsb_get_timings(msrsb_ctx *c, double *ms, int32_t n_phases)
{
    if (!c || !ms || n_phases < 0) return MSRSB_E_ARG;
    DeviceGuard g(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MSRSB_E_HIP, "sync failed");
    for (int p = 0; p < n_phases; ++p) {
        ms[p] = 0.0;
        if (p < MSRSB_N_PHASES && c->ev_used[p]) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, c->ev_start[p], c->ev_stop[p]) == hipSuccess) ms[p] = t;
        }
    }
    return MSRSB_OK;
}

}  // extern "C"
