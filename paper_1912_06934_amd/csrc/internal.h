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
constexpr int kMaxCoarse = 4096;      // dense coarse inverse limit (the last level)
constexpr int kMaxCoarseLevel = 32768;  // coarse size of a level that has a further level
constexpr int kReduceBlocks = 1024;   // partial-sum slots of two-stage reductions
constexpr int kMaxCoarseNeighbours = 96;  // LDS slots per coarse row in R A P
constexpr int kMaxDiag = 32;          // most diagonals of a DIA operator
constexpr int kMapWidth = 8;          // P rows up to this width use slot maps
constexpr int kNoAllocMaxN = 1 << 18; // most rows of msrsb_apply_preconditioner_noalloc

// Offsets of a diagonal (DIA) operator, passed to kernels by value.
struct DiaOffsets {
    int n = 0;
    int off[kMaxDiag] = {};
    // 1: the operator is symmetric and its offsets come in +- pairs, so the
    // lower diagonals may be read from the upper ones
    int sym = 0;
};

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

// Node-block stencil (NBS) form of a vector operator with interleaved dofs
// (dof = bs * node + l): every row reaches, for each of at most 27 node
// offsets, the bs dofs of that neighbour node.  Values are stored as
// [n_off * bs][n] "diagonals" (slot o * bs + l' of row r holds the entry in
// column bs * (r / bs + off[o]) + l'), zero where a row has no such entry, so
// the kernels read no indices and every slot is one coalesced stream.
constexpr int kMaxNodeOffsets = 27;
struct NodeStencil {
    int n = 0;      // node offsets (0: no NBS form)
    int bs = 1;
    int nn = 0;     // nodes
    int off[kMaxNodeOffsets] = {};
};

// Launch segment of a level-scheduled triangular sweep: one wide level (a
// launch across the GPU) or a run of narrow levels (one work-group).
struct TriSegment {
    int lev0, lev1;
    bool wide;
};

// Symbolic data of the triangular smoothers for one sweep order (k_tri.hip):
// formed from A's pattern only.
struct TriOrder {
    bool built = false;
    bool sym_pattern = false;  // A_ij stored <=> A_ji stored
    int ncolours = 0;          // multicolour order: number of colours
    int n = 0;                 // rows
    const int *rp = nullptr, *ci = nullptr, *dpos = nullptr;  // A's pattern (not owned)
    int *rank = nullptr;       // position of each row in the order
    int8_t *side = nullptr;    // per entry: -1 earlier column, 0 diagonal, +1 later
    int *lord = nullptr;       // earlier entries of each row sorted by the column's rank
    int *nlow = nullptr;       // their count per row
    int *tpos = nullptr;       // index of the transposed entry, -1 if not stored
    int *rows_l = nullptr, *rows_u = nullptr;  // rows by level (lower / upper)
    int *ptr_l = nullptr, *ptr_u = nullptr;    // level pointers (device copies)
    std::vector<int> h_lev_l, h_lev_u;
    std::vector<TriSegment> seg_l, seg_u;
    void *packed = nullptr;    // natural order: per level position, the row's
                               // entries on the solved side (k_tri.hip)
    int max_lo = 0, max_up = 0;            // most entries of a row on each side
    int max_w_l = 0, max_w_u = 0;          // widest level of each triangle
};

// P's rows in two halves for the smoothing iteration, when the supports are
// boxes on an nx x ny x nz grid (every row's pattern is a product of one or
// two candidates per axis, 8 entries only where all three axes have two):
// slots 0-3 of every row ([n][4]), then slots 4-7 of the 8-entry rows in row
// order ([n8][4]), so that the zero slots of the narrower rows are neither
// read nor written.  tab holds, per axis position, the number of two-
// candidate positions before it on that axis, premultiplied by the counts of
// the faster axes (x: 1, y: A_x, z: A_x A_y), with bit 31 set where the
// position has two candidates: the second half of row (x, y, z) sits at
// tx[x] + ty[y] + tz[z] (low 31 bits) when all three bits are set.
struct SplitRows {
    const int *tab = nullptr;  // [nx + ny + nz]; null: rows are not split
    int nx = 0, ny = 0, nz = 0;
    double rnx = 0.0, rny = 0.0;  // 1 / nx, 1 / ny
    int64_t n8 = 0;
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
    bool a_symmetric = false;           // A_ij == A_ji exactly (checked on the device)

    // transpose of A (for msrsb_solve_transpose), values gathered from A
    int *at_rp = nullptr, *at_ci = nullptr, *at_src = nullptr, *at_diag = nullptr;
    double *at = nullptr;
    bool at_pattern = false;
    bool a_symmetric_pattern_checked = false;

    // NBS form of A (vector operators whose node pattern is a stencil)
    msrsb::NodeStencil a_ns;
    int8_t *ns_slot = nullptr;          // NBS slot of every CSR entry
    double *a_ns_val = nullptr;         // [a_ns.n * bs][n]
    float *a_ns_val32 = nullptr;
    // DIA form of A (when its rows use few distinct column offsets)
    msrsb::DiaOffsets a_off;
    int8_t *a_slot = nullptr;           // DIA slot of every CSR entry
    double *a_dia = nullptr;            // [a_off.n][n]
    float *a_dia32 = nullptr;
    bool a_dia32_valid = false;
    msrsb::DiaOffsets at_off;           // DIA form of A^T (built with the transpose)
    int8_t *at_slot = nullptr;
    double *at_dia = nullptr;
    float *at_dia32 = nullptr;
    bool at_dia32_valid = false;

    // Jacobi operator J (filtered): CSR pattern (aliases rp/ci when bs == 1)
    // and ELL values [jw][n], in DIA order (k = i + j_off.off[o]) or with
    // explicit ELL columns jcol_ell
    int *jrp = nullptr, *jci = nullptr;
    int64_t jnnz = 0;
    bool j_own_pattern = false;
    int jw = 0;
    msrsb::DiaOffsets j_off;
    bool j_dia = false;
    int *jcol_ell = nullptr;            // [jw][n], -1 = empty (only when !j_dia)
    double *jv = nullptr;               // [jw][n]
    float *jv32 = nullptr;
    // slot maps of the smoothing product: for J entry (o, i) and output slot
    // s of row i, the slot of row k's pattern that holds the same coarse
    // column (4 bits each, 0xF = none), stored as indices into a table
    int jmap_kind = 0;                  // 0 none, 1 uint8 index, 2 uint16 index, 3 full
    void *jmap_idx = nullptr;
    uint32_t *jmap_tab = nullptr;
    int jmap_ntab = 0;

    // coarse partition and P (frozen pattern)
    int nc = 0;
    int *part = nullptr, *prp = nullptr, *pci = nullptr;
    uint8_t *interior = nullptr;
    int64_t pnnz = 0;
    int pmaxw = 0;
    std::vector<int> h_prp, h_pci;
    // P values live in row-major ELL layout (slot s of row i at i*pw + s, pw =
    // 4 or 8 when the pattern allows, else its width), the slots of a row in
    // ascending coarse column order, padding = 0 / col -1
    int pw = 0;
    int *pcol_ell = nullptr;
    uint16_t *pcol16 = nullptr;   // 16-bit copy for the prolongation (pw 4 or 8)
    double *p64[2] = {nullptr, nullptr};
    float *p32[2] = {nullptr, nullptr};
    int pcur = 0;          // which buffer holds the current P
    bool p_is32 = false;   // current P lives in p32[pcur]
    double *p_csr_tmp = nullptr;  // CSR copy for msrsb_get_prolongation

    // R = P^T (CSR over coarse rows) with the source index into P
    // R = P^T by coarse rows, each row padded to a multiple of 64 entries
    // (pads repeat the row's last column with value 0, rsrc = -1); rnnz
    // entries in all.  With roff16, the columns are also kept as 16-bit
    // offsets from a base per 64-entry group (rbase), for the restriction.
    int *rrp = nullptr, *rci = nullptr, *rsrc = nullptr;
    int rmaxlen = 0;  // longest row of R, pads included
    uint16_t *roff16 = nullptr;
    int *rbase = nullptr;
    // supports that are boxes of the assembled grid: per coarse row the first
    // fine row, bx, bx * by and the entry count (null when any is not)
    int *rbox = nullptr;
    // P's columns as products of per-axis coarse candidates (see ProlongAxes;
    // null unless every row of the pattern was checked to be one)
    int *paxes = nullptr;
    int pax_ncx = 0, pax_ncxy = 0;
    // P split in halves for the smoothing iteration (see SplitRows; tab null
    // unless the supports are boxes on a 3D grid with 8-slot rows), and the
    // two split buffers of the iteration
    int *psplit_tab = nullptr;
    int4 *psplit_wtab = nullptr;  // per 64 rows (ProlongAxes::wtab)
    msrsb::SplitRows psplit;
    double *ps64[2] = {nullptr, nullptr};
    float *ps32[2] = {nullptr, nullptr};
    bool ps_valid = false;  // ps64/ps32[pcur] hold the current P (the prolongation reads it)
    int64_t rnnz = 0;
    double *r64 = nullptr;
    float *r32 = nullptr;
    int rmaxnb = 0;  // max coarse neighbours of a coarse row (RAP)
    // R A P's column lists by coarse row, formed once per pattern when the
    // ELL form of the RAP applies ([nc][kMaxCoarseNeighbours] and counts)
    int *rap_cols = nullptr, *rap_ncol = nullptr;
    bool rap_cols_valid = false;
    // coarse rows of a Cartesian coarse grid listed brick by brick (4 x 4 x 4
    // nodes, bricks in lexicographic order): the stencil product's row order
    int *rap_order = nullptr;
    // threads of the box form of R A P (0: its conditions on the supports
    // and P's candidates do not hold)
    int rap_box_threads = 0;
    // the same at node level for a node-block operator (3 components per
    // node, 27 node offsets): per coarse node the first fine node, bx,
    // bx * by and the node count of its support box; P's per-axis candidate
    // coarse nodes (ProlongAxes layout over the node grid); the node grid
    // and the coarse node grid
    int *nrbox = nullptr, *npaxes = nullptr;
    int ndims[3] = {0, 0, 0}, ncdims[3] = {0, 0, 0};
    int rap_nbox_threads = 0;
    // the dense A_c holds zeros outside every row's 27-column neighbourhood
    // (a box-form product wrote it since the last fill): the next box-form
    // product need not clear it again
    bool ac_outside_zero = false;
    int *band = nullptr;  // lower and upper bandwidth of A_c (device)
    int h_band[2] = {0, 0};

    // coarse operator and its inverse
    double *ac = nullptr, *acinv = nullptr, *gj_b = nullptr;
    // the SPD path's inverse: lower 64 x 64 tiles (I >= J) packed in
    // I (I + 1) / 2 + J order, each row-major and whole (diagonal tiles hold
    // both triangles, zeros past nc); and the partials of its product
    double *acinv_pk = nullptr, *symv_part = nullptr;
    bool acinv_sym = false;  // acinv came from the SPD (symmetric) path
    double *spd_buf = nullptr;  // inverse Cholesky factors of the diagonal blocks (SPD path)
    int *piv = nullptr, *colsrc = nullptr, *dev_flag = nullptr;

    // smoothers (diagonal inverses of A, and of A^T for the transposed solve)
    double *dinv_jac = nullptr, *dinv_l1 = nullptr;
    float *dinv_jac32 = nullptr, *dinv_l1_32 = nullptr;
    double *dinv_jac_t = nullptr, *dinv_l1_t = nullptr;
    float *dinv_jac32_t = nullptr, *dinv_l1_32_t = nullptr;
    float *at32 = nullptr;
    bool smoother32_valid = false, smoother_t_valid = false, smoother32_t_valid = false;
    // triangular smoothers by sweep order (MSRSB_ORDER_*): symbolic data, and
    // the ILU(0) and IC(0) factors on A's pattern (IC(0): L below and on the
    // diagonal, its transpose mirrored above)
    msrsb::TriOrder tri[2];
    double *ilu_f[2] = {nullptr, nullptr}, *ic_f[2] = {nullptr, nullptr};
    bool ilu_ok[2] = {false, false}, ic_ok[2] = {false, false};

    // restriction of the coarse operator (MSRSB_RESTRICT_*)
    int restriction = MSRSB_RESTRICT_GALERKIN;

    // multilevel: the next level is a context of its own whose matrix is A_c
    // (CSR on R A P's column lists, written there by the product) and whose
    // two-stage preconditioner replaces the coarse inverse of this level
    msrsb_ctx *child = nullptr;
    bool dense_coarse = false;       // ac / acinv are allocated (last level)
    msrsb_basis_opts basis_opts = {};  // of the last setup_basis (used by the levels below)
    msrsb_solve_opts child_opts = {};  // the next level's apply options (set per solve)

    // Krylov workspace
    double *w[15] = {};
    float *wf[3] = {};            // FP32 work vectors of the precision-form preconditioner
    double *vc = nullptr, *wc = nullptr;
    double *partials = nullptr, *scal = nullptr;
    double *partials_rr = nullptr;  // r.r partials of the PCG update
    double *gm_v = nullptr, *gm_h = nullptr;  // GMRES basis and small arrays
    int gm_cap = 0;
    double *h_pinned = nullptr;
    double *eit_val = nullptr;  // last e_it (device)

    // TPFA assembly description (set by msrsb_assemble_tpfa)
    bool tpfa = false;
    int tdim = 0, tdims[3] = {1, 1, 1};
    double th[3] = {1, 1, 1}, tbc[6] = {0, 0, 0, 0, 0, 0};
    double *tlogk = nullptr;

    // Q1 elasticity description (set by msrsb_assemble_q1)
    bool q1 = false;
    int qdim = 0, qelems[3] = {1, 1, 1};
    double qh[3] = {1, 1, 1}, qnu = 0.0;
    double *qk0 = nullptr;       // element stiffness for E = 1, (dim 2^dim)^2
    double *qlogE = nullptr;     // log E per element
    uint8_t *qfixed = nullptr;   // Dirichlet flag per dof (null: none)

    // device address of this device's static scratch array (noalloc.hip)
    double *scratch = nullptr;

    // timings
    hipEvent_t ev_start[MSRSB_N_PHASES] = {}, ev_stop[MSRSB_N_PHASES] = {};
    bool ev_used[MSRSB_N_PHASES] = {};
};

namespace msrsb {

// ---- basis kernels (k_basis.hip) ----
// Work-groups are dispatched to the eight XCDs in turn (group b to XCD b % 8)
// and every XCD has its own L2.  Renumbering the groups so that each XCD walks
// one contiguous range of rows keeps a stencil's neighbour rows (i +- nx,
// i +- nx ny) in the L2 that already loaded them.
__device__ __forceinline__ int xcd_group(int b, int g)
{
    const int q = g >> 3, r = g & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}
// (for kernels launched with kBlock threads per work-group: the constant
// stands in for blockDim.x, which is read from the dispatch packet by a
// vector load that every wavefront would wait for before its first real one)
__device__ __forceinline__ int xcd_row()
{
    return xcd_group(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
}

// Work-group order of a sweep over a 3D grid (rows numbered x fastest):
// the y lines are cut into eight slabs, one per XCD, and each XCD walks its
// slab layer by layer in z, kBlock rows of one layer per work-group.  The
// rows that a row's z-neighbours share an L2 with are then read a few
// dispatch steps apart rather than a whole grid plane apart.  nx == 0: the
// plain order (as xcd_row).
struct GridOrder {
    int nx = 0, ny = 0, nz = 0;
    int lines = 0;  // y lines per slab (ny / 8)
    int bps = 0;    // work-groups per slab layer (lines * nx / kBlock)
};
// first row of this work-group (uniform: kept in a scalar register)
__device__ __forceinline__ int grid_row0(const GridOrder &g)
{
    const int q = xcd_group(blockIdx.x, gridDim.x);
    if (g.nx == 0) return __builtin_amdgcn_readfirstlane(q * kBlock);
    const int sub = q % g.bps, rest = q / g.bps;
    const int z = rest % g.nz, st = rest / g.nz;
    return __builtin_amdgcn_readfirstlane((z * g.ny + st * g.lines) * g.nx + sub * kBlock);
}
// The order for n rows with DIA offsets d, when d is the 7-point stencil
// {-nx ny, -nx, -1, 0, 1, nx, nx ny} of an nx x ny x nz grid whose slabs
// split into whole work-groups (then the grid has exactly n / kBlock of them)
GridOrder grid_order_for(int n, const DiaOffsets &d);

struct SmoothArgs {
    int n = 0, pw = 0, jw = 0;
    DiaOffsets joff;
    const int *jcol = nullptr;          // explicit J columns, or null for DIA order
    const int *pcol = nullptr;          // P's ELL columns
    int jmap_kind = 0;
    const void *jmap_idx = nullptr;
    const uint32_t *jmap_tab = nullptr;
    int jmap_ntab = 0;
    const uint8_t *interior = nullptr;
    double *eit_part = nullptr;  // per-work-group maxima; null: no e_it this iteration
    double *eit_out = nullptr;   // e_it (one double)
    bool sym = false;            // J stored factored (k_filter_jacobi's sym form)
    double omega = 0.0;
    GridOrder go;                // work-group order (nx == 0: plain)
    SplitRows split;             // tab non-null: P in and out in the split form
};
void launch_filter_jacobi(hipStream_t s, int n, int bs, int filter, double omega, const int *rp,
                          const int *ci, const double *a, int jw, const DiaOffsets &joff,
                          bool use_dia, bool sym, double *jv64, float *jv32,
                          const double *ad = nullptr, const NodeStencil *ns = nullptr,
                          const double *nsv = nullptr);
void launch_init_basis(hipStream_t s, int n, int pw, const int *pcol, const int *part,
                       double *p64, float *p32);
void launch_smooth(hipStream_t s, const SmoothArgs &a, bool fp32, const double *jv64,
                   const float *jv32, const double *pin64, double *pout64, const float *pin32,
                   float *pout32);
// padded rows [n][8] <-> the split form (q: [n][4] then [n8][4]); merging
// writes zeros to the slots 4-7 of the narrower rows
void launch_p_split(hipStream_t s, int n, const SplitRows &g, bool fp32, const double *p64,
                    const float *p32, double *q64, float *q32);
void launch_p_merge(hipStream_t s, int n, const SplitRows &g, bool fp32, const double *q64,
                    const float *q32, double *p64, float *p32);
void launch_basis_stats(hipStream_t s, int n, int pw, const int *pcol, bool fp32,
                        const double *p64, const float *p32, double *partials, double *out3);
void launch_p_convert(hipStream_t s, int64_t m, const float *src, double *dst);
void launch_p_convert_down(hipStream_t s, int64_t m, const double *src, float *dst);
void launch_ell_to_csr(hipStream_t s, int n, int pw, const int *prp, bool fp32,
                       const double *pe64, const float *pe32, double *pcsr);
void launch_csr_to_ell(hipStream_t s, int n, int pw, const int *prp, const double *pcsr,
                       double *pe64);
void launch_build_maps(hipStream_t s, int n, int pw, int jw, const DiaOffsets &joff,
                       const int *jcol, const int *jrp, const int *jci, const int *pcol,
                       uint32_t *maps);

// ---- coarse kernels (k_coarse.hip) ----
void launch_gather_r(hipStream_t s, int64_t m, const int *rsrc, bool fp32, const double *p64,
                     const float *p32, double *r64, float *r32);
// whether launch_rap takes the stencil/ELL form (which needs no CSR copy of P)
bool rap_uses_ell(int maxnb, const DiaOffsets &d, int pw, const uint16_t *pcol16);
// R A P by coarse-row boxes (see k_rap_box): the supports as boxes, P's
// per-axis candidate tables (ProlongAxes layout) on an nx x ny x nz grid of
// fine cells and an ncx x ncy x ncz grid of coarse nodes, and the work-group
// size (one thread per column of a support box widened by one cell)
struct RapBoxGeom {
    const int *box = nullptr, *tab = nullptr;
    int nx = 0, ny = 0, nz = 0, ncx = 0, ncy = 0, ncz = 0;
    int threads = 0;
};
// whether launch_rap takes the box form (dense A_c, every column of a row in
// its 27-column coarse neighbourhood), and the half bandwidth that
// neighbourhood gives A_c in the lexicographic coarse numbering
bool rap_uses_box(const DiaOffsets &d, int pw, const RapBoxGeom *g);
int rap_box_band(const RapBoxGeom &g);
void launch_rap(hipStream_t s, int n, int nc, int maxnb, const int *rrp, const int *rci,
                bool fp32, const double *r64, const float *r32, const int *rp, const int *ci,
                const double *a, const DiaOffsets &d, const double *ad, const int *prp,
                const int *pci, const double *pcsr, int pw, const uint16_t *pcol16,
                const double *pe64, const float *pe32, double *ac, int *flag, int *band,
                const int *cols = nullptr, const int *ncol = nullptr,
                const int *csr_rp = nullptr, const NodeStencil *ns = nullptr,
                const double *nsv = nullptr, const int *order = nullptr,
                const RapBoxGeom *boxg = nullptr, const RapBoxGeom *nboxg = nullptr);
// whether the node-block stencil form of A (ns, values in FP64) takes the
// stencil/ELL product (k_rap_nbs; needs its column lists, no CSR copy of P)
bool rap_uses_nbs(const NodeStencil &ns, int pw, const uint16_t *pcol16);
// the column lists of R A P by coarse row (stencil forms only; see
// k_rap_cols, k_rap_nbs_cols): cols [nc][kMaxCoarseNeighbours], ncol [nc];
// with ns (node-block form) nsv holds its values and d, ad are not used
void launch_rap_cols(hipStream_t s, int n, int nc, const int *rrp, const int *rci,
                     const DiaOffsets &d, const double *ad, const uint16_t *pcol16, int *cols,
                     int *ncol, const NodeStencil *ns = nullptr, const double *nsv = nullptr);
// A^{-1} of a symmetric positive definite band matrix A (dense n x n, half
// bandwidth bl) into pk (packed lower tiles); X is the factorisation's
// workspace (n x n, only the tiles within the band are written)
msrsb_status coarse_inverse_spd(hipStream_t s, int n, const double *A, double *X, int bl,
                                double *Linv, double *W, double *pk, int *flag, int *host_flag);
// y = S x for the symmetric S in the packed lower-tile form (acinv_pk)
void launch_symv_packed(hipStream_t s, int n, const double *pk, const double *x, double *y,
                        double *part);
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
// Coarse rows whose entries (fine rows ascending) are the cells of a box of
// an nx x ny x nz grid: box[4 j ..] = first row, bx, bx * by, entry count.
// maxlen: R's longest row with its pads (0 when unknown), which sets the
// restriction's entries per lane; used with or without boxes.
struct RestrictBoxes {
    const int *box = nullptr;
    int nx = 0, nxy = 0;
    int maxlen = 0;
};
// P's pattern on an nx x ny x nz grid whose row (x, y, z) reaches the coarse
// nodes (ax + ix) + ncx (ay + iy) + ncxy (az + iz) for ix < cx, iy < cy,
// iz < cz in ascending order, with tab[x] = ax | cx << 16, tab[nx + y] =
// ay | cy << 16, tab[nx + ny + z] = az | cz << 16 and cx, cy in {1, 2}.
struct ProlongAxes {
    const int *tab = nullptr;
    int nx = 0, ny = 0, ncx = 0, ncxy = 0;
    // non-null: P is given in the split form (SplitRows, n8 rows of 8
    // entries), located through a table with one entry per 64 rows: the
    // second-half index of their first 8-entry row and a 64-bit mask of
    // their 8-entry rows (low, high words)
    const int4 *wtab = nullptr;
    int64_t n8 = 0;
};
// xc = R x; columns from the boxes when given, else from rci, or (roff16
// non-null) rbase[e / 64] + roff16[e]
void launch_restrict(hipStream_t s, int nc, const int *rrp, const int *rci,
                     const uint16_t *roff16, const int *rbase, bool fp32, const double *r64,
                     const float *r32, const double *x, double *xc,
                     const RestrictBoxes &boxes = RestrictBoxes{});
void launch_dot(hipStream_t s, int n, const double *x, const double *y, double *partials,
                double *out);
void launch_copy(hipStream_t s, int n, const double *x, double *y);
void launch_axpy(hipStream_t s, int n, double alpha_host, const double *x, double *y);
void launch_diag_inverses(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                          double *dj, double *dl1, float *dj32, float *dl1_32, float *a32,
                          int64_t nnz, int *flag);
void launch_gather_values(hipStream_t s, int64_t m, const int *src, const double *a, double *out);

// ---- node-block stencil kernels (k_krylov.hip) ----
void launch_csr_to_nbs(hipStream_t s, int n, int nslot, const int *rp, const int8_t *slot,
                       const double *a, double *v64, float *v32);
void launch_nbs_spmv(hipStream_t s, int n, const NodeStencil &ns, const double *v, const double *x,
                     double *y);
// r = f - A x; with v32 (non-null) the FP32 values and arithmetic
void launch_nbs_residual(hipStream_t s, int n, const NodeStencil &ns, const double *v,
                         const float *v32, const double *f, const double *x, double *r);
void launch_nbs_sweep(hipStream_t s, int n, const NodeStencil &ns, bool fp32, const double *v,
                      const float *v32, const double *dinv, const float *dinv32,
                      const double *vin, const double *zin, double *zout, bool zero_start);
void launch_nbs_pcg_p_spmv(hipStream_t s, int n, const NodeStencil &ns, const double *v,
                           const double *z, const double *pold, double *pnew, double *q,
                           double *part, double *scal);

// ---- DIA / fused PCG kernels (k_krylov.hip) ----
void launch_dia_spmv(hipStream_t s, int n, const DiaOffsets &d, const double *a, const double *x,
                     double *y);
void launch_dia_residual(hipStream_t s, int n, const DiaOffsets &d, const double *a,
                         const float *a32, const double *f, const double *x, double *r);
// The PCG update x += alpha p, rout = rin - alpha q with the r.r partials
// (alpha = scal[S_ALPHA]).  Passed to the first kernel of the next
// preconditioner application, which performs it where it can read the
// residual at the stencil's rows (rout is that application's input and must
// not alias rin).
struct UpdArgs {
    double *x = nullptr;
    const double *rin = nullptr;
    const double *p = nullptr, *q = nullptr;
    double *rout = nullptr;
    double *part = nullptr;
    const double *scal = nullptr;
};
void launch_dia_sweep(hipStream_t s, int n, const DiaOffsets &d, bool fp32, const double *a64,
                      const float *a32, const double *dinv64, const float *dinv32,
                      const double *v, const double *zin, double *zout, bool zero2,
                      const UpdArgs *upd = nullptr);
void launch_dia_sweep_dots(hipStream_t s, int n, const DiaOffsets &d, bool fp32,
                           const double *a64, const float *a32, const double *dinv64,
                           const float *dinv32, const double *r, const double *zin, double *zout,
                           const double *zold, double *part, double *scal,
                           const double *part_rr, double *host_out, int tag);
// beta and, with host_out, the step's r.r mailbox (see k_fin_beta)
void launch_dots_beta(hipStream_t s, int n, const double *r, const double *z, const double *zold,
                      double *part, double *scal, const double *part_rr, double *host_out,
                      int tag);
void launch_pcg_p_spmv(hipStream_t s, int n, const DiaOffsets &d, const double *ad,
                       const int *rp, const int *ci, const double *a, const double *z,
                       const double *pold, double *pnew, double *q, double *part, double *scal);
// x += alpha p, r -= alpha q; the r.r partials (one per block) go to
// part_rr and are summed by the step's k_fin_beta
void launch_pcg_update(hipStream_t s, int n, const UpdArgs &u);
void launch_prec_f32_pre(hipStream_t s, int n, const DiaOffsets &d, const float *a32,
                         const float *dinv32, const double *v, float *z1, float *tmp, int nc,
                         const int *rrp, const int *rci, const uint16_t *roff16,
                         const int *rbase, const float *r32, double *vc,
                         const RestrictBoxes &boxes = RestrictBoxes{},
                         const UpdArgs *upd = nullptr);
void launch_prec_f32_post(hipStream_t s, int n, const DiaOffsets &d, const float *a32,
                          const float *dinv32, const double *v, float *z1, float *z2, int pw,
                          const uint16_t *pcol16, const float *p32, const double *wc,
                          double *zout, const double *zold, double *partials, double *scal,
                          const double *part_rr, double *host_out, int tag,
                          const ProlongAxes &axes = ProlongAxes{});
void launch_prolong_ell(hipStream_t s, int n, int pw, const int *pcol, const uint16_t *pcol16,
                        bool fp32, const double *p64, const float *p32, const double *wc,
                        double *z, bool zero,
                        const ProlongAxes &axes = ProlongAxes{});
void launch_csr_to_dia(hipStream_t s, int n, int noff, const int *rp, const int8_t *slot,
                       const double *a, double *ad64, float *ad32);

void launch_check_symmetric(hipStream_t s, int n, const int *rp, const int *ci, const double *a,
                            int *flag);

// ---- GMRES helpers (k_krylov.hip) ----
void launch_multi_dot(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                      const double *w, double *partials, double *out);
void launch_multi_axpy(hipStream_t s, int n, int k, const double *V, int64_t ldv,
                       const double *h, double *w, double sign);
void launch_norm_scale(hipStream_t s, int n, const double *w, double *vout, double *partials,
                       double *out_norm);

// ---- static scratch of the allocation-free apply (noalloc.hip) ----
double *static_scratch_init(int device);

// ---- triangular smoothers (k_tri.hip) ----
msrsb_status tri_order_setup(msrsb_ctx *c, int ordering);
void free_tri_order(TriOrder &t);
// ILU(0) or IC(0) factors in the order; E_BREAKDOWN on a zero (ILU) or
// non-positive (IC) pivot
msrsb_status tri_factor(msrsb_ctx *c, int ordering, int kind);
// z += M^{-1} res for ILU(0) / IC(0); res is overwritten
void tri_apply(msrsb_ctx *c, int ordering, int kind, double *res, double *z);
// z += (D + L)^{-1} res (lower) or (D + U)^{-1} res, A's values; res overwritten
void tri_gs_half(msrsb_ctx *c, int ordering, bool lower, double *res, double *z);
// R's values of the MsFV restriction: 1 where the entry's fine row lies in
// the coarse row's block, else 0
void launch_r_indicator(hipStream_t s, int nc, int64_t rnnz, const int *rrp, const int *rci,
                        const int *rsrc, const int *part, bool fp32, double *r64, float *r32);

// ---- TPFA (k_tpfa.hip) ----
void launch_tpfa_values(hipStream_t s, int dim, const int *dims, const double *h,
                        const double *bc, const double *logk, const int *rp, double *val,
                        double *rhs);
void launch_tpfa_grad(hipStream_t s, int dim, const int *dims, const double *h, const double *bc,
                      const double *logk, const double *p, const double *lam, double *grad);

// ---- Q1 elasticity (k_q1.hip) ----
void q1_element_stiffness(int dim, const double *h, double nu, double *K);
void launch_q1_values(hipStream_t s, int dim, const int *elems, const double *k0,
                      const double *logE, const uint8_t *fixed, const int *rp, double *val);
void launch_q1_grad(hipStream_t s, int dim, const int *elems, const double *k0,
                    const double *logE, const uint8_t *fixed, const double *u, const double *lam,
                    double *grad);

}  // namespace msrsb
