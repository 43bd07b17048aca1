/*
 * msrsb.h - C ABI of the MI355X (gfx950) enhanced MsRSB preconditioner.
 *
 * Method: Bosma, Klevtsov, Moyner, Castelletto, "Enhanced multiscale
 * restriction-smoothed basis (MsRSB) preconditioning with applications to
 * porous media flow and geomechanics", arXiv:1912.06934.
 *
 * The calls follow the paper's statement of the problem:
 *   A u = f                                   (eq. linsys_general)
 *   SetupMsRSBpreconditioner(A)               (Alg. 2)
 *     P = EnhancedMsRSB(A, P)                 (Alg. 1)  -> msrsb_setup_basis
 *     R = P^T, A_c = R A P, M_c^{-1}          (Alg. 2)  -> msrsb_build_coarse
 *   ApplyMsRSBTwoLevelPreconditioner(A, v)    (Alg. 3, Alg. 4)
 *                                                       -> msrsb_apply_preconditioner
 *   Krylov acceleration (PCG, GMRES)          (Sec. 3.2, Sec. 4.1)
 *                                                       -> msrsb_solve
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns msrsb_status; the message of the last failure is
 *   msrsb_last_error().  Nothing aborts and no C++ exception crosses the ABI.
 * - `where` says where caller buffers live: MSRSB_HOST (pageable or pinned
 *   host memory) or MSRSB_DEVICE (device memory on the context's GPU).
 * - Inputs are copied into context-owned device memory before the call
 *   returns; the caller may free or reuse its buffers afterwards.  Outputs
 *   go into caller buffers.  The context owns P, J, A_c, its inverse, the
 *   smoother data and all workspaces; msrsb_destroy frees them.
 * - All device work is ordered on the context's stream (set at creation or
 *   with msrsb_set_stream).  Calls that return host-visible results
 *   synchronise that stream; the others return once the work is queued.
 * - Sparse matrices are CSR with int32 row pointers and column indices,
 *   columns strictly ascending within a row, the diagonal present, FP64
 *   values.  Vectors are FP64.
 * - Order of calls: set_matrix (or assemble_tpfa) -> set_coarse ->
 *   setup_basis -> build_coarse -> apply / solve.  A call out of order
 *   returns MSRSB_E_STATE.  update_values keeps P and the coarse solver as a
 *   (stale) preconditioner until setup is run again.
 * - One context per host thread.  The only state shared between contexts is
 *   the static scratch array of msrsb_apply_preconditioner_noalloc (one per
 *   device, its address looked up once under a lock).
 */
#ifndef MSRSB_H
#define MSRSB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msrsb_ctx msrsb_ctx;

typedef enum {
    MSRSB_OK = 0,
    MSRSB_E_ARG = -1,              /* invalid argument or input data */
    MSRSB_E_STATE = -2,            /* call out of order */
    MSRSB_E_HIP = -3,              /* HIP runtime error */
    MSRSB_E_NOMEM = -4,            /* device allocation failed */
    MSRSB_E_BASIS_DIVERGED = -5,   /* e_it non-finite, or P left [0,1] */
    MSRSB_E_COARSE_SINGULAR = -6,  /* zero pivot in the coarse factorisation */
    MSRSB_E_BREAKDOWN = -7,        /* non-finite scalar, or p^T A p <= 0 in CG */
    MSRSB_E_NOT_CONVERGED = -8     /* iteration limit reached */
} msrsb_status;

enum { MSRSB_HOST = 0, MSRSB_DEVICE = 1 };

/* Smoothers of the two-stage preconditioner (Alg. 4).  The paper uses
 * Jacobi-type smoothers, ILU(0) and symmetric Gauss-Seidel as the second
 * stage (Sec. 3.2), and IC(0) and l1-Jacobi in Sec. 4.  One sweep is
 * z += M^{-1} (v - A z); for SGS, M = (D + L) D^{-1} (D + U), i.e. a forward
 * and a backward Gauss-Seidel sweep.  ILU(0), IC(0) and SGS visit the rows
 * in the order msrsb_solve_opts.ordering selects. */
enum {
    MSRSB_SMOOTH_NONE = 0,
    MSRSB_SMOOTH_JACOBI = 1,     /* M = diag(A) */
    MSRSB_SMOOTH_L1JACOBI = 2,   /* M_ii = sum_j |A_ij| */
    MSRSB_SMOOTH_ILU0 = 3,       /* M = L U, no-fill incomplete LU on A's pattern */
    MSRSB_SMOOTH_SGS = 4,        /* symmetric Gauss-Seidel */
    MSRSB_SMOOTH_IC0 = 5         /* M = L L^T, no-fill incomplete Cholesky (symmetric A) */
};

/* Sweep orders of ILU(0), IC(0) and SGS (the paper does not fix one).
 * NATURAL: ascending row index.  MULTICOLOR: first-fit colouring in
 * ascending row order on the symmetrised pattern of A (row i takes the
 * smallest colour none of its already coloured neighbours has; j is a
 * neighbour when A_ij or A_ji is stored), rows visited colour by colour,
 * ascending within a colour.  Rows of one colour never couple, so each
 * colour is processed in parallel over the whole GPU; in the natural order
 * a sweep is limited by the chain of dependencies between rows. */
enum { MSRSB_ORDER_NATURAL = 0, MSRSB_ORDER_MULTICOLOR = 1 };

/* Krylov accelerators and the stand-alone iteration (Sec. 3.2: Richardson
 * x += B (f - A x) and right-preconditioned GMRES; Sec. 4: PCG and BiCGStab). */
enum {
    MSRSB_KRYLOV_PCG = 0,
    MSRSB_KRYLOV_GMRES = 1,
    MSRSB_KRYLOV_RICHARDSON = 2,
    MSRSB_KRYLOV_BICGSTAB = 3
};

/* Restriction operators of Alg. 2. */
enum {
    MSRSB_RESTRICT_GALERKIN = 0, /* R = P^T (Sec. 2) */
    MSRSB_RESTRICT_MSFV = 1      /* Petrov-Galerkin: R_ji = 1 when fine row i lies in
                                    coarse block j (part[i] = j), else 0, so the coarse
                                    problem conserves mass block by block (Sec. 2) */
};

/* Phases reported by msrsb_get_timings (milliseconds, last run of each). */
enum {
    MSRSB_PHASE_FILTER = 0,      /* filter + Jacobi operator */
    MSRSB_PHASE_INIT = 1,        /* initial basis */
    MSRSB_PHASE_SMOOTH = 2,      /* all restricted smoothing iterations */
    MSRSB_PHASE_RAP = 3,         /* R = P^T values and A_c = R A P */
    MSRSB_PHASE_FACTOR = 4,      /* coarse factorisation (inverse of A_c) */
    MSRSB_PHASE_SOLVE = 5,       /* last msrsb_solve */
    MSRSB_PHASE_SOLVE_T = 6,     /* last msrsb_solve_transpose */
    MSRSB_PHASE_GRAD = 7,        /* last adjoint gradient kernel */
    MSRSB_PHASE_ASSEMBLE = 8,    /* last msrsb_assemble_tpfa / msrsb_assemble_q1 */
    MSRSB_PHASE_SMOOTHER_SETUP = 9, /* smoother data (diagonals, ILU(0)) */
    MSRSB_N_PHASES = 10
};

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (NULL = the null stream).  The stream must stay valid while the context
 * uses it. */
msrsb_status msrsb_create(msrsb_ctx **out, int device, void *hip_stream);
/* Free the context and all its device memory (synchronises its stream). */
void msrsb_destroy(msrsb_ctx *ctx);
/* Message of the last failed call on ctx ("" if none).  Never NULL. */
const char *msrsb_last_error(const msrsb_ctx *ctx);
/* Re-target the context to another stream of the same device. */
msrsb_status msrsb_set_stream(msrsb_ctx *ctx, void *hip_stream);

/* Fine operator A of eq. (linsys_general): n x n CSR.  block_size is 1 for
 * scalar problems, or the number of displacement components (2 or 3) for
 * vector problems with interleaved numbering dof = block_size*node + l; the
 * basis is then built from the separate-displacement-component
 * approximation (Sec. 4, eq. blk_stiff_SDC): couplings between different
 * components are ignored by the filter.  Replaces any previous matrix and
 * resets the state to "matrix set".
 * Errors: E_ARG for n < 1, nnz != rowptr[n], unsorted or out-of-range
 * columns, a missing diagonal or block_size not dividing n. */
msrsb_status msrsb_set_matrix(msrsb_ctx *ctx, int32_t n, int64_t nnz,
                              const int32_t *rowptr, const int32_t *col,
                              const double *val, int32_t block_size, int where);

/* New values on the same pattern (nnz values): the next time step of
 * Alg. 2, whose set-up runs again on the changed operator while the
 * partition, the supports and P's frozen pattern (Sec. 2.1) stay.  P, A_c
 * and the smoother keep their old values until the next setup_basis /
 * build_coarse, so the smoothing may warm-start from the previous P.
 * Errors: E_STATE before set_matrix. */
msrsb_status msrsb_update_values(msrsb_ctx *ctx, const double *val, int where);

/* Copy the current A out: rowptr (n+1), col (nnz) and val (nnz) buffers,
 * any of which may be NULL. */
msrsb_status msrsb_get_matrix(msrsb_ctx *ctx, int32_t *rowptr, int32_t *col,
                              double *val, int where);

/* Two-point flux approximation (App. B.1, flux split eq. num_flux_split)
 * on a Cartesian grid of dims[0] x dims[1] (x dims[2] if dim == 3) cells of
 * size h[0] x h[1] (x h[2]), numbered x + nx*(y + ny*z), unit depth in 2D.
 * k = exp(log_k) per cell (n values).  bc[2d] / bc[2d+1] are Dirichlet
 * pressures on the low / high domain face of axis d; NaN means no flow.
 * Face transmissibility T = t_K t_L / (t_K + t_L), t = 2 k area / h; a
 * Dirichlet face adds T_b = 2 k_K area / h to A_KK and T_b g to f_K.
 * The result becomes the context's matrix exactly as msrsb_set_matrix would
 * (same pattern on a repeated call with the same grid: then it acts as
 * msrsb_update_values and keeps P for a warm start).  rhs_out (n values,
 * may be NULL) receives f. */
msrsb_status msrsb_assemble_tpfa(msrsb_ctx *ctx, int32_t dim, const int32_t dims[3],
                                 const double h[3], const double *log_k,
                                 const double bc[6], double *rhs_out, int where);

/* Coarse partition and support regions (Sec. 2.1).  part[n] in [0, nc) is
 * the coarse block of each fine row (the initial basis is its
 * characteristic function).  The support pattern is CSR over fine rows:
 * sup_col[sup_rowptr[i] .. sup_rowptr[i+1]) lists, ascending, the coarse
 * basis functions whose support contains row i; it is P's frozen sparsity
 * pattern and must contain part[i].  interior[i] != 0 marks rows that count
 * in the convergence measure e_it (rows not on a support edge, Alg. 1).
 * At most 32 entries per row.
 * When the matrix came from msrsb_assemble_tpfa and every support is a box
 * of grid cells whose pattern rows are products of per-axis coarse nodes,
 * the restriction and prolongation form their column indices from the grid
 * instead of loading them (checked for every row here; results unchanged),
 * and on a 3D grid the basis iteration (and the FP64 prolongation) hold P
 * without the unused slots of rows with fewer than 8 entries (results
 * unchanged; msrsb_setup_basis then also allocates two such copies).
 * Errors: E_ARG for nc < 1 or nc > 32768 (more than 4096 needs a further
 * level, see msrsb_set_coarse_level), empty rows, unsorted or out-of-range
 * columns, part[i] not in row i's pattern, a coarse block without rows. */
msrsb_status msrsb_set_coarse(msrsb_ctx *ctx, int32_t nc, const int32_t *part,
                              const int32_t *sup_rowptr, const int32_t *sup_col,
                              const uint8_t *interior, int where);

/* Multilevel MsRSB (Conclusion: the filter makes the multipoint coarse
 * operator a valid input of the enhanced method, so it can be applied again
 * to A_c).  Level 0 is the fine level of msrsb_set_coarse; level L >= 1 gives
 * the coarse space of level L's unknowns, the nc_L coarse nodes of the level
 * above: part (nc_L values), the support pattern and the interior flags as
 * in msrsb_set_coarse.  Level L - 1 must be set first.  build_coarse then
 * writes A_c straight into level 1's sparse matrix (CSR on the column
 * pattern of R A P) instead of a dense matrix, and the coarse solver of
 * Alg. 2 becomes level 1's own set-up: the filter and basis (with the
 * options of the last msrsb_setup_basis) and its coarse operator, down to
 * the last level, whose A_c is inverted exactly.  Every apply then replaces
 * A_c^{-1} by one two-stage application (Alg. 4) of the next level, with the
 * same smoothers in FP64.  A level that has a further level may have up to
 * 32768 coarse unknowns (the last level up to 4096).
 * Limits: the operator of a level that gets a further level must be a
 * stencil with 3, 5, 7 or 9 diagonals and supports of at most 8 coarse nodes
 * per row (E_ARG otherwise); coarse levels take Jacobi-type smoothers only
 * (E_ARG at solve time).  Errors: E_STATE before msrsb_set_coarse or with
 * level L - 1 missing; as msrsb_set_coarse for the partition. */
msrsb_status msrsb_set_coarse_level(msrsb_ctx *ctx, int32_t level, int32_t nc,
                                    const int32_t *part, const int32_t *sup_rowptr,
                                    const int32_t *sup_col, const uint8_t *interior, int where);
/* The context of level `level` (0 = ctx itself): borrowed, owned by ctx and
 * valid until ctx or its coarse space changes; it answers msrsb_get_matrix
 * (level L's matrix is A_c of level L - 1), msrsb_get_prolongation and
 * msrsb_get_coarse_matrix.  Errors: E_ARG for a level that does not exist. */
msrsb_status msrsb_get_level(msrsb_ctx *ctx, int32_t level, msrsb_ctx **out);

typedef struct {
    double omega;        /* relaxation factor, the paper uses 2/3 (Sec. 2.1) */
    int32_t max_iter;    /* iteration cap */
    double tol;          /* stop when e_it <= tol; negative = run max_iter */
    int32_t check_every; /* n_it: e_it is computed when k mod n_it == 0 */
    int32_t filter;      /* 1 = enhanced (filtered, eq. negoffdiag), 0 = naive */
    int32_t fp32_basis;  /* 1 = J, P and the smoothing arithmetic in FP32
                            (row sums and the division stay FP64) */
    int32_t warm_start;  /* 1 = keep the current P as the start (Alg. 2) */
} msrsb_basis_opts;

typedef struct {
    int32_t iters;        /* iterations done */
    double e_it;          /* last computed e_it */
    double max_rowsum_err;/* max_i |sum_j P_ij - 1| (FP64 sums) */
    double p_min, p_max;  /* range of P's entries */
} msrsb_basis_info;

/* Alg. 1: filter (eq. negoffdiag) and zero-row-sum diagonal
 * (eq. Dhat_zero_rowsum), then restricted Jacobi smoothing (eq. smoother)
 * of the basis on its frozen support with renormalisation of every row of
 * P to one.  Without warm_start P starts from the characteristic functions
 * of the coarse blocks.  Synchronises; info may be NULL.
 * Errors: E_STATE before set_coarse; E_BASIS_DIVERGED when e_it is not
 * finite (typically the naive method on a non-M-matrix). */
msrsb_status msrsb_setup_basis(msrsb_ctx *ctx, const msrsb_basis_opts *opts,
                               msrsb_basis_info *info);

/* Overwrite P's values (nnz_P values on the support pattern, FP64), e.g. to
 * resume from a saved basis: Alg. 2 initialises the basis only when none
 * exists, so a P put back here is the start of the next warm-started
 * smoothing (Alg. 1).  Marks the basis as set up; the caller owns val.
 * Errors: E_STATE before set_coarse. */
msrsb_status msrsb_set_prolongation(msrsb_ctx *ctx, const double *val, int where);
/* Copy P out (FP64 values; any pointer may be NULL): the prolongation of
 * Sec. 2.1 as Alg. 1 left it, rowptr (n + 1) and col (nnz_P) its frozen
 * support pattern.  Errors: E_STATE before set_coarse, or for val before
 * the basis exists. */
msrsb_status msrsb_get_prolongation(msrsb_ctx *ctx, int32_t *rowptr, int32_t *col,
                                    double *val, int where);

/* How the exact coarse solver A_c^{-1} of Alg. 2 is formed (the paper asks
 * only for a coarse solver; both forms give the exact inverse up to
 * rounding). */
enum {
    MSRSB_FACTOR_AUTO = 0,     /* Cholesky for a symmetric A with the Galerkin
                                  restriction, falling back to PIVOTED on a
                                  non-positive pivot; PIVOTED otherwise */
    MSRSB_FACTOR_PIVOTED = 1,  /* Gauss-Jordan with partial pivoting (the
                                  elimination of LU with partial pivoting) */
    MSRSB_FACTOR_CHOLESKY = 2  /* Cholesky only: A_c must be symmetric positive
                                  definite */
};

typedef struct {
    int32_t restriction; /* MSRSB_RESTRICT_GALERKIN or MSRSB_RESTRICT_MSFV */
    int32_t factor;      /* MSRSB_FACTOR_* */
} msrsb_coarse_opts;

/* Alg. 2: the restriction R (R = P^T, or the MsFV block indicator; opts may
 * be NULL for Galerkin), A_c = R A P with the unfiltered A (eq.
 * lin_system_coarse), and the coarse solver M_c^{-1} = A_c^{-1} formed
 * explicitly in FP64 (applied as a dense product).  With the Galerkin
 * restriction and symmetric A, A_c is symmetric positive definite for the
 * SPD problems of the paper and the inverse comes from its Cholesky factor,
 * A_c^{-1} = L^{-T} L^{-1} (a band Cholesky, L^{-1} by forward
 * substitution, the product on the FP64 matrix cores), kept as its lower
 * 64 x 64 tiles; a non-positive pivot falls back to Gauss-Jordan with
 * partial pivoting, which is also used for non-symmetric A and for the MsFV
 * restriction (whose A_c is not symmetric); opts->factor can force either
 * form.  With a further level (msrsb_set_coarse_level) the coarse solver is
 * that level's preconditioner and the factor choice passes down to the last
 * level.  Synchronises.
 * Errors: E_STATE before setup_basis; E_ARG for an unknown restriction or
 * factor, or MSRSB_FACTOR_CHOLESKY with a non-symmetric A or the MsFV
 * restriction; E_COARSE_SINGULAR on a zero pivot (pivoting form) or a
 * non-positive pivot (MSRSB_FACTOR_CHOLESKY). */
msrsb_status msrsb_build_coarse(msrsb_ctx *ctx, const msrsb_coarse_opts *opts);
/* Copy A_c = R A P (eq. lin_system_coarse, Alg. 2) out as a dense row-major
 * nc x nc FP64 matrix; the caller owns dense (nc * nc values).
 * Errors: E_STATE before build_coarse, or when a further level holds A_c
 * (then msrsb_get_matrix on that level's context). */
msrsb_status msrsb_get_coarse_matrix(msrsb_ctx *ctx, double *dense, int where);

typedef struct {
    int32_t krylov;          /* MSRSB_KRYLOV_* */
    int32_t restart;         /* GMRES restart length */
    double rtol;             /* stop at ||f - A u|| <= rtol ||f|| */
    int32_t max_iter;
    int32_t pre_smoother, pre_sweeps;
    int32_t post_smoother, post_sweeps;
    int32_t fp32_smoother;   /* 1 = Jacobi-type smoother values and arithmetic in FP32
                                (ILU(0), IC(0) and SGS always run in FP64) */
    int32_t use_multiscale;  /* 0 = smoother-only preconditioner */
    int32_t ordering;        /* MSRSB_ORDER_*: sweep order of ILU(0), IC(0), SGS */
} msrsb_solve_opts;

typedef struct {
    int32_t iters;           /* iterations: products A p (PCG), Arnoldi steps (GMRES),
                                applications of B (Richardson), passes of the loop
                                with two applications of B each (BiCGStab; a pass
                                that converges after its first half counts one) */
    double true_rel_res;     /* ||f - A u|| / ||f||, recomputed at exit */
    double *history;         /* optional host buffer: relative residual per
                                iteration (recursive estimate) */
    int32_t history_cap;     /* its capacity */
} msrsb_solve_info;

/* z = B v with B the two-stage preconditioner of Alg. 4: z = 0; pre-sweeps
 * z += M_pre^{-1}(v - A z); z += P A_c^{-1} R (v - A z) (Alg. 3);
 * post-sweeps.  n values each.  Errors: E_STATE before build_coarse (unless
 * use_multiscale == 0); E_ARG for IC(0) on a non-symmetric A;
 * E_BREAKDOWN when ILU(0) meets a zero pivot or IC(0) a non-positive one. */
msrsb_status msrsb_apply_preconditioner(msrsb_ctx *ctx, const msrsb_solve_opts *opts,
                                        const double *v, double *z, int where);

/* msrsb_apply_preconditioner for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): z = B v exactly as
 * msrsb_apply_preconditioner computes it (the same kernels), with v and z
 * device pointers of n values on the context's device and every temporary in
 * a static device array of the library (about 11 MB per device, held until
 * the process ends) instead of the context's workspace.  Nothing is
 * allocated or freed; the call only queues work on the context's stream and
 * does not synchronise.
 * Limits: n <= 262144 rows (E_ARG beyond), and the smoother's data must
 * already exist (E_STATE otherwise): run msrsb_apply_preconditioner or
 * msrsb_solve once with the same smoother options first.  All calls on one
 * device share the array, so calls that overlap in time on one device (two
 * streams, or two host threads) race; consecutive calls on one stream do
 * not. */
msrsb_status msrsb_apply_preconditioner_noalloc(msrsb_ctx *ctx, const msrsb_solve_opts *opts,
                                                const double *v, double *z);

/* Solve A u = f (n values) with the preconditioned Krylov method or the
 * stand-alone iteration; u holds the initial guess on entry and the
 * solution on exit.  PCG uses the flexible Polak-Ribiere beta; GMRES and
 * BiCGStab are right-preconditioned; Richardson is x += B (f - A x)
 * (Sec. 3.2), stopped on its true residual.  Convergence of the Krylov
 * methods is tested on the recursive residual and confirmed on the true
 * residual.  Synchronises; info may be NULL.  Errors: E_BREAKDOWN,
 * E_NOT_CONVERGED (u still holds the last iterate and info the achieved
 * residual). */
msrsb_status msrsb_solve(msrsb_ctx *ctx, const double *f, double *u,
                         const msrsb_solve_opts *opts, msrsb_solve_info *info,
                         int where);

/* Solve A^T lambda = g, e.g. the adjoint system of a gradient computation.
 * The preconditioner is the two-stage preconditioner of A^T: A^T in the
 * residuals, the smoothers built from A^T with the pre and post sweeps
 * exchanged, and the coarse correction P A_c^{-T} P^T (P, R and the coarse
 * inverse are reused).  For symmetric A, and for point Jacobi on any A, this
 * is exactly B^T.  ILU(0), IC(0), SGS and the MsFV restriction are not
 * available here (E_ARG).  Other arguments and errors as msrsb_solve. */
msrsb_status msrsb_solve_transpose(msrsb_ctx *ctx, const double *g, double *lambda,
                                   const msrsb_solve_opts *opts, msrsb_solve_info *info,
                                   int where);

/* Gradient of an objective with respect to log k through the TPFA system
 * of the last msrsb_assemble_tpfa, given the pressure p and the adjoint
 * lambda (A^T lambda = dJ/dp):
 *   grad_K = -[ sum_{faces (K,L)} T k_L/(k_K+k_L) (p_K-p_L)(lam_K-lam_L)
 *               + sum_{Dirichlet faces of K} T_b (p_K - g_b) lam_K ].
 * (Derived from the TPFA transmissibilities; the paper has no adjoint.)
 * All vectors n values.  Errors: E_STATE if A was not assembled by
 * msrsb_assemble_tpfa. */
msrsb_status msrsb_tpfa_adjoint_grad(msrsb_ctx *ctx, const double *log_k, const double *p,
                                     const double *lambda, double *grad, int where);

/* Q1 (bi/trilinear) finite element linear elasticity (App. "Linear
 * elastostatics: Galerkin finite element formulation", eq.
 * model_elastostatics_bilin_FE) on a Cartesian grid of dim = 2 (plane
 * strain) or 3 dimensions: elems[d] equal elements of size h[d] per axis,
 * Young's modulus E_e = exp(log_E[e]) per element (x fastest, prod(elems)
 * values) and Poisson ratio nu in (-1, 1/2).  Nodes are numbered
 * x + (nx+1)(y + (ny+1) z) and the dofs are interleaved, dof = dim*node + l.
 * fixed (n = dim * #nodes bytes, may be NULL) marks homogeneous Dirichlet
 * dofs, imposed by symmetric diagonalisation (Remark "FEM_Dir_BC"): their
 * row and column are zero except for the diagonal.  Each row keeps the full
 * pattern of its 3^dim neighbouring nodes (zeros included).  The result
 * becomes the context's matrix with block_size = dim, as msrsb_set_matrix
 * would set it (same pattern on a repeated call with the same grid: then it
 * acts as msrsb_update_values and keeps P for a warm start).  Loads (the
 * right-hand side) are the caller's.
 * Errors: E_ARG for a bad dimension, grid, sizes or nu. */
msrsb_status msrsb_assemble_q1(msrsb_ctx *ctx, int32_t dim, const int32_t elems[3],
                               const double h[3], double nu, const double *log_E,
                               const uint8_t *fixed, int where);

/* Gradient with respect to log E of an objective through the elasticity
 * system of the last msrsb_assemble_q1, given the displacement u and the
 * adjoint lambda (A^T lambda = dJ/du), both n values:
 *   grad_e = -E_e lambda_e^T K0_e u_e
 * with K0_e the element stiffness for E = 1 and fixed dofs taken as zero
 * (the right-hand side must not depend on E).  grad has prod(elems) values.
 * (Derived from the element assembly; the paper has no adjoint.)
 * Errors: E_STATE if A was not assembled by msrsb_assemble_q1. */
msrsb_status msrsb_q1_adjoint_grad(msrsb_ctx *ctx, const double *u, const double *lambda,
                                   double *grad, int where);

/* Milliseconds of the last run of each phase (MSRSB_PHASE_*), measured
 * with HIP events on the context's stream: the set-up steps of Alg. 1 and
 * Alg. 2 and the solves around Alg. 3-4 (instrumentation, not part of the
 * method).  Writes n_phases values, zero for phases past MSRSB_N_PHASES
 * or not run yet.  Synchronises. */
msrsb_status msrsb_get_timings(msrsb_ctx *ctx, double *ms_by_phase, int32_t n_phases);

#ifdef __cplusplus
}
#endif

#endif /* MSRSB_H */
