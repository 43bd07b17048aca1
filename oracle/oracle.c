/*
 * Plain FP64 CPU oracle for enhanced MsRSB preconditioning
 * (Bosma, Klevtsov, Moyner, Castelletto, arXiv:1912.06934).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source with the HIP library and is deliberately slow and literal: plain
 * loops, double precision, no blocking, no fusion, built with
 * -ffp-contract=off so every product and sum is rounded as written.
 * OpenMP is used only over independent rows (each row's arithmetic is done
 * in a fixed order by one thread), so results do not depend on the number
 * of threads.
 *
 * Every function names the passage of the paper it follows.  Sparse
 * matrices are CSR (int32 row pointers and column indices, columns sorted
 * ascending, FP64 values).
 *
 * Return codes: 0 ok, -1 bad argument, -6 singular coarse matrix,
 * -7 Krylov breakdown (non-finite value or non-positive curvature in CG),
 * -8 iteration limit reached.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EARG (-1)
#define ORC_ESING (-6)
#define ORC_EBREAK (-7)
#define ORC_ENOCONV (-8)

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Filter and Jacobi operator: eq. (negoffdiag), eq. (Dhat_zero_rowsum),
 * Alg. 1 (first three statements), SDC block diagonal (Sec. 4).
 *
 * G is A restricted to same-component couplings (comp = index % bs).  With
 * filter != 0 its off-diagonal entries are min(A_ij, 0).  Dhat_ii is minus
 * the sum of G's off-diagonal entries of row i, so L + Dhat + U has zero
 * row sums.  The smoothing update P - omega Dhat^{-1} Ghat P equals J P with
 *   J_ii = 1 - omega,   J_ij = -omega G_ij / Dhat_ii   (j != i).
 * A row with Dhat_ii == 0 has nothing to smooth against and is frozen
 * (J_i = e_i).  J is returned on A's pattern (cross-component and frozen
 * entries are explicit zeros).  dhat may be NULL.
 */
int orc_filter_jacobi(int n, const int *rp, const int *ci, const double *a,
                      int bs, int filter, double omega, double *jv,
                      double *dhat)
{
    if (n < 0 || bs < 1) return ORC_EARG;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        int has_diag = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j == i) { has_diag = 1; continue; }
            if (j % bs != i % bs) continue;
            double g = a[e];
            if (filter && g > 0.0) g = 0.0;
            d -= g;
        }
        if (!has_diag) bad = 1;
        if (dhat) dhat[i] = d;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (d == 0.0) {
                jv[e] = (j == i) ? 1.0 : 0.0;
            } else if (j == i) {
                jv[e] = 1.0 - omega;
            } else if (j % bs != i % bs) {
                jv[e] = 0.0;
            } else {
                double g = a[e];
                if (filter && g > 0.0) g = 0.0;
                jv[e] = -omega * g / d;
            }
        }
    }
    return bad ? ORC_EARG : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Initial basis (Sec. 2.1): column j is the characteristic function of
 * coarse block j, so P_ij = 1 if j == part(i), else 0, on P's pattern.
 * Fails if part(i) is not in row i's pattern. */
int orc_init_basis(int n, const int *prp, const int *pci, const int *part,
                   double *pv)
{
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        int found = 0;
        for (int e = prp[i]; e < prp[i + 1]; ++e) {
            pv[e] = (pci[e] == part[i]) ? 1.0 : 0.0;
            if (pci[e] == part[i]) found = 1;
        }
        if (!found) bad = 1;
    }
    return bad ? ORC_EARG : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* One restricted smoothing iteration (eq. (smoother) with the support
 * restriction and the renormalisation of Alg. 1).
 *
 * For each row i and each j in row i's (frozen) pattern:
 *   T_ij = sum over the J-neighbours k of i, in ascending k, of J_ik P_kj.
 * Products P_kj whose column j is not in row i's pattern are dropped: that
 * keeps every basis function inside its support.  Then
 *   delta_ij = T_ij - P_ij          (the restricted update)
 *   s_i      = sum_j T_ij           (ascending j)
 *   Pnew_ij  = T_ij / s_i           (rescale the updated values, so every
 *                                    row of P sums to one).
 * If eit != NULL, *eit = max |delta_ij| over rows with interior[i] != 0.
 */
int orc_smooth_step(int n, const int *rp, const int *ci, const double *jv,
                    const int *prp, const int *pci, const double *pin,
                    double *pout, const uint8_t *interior, double *eit)
{
    double emax = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : emax) reduction(| : bad)
    for (int i = 0; i < n; ++i) {
        int p0 = prp[i], np = prp[i + 1] - prp[i];
        double t[64];
        if (np > 64 || np < 1) { bad = 1; continue; }
        for (int s = 0; s < np; ++s) t[s] = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int k = ci[e];
            double w = jv[e];
            for (int q = prp[k]; q < prp[k + 1]; ++q) {
                int c = pci[q];
                for (int s = 0; s < np; ++s) {
                    if (pci[p0 + s] == c) {
                        double prod = w * pin[q];
                        t[s] = t[s] + prod;
                        break;
                    }
                }
            }
        }
        double rs = 0.0;
        for (int s = 0; s < np; ++s) rs = rs + t[s];
        for (int s = 0; s < np; ++s) {
            double d = t[s] - pin[p0 + s];
            if (interior && interior[i]) {
                double ad = fabs(d);
                if (ad > emax || ad != ad) emax = (ad != ad) ? INFINITY : ad;
            }
            pout[p0 + s] = t[s] / rs;
        }
    }
    if (eit) *eit = emax;
    return bad ? ORC_EARG : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 loop: iterate the restricted smoothing from the P given in pv
 * (warm start, Alg. 2) for k = 0, 1, ...; after iteration k, when
 * k mod nit == 0, e_it is computed and the loop stops if e_it <= tol.
 * At most kmax iterations.  A negative tol never stops early.
 * *iters = iterations done; eit_hist[k] = e_it after iteration k, or -1
 * when it was not computed (eit_hist may be NULL). */
int orc_basis(int n, const int *rp, const int *ci, const double *jv,
              const int *prp, const int *pci, double *pv,
              const uint8_t *interior, int kmax, double tol, int nit,
              int *iters, double *eit_last, double *eit_hist)
{
    if (nit < 1 || kmax < 0) return ORC_EARG;
    int64_t nnzp = prp[n];
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(nnzp > 0 ? nnzp : 1));
    if (!tmp) return ORC_EARG;
    double *src = pv, *dst = tmp;
    int k = 0, rc = ORC_OK;
    double e = INFINITY;
    for (k = 0; k < kmax; ++k) {
        int check = (k % nit) == 0;
        double ek = -1.0;
        rc = orc_smooth_step(n, rp, ci, jv, prp, pci, src, dst, interior,
                             check ? &ek : NULL);
        if (rc) break;
        if (eit_hist) eit_hist[k] = check ? ek : -1.0;
        double *sw = src; src = dst; dst = sw;
        if (check) {
            e = ek;
            if (e <= tol) { ++k; break; }
        }
    }
    if (src != pv) memcpy(pv, src, sizeof(double) * (size_t)nnzp);
    free(tmp);
    if (iters) *iters = k;
    if (eit_last) *eit_last = e;
    return rc;
}

/* ------------------------------------------------------------------ */
/* Galerkin coarse operator, eq. (lin_system_coarse) with R = P^T (Alg. 2):
 *   Ac[j,l] = sum_i P_ij * ( sum_k A_ik P_kl )
 * with the full, unfiltered A.  i runs ascending, and the inner sum over k
 * ascending.  Ac is dense, row-major, nc x nc.  Coarse rows are
 * independent, so they are computed in parallel from the transpose of P's
 * pattern. */
int orc_rap(int n, const int *rp, const int *ci, const double *a, int nc,
            const int *prp, const int *pci, const double *pv, double *ac)
{
    int64_t nnzp = prp[n];
    /* transpose of P: for each coarse j, the fine rows i (ascending) */
    int *cnt = (int *)calloc((size_t)nc + 1, sizeof(int));
    int *ti = (int *)malloc(sizeof(int) * (size_t)(nnzp > 0 ? nnzp : 1));
    int64_t *te = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnzp > 0 ? nnzp : 1));
    if (!cnt || !ti || !te) { free(cnt); free(ti); free(te); return ORC_EARG; }
    for (int64_t e = 0; e < nnzp; ++e) {
        if (pci[e] < 0 || pci[e] >= nc) { free(cnt); free(ti); free(te); return ORC_EARG; }
        cnt[pci[e] + 1]++;
    }
    for (int j = 0; j < nc; ++j) cnt[j + 1] += cnt[j];
    int *pos = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    memcpy(pos, cnt, sizeof(int) * (size_t)nc);
    for (int i = 0; i < n; ++i)
        for (int e = prp[i]; e < prp[i + 1]; ++e) {
            int j = pci[e];
            ti[pos[j]] = i;
            te[pos[j]] = e;
            pos[j]++;
        }
    free(pos);
    memset(ac, 0, sizeof(double) * (size_t)nc * (size_t)nc);
#pragma omp parallel
    {
        double *ap = (double *)calloc((size_t)nc, sizeof(double));
        int *touched = (int *)malloc(sizeof(int) * (size_t)nc);
        char *mark = (char *)calloc((size_t)nc, 1);
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < nc; ++j) {
            double *row = ac + (size_t)j * nc;
            for (int t = cnt[j]; t < cnt[j + 1]; ++t) {
                int i = ti[t];
                double pij = pv[te[t]];
                /* row i of A P, accumulated over k ascending */
                int nt = 0;
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    int k = ci[e];
                    for (int q = prp[k]; q < prp[k + 1]; ++q) {
                        int l = pci[q];
                        double prod = a[e] * pv[q];
                        if (!mark[l]) { mark[l] = 1; touched[nt++] = l; ap[l] = 0.0; }
                        ap[l] = ap[l] + prod;
                    }
                }
                for (int u = 0; u < nt; ++u) {
                    int l = touched[u];
                    double prod = pij * ap[l];
                    row[l] = row[l] + prod;
                    mark[l] = 0;
                }
            }
        }
        free(ap); free(touched); free(mark);
    }
    free(cnt); free(ti); free(te);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Coarse solver M_c^{-1} = A_c^{-1} (Alg. 2): dense LU with partial
 * pivoting, in place, row-major.  At step k the pivot is the first row
 * r >= k with the largest |a_rk|; an exact zero pivot means A_c is
 * singular.  piv[k] = the row swapped with row k. */
int orc_lu(int nc, double *a, int *piv)
{
    for (int k = 0; k < nc; ++k) {
        int p = k;
        double best = fabs(a[(size_t)k * nc + k]);
        for (int r = k + 1; r < nc; ++r) {
            double v = fabs(a[(size_t)r * nc + k]);
            if (v > best) { best = v; p = r; }
        }
        piv[k] = p;
        if (best == 0.0 || best != best) return ORC_ESING;
        if (p != k)
            for (int c = 0; c < nc; ++c) {
                double t = a[(size_t)k * nc + c];
                a[(size_t)k * nc + c] = a[(size_t)p * nc + c];
                a[(size_t)p * nc + c] = t;
            }
        double d = a[(size_t)k * nc + k];
#pragma omp parallel for schedule(static)
        for (int r = k + 1; r < nc; ++r) {
            double l = a[(size_t)r * nc + k] / d;
            a[(size_t)r * nc + k] = l;
            for (int c = k + 1; c < nc; ++c) {
                double prod = l * a[(size_t)k * nc + c];
                a[(size_t)r * nc + c] = a[(size_t)r * nc + c] - prod;
            }
        }
    }
    return ORC_OK;
}

/* Solve (LU) x = Pm b in place (trans == 0), or the transposed system
 * A^T x = b (trans != 0), from orc_lu's factors. */
void orc_lu_solve(int nc, const double *lu, const int *piv, double *b, int trans)
{
    if (!trans) {
        for (int k = 0; k < nc; ++k)
            if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
        for (int r = 0; r < nc; ++r) {
            double s = b[r];
            for (int c = 0; c < r; ++c) s = s - lu[(size_t)r * nc + c] * b[c];
            b[r] = s;
        }
        for (int r = nc - 1; r >= 0; --r) {
            double s = b[r];
            for (int c = r + 1; c < nc; ++c) s = s - lu[(size_t)r * nc + c] * b[c];
            b[r] = s / lu[(size_t)r * nc + r];
        }
    } else {
        /* A = Pm^T L U  =>  A^T = U^T L^T Pm:  solve U^T y = b, L^T w = y, x = Pm^T w */
        for (int r = 0; r < nc; ++r) {
            double s = b[r];
            for (int c = 0; c < r; ++c) s = s - lu[(size_t)c * nc + r] * b[c];
            b[r] = s / lu[(size_t)r * nc + r];
        }
        for (int r = nc - 1; r >= 0; --r) {
            double s = b[r];
            for (int c = r + 1; c < nc; ++c) s = s - lu[(size_t)c * nc + r] * b[c];
            b[r] = s;
        }
        for (int k = nc - 1; k >= 0; --k)
            if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    }
}

/* ------------------------------------------------------------------ */
/* ILU(0): incomplete LU on A's own pattern, natural order (the IKJ
 * elimination restricted to existing entries).  lu holds L (unit
 * diagonal, not stored) strictly below the diagonal and U on and above
 * it, on A's pattern, so (L U)_ij = A_ij wherever A has an entry. */
int orc_ilu0(int n, const int *rp, const int *ci, const double *a, double *lu)
{
    int64_t nnz = rp[n];
    memcpy(lu, a, sizeof(double) * (size_t)nnz);
    int *diag = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *where = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) { diag[i] = -1; where[i] = -1; }
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] == i) diag[i] = e;
    int rc = ORC_OK;
    for (int i = 0; i < n && rc == ORC_OK; ++i) {
        if (diag[i] < 0) { rc = ORC_EARG; break; }
        for (int e = rp[i]; e < rp[i + 1]; ++e) where[ci[e]] = e;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int k = ci[e];
            if (k >= i) break;
            double pivot = lu[diag[k]];
            if (pivot == 0.0) { rc = ORC_ESING; break; }
            double lik = lu[e] / pivot;
            lu[e] = lik;
            for (int f = diag[k] + 1; f < rp[k + 1]; ++f) {
                int w = where[ci[f]];
                if (w >= 0) {
                    double prod = lik * lu[f];
                    lu[w] = lu[w] - prod;
                }
            }
        }
        for (int e = rp[i]; e < rp[i + 1]; ++e) where[ci[e]] = -1;
    }
    free(diag);
    free(where);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sweep orders of the triangular smoothers (ILU(0), IC(0), symmetric
 * Gauss-Seidel).  The paper names the smoothers but not the order in which
 * they visit the unknowns.  Two orders are used: the natural one, and a
 * multicolour order in which rows of one colour never couple, so that all
 * rows of a colour can be processed at once.
 *
 * Colouring: first fit in ascending row order on the symmetrised pattern of
 * A (j is a neighbour of i when A_ij or A_ji is stored, j != i): row i gets
 * the smallest colour that none of its already coloured neighbours has.
 * Returns the number of colours. */
int orc_color(int n, const int *rp, const int *ci, int *color)
{
    int64_t nnz = rp[n];
    /* pattern of A^T */
    int *trp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *tci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *pos = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *stamp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    if (!trp || !tci || !pos || !stamp) { free(trp); free(tci); free(pos); free(stamp); return ORC_EARG; }
    for (int64_t e = 0; e < nnz; ++e) trp[ci[e] + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    for (int i = 0; i < n; ++i) pos[i] = trp[i];
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) tci[pos[ci[e]]++] = i;
    for (int c = 0; c <= n; ++c) stamp[c] = -1;
    int ncol = 0;
    for (int i = 0; i < n; ++i) {
        /* colours taken by neighbours that come before i */
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] < i) stamp[color[ci[e]]] = i;
        for (int e = trp[i]; e < trp[i + 1]; ++e)
            if (tci[e] < i) stamp[color[tci[e]]] = i;
        int c = 0;
        while (stamp[c] == i) ++c;
        color[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(trp); free(tci); free(pos); free(stamp);
    return ncol;
}

/* The multicolour order: rows sorted by colour, ascending row index within a
 * colour.  order[k] = the k-th row visited. */
void orc_color_order(int n, const int *color, int ncol, int *order)
{
    int k = 0;
    for (int c = 0; c < ncol; ++c)
        for (int i = 0; i < n; ++i)
            if (color[i] == c) order[k++] = i;
}

/* B = Q A Q^T for the order: row k of B is row order[k] of A, with every
 * column j renumbered to its position in the order; columns sorted
 * ascending.  brp (n+1), bci and ba (nnz) are the caller's. */
int orc_permute(int n, const int *rp, const int *ci, const double *a, const int *order,
                int *brp, int *bci, double *ba)
{
    int *rank = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!rank) return ORC_EARG;
    for (int k = 0; k < n; ++k) rank[order[k]] = k;
    brp[0] = 0;
    for (int k = 0; k < n; ++k) {
        int i = order[k], b0 = brp[k];
        int len = rp[i + 1] - rp[i];
        for (int t = 0; t < len; ++t) {
            /* insertion in ascending new column */
            int col = rank[ci[rp[i] + t]];
            double v = a[rp[i] + t];
            int q = b0 + t;
            while (q > b0 && bci[q - 1] > col) {
                bci[q] = bci[q - 1];
                ba[q] = ba[q - 1];
                --q;
            }
            bci[q] = col;
            ba[q] = v;
        }
        brp[k + 1] = b0 + len;
    }
    free(rank);
    return ORC_OK;
}

/* IC(0): incomplete Cholesky on the lower part of a symmetric A's own
 * pattern, natural order (the no-fill factorisation of Sec. 4.1 and
 * Sec. 4.2).  For i ascending and each stored j < i, ascending,
 *   L_ij = (A_ij - sum_{k < j} L_ik L_jk) / L_jj,
 * the sum running over the k stored in both rows, then
 *   L_ii = sqrt(A_ii - sum_{k < i} L_ik^2),
 * so (L L^T)_ij = A_ij wherever the lower pattern has an entry.  l holds L
 * on A's pattern (entries above the diagonal are set to zero).  A
 * non-positive square-root argument is a breakdown (ORC_ESING). */
int orc_ic0(int n, const int *rp, const int *ci, const double *a, double *l)
{
    int64_t nnz = rp[n];
    for (int64_t e = 0; e < nnz; ++e) l[e] = 0.0;
    for (int i = 0; i < n; ++i) {
        int dpos = -1;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (j > i) break;
            if (j == i) { dpos = e; break; }
            /* sum over k < j stored in rows i and j (both ascending) */
            double s = a[e];
            int p = rp[i], q = rp[j];
            while (p < e && q < rp[j + 1] && ci[q] < j) {
                if (ci[p] < ci[q]) ++p;
                else if (ci[p] > ci[q]) ++q;
                else { double prod = l[p] * l[q]; s = s - prod; ++p; ++q; }
            }
            int jd = -1;
            for (int f = rp[j]; f < rp[j + 1]; ++f) if (ci[f] == j) jd = f;
            if (jd < 0) return ORC_EARG;
            l[e] = s / l[jd];
        }
        if (dpos < 0) return ORC_EARG;
        double s = a[dpos];
        for (int e = rp[i]; e < dpos; ++e) { double prod = l[e] * l[e]; s = s - prod; }
        if (!(s > 0.0)) return ORC_ESING;
        l[dpos] = sqrt(s);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Two-stage preconditioner (Alg. 3 and Alg. 4). */
typedef struct orc_prec_s {
    int n;
    const int *rp, *ci;
    const double *a;          /* fine operator (A, or A^T for the adjoint) */
    int nc;
    const int *prp, *pci;
    const double *pv;         /* prolongation P; R = P^T */
    const double *lu;         /* LU of A_c (nc x nc) */
    const int *piv;
    int lu_trans;             /* solve with A_c^T instead of A_c */
    int use_ms;               /* 0: smoother only (no coarse stage) */
    int pre_kind, pre_sweeps; /* 0 none, 1 Jacobi, 2 l1-Jacobi, 3 ILU(0),
                                 4 symmetric Gauss-Seidel, 5 IC(0) */
    int post_kind, post_sweeps;
    /* kinds 3-5 work on B = Q A Q^T in natural order, i.e. on A in the
     * order `order` (NULL: natural, and then B = A) */
    const int *order;
    const int *brp, *bci;
    const double *ba;
    const double *ilu;        /* ILU(0) factors of B (kind 3) */
    const double *ic;         /* IC(0) factor L of B (kind 5) */
    /* restriction: NULL = Galerkin R = P^T; otherwise the coarse block of
     * every fine row, and R is the block indicator (Petrov-Galerkin, MsFV) */
    const int *part;
    /* multilevel MsRSB (the conclusion's multilevel use of the enhanced
     * method): when not NULL, the coarse solve M_c^{-1} is the two-stage
     * preconditioner of the next level, built on A_c, instead of the LU */
    const struct orc_prec_s *next;
} orc_prec;

static void spmv(int n, const int *rp, const int *ci, const double *a,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) s = s + a[e] * x[ci[e]];
        y[i] = s;
    }
}

/* z += M^{-1} (v - A z) for one sweep of the given smoother.  tmp needs n
 * doubles, perm 3n (kinds 3-5). */
static void smooth_sweep(const orc_prec *m, int kind, const double *v,
                         double *z, double *tmp, double *perm)
{
    int n = m->n;
    const int *rp = m->rp, *ci = m->ci;
    const double *a = m->a;
    if (kind >= 3) {
        /* in B's numbering: vb = Q v, zb = Q z */
        const int *brp = m->order ? m->brp : rp, *bci = m->order ? m->bci : ci;
        const double *ba = m->order ? m->ba : a;
        double *vb = perm, *zb = perm + n, *rb = perm + 2 * (size_t)n;
        for (int k = 0; k < n; ++k) {
            int i = m->order ? m->order[k] : k;
            vb[k] = v[i];
            zb[k] = z[i];
        }
        if (kind == 4) {
            /* symmetric Gauss-Seidel: a forward sweep over the rows, each
             * row corrected by its own residual with the values already
             * updated, then the same backwards */
            for (int pass = 0; pass < 2; ++pass)
                for (int t = 0; t < n; ++t) {
                    int k = pass == 0 ? t : n - 1 - t;
                    double r = vb[k], d = 0.0;
                    for (int e = brp[k]; e < brp[k + 1]; ++e) {
                        r = r - ba[e] * zb[bci[e]];
                        if (bci[e] == k) d = ba[e];
                    }
                    zb[k] = zb[k] + r / d;
                }
        } else {
            /* rb = vb - B zb, then the two triangular solves */
            for (int k = 0; k < n; ++k) {
                double r = vb[k];
                for (int e = brp[k]; e < brp[k + 1]; ++e) r = r - ba[e] * zb[bci[e]];
                rb[k] = r;
            }
            if (kind == 3) {
                /* L y = rb (unit lower), U w = y */
                for (int k = 0; k < n; ++k) {
                    double s = rb[k];
                    for (int e = brp[k]; e < brp[k + 1] && bci[e] < k; ++e)
                        s = s - m->ilu[e] * rb[bci[e]];
                    rb[k] = s;
                }
                for (int k = n - 1; k >= 0; --k) {
                    double s = rb[k], d = 0.0;
                    for (int e = brp[k]; e < brp[k + 1]; ++e) {
                        if (bci[e] == k) d = m->ilu[e];
                        else if (bci[e] > k) s = s - m->ilu[e] * rb[bci[e]];
                    }
                    rb[k] = s / d;
                }
            } else {
                /* L y = rb, then L^T w = y by columns: w_k = y_k / L_kk,
                 * then y_j -= L_kj w_k for the stored j < k */
                const double *L = m->ic;
                for (int k = 0; k < n; ++k) {
                    double s = rb[k], d = 0.0;
                    for (int e = brp[k]; e < brp[k + 1] && bci[e] <= k; ++e) {
                        if (bci[e] == k) d = L[e];
                        else s = s - L[e] * rb[bci[e]];
                    }
                    rb[k] = s / d;
                }
                for (int k = n - 1; k >= 0; --k) {
                    double d = 0.0;
                    for (int e = brp[k]; e < brp[k + 1] && bci[e] <= k; ++e)
                        if (bci[e] == k) d = L[e];
                    rb[k] = rb[k] / d;
                    for (int e = brp[k]; e < brp[k + 1] && bci[e] < k; ++e) {
                        double prod = L[e] * rb[k];
                        rb[bci[e]] = rb[bci[e]] - prod;
                    }
                }
            }
            for (int k = 0; k < n; ++k) zb[k] = zb[k] + rb[k];
        }
        for (int k = 0; k < n; ++k) z[m->order ? m->order[k] : k] = zb[k];
        return;
    }
    spmv(n, rp, ci, a, z, tmp);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) tmp[i] = v[i] - tmp[i];
    if (kind == 1 || kind == 2) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double d = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                if (kind == 1) { if (ci[e] == i) d = a[e]; }
                else d = d + fabs(a[e]);
            }
            z[i] = z[i] + tmp[i] / d;
        }
    }
}

/* z = B v, Alg. 4: z = 0; pre-smoothing; z += P A_c^{-1} R (v - A z);
 * post-smoothing.  work needs PREC_WORK(n, nc) doubles. */
#define PREC_WORK(n, nc) (5 * (size_t)(n) + (size_t)(nc) + 1)
static void prec_apply(const orc_prec *m, const double *v, double *z, double *work)
{
    int n = m->n;
    double *tmp = work, *res = work + n, *perm = work + 2 * (size_t)n,
           *vc = work + 5 * (size_t)n;
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    for (int s = 0; s < m->pre_sweeps; ++s) smooth_sweep(m, m->pre_kind, v, z, tmp, perm);
    if (m->use_ms) {
        spmv(n, m->rp, m->ci, m->a, z, res);
        for (int i = 0; i < n; ++i) res[i] = v[i] - res[i];
        for (int j = 0; j < m->nc; ++j) vc[j] = 0.0;
        if (m->part) {                                     /* v_c = R r, R = block indicator */
            for (int i = 0; i < n; ++i) vc[m->part[i]] = vc[m->part[i]] + res[i];
        } else {                                           /* v_c = R r, R = P^T */
            for (int i = 0; i < n; ++i)
                for (int e = m->prp[i]; e < m->prp[i + 1]; ++e)
                    vc[m->pci[e]] = vc[m->pci[e]] + m->pv[e] * res[i];
        }
        if (m->next) {                                      /* w_c = B_next v_c */
            double *wc = (double *)malloc(sizeof(double) * (size_t)(m->nc > 0 ? m->nc : 1));
            double *w2 = (double *)malloc(sizeof(double) * PREC_WORK(m->nc, m->next->nc));
            prec_apply(m->next, vc, wc, w2);
            for (int j = 0; j < m->nc; ++j) vc[j] = wc[j];
            free(wc);
            free(w2);
        } else {
            orc_lu_solve(m->nc, m->lu, m->piv, vc, m->lu_trans); /* w_c = M_c^{-1} v_c */
        }
        for (int i = 0; i < n; ++i) {                      /* z += P w_c */
            double s = 0.0;
            for (int e = m->prp[i]; e < m->prp[i + 1]; ++e) s = s + m->pv[e] * vc[m->pci[e]];
            z[i] = z[i] + s;
        }
    }
    for (int s = 0; s < m->post_sweeps; ++s) smooth_sweep(m, m->post_kind, v, z, tmp, perm);
}

int orc_apply(const orc_prec *m, const double *v, double *z)
{
    double *work = (double *)malloc(sizeof(double) * PREC_WORK(m->n, m->nc));
    if (!work) return ORC_EARG;
    prec_apply(m, v, z, work);
    free(work);
    return ORC_OK;
}

static double dot(int n, const double *x, const double *y)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = s + x[i] * y[i];
    return s;
}

static int is_finite(double x) { return x == x && x - x == 0.0; }

/* Preconditioned CG with the flexible (Polak-Ribiere) beta
 *   beta = r_{k+1}^T (z_{k+1} - z_k) / r_k^T z_k,
 * which stays valid for a non-symmetric or inexact preconditioner.
 * x holds x0 on entry.  The loop stops when the recursive residual drops
 * below rtol ||f||; the true residual ||f - A x|| is then recomputed and
 * the iteration restarts from x if it is still above.  Iterations count
 * products A p.  hist (may be NULL) receives ||r_k||/||f|| for
 * k = 0..iters. */
int orc_pcg(const orc_prec *m, const double *f, double *x, double rtol,
            int maxit, int *iters, double *true_rel, double *hist, int hist_cap)
{
    int n = m->n;
    size_t N = (size_t)n;
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N),
           *zold = malloc(sizeof(double) * N), *p = malloc(sizeof(double) * N),
           *q = malloc(sizeof(double) * N),
           *work = malloc(sizeof(double) * PREC_WORK(n, m->nc));
    int rc = ORC_ENOCONV, it = 0;
    double fn = sqrt(dot(n, f, f));
    if (fn == 0.0) fn = 1.0;
    double rr = 0.0;
    int restart = 1;
    double rz = 0.0;
    while (it <= maxit) {
        if (restart) {
            spmv(n, m->rp, m->ci, m->a, x, q);
            for (int i = 0; i < n; ++i) r[i] = f[i] - q[i];
            rr = sqrt(dot(n, r, r));
            if (hist && it < hist_cap) hist[it] = rr / fn;
            if (!is_finite(rr)) { rc = ORC_EBREAK; break; }
            if (rr <= rtol * fn) { rc = ORC_OK; break; }
            if (it == maxit) break;
            prec_apply(m, r, z, work);
            for (int i = 0; i < n; ++i) p[i] = z[i];
            rz = dot(n, r, z);
            restart = 0;
        }
        spmv(n, m->rp, m->ci, m->a, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !is_finite(pq) || !is_finite(rz)) { rc = ORC_EBREAK; break; }
        double alpha = rz / pq;
        for (int i = 0; i < n; ++i) { x[i] = x[i] + alpha * p[i]; r[i] = r[i] - alpha * q[i]; }
        ++it;
        rr = sqrt(dot(n, r, r));
        if (hist && it < hist_cap) hist[it] = rr / fn;
        if (!is_finite(rr)) { rc = ORC_EBREAK; break; }
        if (rr <= rtol * fn) { restart = 1; continue; }
        if (it >= maxit) break;
        for (int i = 0; i < n; ++i) zold[i] = z[i];
        prec_apply(m, r, z, work);
        double num = 0.0;
        for (int i = 0; i < n; ++i) num = num + r[i] * (z[i] - zold[i]);
        double rznew = dot(n, r, z);
        double beta = num / rz;
        rz = rznew;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    spmv(n, m->rp, m->ci, m->a, x, q);
    for (int i = 0; i < n; ++i) r[i] = f[i] - q[i];
    if (true_rel) *true_rel = sqrt(dot(n, r, r)) / fn;
    if (iters) *iters = it;
    free(r); free(z); free(zold); free(p); free(q); free(work);
    return rc;
}

/* Right-preconditioned restarted GMRES(m): Arnoldi with modified
 * Gram-Schmidt on A B, Givens rotations for the least-squares problem,
 * x = x0 + B (V y) at the end of each cycle.  Stops on the recursive
 * residual, then checks the true residual as in orc_pcg.  Iterations count
 * Arnoldi steps. */
int orc_gmres(const orc_prec *m, const double *f, double *x, int restart,
              double rtol, int maxit, int *iters, double *true_rel,
              double *hist, int hist_cap)
{
    int n = m->n, mm = restart;
    size_t N = (size_t)n;
    if (mm < 1) return ORC_EARG;
    double *V = malloc(sizeof(double) * N * (size_t)(mm + 1));
    double *H = calloc((size_t)(mm + 1) * (size_t)mm, sizeof(double));
    double *cs = malloc(sizeof(double) * (size_t)mm), *sn = malloc(sizeof(double) * (size_t)mm);
    double *g = malloc(sizeof(double) * (size_t)(mm + 1)), *y = malloc(sizeof(double) * (size_t)mm);
    double *w = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *work = malloc(sizeof(double) * PREC_WORK(n, m->nc));
    double fn = sqrt(dot(n, f, f));
    if (fn == 0.0) fn = 1.0;
    int it = 0, rc = ORC_ENOCONV;
    for (;;) {
        spmv(n, m->rp, m->ci, m->a, x, w);
        for (int i = 0; i < n; ++i) w[i] = f[i] - w[i];
        double beta = sqrt(dot(n, w, w));
        if (hist && it < hist_cap) hist[it] = beta / fn;
        if (!is_finite(beta)) { rc = ORC_EBREAK; break; }
        if (beta <= rtol * fn) { rc = ORC_OK; break; }
        if (it >= maxit) break;
        for (int i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int k = 0; k <= mm; ++k) g[k] = 0.0;
        g[0] = beta;
        int j = 0;
        int converged = 0;
        for (j = 0; j < mm && it < maxit; ++j) {
            double *vj = V + (size_t)j * N, *vn = V + (size_t)(j + 1) * N;
            prec_apply(m, vj, z, work);
            spmv(n, m->rp, m->ci, m->a, z, w);
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * N;
                double h = dot(n, w, vi);
                H[(size_t)i * mm + j] = h;
                for (int t = 0; t < n; ++t) w[t] = w[t] - h * vi[t];
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(j + 1) * mm + j] = hn;
            if (hn != 0.0)
                for (int t = 0; t < n; ++t) vn[t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {
                double h0 = H[(size_t)i * mm + j], h1 = H[(size_t)(i + 1) * mm + j];
                H[(size_t)i * mm + j] = cs[i] * h0 + sn[i] * h1;
                H[(size_t)(i + 1) * mm + j] = -sn[i] * h0 + cs[i] * h1;
            }
            double h0 = H[(size_t)j * mm + j], h1 = H[(size_t)(j + 1) * mm + j];
            double den = sqrt(h0 * h0 + h1 * h1);
            if (den == 0.0 || !is_finite(den)) { rc = ORC_EBREAK; converged = -1; break; }
            cs[j] = h0 / den;
            sn[j] = h1 / den;
            H[(size_t)j * mm + j] = den;
            H[(size_t)(j + 1) * mm + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            double res = fabs(g[j + 1]);
            if (hist && it < hist_cap) hist[it] = res / fn;
            if (res <= rtol * fn || hn == 0.0) { converged = 1; ++j; break; }
        }
        /* back substitution for y, then x += B (V y) */
        for (int r = j - 1; r >= 0; --r) {
            double s = g[r];
            for (int c = r + 1; c < j; ++c) s = s - H[(size_t)r * mm + c] * y[c];
            y[r] = s / H[(size_t)r * mm + r];
        }
        for (int t = 0; t < n; ++t) {
            double s = 0.0;
            for (int r = 0; r < j; ++r) s = s + V[(size_t)r * N + t] * y[r];
            w[t] = s;
        }
        prec_apply(m, w, z, work);
        for (int t = 0; t < n; ++t) x[t] = x[t] + z[t];
        if (converged < 0) break;
    }
    spmv(n, m->rp, m->ci, m->a, x, w);
    for (int i = 0; i < n; ++i) w[i] = f[i] - w[i];
    if (true_rel) *true_rel = sqrt(dot(n, w, w)) / fn;
    if (iters) *iters = it;
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(w); free(z); free(work);
    return rc;
}

/* Stand-alone (Richardson) iteration with the two-stage preconditioner, the
 * "non-accelerated stand-alone solver" of Sec. 3.2:
 *   x_{k+1} = x_k + B (f - A x_k).
 * Stops when ||f - A x_k|| <= rtol ||f||; iterations count applications of
 * B.  hist (may be NULL) receives ||f - A x_k|| / ||f|| for k = 0..iters. */
int orc_richardson(const orc_prec *m, const double *f, double *x, double rtol, int maxit,
                   int *iters, double *true_rel, double *hist, int hist_cap)
{
    int n = m->n;
    size_t N = (size_t)n;
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N),
           *work = malloc(sizeof(double) * PREC_WORK(n, m->nc));
    double fn = sqrt(dot(n, f, f));
    if (fn == 0.0) fn = 1.0;
    int it = 0, rc = ORC_ENOCONV;
    double rr = 0.0;
    for (;;) {
        spmv(n, m->rp, m->ci, m->a, x, r);
        for (int i = 0; i < n; ++i) r[i] = f[i] - r[i];
        rr = sqrt(dot(n, r, r));
        if (hist && it < hist_cap) hist[it] = rr / fn;
        if (!is_finite(rr)) { rc = ORC_EBREAK; break; }
        if (rr <= rtol * fn) { rc = ORC_OK; break; }
        if (it >= maxit) break;
        prec_apply(m, r, z, work);
        for (int i = 0; i < n; ++i) x[i] = x[i] + z[i];
        ++it;
    }
    if (true_rel) *true_rel = rr / fn;
    if (iters) *iters = it;
    free(r); free(z); free(work);
    return rc;
}

/* Right-preconditioned BiCGStab (Sec. 4.1: the preconditioner is applied
 * twice per iteration).  With rhat = r_0, rho = rhat^T r:
 *   p = r + beta (p - omega v),  beta = (rho_k / rho_{k-1}) (alpha / omega)
 *   y = B p,  v = A y,  alpha = rho_k / rhat^T v,  s = r - alpha v
 *   z = B s,  t = A z,  omega = t^T s / t^T t
 *   x += alpha y + omega z,  r = s - omega t.
 * An iteration that already meets the tolerance after its first half ends
 * there (x += alpha y).  Convergence of the recursive residual is confirmed
 * on the true one; if that is still above the tolerance the iteration starts
 * again from x.  Iterations count passes of the loop (a half pass counts
 * one).  hist receives the recursive relative residual per iteration.
 * Breakdown: rhat^T r is negligible, |rho_k| <= 1e-14 ||rhat|| ||r||
 * (rounding keeps an exact zero from showing), or rhat^T v or t^T t is
 * zero. */
int orc_bicgstab(const orc_prec *m, const double *f, double *x, double rtol, int maxit,
                 int *iters, double *true_rel, double *hist, int hist_cap)
{
    int n = m->n;
    size_t N = (size_t)n;
    double *r = malloc(sizeof(double) * N), *rh = malloc(sizeof(double) * N),
           *p = malloc(sizeof(double) * N), *v = malloc(sizeof(double) * N),
           *y = malloc(sizeof(double) * N), *sv = malloc(sizeof(double) * N),
           *z = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * N),
           *work = malloc(sizeof(double) * PREC_WORK(n, m->nc));
    double fn = sqrt(dot(n, f, f));
    if (fn == 0.0) fn = 1.0;
    int it = 0, rc = ORC_ENOCONV, restart = 1;
    double rho = 1.0, alpha = 1.0, omega = 1.0, rhn = 0.0, rn = 0.0;
    while (it <= maxit) {
        if (restart) {
            spmv(n, m->rp, m->ci, m->a, x, r);
            for (int i = 0; i < n; ++i) r[i] = f[i] - r[i];
            double rr = sqrt(dot(n, r, r));
            if (hist && it < hist_cap) hist[it] = rr / fn;
            if (!is_finite(rr)) { rc = ORC_EBREAK; break; }
            if (rr <= rtol * fn) { rc = ORC_OK; break; }
            if (it >= maxit) break;
            for (int i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = r[i]; v[i] = 0.0; }
            rho = dot(n, rh, r);
            rhn = rr;
            restart = 0;
        } else {
            double rho_new = dot(n, rh, r);
            if (!(fabs(rho_new) > 1e-14 * rhn * rn)) { rc = ORC_EBREAK; break; }
            double beta = (rho_new / rho) * (alpha / omega);
            for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            rho = rho_new;
        }
        prec_apply(m, p, y, work);
        spmv(n, m->rp, m->ci, m->a, y, v);
        double sig = dot(n, rh, v);
        if (sig == 0.0 || !is_finite(sig)) { rc = ORC_EBREAK; break; }
        alpha = rho / sig;
        for (int i = 0; i < n; ++i) sv[i] = r[i] - alpha * v[i];
        ++it;
        double ss = sqrt(dot(n, sv, sv));
        if (ss <= rtol * fn) {
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * y[i];
            if (hist && it < hist_cap) hist[it] = ss / fn;
            restart = 1;
            continue;
        }
        prec_apply(m, sv, z, work);
        spmv(n, m->rp, m->ci, m->a, z, t);
        double tt = dot(n, t, t);
        if (tt == 0.0 || !is_finite(tt)) { rc = ORC_EBREAK; break; }
        omega = dot(n, t, sv) / tt;
        for (int i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * y[i] + omega * z[i];
            r[i] = sv[i] - omega * t[i];
        }
        double rr = sqrt(dot(n, r, r));
        rn = rr;
        if (hist && it < hist_cap) hist[it] = rr / fn;
        if (!is_finite(rr)) { rc = ORC_EBREAK; break; }
        if (rr <= rtol * fn) { restart = 1; continue; }
        if (omega == 0.0) { rc = ORC_EBREAK; break; }
        if (it >= maxit) break;
    }
    spmv(n, m->rp, m->ci, m->a, x, r);
    for (int i = 0; i < n; ++i) r[i] = f[i] - r[i];
    if (true_rel) *true_rel = sqrt(dot(n, r, r)) / fn;
    if (iters) *iters = it;
    free(r); free(rh); free(p); free(v); free(y); free(sv); free(z); free(t); free(work);
    return rc;
}

/* Petrov-Galerkin coarse operator of the MsFV kind (Sec. 2: the rows of R
 * make the coarse problem conserve mass over every coarse block; Alg. 2's
 * Petrov-Galerkin branch): R_ji = 1 when fine row i lies in coarse block j
 * (part[i] = j), else 0, so
 *   Ac[j,l] = sum_{i : part(i) = j} sum_k A_ik P_kl,
 * i ascending and k ascending, with the full, unfiltered A.  Dense,
 * row-major, nc x nc. */
int orc_rap_pg(int n, const int *rp, const int *ci, const double *a, int nc,
               const int *part, const int *prp, const int *pci, const double *pv,
               double *ac)
{
    for (int i = 0; i < n; ++i)
        if (part[i] < 0 || part[i] >= nc) return ORC_EARG;
    memset(ac, 0, sizeof(double) * (size_t)nc * (size_t)nc);
#pragma omp parallel
    {
        double *ap = (double *)calloc((size_t)nc, sizeof(double));
        int *touched = (int *)malloc(sizeof(int) * (size_t)nc);
        char *mark = (char *)calloc((size_t)nc, 1);
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < nc; ++j) {
            double *row = ac + (size_t)j * nc;
            for (int i = 0; i < n; ++i) {
                if (part[i] != j) continue;
                int nt = 0;
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    int k = ci[e];
                    for (int q = prp[k]; q < prp[k + 1]; ++q) {
                        int l = pci[q];
                        double prod = a[e] * pv[q];
                        if (!mark[l]) { mark[l] = 1; touched[nt++] = l; ap[l] = 0.0; }
                        ap[l] = ap[l] + prod;
                    }
                }
                for (int u = 0; u < nt; ++u) {
                    int l = touched[u];
                    row[l] = row[l] + ap[l];
                    mark[l] = 0;
                }
            }
        }
        free(ap); free(touched); free(mark);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Two-point flux approximation on a Cartesian grid (App. B.1 with the
 * flux split eq. (num_flux_split)).  Cells are numbered x + nx (y + ny z);
 * dim = 2 uses nz = 1 and unit depth.  k = exp(logk).  For the face between
 * neighbouring cells K, L in axis d, with area a_d and spacing h_d, each
 * half-cell contributes t = 2 k a_d / h_d and the face transmissibility is
 * the series (harmonic) combination T = t_K t_L / (t_K + t_L).  A domain
 * face with Dirichlet value g (bc[2d] for the low side, bc[2d+1] for the
 * high side; NaN = no flow) adds T_b = 2 k_K a_d / h_d to A_KK and T_b g
 * to f_K.  Columns are sorted; the diagonal is always present.
 * rp must hold n+1 ints and ci/val up to 7n entries. */
int orc_tpfa(int dim, int nx, int ny, int nz, double hx, double hy, double hz,
             const double *logk, const double *bc, int *rp, int *ci,
             double *val, double *rhs)
{
    if (dim == 2) nz = 1;
    if (dim != 2 && dim != 3) return ORC_EARG;
    int n = nx * ny * nz;
    int nd[3] = {nx, ny, nz};
    double h[3] = {hx, hy, dim == 3 ? hz : 1.0};
    double area[3] = {h[1] * h[2], h[0] * h[2], h[0] * h[1]};
    if (dim == 2) { area[0] = h[1]; area[1] = h[0]; }
    int64_t e = 0;
    rp[0] = 0;
    for (int c = 0; c < n; ++c) {
        int xyz[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
        int stride[3] = {1, nx, nx * ny};
        double kk = exp(logk[c]);
        double diag = 0.0, f = 0.0;
        /* neighbours in ascending index: z-, y-, x-, self, x+, y+, z+ */
        int order[7][2] = {{2, -1}, {1, -1}, {0, -1}, {-1, 0}, {0, 1}, {1, 1}, {2, 1}};
        int64_t diag_pos = -1;
        for (int t = 0; t < 7; ++t) {
            int d = order[t][0], s = order[t][1];
            if (d < 0) { diag_pos = e; ci[e] = c; val[e] = 0.0; ++e; continue; }
            if (d >= dim) continue;
            int nb = xyz[d] + s;
            if (nb < 0 || nb >= nd[d]) {
                double g = bc[2 * d + (s > 0 ? 1 : 0)];
                if (g == g) {
                    double tb = 2.0 * kk * area[d] / h[d];
                    diag = diag + tb;
                    f = f + tb * g;
                }
                continue;
            }
            int L = c + s * stride[d];
            double kl = exp(logk[L]);
            double tK = 2.0 * kk * area[d] / h[d], tL = 2.0 * kl * area[d] / h[d];
            double T = tK * tL / (tK + tL);
            diag = diag + T;
            ci[e] = L;
            val[e] = -T;
            ++e;
        }
        val[diag_pos] = diag;
        rhs[c] = f;
        rp[c + 1] = (int)e;
    }
    return ORC_OK;
}

/* Gradient of an objective J(p) with respect to log k through the TPFA
 * system A(k) p = f(k), given the adjoint lambda solving A^T lambda = dJ/dp:
 *   dJ/dlog k_K = -lambda^T (dA/dlog k_K p - df/dlog k_K).
 * With T = t_K t_L / (t_K + t_L) and t = 2 k a/h one has
 * dT/dlog k_K = T t_L/(t_K + t_L) = T k_L/(k_K + k_L), and a Dirichlet face
 * has dT_b/dlog k_K = T_b, so
 *   g_K = -[ sum over faces (K,L) of T k_L/(k_K+k_L) (p_K - p_L)(lam_K - lam_L)
 *            + sum over Dirichlet faces of K of T_b (p_K - g_b) lam_K ].
 * This derivation is not in the paper (which has no adjoint); it follows
 * from the TPFA transmissibilities above. */
int orc_tpfa_grad(int dim, int nx, int ny, int nz, double hx, double hy, double hz,
                  const double *logk, const double *bc, const double *p,
                  const double *lam, double *grad)
{
    if (dim == 2) nz = 1;
    int n = nx * ny * nz;
    int nd[3] = {nx, ny, nz};
    double h[3] = {hx, hy, dim == 3 ? hz : 1.0};
    double area[3] = {h[1] * h[2], h[0] * h[2], h[0] * h[1]};
    if (dim == 2) { area[0] = h[1]; area[1] = h[0]; }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < n; ++c) {
        int xyz[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
        int stride[3] = {1, nx, nx * ny};
        double kk = exp(logk[c]);
        double s = 0.0;
        for (int d = 0; d < dim; ++d)
            for (int sg = -1; sg <= 1; sg += 2) {
                int nb = xyz[d] + sg;
                if (nb < 0 || nb >= nd[d]) {
                    double g = bc[2 * d + (sg > 0 ? 1 : 0)];
                    if (g == g) {
                        double tb = 2.0 * kk * area[d] / h[d];
                        s = s + tb * (p[c] - g) * lam[c];
                    }
                    continue;
                }
                int L = c + sg * stride[d];
                double kl = exp(logk[L]);
                double tK = 2.0 * kk * area[d] / h[d], tL = 2.0 * kl * area[d] / h[d];
                double T = tK * tL / (tK + tL);
                double dT = T * kl / (kk + kl);
                s = s + dT * (p[c] - p[L]) * (lam[c] - lam[L]);
            }
        grad[c] = -s;
    }
    return ORC_OK;
}

/* Gradient of an objective J(u) with respect to log E through the Q1
 * elasticity system A(E) u = f with E-independent loads (App. "Linear
 * elastostatics: Galerkin finite element formulation"): A = sum_e E_e K_e,
 * so dJ/dlog E_e = -lambda^T (E_e K_e) u, with lambda solving A^T lambda =
 * dJ/du.  Dofs fixed by symmetric diagonalisation are zero in u and
 * lambda (homogeneous data, an objective on free dofs) and are skipped.
 *
 * The element matrix is integrated here directly from the bilinear form
 *   a(v, u) = int lambda_L div v div u + 2 G eps(v) : eps(u),
 * whose entry for v = N_a e_l, u = N_b e_m reads
 *   lambda_L dN_a/dx_l dN_b/dx_m + G dN_a/dx_m dN_b/dx_l
 *   + G delta_lm grad N_a . grad N_b,
 * with 2-point Gauss quadrature per axis on the dim-cube of sizes h.  Nodes
 * of element (ex, ey, ez) are (ex + bx, ey + by, ez + bz), local index
 * bx + 2 by + 4 bz; dof = dim * node + l.  (Not in the paper, which has no
 * adjoint.) */
int orc_q1_grad(int dim, const int *elems, const double *h, double nu, const double *logE,
                const unsigned char *fixed, const double *u, const double *lam, double *grad)
{
    if (dim != 2 && dim != 3) return ORC_EARG;
    int ne[3] = {1, 1, 1}, nn[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) {
        ne[k] = elems[k];
        nn[k] = elems[k] + 1;
    }
    int nloc = 1 << dim, nd = dim * nloc;
    double lamL = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), G = 1.0 / (2.0 * (1.0 + nu));
    double K[24 * 24];
    memset(K, 0, sizeof(K));
    double gpt = 1.0 / sqrt(3.0);
    double wdet = 1.0;
    for (int k = 0; k < dim; ++k) wdet = wdet * (h[k] / 2.0);
    for (int p = 0; p < nloc; ++p) {
        double xi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) xi[k] = (p >> k & 1) ? gpt : -gpt;
        double dN[8][3];
        for (int a = 0; a < nloc; ++a)
            for (int k = 0; k < dim; ++k) {
                /* d/dx_k of prod_m (1 + s_m xi_m)/2, with dxi/dx = 2/h */
                double v = 1.0;
                for (int m = 0; m < dim; ++m) {
                    double sm = (a >> m & 1) ? 1.0 : -1.0;
                    v = v * (m == k ? sm / 2.0 : (1.0 + sm * xi[m]) / 2.0);
                }
                dN[a][k] = v * 2.0 / h[k];
            }
        for (int a = 0; a < nloc; ++a)
            for (int l = 0; l < dim; ++l)
                for (int b = 0; b < nloc; ++b)
                    for (int m = 0; m < dim; ++m) {
                        double gg = 0.0;
                        for (int k = 0; k < dim; ++k) gg = gg + dN[a][k] * dN[b][k];
                        double v = lamL * dN[a][l] * dN[b][m] + G * dN[a][m] * dN[b][l];
                        if (l == m) v = v + G * gg;
                        K[(dim * a + l) * nd + dim * b + m] += v * wdet;
                    }
    }
    int nel = ne[0] * ne[1] * ne[2];
#pragma omp parallel for schedule(static)
    for (int e = 0; e < nel; ++e) {
        int o[3] = {e % ne[0], (e / ne[0]) % ne[1], e / (ne[0] * ne[1])};
        double ue[24], le[24];
        for (int a = 0; a < nloc; ++a) {
            int node = (o[0] + (a & 1)) + nn[0] * ((o[1] + (a >> 1 & 1)) + nn[1] * (o[2] + (a >> 2 & 1)));
            for (int l = 0; l < dim; ++l) {
                int dof = dim * node + l;
                int f = fixed ? fixed[dof] != 0 : 0;
                ue[dim * a + l] = f ? 0.0 : u[dof];
                le[dim * a + l] = f ? 0.0 : lam[dof];
            }
        }
        double s = 0.0;
        for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nd; ++j) s = s + le[i] * K[i * nd + j] * ue[j];
        grad[e] = -exp(logE[e]) * s;
    }
    return ORC_OK;
}
