"""Pins of the oracle's further solver options (the paper's solver matrix):
sweep orders, symmetric Gauss-Seidel, IC(0), the stand-alone (Richardson)
iteration, BiCGStab and the Petrov-Galerkin (MsFV) restriction.

Every check compares the oracle with something other than itself: dense
linear algebra (the closed form of the smoother's operator, dense triangular
solves, numpy's Cholesky and direct solves), the number of colours that
first-fit colouring gives on structured stencils, and properties the paper
states (the coarse problem of the MsFV restriction conserves mass block by
block; an exact preconditioner makes the stand-alone iteration exact)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

SGS, IC0, ILU0 = 4, 5, 3


def csr(rp, ci, a, n=None):
    n = n or rp.size - 1
    return sp.csr_matrix((a, ci, rp), shape=(n, n))


def stencil(dims, offsets, seed=0, spd=True):
    """A random matrix on a structured stencil: symmetric positive definite
    (weighted graph Laplacian plus a positive shift) or, with spd=False,
    with non-symmetric couplings of mixed sign."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    idx = np.arange(n).reshape(tuple(reversed(dims)))
    rows, cols, vals = [], [], []
    nd = len(dims)
    for off in offsets:
        o = tuple(reversed(off))
        src = idx[tuple(slice(max(0, -d), s - max(0, d)) for d, s in zip(o, idx.shape))]
        dst = idx[tuple(slice(max(0, d), s - max(0, -d)) for d, s in zip(o, idx.shape))]
        w = rng.uniform(0.5, 1.5, src.size)
        rows += [src.ravel(), dst.ravel()]
        cols += [dst.ravel(), src.ravel()]
        if spd:
            vals += [-w, -w]
        else:
            vals += [-w, rng.uniform(-1.0, 0.3, src.size)]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    d = np.abs(A).sum(axis=1).A1 + rng.uniform(0.05, 0.5, n)
    A = (A + sp.diags(d)).tocsr()
    A.sort_indices()
    return A


FIVE = [(1, 0), (0, 1)]
NINE = [(1, 0), (0, 1), (1, 1), (1, -1)]
SEVEN = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
TWENTYSEVEN = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
               if (a, b, c) > (0, 0, 0)]


# --------------------------------------------------------------------------
# colouring and orders
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims,offs,ncol", [((9, 7), FIVE, 2), ((9, 7), NINE, 4),
                                            ((6, 5, 4), SEVEN, 2), ((6, 5, 4), TWENTYSEVEN, 8)])
def test_first_fit_colouring_of_stencils(dims, offs, ncol):
    # first fit in natural order colours a 5- or 7-point grid red-black, a
    # 9-point grid by the parities (x mod 2, y mod 2), a 27-point grid by
    # (x, y, z) mod 2
    A = stencil(dims, offs)
    col, nc = oracle.color(A.indptr, A.indices)
    assert nc == ncol
    coo = A.tocoo()
    off = coo.row != coo.col
    assert np.all(col[coo.row[off]] != col[coo.col[off]])
    # rows share a colour exactly when they share the parity class
    x = np.indices(tuple(reversed(dims))).reshape(len(dims), -1)[::-1] % 2
    if ncol == 2:
        key = x.sum(axis=0) % 2
    else:
        key = sum(x[d] << d for d in range(len(dims)))
    for c in range(ncol):
        assert len(set(key[col == c])) == 1


def test_colouring_of_a_nonsymmetric_pattern_uses_both_triangles():
    # j is a neighbour of i when A_ij or A_ji is stored
    A = sp.csr_matrix(np.array([[2.0, 0, 0, 0], [0, 2, 0, 0], [1, 1, 2, 0], [0, 0, 1, 2]]))
    A.sort_indices()
    col, nc = oracle.color(A.indptr, A.indices)
    assert list(col) == [0, 0, 1, 0] and nc == 2


def test_permutation_is_symmetric_reordering():
    A = stencil((7, 6), NINE, seed=2, spd=False)
    order = oracle.sweep_order(A.indptr, A.indices, "multicolor")
    assert sorted(order) == list(range(42))
    brp, bci, ba = oracle.permute(A.indptr, A.indices, A.data, order)
    np.testing.assert_array_equal(csr(brp, bci, ba).toarray(), A.toarray()[order][:, order])
    assert all(np.all(np.diff(bci[brp[k]:brp[k + 1]]) > 0) for k in range(42))


# --------------------------------------------------------------------------
# smoothers in a given order against dense algebra
# --------------------------------------------------------------------------

def _smoother_only(A):
    n = A.shape[0]
    m = oracle.Msrsb(A.indptr, A.indices, A.data)
    part = np.zeros(n, np.int32)
    m.set_coarse(1, part, np.arange(n + 1, dtype=np.int32), part, np.ones(n, np.uint8))
    m.setup_basis(kmax=1)
    m.build_coarse()
    return m


def _qmat(order):
    n = order.size
    Q = np.zeros((n, n))
    Q[np.arange(n), order] = 1.0     # (Q x)_k = x[order[k]]
    return Q


@pytest.mark.parametrize("ordering", ["natural", "multicolor"])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_sgs_sweep_is_the_symmetric_gauss_seidel_operator(ordering, sweeps):
    # one SGS sweep is z += M^{-1} (v - A z) with
    # M = (D + L) D^{-1} (D + U) of the reordered matrix Q A Q^T
    A = stencil((8, 7), NINE, seed=3, spd=False)
    n = 56
    order = oracle.sweep_order(A.indptr, A.indices, ordering)
    Q = _qmat(order)
    B = Q @ A.toarray() @ Q.T
    D = np.diag(np.diag(B))
    M = (np.tril(B, -1) + D) @ np.linalg.inv(D) @ (np.triu(B, 1) + D)
    Minv = Q.T @ np.linalg.inv(M) @ Q
    v = np.random.default_rng(4).standard_normal(n)
    ref = np.zeros(n)
    for _ in range(sweeps):
        ref = ref + Minv @ (v - A.toarray() @ ref)
    z = _smoother_only(A).apply(v, post=(SGS, sweeps), use_ms=False, ordering=ordering)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    if ordering == "multicolor":
        # the order matters: natural order gives another operator
        zn = _smoother_only(A).apply(v, post=(SGS, sweeps), use_ms=False)
        assert np.abs(zn - z).max() > 1e-4 * np.abs(z).max()


def test_ilu0_in_colour_order():
    # ILU(0) of Q A Q^T: (L U)_kl = B_kl on B's pattern, and the sweep applies
    # Q^T (L U)^{-1} Q
    A = stencil((9, 8), NINE, seed=5, spd=False)
    n = 72
    order = oracle.sweep_order(A.indptr, A.indices, "multicolor")
    brp, bci, ba = oracle.permute(A.indptr, A.indices, A.data, order)
    F = csr(brp, bci, oracle.ilu0(brp, bci, ba)).toarray()
    L, U = np.tril(F, -1) + np.eye(n), np.triu(F)
    B = csr(brp, bci, ba).toarray()
    mask = B != 0
    np.testing.assert_allclose((L @ U)[mask], B[mask], rtol=1e-13, atol=1e-13)
    Q = _qmat(order)
    v = np.random.default_rng(6).standard_normal(n)
    ref = Q.T @ np.linalg.solve(U, np.linalg.solve(L, Q @ v))
    z = _smoother_only(A).apply(v, post=(ILU0, 1), use_ms=False, ordering="multicolor")
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_ic0_defining_property_and_tridiagonal_cholesky():
    A = stencil((7, 6, 4), SEVEN, seed=7)
    l = oracle.ic0(A.indptr, A.indices, A.data)
    L = csr(A.indptr, A.indices, l).toarray()
    assert np.all(np.triu(L, 1) == 0.0)
    mask = np.tril(A.toarray()) != 0
    np.testing.assert_allclose((L @ L.T)[mask], A.toarray()[mask], rtol=1e-13, atol=1e-13)
    # no fill on a tridiagonal matrix: IC(0) is the Cholesky factor
    T = stencil((40,), [(1,)], seed=8)
    lt = oracle.ic0(T.indptr, T.indices, T.data)
    np.testing.assert_allclose(csr(T.indptr, T.indices, lt).toarray(),
                               np.linalg.cholesky(T.toarray()), rtol=1e-13, atol=1e-14)


def test_ic0_breakdown_is_reported():
    A = sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.ic0(A.indptr, A.indices, A.data)
    assert e.value.code == oracle.E_SING


@pytest.mark.parametrize("ordering", ["natural", "multicolor"])
def test_ic0_sweep(ordering):
    # z += Q^T (L L^T)^{-1} Q (v - A z), and L L^T equals the ILU(0) product
    # of the same (symmetric) matrix up to rounding
    A = stencil((6, 5, 4), SEVEN, seed=9)
    n = 120
    order = oracle.sweep_order(A.indptr, A.indices, ordering)
    brp, bci, ba = oracle.permute(A.indptr, A.indices, A.data, order)
    L = csr(brp, bci, oracle.ic0(brp, bci, ba)).toarray()
    Q = _qmat(order)
    v = np.random.default_rng(10).standard_normal(n)
    Ad = A.toarray()
    ref = Q.T @ np.linalg.solve(L @ L.T, Q @ v)
    ref = ref + Q.T @ np.linalg.solve(L @ L.T, Q @ (v - Ad @ ref))
    m = _smoother_only(A)
    z = m.apply(v, pre=(IC0, 1), post=(IC0, 1), use_ms=False, ordering=ordering)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    zi = m.apply(v, pre=(ILU0, 1), post=(ILU0, 1), use_ms=False, ordering=ordering)
    np.testing.assert_allclose(zi, z, rtol=1e-11, atol=1e-11 * np.abs(z).max())


# --------------------------------------------------------------------------
# Krylov variants and the stand-alone iteration
# --------------------------------------------------------------------------

def tpfa_case(dims, block, sigma=1.0, seed=0):
    rng = np.random.default_rng(seed)
    logk = sigma * rng.standard_normal(int(np.prod(dims)))
    h = tuple(1.0 / d for d in dims)
    bc = np.array([1.0, 0.0] + [np.nan] * 4)
    rp, ci, a, f = oracle.tpfa(dims, h, logk, bc)
    sup = synth.cell_supports(dims, block)
    m = oracle.Msrsb(rp, ci, a)
    m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    return m, csr(rp, ci, a), f, sup


def test_richardson_iterates_are_the_stationary_iteration():
    # x_k = x_{k-1} + B (f - A x_{k-1}); with B from the oracle's own apply,
    # the residual history is that of (I - A B)^k f
    m, A, f, sup = tpfa_case((16, 12), 4, seed=1)
    m.setup_basis(kmax=30)
    m.build_coarse()
    n = 192
    Bm = np.column_stack([m.apply(e, post=(SGS, 1)) for e in np.eye(n)])
    r = m.solve(f, krylov="richardson", post=(SGS, 1), rtol=1e-10, maxit=200, hist_cap=201)
    assert r["status"] == 0
    E = np.eye(n) - A.toarray() @ Bm
    res = [np.linalg.norm(np.linalg.matrix_power(E, k) @ f) / np.linalg.norm(f)
           for k in range(min(8, r["iters"]))]
    np.testing.assert_allclose(r["hist"][:len(res)], res, rtol=1e-9)
    np.testing.assert_allclose(r["x"], np.linalg.solve(A.toarray(), f), rtol=1e-8,
                               atol=1e-8 * np.abs(f).max())


def test_richardson_with_exact_preconditioner_is_one_step():
    # one cell per block: P = I, A_c = A and B = A^{-1}
    m, A, f, sup = tpfa_case((6, 5), 1, seed=2)
    m.setup_basis(kmax=2)
    m.build_coarse()
    r = m.solve(f, krylov="richardson", rtol=1e-12, maxit=5)
    assert r["status"] == 0 and r["iters"] == 1


@pytest.mark.parametrize("post", [(ILU0, 1), (SGS, 1), (1, 2)])
def test_bicgstab_matches_dense_solve(post):
    # a non-symmetric operator: TPFA plus a one-sided advection-like coupling
    m0, A, f, sup = tpfa_case((20, 16), 4, seed=3)
    A = A.tolil()
    rng = np.random.default_rng(1)
    for i in range(319):
        if (i + 1) % 20:
            A[i, i + 1] += -0.2 * A[i, i] * rng.uniform(0.0, 0.3)
    A = A.tocsr()
    A.sort_indices()
    m = oracle.Msrsb(A.indptr, A.indices, A.data)
    m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    m.setup_basis(kmax=50)
    m.build_coarse()
    r = m.solve(f, krylov="bicgstab", post=post, rtol=1e-12, maxit=300)
    assert r["status"] == 0 and r["true_rel"] <= 1e-12
    ref = np.linalg.solve(A.toarray(), f)
    np.testing.assert_allclose(r["x"], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_bicgstab_with_exact_preconditioner_ends_after_half_a_step():
    m, A, f, sup = tpfa_case((6, 5), 1, seed=4)
    m.setup_basis(kmax=2)
    m.build_coarse()
    r = m.solve(f, krylov="bicgstab", rtol=1e-12, maxit=5)
    assert r["status"] == 0 and r["iters"] == 1 and r["true_rel"] <= 1e-12


# --------------------------------------------------------------------------
# Petrov-Galerkin (MsFV) restriction
# --------------------------------------------------------------------------

def test_msfv_coarse_operator_is_dense_product():
    m, A, f, sup = tpfa_case((16, 12), 4, seed=5)
    m.setup_basis(kmax=40)
    ac = m.build_coarse(restriction="msfv")
    P = sp.csr_matrix((m.pv, sup["pci"], sup["prp"]), shape=(192, sup["nc"])).toarray()
    R = np.eye(sup["nc"])[sup["part"]].T
    np.testing.assert_allclose(ac, R @ A.toarray() @ P, rtol=1e-14, atol=1e-14 * np.abs(ac).max())
    # the block-indicator restriction gives a non-symmetric coarse operator
    assert np.abs(ac - ac.T).max() > 1e-6 * np.abs(ac).max()


def test_msfv_coarse_solution_conserves_mass_per_block():
    # Sec. 2: with the MsFV restriction the coarse problem is conservative:
    # the fine residual of u = P A_c^{-1} R f sums to zero over every block
    m, A, f, sup = tpfa_case((20, 20), 5, seed=6)
    m.setup_basis(kmax=60)
    Ad = A.toarray()
    for restr, conservative in (("msfv", True), ("galerkin", False)):
        m.build_coarse(restriction=restr)
        u = m.apply(f)                      # Alg. 3 alone: P A_c^{-1} R f
        res = f - Ad @ u
        blk = np.bincount(sup["part"], weights=res, minlength=sup["nc"])
        scale = np.abs(f).sum()
        if conservative:
            assert np.abs(blk).max() <= 1e-12 * scale
        else:
            assert np.abs(blk).max() > 1e-6 * scale


def test_msfv_solves_with_gmres_and_richardson():
    m, A, f, sup = tpfa_case((24, 24), 6, seed=7)
    m.setup_basis(kmax=80)
    m.build_coarse(restriction="msfv")
    ref = np.linalg.solve(A.toarray(), f)
    for kry in ("gmres", "richardson", "bicgstab"):
        r = m.solve(f, krylov=kry, post=(ILU0, 1), rtol=1e-11, maxit=400)
        assert r["status"] == 0, kry
        np.testing.assert_allclose(r["x"], ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())
    with pytest.raises(oracle.OracleError):
        m.solve(f, transpose=True, post=(1, 1))


def test_bicgstab_breakdown_with_point_source():
    # with f = e_0 the shadow residual is e_0; row 0 comes first in either
    # order, row 0 of L U is row 0 of A, so every ILU(0) sweep leaves the
    # residual zero there: rhat^T r vanishes at the second step
    A = stencil((12, 10), NINE, seed=12, spd=False)
    n = 120
    f = np.zeros(n)
    f[0] = 1.0
    m = _smoother_only(A)
    for ordering in ("natural", "multicolor"):
        z = m.apply(f, post=(ILU0, 1), use_ms=False, ordering=ordering)
        assert abs((f - A @ z)[0]) <= 1e-15
        r = m.solve(f, krylov="bicgstab", post=(ILU0, 1), use_ms=False, ordering=ordering,
                    rtol=1e-10, maxit=50)
        assert r["status"] == oracle.E_BREAK and r["iters"] == 1
