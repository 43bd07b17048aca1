"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (linear hats, linear pressure), invariants the paper states (row sums
of P, range of P, M-matrices unchanged by the filter, SPD coarse operator),
special cases that reduce to a library routine (dense products, dense LU,
dense direct solves) and finite differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def csr(rp, ci, a, n=None):
    n = n or rp.size - 1
    return sp.csr_matrix((a, ci, rp), shape=(n, n))


def pmat(sup, pv, n):
    return sp.csr_matrix((pv, sup["pci"], sup["prp"]), shape=(n, sup["nc"]))


def tpfa_case(dims, block, sigma=1.0, seed=0, bc=None, h=None):
    rng = np.random.default_rng(seed)
    logk = sigma * rng.standard_normal(int(np.prod(dims)))
    h = h or tuple(1.0 / d for d in dims)
    if bc is None:
        bc = np.array([1.0, 0.0] + [np.nan] * 4)
    rp, ci, a, f = oracle.tpfa(dims, h, logk, bc)
    sup = synth.cell_supports(dims, block)
    return dict(rp=rp, ci=ci, a=a, f=f, sup=sup, logk=logk, h=h, bc=bc, dims=dims)


def random_non_m(n, seed, bs=1, density=0.3):
    """Random matrix with a positive diagonal and mixed-sign off-diagonals."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    M.data = rng.uniform(-1.0, 0.4, M.data.size)
    M = M + sp.diags(rng.uniform(1, 3, n) + np.abs(M).sum(axis=1).A1)
    M = M.tocsr()
    M.sort_indices()
    return M


# --------------------------------------------------------------------------
# filter and Jacobi operator: eq. (negoffdiag), eq. (Dhat_zero_rowsum)
# --------------------------------------------------------------------------

def test_filter_leaves_m_matrix_unchanged():
    # Sec. 3.1: the filter does not affect an M-matrix (TPFA gives one)
    c = tpfa_case((12, 9, 5), 4, sigma=1.5, seed=3)
    j1, d1 = oracle.filter_jacobi(c["rp"], c["ci"], c["a"], filt=True)
    j0, d0 = oracle.filter_jacobi(c["rp"], c["ci"], c["a"], filt=False)
    assert np.array_equal(j1, j0) and np.array_equal(d1, d0)


@pytest.mark.parametrize("bs", [1, 2, 3])
def test_filtered_operator_invariants(bs):
    # Sec. 3.1: Ghat has zero row sums and non-positive off-diagonals, so
    # J = I - omega Dhat^{-1} Ghat is non-negative with unit row sums.
    n = 60
    M = random_non_m(n, seed=10 + bs)
    omega = 2.0 / 3.0
    jv, dh = oracle.filter_jacobi(M.indptr, M.indices, M.data, bs=bs, filt=True, omega=omega)
    J = csr(M.indptr, M.indices, jv).toarray()
    A = M.toarray()
    I = np.eye(n)
    rows = np.arange(n)
    same = (rows[:, None] % bs) == (rows[None, :] % bs)
    active = dh > 0
    # reconstruct Ghat = Dhat (I - J) / omega on the active rows
    G = (dh[:, None] * (I - J)) / omega
    off = ~np.eye(n, dtype=bool)
    assert np.all(G[active][off[active]] <= 1e-15)
    np.testing.assert_allclose(G[active].sum(axis=1), 0.0, atol=1e-13 * dh.max())
    # off-diagonals of Ghat are min(A, 0) restricted to the same component
    expect = np.where(same & off & (A != 0), np.minimum(A, 0.0), 0.0)
    np.testing.assert_allclose(G[active][off[active]], expect[active][off[active]],
                               rtol=1e-13, atol=1e-15)
    assert np.all(J >= 0.0)
    np.testing.assert_allclose(J.sum(axis=1), 1.0, rtol=0, atol=4e-16 * 8)
    # cross-component couplings never enter J
    assert np.all(J[~same] == 0.0)


def test_frozen_rows():
    # a row whose off-diagonals are all positive has Dhat = 0 once filtered
    n = 5
    A = np.diag([2.0, 2, 2, 2, 2])
    A[2, 1] = A[2, 3] = 0.5
    A[0, 1] = A[1, 0] = -1.0
    M = sp.csr_matrix(A)
    M.sort_indices()
    jv, dh = oracle.filter_jacobi(M.indptr, M.indices, M.data)
    J = csr(M.indptr, M.indices, jv).toarray()
    assert dh[2] == 0.0
    np.testing.assert_array_equal(J[2], np.eye(n)[2])


# --------------------------------------------------------------------------
# initial basis and one smoothing step against dense linear algebra
# --------------------------------------------------------------------------

def test_initial_basis_is_block_indicator():
    c = tpfa_case((16, 12), 4)
    sup = c["sup"]
    n = 16 * 12
    P = pmat(sup, oracle.init_basis(sup["prp"], sup["pci"], sup["part"]), n).toarray()
    np.testing.assert_array_equal(P, np.eye(sup["nc"])[sup["part"]])


def test_smoothing_step_matches_dense_masked_product():
    c = tpfa_case((20, 12), 4, sigma=2.0, seed=5)
    sup = c["sup"]
    n = 240
    jv, _ = oracle.filter_jacobi(c["rp"], c["ci"], c["a"])
    rng = np.random.default_rng(1)
    # a generic P on the pattern (not a fixed point) to exercise every product
    pv = rng.uniform(0.1, 1.0, sup["pci"].size)
    out, e = oracle.smooth_step(c["rp"], c["ci"], jv, sup["prp"], sup["pci"], pv,
                                sup["interior"])
    J = csr(c["rp"], c["ci"], jv).toarray()
    P = pmat(sup, pv, n).toarray()
    mask = pmat(sup, np.ones_like(pv), n).toarray() > 0
    T = np.where(mask, J @ P, 0.0)
    expect = T / T.sum(axis=1, keepdims=True)
    np.testing.assert_allclose(pmat(sup, out, n).toarray(), expect, rtol=1e-14, atol=1e-15)
    delta = np.where(mask, T - P, 0.0)
    np.testing.assert_allclose(e, np.abs(delta[sup["interior"] > 0]).max(), rtol=1e-14)


# --------------------------------------------------------------------------
# closed forms: the basis of a homogeneous Cartesian problem converges to
# (tensor-product) linear hats (stated for Q1 in Sec. 4; it holds for any
# reflection-symmetric zero-row-sum stencil)
# --------------------------------------------------------------------------

def hat_1d(N, b):
    m = -(-N // b)
    nodes = np.minimum(np.arange(m) * b + b // 2, N - 1)
    x = np.arange(N)
    H = np.zeros((N, m))
    for a in range(m):
        lo = nodes[a - 1] if a > 0 else None
        hi = nodes[a + 1] if a + 1 < m else None
        for xi in x:
            if xi == nodes[a]:
                H[xi, a] = 1.0
            elif xi < nodes[a]:
                H[xi, a] = 1.0 if lo is None else max(0.0, (xi - lo) / (nodes[a] - lo))
            else:
                H[xi, a] = 1.0 if hi is None else max(0.0, (hi - xi) / (hi - nodes[a]))
    return H


def converge_basis(c, tol=1e-14, kmax=20000):
    sup = c["sup"]
    jv, _ = oracle.filter_jacobi(c["rp"], c["ci"], c["a"])
    p0 = oracle.init_basis(sup["prp"], sup["pci"], sup["part"])
    pv, it, e, _ = oracle.basis(c["rp"], c["ci"], jv, sup["prp"], sup["pci"], p0,
                                sup["interior"], kmax=kmax, tol=tol, nit=10)
    assert e <= tol, (it, e)
    return pv


@pytest.mark.parametrize("N,b", [(16, 4), (24, 8), (20, 5)])
def test_hats_1d(N, b):
    c = tpfa_case((N, 1), b, sigma=0.0)
    c["sup"] = synth.cell_supports((N,), b)
    pv = converge_basis(c)
    P = pmat(c["sup"], pv, N).toarray()
    np.testing.assert_allclose(P, hat_1d(N, b), atol=1e-11)


@pytest.mark.parametrize("dims,block,h", [((16, 12), (4, 4), None),
                                          ((16, 12), (4, 4), (1.0, 7.0)),
                                          ((12, 8, 8), (4, 4, 4), None)])
def test_hats_tensor_product(dims, block, h):
    c = tpfa_case(dims, block, sigma=0.0, h=h)
    c["sup"] = synth.cell_supports(dims, block)
    pv = converge_basis(c)
    n = int(np.prod(dims))
    P = pmat(c["sup"], pv, n).toarray()
    H = hat_1d(dims[0], block[0])
    for d in range(1, len(dims)):
        H = np.kron(hat_1d(dims[d], block[d]), H)
    np.testing.assert_allclose(P, H, atol=1e-10)


def test_partition_of_unity_and_range():
    # Alg. 1 renormalisation: rows sum to one; with the filter P in [0, 1]
    cfg = synth.make_config("c1")
    rp, ci, a, f = oracle.tpfa(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"])
    sup = cfg["supports"]
    jv, _ = oracle.filter_jacobi(rp, ci, a)
    p0 = oracle.init_basis(sup["prp"], sup["pci"], sup["part"])
    pv, it, e, hist = oracle.basis(rp, ci, jv, sup["prp"], sup["pci"], p0, sup["interior"],
                                   kmax=100)
    assert it == 100 and np.all(hist >= 0)
    rs = np.add.reduceat(pv, sup["prp"][:-1])
    assert np.max(np.abs(rs - 1.0)) <= 4 * np.finfo(float).eps
    assert pv.min() >= 0.0 and pv.max() <= 1.0


def test_eit_decreases_on_m_matrix():
    cfg = synth.make_config("c1")
    rp, ci, a, f = oracle.tpfa(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"])
    sup = cfg["supports"]
    jv, _ = oracle.filter_jacobi(rp, ci, a)
    p0 = oracle.init_basis(sup["prp"], sup["pci"], sup["part"])
    _, it, e, hist = oracle.basis(rp, ci, jv, sup["prp"], sup["pci"], p0, sup["interior"],
                                  kmax=400, nit=50)
    checked = hist[hist >= 0]
    assert checked.size == 8 and checked[-1] < 1e-3 * checked[0]


# --------------------------------------------------------------------------
# coarse operator (eq. (lin_system_coarse)), LU, ILU(0)
# --------------------------------------------------------------------------

def _basis_for(c, kmax=30):
    sup = c["sup"]
    jv, _ = oracle.filter_jacobi(c["rp"], c["ci"], c["a"])
    p0 = oracle.init_basis(sup["prp"], sup["pci"], sup["part"])
    return oracle.basis(c["rp"], c["ci"], jv, sup["prp"], sup["pci"], p0, sup["interior"],
                        kmax=kmax)[0]


@pytest.mark.parametrize("dims,block", [((20, 16), 4), ((8, 12, 8), 4)])
def test_rap_matches_dense_product(dims, block):
    c = tpfa_case(dims, block, sigma=1.0, seed=2)
    pv = _basis_for(c)
    sup = c["sup"]
    n = int(np.prod(dims))
    ac = oracle.rap(c["rp"], c["ci"], c["a"], sup["nc"], sup["prp"], sup["pci"], pv)
    A = csr(c["rp"], c["ci"], c["a"]).toarray()
    P = pmat(sup, pv, n).toarray()
    ref = P.T @ A @ P
    np.testing.assert_allclose(ac, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    # symmetric A -> symmetric, positive definite A_c (Sec. 2)
    np.testing.assert_allclose(ac, ac.T, rtol=0, atol=1e-14 * np.abs(ref).max())
    assert np.linalg.eigvalsh(0.5 * (ac + ac.T)).min() > 0
    # A_c 1 = P^T (A 1) because P 1_c = 1_f
    np.testing.assert_allclose(ac.sum(axis=1), P.T @ (A.sum(axis=1)), rtol=1e-12,
                               atol=1e-13 * np.abs(ref).max())
    # coarse stencil: 9-point in 2D, 27-point in 3D
    nnz_row = (ac != 0).sum(axis=1)
    assert nnz_row.max() == np.prod([min(3, m) for m in sup["coarse_dims"]])


def test_rap_nonsymmetric_matches_dense():
    M = random_non_m(80, seed=4, density=0.08)
    sup = synth.cell_supports((80,), 8)
    pv = np.random.default_rng(0).uniform(0, 1, sup["pci"].size)
    ac = oracle.rap(M.indptr, M.indices, M.data, sup["nc"], sup["prp"], sup["pci"], pv)
    P = pmat(sup, pv, 80).toarray()
    ref = P.T @ M.toarray() @ P
    np.testing.assert_allclose(ac, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (40, 2), (120, 3)])
def test_lu_matches_numpy_solve(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A[0, 0] = 0.0 if n > 1 else A[0, 0]  # forces a row swap at the first step
    b = rng.standard_normal(n)
    lu, piv = oracle.lu(A)
    x = oracle.lu_solve(lu, piv, b)
    ref = np.linalg.solve(A, b)
    np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    xt = oracle.lu_solve(lu, piv, b, trans=True)
    np.testing.assert_allclose(xt, np.linalg.solve(A.T, b), rtol=1e-11,
                               atol=1e-12 * np.abs(ref).max())


def test_lu_pivot_choice_and_singular():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    lu, piv = oracle.lu(A)
    assert list(piv) == [1, 1]
    with pytest.raises(oracle.OracleError) as ei:
        oracle.lu(np.array([[1.0, 2.0], [2.0, 4.0]]))
    assert ei.value.code == oracle.E_SING


def test_ilu0_defining_property():
    M = random_non_m(50, seed=7, density=0.1)
    lu = oracle.ilu0(M.indptr, M.indices, M.data)
    F = csr(M.indptr, M.indices, lu).toarray()
    L = np.tril(F, -1) + np.eye(50)
    U = np.triu(F)
    LU = L @ U
    mask = M.toarray() != 0
    np.testing.assert_allclose(LU[mask], M.toarray()[mask], rtol=1e-13, atol=1e-13)


def test_ilu0_exact_on_tridiagonal():
    n = 30
    rng = np.random.default_rng(3)
    A = sp.diags([rng.uniform(-1, 0, n - 1), rng.uniform(3, 4, n), rng.uniform(-1, 0, n - 1)],
                 [-1, 0, 1], format="csr")
    A.sort_indices()
    lu = oracle.ilu0(A.indptr, A.indices, A.data)
    F = csr(A.indptr, A.indices, lu).toarray()
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    np.testing.assert_allclose(L @ U, A.toarray(), atol=1e-14)


# --------------------------------------------------------------------------
# smoother sweeps of Alg. 4 against dense algebra: z += M^{-1} (v - A z)
# --------------------------------------------------------------------------

def _smoother_only(M):
    """The oracle's preconditioner on M with one coarse block (its coarse
    stage is switched off below, so only the sweeps act)."""
    n = M.shape[0]
    m = oracle.Msrsb(M.indptr, M.indices, M.data)
    part = np.zeros(n, np.int32)
    m.set_coarse(1, part, np.arange(n + 1, dtype=np.int32), part, np.ones(n, np.uint8))
    m.setup_basis(kmax=1)
    m.build_coarse()
    return m


def _dense_sweeps(A, v, solve_m, pre, post):
    z = np.zeros_like(v)
    for _ in range(pre + post):
        z = z + solve_m(v - A @ z)
    return z


@pytest.mark.parametrize("pre,post", [(1, 0), (3, 0), (2, 1), (0, 2)])
def test_l1_jacobi_sweeps_match_dense(pre, post):
    # l1-Jacobi: M = diag(sum_j |A_ij|) (Sec. 4.2, two sweeps each side);
    # a non-symmetric operator with negative off-diagonals, so sum_j A_ij,
    # A_ii + sum_{j != i} |A_ij| / 2 and sum_j |A_ij| all differ
    M = random_non_m(70, seed=21, density=0.15)
    A = M.toarray()
    assert np.abs(A - A.T).max() > 0.1
    v = np.random.default_rng(5).standard_normal(70)
    d = np.abs(A).sum(axis=1)
    ref = _dense_sweeps(A, v, lambda r: r / d, pre, post)
    z = _smoother_only(M).apply(v, pre=(2, pre), post=(2, post), use_ms=False)
    np.testing.assert_allclose(z, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("pre,post", [(1, 0), (0, 1), (2, 2)])
def test_ilu0_sweeps_match_dense(pre, post):
    # ILU(0) as the second stage (Sec. 3.2): z += U^{-1} L^{-1} (v - A z) with
    # the factors of the pinned natural-order ILU(0), applied as dense
    # triangular solves (L first); the operator is non-symmetric and not an
    # M-matrix, so U^{-1} L^{-1} and L^{-1} U^{-1} differ
    M = random_non_m(60, seed=23, density=0.12)
    A = M.toarray()
    F = csr(M.indptr, M.indices, oracle.ilu0(M.indptr, M.indices, M.data)).toarray()
    L = np.tril(F, -1) + np.eye(60)
    U = np.triu(F)
    v = np.random.default_rng(6).standard_normal(60)
    ref = _dense_sweeps(A, v, lambda r: np.linalg.solve(U, np.linalg.solve(L, r)), pre, post)
    # (one sweep in the wrong order differs visibly; more sweeps of either
    # order approach A^{-1} v)
    one = np.linalg.solve(U, np.linalg.solve(L, v))
    swapped = np.linalg.solve(L, np.linalg.solve(U, v))
    assert np.abs(swapped - one).max() > 1e-3 * np.abs(one).max()
    z = _smoother_only(M).apply(v, pre=(3, pre), post=(3, post), use_ms=False)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


# --------------------------------------------------------------------------
# solves: Alg. 4 inside PCG / GMRES against dense direct solves
# --------------------------------------------------------------------------

def _setup(c, kmax=100):
    m = oracle.Msrsb(c["rp"], c["ci"], c["a"])
    s = c["sup"]
    m.set_coarse(s["nc"], s["part"], s["prp"], s["pci"], s["interior"])
    m.setup_basis(kmax=kmax)
    m.build_coarse()
    return m


def test_tpfa_homogeneous_linear_pressure():
    # closed form: homogeneous k with p = 1 / 0 on x = 0 / 1 gives p = 1 - x
    for dims in [(16, 8), (8, 6, 4)]:
        c = tpfa_case(dims, 4, sigma=0.0)
        m = _setup(c, kmax=20)
        r = m.solve(c["f"], rtol=1e-13, pre=(2, 2), post=(2, 2))
        x = (np.arange(int(np.prod(dims))) % dims[0] + 0.5) / dims[0]
        np.testing.assert_allclose(r["x"], 1.0 - x, atol=1e-12)


@pytest.mark.parametrize("dims,block,pre,post", [((32, 32), 8, (0, 0), (1, 1)),
                                                 ((32, 32), 8, (1, 1), (1, 1)),
                                                 ((8, 8, 8), 4, (2, 2), (2, 2))])
def test_pcg_matches_dense_solve(dims, block, pre, post):
    c = tpfa_case(dims, block, sigma=1.0, seed=11)
    m = _setup(c)
    r = m.solve(c["f"], rtol=1e-12, pre=pre, post=post)
    assert r["status"] == 0 and r["true_rel"] <= 1e-12
    ref = np.linalg.solve(csr(c["rp"], c["ci"], c["a"]).toarray(), c["f"])
    np.testing.assert_allclose(r["x"], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_pcg_exact_with_identity_prolongation():
    # one cell per block: P = I, A_c = A, the preconditioner is A^{-1}
    c = tpfa_case((6, 5), 1, sigma=1.0, seed=4)
    m = _setup(c, kmax=3)
    P = pmat(c["sup"], m.pv, 30).toarray()
    np.testing.assert_array_equal(P, np.eye(30))
    np.testing.assert_allclose(m.ac, csr(c["rp"], c["ci"], c["a"]).toarray(), rtol=1e-15)
    r = m.solve(c["f"], rtol=1e-10)
    assert r["iters"] == 1 and r["true_rel"] < 1e-12


def test_gmres_ilu0_nonsymmetric_matches_dense():
    # a non-symmetric, non-M operator on a 2D grid pattern
    c = tpfa_case((24, 24), 6, sigma=1.0, seed=6)
    A = csr(c["rp"], c["ci"], c["a"]).tolil()
    rng = np.random.default_rng(0)
    n = 576
    for i in range(n):
        if i + 1 < n and (i + 1) % 24:
            A[i, i + 1] += 0.3 * A[i, i] * rng.uniform(0, 0.2)
    A = A.tocsr()
    A.sort_indices()
    c2 = dict(c, rp=A.indptr, ci=A.indices, a=A.data)
    m = _setup(c2)
    r = m.solve(c["f"], krylov="gmres", restart=30, rtol=1e-12, post=(3, 1))
    assert r["status"] == 0
    ref = np.linalg.solve(A.toarray(), c["f"])
    np.testing.assert_allclose(r["x"], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    rt = m.solve(c["f"], krylov="gmres", restart=30, rtol=1e-12, pre=(1, 1), post=(1, 1),
                 transpose=True)
    reft = np.linalg.solve(A.toarray().T, c["f"])
    np.testing.assert_allclose(rt["x"], reft, rtol=1e-9, atol=1e-9 * np.abs(reft).max())


def test_apply_is_alg4_composition():
    # Alg. 4 with no smoothing reduces to Alg. 3: z = P A_c^{-1} P^T v
    c = tpfa_case((16, 16), 4, sigma=1.0, seed=9)
    m = _setup(c, kmax=20)
    v = np.random.default_rng(2).standard_normal(256)
    z = m.apply(v)
    P = pmat(c["sup"], m.pv, 256).toarray()
    ref = P @ np.linalg.solve(P.T @ csr(c["rp"], c["ci"], c["a"]).toarray() @ P, P.T @ v)
    np.testing.assert_allclose(z, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    # one Jacobi post-sweep: z += D^{-1} (v - A z)
    A = csr(c["rp"], c["ci"], c["a"]).toarray()
    z1 = m.apply(v, post=(1, 1))
    np.testing.assert_allclose(z1, ref + (v - A @ ref) / np.diag(A), rtol=1e-11,
                               atol=1e-12 * np.abs(ref).max())


# --------------------------------------------------------------------------
# adjoint gradient against central finite differences
# --------------------------------------------------------------------------

def test_tpfa_adjoint_gradient_matches_fd():
    dims = (6, 5, 4)
    h = (1 / 6, 1 / 5, 1 / 4)
    rng = np.random.default_rng(12)
    logk = 1.5 * rng.standard_normal(120)
    bc = np.array([1.0, 0.0, np.nan, 0.3, np.nan, np.nan])
    obs = rng.choice(120, 10, replace=False)
    d = rng.uniform(0, 1, 10)

    def objective(lk):
        rp, ci, a, f = oracle.tpfa(dims, h, lk, bc)
        p = np.linalg.solve(csr(rp, ci, a).toarray(), f)
        return np.sum((p[obs] - d) ** 2), p, csr(rp, ci, a).toarray()

    J0, p, A = objective(logk)
    g_p = np.zeros(120)
    g_p[obs] = 2 * (p[obs] - d)
    lam = np.linalg.solve(A.T, g_p)
    g = oracle.tpfa_grad(dims, h, logk, bc, p, lam)
    eps = 1e-5
    fd = np.empty(120)
    for k in range(120):
        e = np.zeros(120)
        e[k] = eps
        fd[k] = (objective(logk + e)[0] - objective(logk - e)[0]) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
