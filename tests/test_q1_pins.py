"""The Q1 elasticity input generator and the SDC filter, pinned on the CPU.

* The unconstrained stiffness annihilates the rigid-body modes (3 in 2D,
  6 in 3D) and is symmetric.
* Patch test: a linear displacement field leaves zero residual at every
  node off the boundary (homogeneous modulus).
* Remark "SDC": each same-component block A_ll is the Q1 discretisation of
  -div(Lambda grad u) with Lambda = G I + (G + lambda) e_l e_l^T; the blocks
  are compared with a scalar diffusion assembly written here from that
  statement (element integrals by 3-point Gauss rules).
* Symmetric diagonalisation: fixed dofs keep only their diagonal, and the
  matrix stays symmetric.
* The paper's geomechanics basis experiment (Sec. "FE simulation of linear
  elastic geomechanics"): 12 x 12 elements, E = 1, nu = 0.25, 5 coarse
  nodes per direction, stretched 20 times in y.  The naive basis leaves
  [0, 1] within 20 iterations; the enhanced (SDC-filtered) basis converges
  to the bilinear interpolators of a homogeneous Cartesian problem.
* The oracle's log-E adjoint gradient (element matrix integrated from the
  index form of the bilinear form) against central finite differences of
  the objective through direct solves of the generator's (Voigt-form)
  matrices, per element and along a random direction.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from synth.q1 import q1_elasticity, lame


def _csr(rp, ci, a):
    n = rp.size - 1
    return sp.csr_matrix((a, ci, rp), shape=(n, n))


def _node_coords(elems, h):
    d = len(elems)
    axes = [np.arange(e + 1) * h[k] for k, e in enumerate(elems)]
    g = np.meshgrid(*reversed(axes), indexing="ij")
    return np.stack([x.ravel() for x in reversed(g)], axis=1)   # columns x, y, (z)


@pytest.mark.parametrize("elems", [(3, 4, 2), (4, 3)])
def test_rigid_body_modes_and_symmetry(elems):
    d = len(elems)
    h = tuple(0.1 * (k + 1) for k in range(d))
    rng = np.random.default_rng(2)
    A = _csr(*q1_elasticity(elems, h, np.exp(rng.standard_normal(int(np.prod(elems)))), 0.25))
    X = _node_coords(elems, h)
    modes = [np.eye(d)[l][None, :].repeat(X.shape[0], 0).ravel() for l in range(d)]
    if d == 3:
        modes += [np.cross(w, X).ravel() for w in np.eye(3)]
    else:
        modes.append(np.stack([-X[:, 1], X[:, 0]], axis=1).ravel())
    scale = np.max(np.abs(A.data))
    for m in modes:
        assert np.max(np.abs(A @ m)) <= 1e-13 * scale * max(1.0, np.max(np.abs(m)))
    assert abs(A - A.T).max() <= 1e-15 * scale
    # full pattern: 3^d neighbour nodes times d components in the interior
    assert A.nnz == d * d * np.prod([4 + 3 * (e - 1) for e in elems])


@pytest.mark.parametrize("elems", [(4, 3, 3), (5, 4)])
def test_patch_test_linear_displacement(elems):
    d = len(elems)
    h = tuple(1.0 / e for e in elems)
    A = _csr(*q1_elasticity(elems, h, np.ones(int(np.prod(elems))), 0.3))
    X = _node_coords(elems, h)
    B = np.random.default_rng(1).standard_normal((d, d))
    r = (A @ (X @ B.T + 0.3).ravel()).reshape(-1, d)
    inner = np.all((X > 1e-12) & (X < 1.0 - 1e-12), axis=1)
    assert np.max(np.abs(r[inner])) <= 1e-13 * np.max(np.abs(A.data))
    assert np.max(np.abs(r[~inner])) > 1e-3


def _q1_diffusion(elems, h, Lam, coef):
    """Scalar Q1 matrix of -div(coef_e Lam grad u), dense, by 3-point Gauss."""
    d = len(elems)
    nodes = [e + 1 for e in elems]
    nn = int(np.prod(nodes))
    A = np.zeros((nn, nn))
    gp = [-np.sqrt(0.6), 0.0, np.sqrt(0.6)]
    gw = [5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0]
    corners = list(itertools.product((0, 1), repeat=d))   # (b_last, ..., b_x)
    for eidx, e in enumerate(itertools.product(*[range(m) for m in reversed(elems)])):
        org = list(reversed(e))                            # element origin (x, y, z)
        loc = []
        for c in corners:
            bits = list(reversed(c))
            node = 0
            for k in reversed(range(d)):
                node = node * nodes[k] + org[k] + bits[k]
            loc.append((node, bits))
        Ke = np.zeros((len(loc), len(loc)))
        for pt in itertools.product(range(3), repeat=d):
            xi = [gp[q] for q in pt]
            w = np.prod([gw[q] for q in pt]) * np.prod(h) / 2 ** d
            grads = []
            for _, bits in loc:
                s = [2 * b - 1 for b in bits]
                g = np.array([s[k] / 2 * np.prod([(1 + s[m] * xi[m]) / 2
                                                  for m in range(d) if m != k]) * 2 / h[k]
                              for k in range(d)])
                grads.append(g)
            G = np.array(grads)
            Ke += w * G @ Lam @ G.T
        idx = [nd for nd, _ in loc]
        A[np.ix_(idx, idx)] += coef[eidx] * Ke
    return A


@pytest.mark.parametrize("elems", [(3, 2, 2), (4, 3)])
def test_sdc_blocks_are_anisotropic_diffusion(elems):
    d = len(elems)
    h = tuple(0.5 / (k + 1) for k in range(d))
    nu = 0.25
    E = np.exp(np.random.default_rng(3).standard_normal(int(np.prod(elems))))
    A = _csr(*q1_elasticity(elems, h, E, nu)).toarray()
    lam, G = lame(1.0, nu)
    for l in range(d):
        Lam = G * np.eye(d) + (G + lam) * np.outer(np.eye(d)[l], np.eye(d)[l])
        ref = _q1_diffusion(elems, h, Lam, E)
        blk = A[l::d, l::d]
        assert np.max(np.abs(blk - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_dirichlet_symmetric_diagonalisation():
    cfg = synth.make_config("c3", dims=(4, 3, 3), block=2)
    A = _csr(*cfg["matrix"])
    fixed = cfg["fixed"]
    assert fixed.sum() == 3 * 5 * 4
    Ad = A.toarray()
    fx = np.nonzero(fixed)[0]
    off = Ad[fx].copy()
    off[np.arange(fx.size), fx] = 0.0
    assert np.all(off == 0.0) and np.all(Ad[:, fx][~fixed] == 0.0)
    assert np.all(Ad[fx, fx] > 0)
    assert abs(A - A.T).max() == 0.0
    # consistent traction loads: total force -1 (unit area), all on z
    f = cfg["rhs"].reshape(-1, 3)
    assert abs(f[:, 2].sum() + 1.0) <= 1e-14 and np.all(f[:, :2] == 0.0)


def test_naive_basis_diverges_sdc_basis_is_bilinear():
    elems, h = (12, 12), (1.0 / 12, 20.0 / 12)
    rp, ci, a = q1_elasticity(elems, h, np.ones(144), 0.25)
    sup = synth.vector_supports(synth.vertex_supports(elems, 3), 2)
    naive = oracle.Msrsb(rp, ci, a, 2)
    naive.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    naive.setup_basis(kmax=20, filt=False)
    assert naive.pv.min() < -0.1 and naive.pv.max() > 1.1
    enh = oracle.Msrsb(rp, ci, a, 2)
    enh.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    enh.setup_basis(kmax=2000, filt=True)
    assert enh.eit < 1e-13
    prp, pci = sup["prp"], sup["pci"]
    err = 0.0
    for r in range(prp.size - 1):
        node = r // 2
        x, y = node % 13, node // 13
        for e in range(prp[r], prp[r + 1]):
            cv = pci[e] // 2
            cx, cy = (cv % 5) * 3, (cv // 5) * 3
            hat = max(0.0, 1 - abs(x - cx) / 3) * max(0.0, 1 - abs(y - cy) / 3)
            err = max(err, abs(enh.pv[e] - hat))
    assert err <= 1e-10


def _q1_objective(cfg, logE, obs, data):
    import scipy.sparse.linalg as spl
    rp, ci, a = q1_elasticity(cfg["dims"], cfg["h"], np.exp(logE), cfg["nu"], cfg["fixed"])
    A = _csr(rp, ci, a).tocsc()
    u = spl.spsolve(A, cfg["rhs"])
    return float(np.sum((u[obs] - data) ** 2)), u, A


@pytest.mark.parametrize("dims", [(3, 3, 2), (4, 2, 3)])
def test_oracle_q1_gradient_matches_finite_differences(dims):
    """The oracle's log-E gradient (element matrix from the index form of the
    bilinear form) against central differences of J through direct solves of
    the generator's matrices (Voigt form), so neither side checks itself."""
    import scipy.sparse.linalg as spl
    cfg = synth.make_config("c3", dims=dims, block=2, seed=7)
    n = cfg["rhs"].size
    rng = np.random.default_rng(0)
    free = np.nonzero(~cfg["fixed"])[0]
    obs = np.sort(rng.choice(free, size=6, replace=False))
    data = 1e-3 * rng.standard_normal(obs.size)
    logE = cfg["logE"]
    J0, u, A = _q1_objective(cfg, logE, obs, data)
    gu = np.zeros(n)
    gu[obs] = 2.0 * (u[obs] - data)
    lam = spl.spsolve(A.T.tocsc(), gu)
    g = oracle.q1_grad(dims, cfg["h"], cfg["nu"], logE, cfg["fixed"], u, lam)
    step = 1e-5
    for e in range(logE.size):
        lp, lm = logE.copy(), logE.copy()
        lp[e] += step
        lm[e] -= step
        fd = (_q1_objective(cfg, lp, obs, data)[0] - _q1_objective(cfg, lm, obs, data)[0]) / (2 * step)
        assert abs(fd - g[e]) <= 1e-6 * np.max(np.abs(g)), (e, fd, g[e])
    # a random direction over all elements
    dvec = rng.standard_normal(logE.size)
    fd = (_q1_objective(cfg, logE + step * dvec, obs, data)[0]
          - _q1_objective(cfg, logE - step * dvec, obs, data)[0]) / (2 * step)
    assert abs(fd - g @ dvec) <= 1e-6 * abs(g @ dvec)
