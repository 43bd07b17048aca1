"""The MPFA-O input generator and the enhanced filter on MPFA matrices,
pinned on the CPU.

* On a K-orthogonal Cartesian grid (isotropic K, unperturbed nodes) MPFA-O
  reduces to the two-point scheme (Sec. "MsRSB for non-M matrices"), so the
  generated matrix must equal the oracle's independently written TPFA
  matrix with no-flow boundaries.
* MPFA-O is consistent: for a homogeneous full tensor on a perturbed grid a
  linear pressure field has zero net flux out of every cell not touching the
  boundary.
* Without sources or wells every row sums to zero (fluxes are conservative).
* The paper's basis experiment (Sec. "Extension to non M-matrices"): a 9x9
  homogeneous grid with perturbed vertices, stretched ten times in y and
  coarsened by three.  The naive basis leaves [0, 1] within 11 iterations,
  the filtered one stays a monotone partition of unity.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from synth.mpfa import perturbed_nodes, rotated_tensors, mpfa_o

NAN = float("nan")


def _csr(rp, ci, a):
    n = rp.size - 1
    return sp.csr_matrix((a, ci, rp), shape=(n, n))


def test_mpfa_equals_tpfa_on_k_orthogonal_grid():
    rng = np.random.default_rng(11)
    dims = (7, 5)
    X = perturbed_nodes(dims, rng, 0.0)
    logk = rng.standard_normal(35)
    K = np.exp(logk)[:, None, None] * np.eye(2)[None]
    A = _csr(*mpfa_o(X, K)).toarray()
    r2, c2, v2, _ = oracle.tpfa(dims, (1 / 7, 1 / 5, 1.0), logk, np.array([NAN] * 6))
    B = _csr(r2, c2, v2).toarray()
    assert np.max(np.abs(A - B)) <= 1e-12 * np.max(np.abs(B))


@pytest.mark.parametrize("seed", [0, 1])
def test_mpfa_reproduces_linear_pressure(seed):
    rng = np.random.default_rng(seed)
    nx, ny = 9, 8
    X = perturbed_nodes((nx, ny), rng, 0.2)
    A = _csr(*mpfa_o(X, rotated_tensors(np.zeros(nx * ny))))
    xc = 0.25 * (X[:-1, :-1] + X[:-1, 1:] + X[1:, 1:] + X[1:, :-1]).reshape(-1, 2)
    p = 1.3 * xc[:, 0] - 0.7 * xc[:, 1] + 0.2
    r = A @ p
    jj, ii = np.divmod(np.arange(nx * ny), nx)
    inner = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1)
    assert np.max(np.abs(r[inner])) <= 1e-12 * np.max(np.abs(A.data))
    # the boundary cells do see the flux of the linear field
    assert np.max(np.abs(r[~inner])) > 1e-3


def test_mpfa_rows_conserve():
    rng = np.random.default_rng(5)
    X = perturbed_nodes((12, 10), rng, 0.2)
    A = _csr(*mpfa_o(X, rotated_tensors(rng.standard_normal(120))))
    assert np.max(np.abs(A @ np.ones(120))) <= 1e-12 * np.max(np.abs(A.data))


def test_c2_workload_structure():
    cfg = synth.make_config("c2", dims=(32, 32))
    rp, ci, a = cfg["matrix"]
    A = _csr(rp, ci, a)
    n = 32 * 32
    # 9-point pattern: (3 m - 2)^2 entries for an m x m grid
    assert rp[-1] == (3 * 32 - 2) ** 2
    off = (A - sp.diags(A.diagonal())).tocsr()
    assert (off.data > 0).sum() > 0           # not an M-matrix: the filter acts
    assert np.all(A.diagonal() > 0)
    assert cfg["rhs"][0] == 1.0 and np.count_nonzero(cfg["rhs"]) == 1
    # the well doubles the sink cell's diagonal
    assert abs(A[n - 1] @ np.ones(n) - A[n - 1, n - 1] / 2) <= 1e-12 * A[n - 1, n - 1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_naive_basis_diverges_filtered_stays_monotone(seed):
    # Sec. 3.1's 9 x 9 grid stretched 10x in y, vertices perturbed by the
    # 0.2 factor of Sec. 3.2 (Sec. 3.1 states no amplitude)
    rng = np.random.default_rng(seed)
    X = perturbed_nodes((9, 9), rng, 0.2, lengths=(1.0, 10.0))
    rp, ci, a = mpfa_o(X, np.eye(2)[None].repeat(81, 0))
    sup = synth.cell_supports((9, 9), 3)
    naive = oracle.Msrsb(rp, ci, a)
    naive.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    naive.setup_basis(kmax=11, filt=False)
    assert naive.pv.min() < -0.05 and naive.pv.max() > 1.05
    # iterated further the naive basis grows until e_it overflows
    grow = oracle.Msrsb(rp, ci, a)
    grow.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    grow.setup_basis(kmax=20000, nit=100, filt=False)
    assert not np.isfinite(grow.eit)
    filt = oracle.Msrsb(rp, ci, a)
    filt.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    filt.setup_basis(kmax=400, filt=True)
    assert filt.pv.min() >= 0.0 and filt.pv.max() <= 1.0
    assert filt.eit < 1e-4
