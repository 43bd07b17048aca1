"""A hand-worked example of the whole method (tests/golden/worked_1d_six_cells.txt):
six cells in 1D, two coarse blocks, two positive off-diagonal couplings.

The expected values were derived by hand from the paper's definitions (the
filter and D-hat of Sec. 2.1/3.1, the smoothing step with dropped
out-of-support products and row rescaling of Alg. 1, A_c = P^T A P of Alg. 2,
the coarse correction of Alg. 3 and a post-smoothing step of Alg. 4); the
file shows the working.  The oracle must reproduce them to rounding (CPU
tests), and so must the HIP library (the GPU test).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_1d_six_cells.txt")
TOL = 1e-14          # every value is O(1) and takes a handful of operations


def _load():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(":", 1)
            vals[key.strip()] = [float(Fraction(t)) for t in rest.split()]
    g = {k: np.array(v) for k, v in vals.items() if "[" not in k}
    for name in ("A", "J_filtered", "Ac"):
        rows = sorted((int(k[len(name) + 1:-1]), v) for k, v in vals.items()
                      if k.startswith(name + "["))
        g[name] = np.array([v for _, v in rows])
    n = int(g["n"][0])
    pat = [np.array(vals[f"pattern[{i}]"], dtype=np.int32) for i in range(n)]
    g["prp"] = np.concatenate([[0], np.cumsum([p.size for p in pat])]).astype(np.int32)
    g["pci"] = np.concatenate(pat).astype(np.int32)
    g["nc"] = int(g["nc"][0])
    g["part"] = g["part"].astype(np.int32)
    g["interior"] = g["interior"].astype(np.uint8)
    A = g["A"]
    rows, cols = np.nonzero(A)
    g["rp"] = np.searchsorted(rows, np.arange(n + 1)).astype(np.int32)
    g["ci"] = cols.astype(np.int32)
    g["a"] = A[rows, cols]
    return g


@pytest.fixture(scope="module")
def gold():
    return _load()


def _dense(g, vals):
    n = g["rp"].size - 1
    M = np.zeros((n, n))
    for i in range(n):
        for e in range(g["rp"][i], g["rp"][i + 1]):
            M[i, g["ci"][e]] = vals[e]
    return M


def test_fixture_is_consistent(gold):
    # the inputs as written: symmetric A with the two positive couplings,
    # every row's support contains its own block, P0 a partition of unity
    A = gold["A"]
    assert np.array_equal(A, A.T) and A[1, 3] == 0.5
    for i in range(A.shape[0]):
        assert gold["part"][i] in gold["pci"][gold["prp"][i]:gold["prp"][i + 1]]
    # hand-derived results that must hold between themselves
    P = np.zeros((6, 2))
    for i in range(6):
        for e in range(gold["prp"][i], gold["prp"][i + 1]):
            P[i, gold["pci"][e]] = gold["P_converged_filtered"][e]
    assert np.allclose(P.sum(1), 1.0, atol=0)
    assert np.allclose(P.T @ A @ P, gold["Ac"], atol=TOL)


def test_oracle_filter_and_jacobi(gold):
    jv, dh = oracle.filter_jacobi(gold["rp"], gold["ci"], gold["a"], filt=True)
    assert np.max(np.abs(dh - gold["dhat_filtered"])) <= TOL
    assert np.max(np.abs(_dense(gold, jv) - gold["J_filtered"])) <= TOL
    _, dh0 = oracle.filter_jacobi(gold["rp"], gold["ci"], gold["a"], filt=False)
    assert np.max(np.abs(dh0 - gold["dhat_unfiltered"])) <= TOL


def test_oracle_smoothing_steps(gold):
    g = gold
    p0 = oracle.init_basis(g["prp"], g["pci"], g["part"])
    jv, _ = oracle.filter_jacobi(g["rp"], g["ci"], g["a"], filt=True)
    p1, e0 = oracle.smooth_step(g["rp"], g["ci"], jv, g["prp"], g["pci"], p0, g["interior"])
    assert np.max(np.abs(p1 - g["P1_filtered"])) <= TOL
    assert abs(e0 - g["eit0_filtered"][0]) <= TOL
    pk, iters, _, hist = oracle.basis(g["rp"], g["ci"], jv, g["prp"], g["pci"], p0,
                                      g["interior"], kmax=100, nit=1)
    assert iters == 100
    assert np.max(np.abs(pk - g["P_converged_filtered"])) <= TOL
    assert abs(hist[0] - g["eit0_filtered"][0]) <= TOL
    assert abs(hist[1] - g["eit1_filtered"][0]) <= TOL
    ju, _ = oracle.filter_jacobi(g["rp"], g["ci"], g["a"], filt=False)
    pu, _ = oracle.smooth_step(g["rp"], g["ci"], ju, g["prp"], g["pci"], p0, g["interior"])
    assert np.max(np.abs(pu - g["P1_unfiltered"])) <= TOL


def test_oracle_coarse_operator_and_apply(gold):
    g = gold
    m = oracle.Msrsb(g["rp"], g["ci"], g["a"])
    m.set_coarse(g["nc"], g["part"], g["prp"], g["pci"], g["interior"])
    m.setup_basis(kmax=100)
    ac = m.build_coarse()
    assert np.max(np.abs(ac - g["Ac"])) <= TOL
    z = m.apply(g["v"])
    assert np.max(np.abs(z - g["z_coarse_only"])) <= TOL
    z = m.apply(g["v"], post=(1, 1))              # one Jacobi post-sweep
    assert np.max(np.abs(z - g["z_post_jacobi"])) <= TOL


@pytest.mark.gpu
def test_library_reproduces_worked_example(gold):
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_1912_06934_amd import Msrsb
    g = gold
    s = Msrsb()
    s.set_matrix(g["rp"], g["ci"], g["a"])
    s.set_coarse(g["nc"], g["part"], g["prp"], g["pci"], g["interior"])
    info = s.setup_basis(max_iter=1)
    assert np.max(np.abs(s.get_prolongation()[2] - g["P1_filtered"])) <= TOL
    assert abs(info["e_it"] - g["eit0_filtered"][0]) <= TOL
    s.setup_basis(max_iter=1, filter=False)
    assert np.max(np.abs(s.get_prolongation()[2] - g["P1_unfiltered"])) <= TOL
    info = s.setup_basis(max_iter=100)
    assert np.max(np.abs(s.get_prolongation()[2] - g["P_converged_filtered"])) <= TOL
    assert abs(info["e_it"] - g["eit1_filtered"][0]) <= TOL
    s.build_coarse()
    assert np.max(np.abs(s.get_coarse_matrix() - g["Ac"])) <= TOL
    z = np.zeros(6)
    s.apply(g["v"], z)
    assert np.max(np.abs(z - g["z_coarse_only"])) <= TOL
    s.apply(g["v"], z, post=(1, 1))
    assert np.max(np.abs(z - g["z_post_jacobi"])) <= TOL
