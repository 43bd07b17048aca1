"""Pins of the oracle's multilevel MsRSB: the enhanced method applied again
to the (multipoint) coarse operator A_c, whose coarse solve becomes the next
level's two-stage preconditioner (the paper's conclusion: the filter makes
multipoint coarse operators usable for a further level).

* A second level in which every coarse node is its own block has P = I and
  an exact coarse solve, so its preconditioner is A_c^{-1} and the
  three-level apply equals the two-level one.
* The second level's coarse operator is the dense product P2^T A_c P2, its
  basis a partition of unity in [0, 1] (A_c is not an M-matrix).
* PCG with three levels solves the fine problem (dense direct solve)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def tpfa(dims, block, sigma=1.5, seed=0):
    rng = np.random.default_rng(seed)
    logk = sigma * rng.standard_normal(int(np.prod(dims)))
    h = tuple(1.0 / d for d in dims)
    bc = np.array([1.0, 0.0] + [np.nan] * 4)
    rp, ci, a, f = oracle.tpfa(dims, h, logk, bc)
    return rp, ci, a, f, synth.cell_supports(dims, block)


def setup(rp, ci, a, sup, levels=(), kmax=60):
    m = oracle.Msrsb(rp, ci, a)
    m.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    for lv, s2 in enumerate(levels, start=1):
        m.set_coarse_level(lv, s2["nc"], s2["part"], s2["prp"], s2["pci"], s2["interior"])
    m.setup_basis(kmax=kmax)
    m.build_coarse()
    return m


def identity_space(nc):
    ar = np.arange(nc, dtype=np.int32)
    return dict(nc=nc, part=ar, prp=np.arange(nc + 1, dtype=np.int32), pci=ar,
                interior=np.ones(nc, np.uint8))


def test_identity_second_level_equals_two_levels():
    rp, ci, a, f, sup = tpfa((24, 20), 4, seed=1)
    two = setup(rp, ci, a, sup)
    three = setup(rp, ci, a, sup, [identity_space(sup["nc"])])
    np.testing.assert_array_equal(three.child.pv, np.ones(sup["nc"]))
    v = np.random.default_rng(2).standard_normal(480)
    for pre, post in (((0, 0), (0, 0)), ((2, 2), (2, 2)), ((1, 1), (1, 1))):
        z2 = two.apply(v, pre=pre, post=post)
        z3 = three.apply(v, pre=pre, post=post)
        np.testing.assert_allclose(z3, z2, rtol=1e-12, atol=1e-12 * np.abs(z2).max())


def test_second_level_operator_and_basis():
    dims = (16, 16, 12)
    rp, ci, a, f, sup = tpfa(dims, 4, sigma=2.0, seed=3)
    sup2 = synth.cell_supports((4, 4, 3), 2)
    m = setup(rp, ci, a, sup, [sup2])
    ac = m.ac
    off = ac - np.diag(np.diag(ac))
    assert (off > 1e-12 * np.abs(ac).max()).sum() > 0     # A_c is not an M-matrix
    c = m.child
    P2 = sp.csr_matrix((c.pv, sup2["pci"], sup2["prp"]), shape=(sup["nc"], sup2["nc"])).toarray()
    np.testing.assert_allclose(P2.sum(axis=1), 1.0, atol=1e-14)
    assert P2.min() >= 0.0 and P2.max() <= 1.0
    np.testing.assert_allclose(c.ac, P2.T @ ac @ P2, rtol=1e-13, atol=1e-13 * np.abs(c.ac).max())


@pytest.mark.parametrize("pre,post", [((2, 2), (2, 2)), ((1, 1), (1, 1))])
def test_three_level_pcg_matches_dense_solve(pre, post):
    dims = (16, 16, 16)
    rp, ci, a, f, sup = tpfa(dims, 4, seed=4)
    m = setup(rp, ci, a, sup, [synth.cell_supports((4, 4, 4), 2)])
    r = m.solve(f, pre=pre, post=post, rtol=1e-12, maxit=500)
    assert r["status"] == 0 and r["true_rel"] <= 1e-12
    A = sp.csr_matrix((a, ci, rp), shape=(4096, 4096)).toarray()
    ref = np.linalg.solve(A, f)
    np.testing.assert_allclose(r["x"], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_four_levels():
    # three coarse levels below the fine one
    dims = (32, 32, 16)
    rp, ci, a, f, sup = tpfa(dims, 4, seed=5)
    lv = [synth.cell_supports((8, 8, 4), 2), synth.cell_supports((4, 4, 2), 2)]
    m = setup(rp, ci, a, sup, lv)
    assert m.child.child is not None and m.child.child.nc == 4
    r = m.solve(f, pre=(2, 2), post=(2, 2), rtol=1e-10, maxit=500)
    assert r["status"] == 0 and r["true_rel"] <= 1e-10
