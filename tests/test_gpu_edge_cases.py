"""GPU parity on the degenerate cases of the method, against the oracle:
fewer rows than a wavefront, a single coarse block, grids one cell wide,
supports without overlap (P stays the block indicator), and frozen rows
(a row with no coupling: D-hat_ii = 0, so J's row is e_i).  Each compares P,
A_c, one preconditioner application and the PCG solution with the
tolerances of the other parity tests."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from _cases import (tpfa_inputs, oracle_setup, gpu_setup_tpfa, gpu_setup_matrix, rel_max)

pytestmark = pytest.mark.gpu


def _compare(s, m, f, pre, post, n):
    _, _, pv = s.get_prolongation()
    assert rel_max(pv, m.pv) <= 1e-12
    assert rel_max(s.get_coarse_matrix(), m.ac) <= 1e-12
    v = np.random.default_rng(7).standard_normal(n)
    z = np.zeros(n)
    s.apply(v, z, pre=pre, post=post)
    assert rel_max(z, m.apply(v, pre=pre, post=post)) <= 1e-11
    ref = m.solve(f, rtol=1e-12, pre=pre, post=post)
    assert ref["status"] == 0
    u = np.zeros(n)
    info = s.solve(f, u, rtol=1e-12, pre=pre, post=post)
    assert info["true_rel_res"] <= 1e-12
    assert rel_max(u, ref["x"]) <= 1e-8
    r8 = m.solve(f, rtol=1e-8, pre=pre, post=post)
    u8 = np.zeros(n)
    i8 = s.solve(f, u8, rtol=1e-8, pre=pre, post=post)
    assert i8["true_rel_res"] <= 1e-8 and abs(i8["iters"] - r8["iters"]) <= 1
    return info["iters"]


CASES = [("c1", (3, 2), 2),              # 6 rows: less than one wavefront
         ("c1", (16, 16), 16),           # a single coarse block (nc = 1)
         ("c1", (64, 1), 8),             # a line of cells
         ("c4", (5, 3, 2), 2),           # tiny 3D with ragged blocks
         ("c4", (1, 1, 40), (1, 1, 8))]  # a column of cells


@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}")
def test_degenerate_grids(case):
    cfg = tpfa_inputs(*case)
    m = oracle_setup(cfg)
    s, _, _ = gpu_setup_tpfa(cfg)
    n = cfg["rp"].size - 1
    it = _compare(s, m, cfg["f"], cfg["pre"], cfg["post"], n)
    print(f"{case}: n {n}, nc {cfg['supports']['nc']}, {it} PCG iterations", flush=True)


def test_supports_without_overlap():
    # every support is its own coarse block: one entry per row of P, which
    # the renormalisation keeps at 1 (the block indicator): exactly in the
    # oracle, which divides by the row sum, and within one unit in the last
    # place in the kernel, which multiplies by the sum's FP64 reciprocal
    cfg = tpfa_inputs("c1", (12, 10), 4)
    n = cfg["rp"].size - 1
    sup = dict(cfg["supports"])
    part = sup["part"].astype(np.int32)
    sup.update(prp=np.arange(n + 1, dtype=np.int32), pci=part.copy(),
               interior=np.ones(n, np.uint8))
    cfg["supports"] = sup
    m = oracle_setup(cfg)
    s, _, _ = gpu_setup_tpfa(cfg)
    _, _, pv = s.get_prolongation()
    np.testing.assert_array_equal(m.pv, np.ones(n))
    np.testing.assert_allclose(pv, 1.0, rtol=0, atol=2.0 ** -52)
    _compare(s, m, cfg["f"], (0, 0), (1, 1), n)


def test_frozen_rows():
    # a TPFA matrix in which two cells lose every coupling (kept as stored
    # zeros; each removed value moved onto the neighbour's diagonal, so its
    # row keeps its sum; the decoupled cells' diagonal set to 1): their
    # filtered diagonal is zero, so their rows of J are e_i and P keeps them
    # at their block's characteristic value
    cfg = tpfa_inputs("c1", (12, 10), 4)
    rp, ci, a = cfg["rp"], cfg["ci"], cfg["a"].copy()
    n = rp.size - 1
    dpos = {i: e for i in range(n) for e in range(rp[i], rp[i + 1]) if ci[e] == i}
    for k in (17, 63):
        for e in range(rp[k], rp[k + 1]):
            j = ci[e]
            if j == k or a[e] == 0.0:
                continue
            w = a[e]
            mirror = next(e2 for e2 in range(rp[j], rp[j + 1]) if ci[e2] == k)
            a[e] = a[mirror] = 0.0
            a[dpos[k]] += w
            a[dpos[j]] += w
        a[dpos[k]] = 1.0     # the decoupled cell's equation: u_k = f_k
    mcfg = dict(rp=rp, ci=ci, a=a, supports=cfg["supports"])
    m = oracle_setup(mcfg)
    assert np.sum(m.dhat == 0.0) >= 2
    s, _ = gpu_setup_matrix(mcfg)
    f = np.random.default_rng(3).standard_normal(n)
    _compare(s, m, f, (2, 2), (2, 2), n)
