"""GPU parity: the HIP library against the FP64 CPU oracle on the same
seeded inputs, through the C ABI.

Tolerances: P and A_c to 1e-12 (relative to their largest entry) in FP64;
solutions to 1e-8 relative with both sides solved to 1e-12; the adjoint
gradient to 1e-8 of its largest entry.  The FP64 kernels use fused
multiply-adds and a different summation order, so agreement is to rounding,
not bitwise; the smoothing iteration is non-expansive (J is non-negative
and row-stochastic once filtered), so the difference after K iterations
stays near K * (stencil size) * 2^-53.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from _cases import (tpfa_inputs, matrix_inputs, oracle_setup, gpu_setup_tpfa,
                    gpu_setup_matrix, rel_max)

pytestmark = pytest.mark.gpu

# (workload recipe, dims, block): several tiles plus a ragged tail
CASES = [("c1", None, None),                 # 32^2, 16 coarse blocks (full size)
         ("c1", (37, 29), 8),                # partial coarse blocks on both axes
         ("c5", (24, 20, 18), 8),            # 3D, ragged last blocks
         ("c4", (32, 32, 32), 8),            # layered channels
         ("c4", (32, 64, 12), 8)]            # slabs of whole work-groups: the
                                             # z-walking smoothing order


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    return torch


def _id(c):
    return f"{c[0]}-{'x'.join(map(str, c[1])) if c[1] else 'full'}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_tpfa_assembly_matches_oracle(torch_cuda, case):
    cfg = tpfa_inputs(*case)
    s, rhs, _ = gpu_setup_tpfa(cfg, kmax=1)
    rp, ci, a = s.get_matrix()
    assert np.array_equal(rp, cfg["rp"]) and np.array_equal(ci, cfg["ci"])
    np.testing.assert_allclose(a, cfg["a"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(rhs.cpu().numpy(), cfg["f"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_basis_and_coarse_operator_match_oracle(torch_cuda, case):
    cfg = tpfa_inputs(*case)
    orc = oracle_setup(cfg)
    s, _, info = gpu_setup_tpfa(cfg)
    _, _, pv = s.get_prolongation()
    assert info["iters"] == 100 and orc.basis_iters == 100
    assert rel_max(pv, orc.pv) <= 1e-12
    assert info["max_rowsum_err"] <= 8 * np.finfo(float).eps
    assert 0.0 <= info["p_min"] and info["p_max"] <= 1.0
    assert abs(info["e_it"] - orc.eit) <= 1e-12 * max(orc.eit, 1e-300) + 1e-15
    ac = s.get_coarse_matrix()
    assert rel_max(ac, orc.ac) <= 1e-12


def test_coarse_pattern_follows_value_changes(torch_cuda):
    """The column lists of R A P are formed with the coarse space, from A's
    values at that time.  Formed on a diagonal A, they miss every coupling
    through a neighbour; once the full values are in place, the product must
    still reach all of A_c (the lists are formed again)."""
    from paper_1912_06934_amd import Msrsb
    cfg = tpfa_inputs("c5", (24, 20, 18), 8)
    orc = oracle_setup(cfg)
    rp, ci, a = cfg["rp"], cfg["ci"], cfg["a"]
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    s = Msrsb(device=0)
    s.set_matrix(rp, ci, np.where(ci == rows, a, 0.0))
    sup = cfg["supports"]
    s.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    s.update_values(a)
    s.setup_basis(max_iter=100)
    s.build_coarse()
    ac = s.get_coarse_matrix()
    assert rel_max(ac, orc.ac) <= 1e-12
    s.build_coarse()
    assert np.array_equal(s.get_coarse_matrix(), ac)


@pytest.mark.parametrize("case", CASES, ids=_id)
@pytest.mark.parametrize("smoother", [((0, 0), (1, 1)), ((2, 2), (2, 2)), ((1, 1), (0, 0))],
                         ids=["jac-post", "l1x2", "jac-pre"])
def test_preconditioner_apply_matches_oracle(torch_cuda, case, smoother):
    cfg = tpfa_inputs(*case)
    orc = oracle_setup(cfg)
    s, _, _ = gpu_setup_tpfa(cfg)
    v = np.random.default_rng(7).standard_normal(cfg["rp"].size - 1)
    pre, post = smoother
    z_ref = orc.apply(v, pre=pre, post=post)
    z = np.zeros_like(v)
    s.apply(v, z, pre=pre, post=post)
    assert rel_max(z, z_ref) <= 1e-11


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_solution_matches_oracle(torch_cuda, case):
    cfg = tpfa_inputs(*case)
    orc = oracle_setup(cfg)
    s, rhs, _ = gpu_setup_tpfa(cfg)
    pre, post = cfg["pre"], cfg["post"]
    ref = orc.solve(cfg["f"], rtol=1e-12, pre=pre, post=post)
    assert ref["status"] == 0
    u = np.zeros(cfg["rp"].size - 1)
    info = s.solve(cfg["f"], u, rtol=1e-12, pre=pre, post=post)
    assert info["true_rel_res"] <= 1e-12
    assert rel_max(u, ref["x"]) <= 1e-8
    # at the benchmark tolerance the iteration counts agree closely
    r8 = orc.solve(cfg["f"], rtol=1e-8, pre=pre, post=post)
    u8 = np.zeros_like(u)
    i8 = s.solve(cfg["f"], u8, rtol=1e-8, pre=pre, post=post)
    assert abs(i8["iters"] - r8["iters"]) <= 1
    assert i8["true_rel_res"] <= 1e-8


def test_device_buffers_and_stream(torch_cuda):
    torch = torch_cuda
    cfg = tpfa_inputs("c1")
    orc = oracle_setup(cfg)
    s, rhs, _ = gpu_setup_tpfa(cfg)
    u = torch.zeros_like(rhs)
    info = s.solve(rhs, u, rtol=1e-12, pre=(0, 0), post=(1, 1))
    ref = orc.solve(cfg["f"], rtol=1e-12, pre=(0, 0), post=(1, 1))
    torch.cuda.synchronize()
    assert rel_max(u.cpu().numpy(), ref["x"]) <= 1e-8
    assert info["iters"] > 0


def test_deterministic(torch_cuda):
    cfg = tpfa_inputs("c4", (32, 32, 32), 8)
    out = []
    for _ in range(2):
        s, rhs, _ = gpu_setup_tpfa(cfg)
        _, _, pv = s.get_prolongation()
        ac = s.get_coarse_matrix()
        u = np.zeros(cfg["rp"].size - 1)
        s.solve(cfg["f"], u, rtol=1e-8, pre=(2, 2), post=(2, 2))
        out.append((pv, ac, u))
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dims", [(32, 32, 32), (32, 64, 12)], ids=["32x32x32", "32x64x12"])
def test_fp32_basis_form(torch_cuda, dims):
    cfg = tpfa_inputs("c4", dims, 8)
    orc = oracle_setup(cfg)
    s, rhs, info = gpu_setup_tpfa(cfg, fp32_basis=True)
    _, _, pv = s.get_prolongation()
    err = np.max(np.abs(pv - orc.pv))
    # FP32 values with FP64 row sums: P error is FP32 rounding accumulated
    assert err <= 1e-5, err
    assert info["max_rowsum_err"] <= 8 * 2.0 ** -24
    u = np.zeros(cfg["rp"].size - 1)
    r = s.solve(cfg["f"], u, rtol=1e-8, pre=(2, 2), post=(2, 2), fp32_smoother=True)
    assert r["true_rel_res"] <= 1e-8
    # the FP64 outer iteration restores full accuracy: solved to 1e-12 the
    # FP32-basis form reaches the same solution as the FP64 oracle
    u = np.zeros(cfg["rp"].size - 1)
    r = s.solve(cfg["f"], u, rtol=1e-12, pre=(2, 2), post=(2, 2), fp32_smoother=True)
    assert r["true_rel_res"] <= 1e-12
    ref = orc.solve(cfg["f"], rtol=1e-12, pre=(2, 2), post=(2, 2))
    assert rel_max(u, ref["x"]) <= 1e-8


def test_transpose_solve_nonsymmetric(torch_cuda):
    cfg = tpfa_inputs("c1", (24, 24), 6)
    A = sp.csr_matrix((cfg["a"], cfg["ci"], cfg["rp"])).tolil()
    rng = np.random.default_rng(0)
    for i in range(575):
        if (i + 1) % 24:
            A[i, i + 1] += 0.06 * A[i, i] * rng.uniform()
    A = A.tocsr()
    A.sort_indices()
    cfg.update(rp=A.indptr.astype(np.int32), ci=A.indices.astype(np.int32), a=A.data)
    orc = oracle_setup(cfg)
    s, _ = gpu_setup_matrix(cfg)
    g = rng.standard_normal(576)
    ref = orc.solve(g, krylov="gmres", rtol=1e-12, pre=(1, 1), post=(1, 1), transpose=True)
    lam = np.zeros(576)
    info = s.solve_transpose(g, lam, krylov="gmres", rtol=1e-12, pre=(1, 1), post=(1, 1))
    assert info["true_rel_res"] <= 1e-12
    assert rel_max(lam, ref["x"]) <= 1e-8
    x = np.zeros(576)
    s.solve(g, x, krylov="gmres", rtol=1e-12, post=(1, 1))
    np.testing.assert_allclose(A @ x, g, atol=1e-10 * np.abs(g).max())


def test_adjoint_gradient_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1912_06934_amd import MsrsbTPFASolve, TPFAProblem
    cfg = tpfa_inputs("c5", (24, 20, 16), 8)
    obs, d = cfg["obs"] % (cfg["rp"].size - 1), cfg["data"]
    sup = cfg["supports"]
    prob = TPFAProblem(dims=cfg["dims"], h=cfg["h"], bc=tuple(cfg["bc"]),
                       coarse=dict(nc=sup["nc"], part=sup["part"], prp=sup["prp"],
                                   pci=sup["pci"], interior=sup["interior"]),
                       rtol=1e-12, fp32_basis=True)
    lk = torch.tensor(cfg["logk"], device="cuda", requires_grad=True)
    p = MsrsbTPFASolve.apply(lk, prob)
    ob = torch.as_tensor(obs, device="cuda")
    J = ((p[ob] - torch.as_tensor(d, device="cuda")) ** 2).sum()
    J.backward()
    g = lk.grad.cpu().numpy()
    # oracle: forward and adjoint solves at 1e-12, then the gradient formula
    orc = oracle_setup(cfg)
    pr = orc.solve(cfg["f"], rtol=1e-12, pre=(2, 2), post=(2, 2))["x"]
    gp = np.zeros_like(pr)
    np.add.at(gp, obs, 2 * (pr[obs] - d))
    lam = orc.solve(gp, rtol=1e-12, pre=(2, 2), post=(2, 2), transpose=True)["x"]
    g_ref = oracle.tpfa_grad(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"], pr, lam)
    assert np.max(np.abs(g - g_ref)) <= 1e-8 * np.max(np.abs(g_ref))


def _nonsymmetric(cfg, seed=0, amount=0.06):
    A = sp.csr_matrix((cfg["a"], cfg["ci"], cfg["rp"])).tolil()
    rng = np.random.default_rng(seed)
    n = A.shape[0]
    nx = cfg["dims"][0]
    for i in range(n - 1):
        if (i + 1) % nx:
            A[i, i + 1] += amount * A[i, i] * rng.uniform()
    A = A.tocsr()
    A.sort_indices()
    cfg.update(rp=A.indptr.astype(np.int32), ci=A.indices.astype(np.int32), a=A.data)
    return cfg


@pytest.mark.parametrize("case", [("c1", (96, 96), 4), ("c5", (48, 48, 48), 4),
                                  ("c1", (100, 92), 4), ("c5", (44, 40, 36), 4)],
                         ids=["2d-576coarse", "3d-1728coarse", "2d-575coarse", "3d-990coarse"])
def test_coarse_inverse_many_panels(torch_cuda, case):
    # coarse problems spanning many 64-wide panels of the band Cholesky
    # inverse, with whole and ragged last panels
    cfg = tpfa_inputs(*case)
    orc = oracle_setup(cfg, kmax=20)
    s, _, _ = gpu_setup_tpfa(cfg, kmax=20)
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    v = np.random.default_rng(3).standard_normal(cfg["rp"].size - 1)
    z_ref = orc.apply(v)
    z = np.zeros_like(v)
    s.apply(v, z)
    assert rel_max(z, z_ref) <= 1e-10


@pytest.mark.parametrize("case", [("c5", (13, 9, 7), 4), ("c5", (7, 5, 4), 2)],
                         ids=["13x9x7", "7x5x4"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_split_basis_small_grids(torch_cuda, case, fp32):
    # the split form on grids whose x lines are much shorter than a
    # wavefront (a wavefront's rows span several lines and planes): P in
    # both precisions and the apply (FP64 P: the split prolongation)
    cfg = tpfa_inputs(*case)
    orc = oracle_setup(cfg, kmax=30)
    s, _, _ = gpu_setup_tpfa(cfg, kmax=30, fp32_basis=fp32)
    assert rel_max(s.get_prolongation()[2], orc.pv) <= (1e-5 if fp32 else 1e-12)
    if not fp32:
        v = np.random.default_rng(7).standard_normal(cfg["rp"].size - 1)
        z_ref = orc.apply(v)
        z = np.zeros_like(v)
        s.apply(v, z)
        assert rel_max(z, z_ref) <= 1e-10


def test_split_basis_warm_start_and_set_prolongation(torch_cuda):
    # box supports on a 3D grid: the smoothing iteration runs on P split in
    # halves and the FP64 prolongation reads that form while it holds the
    # current P.  A warm start continues from the current P; a P set from
    # outside must replace the split copy in the prolongation; a warm start
    # in FP32 converts the set P.  The grid's row count is not a multiple
    # of the work-group size.
    cfg = tpfa_inputs("c5", (44, 40, 36), 4)
    orc = oracle_setup(cfg, kmax=6)
    s, _, _ = gpu_setup_tpfa(cfg, kmax=6)
    n = cfg["rp"].size - 1
    v = np.random.default_rng(5).standard_normal(n)

    def check_apply(tol):
        z_ref = orc.apply(v)
        z = np.zeros_like(v)
        s.apply(v, z)
        assert rel_max(z, z_ref) <= tol

    orc.setup_basis(kmax=5, warm_start=True)
    orc.build_coarse()
    s.setup_basis(max_iter=5, warm_start=True)
    s.build_coarse()
    assert rel_max(s.get_prolongation()[2], orc.pv) <= 1e-12
    check_apply(1e-10)

    pset = orc.pv * (1.0 + 0.01 * np.random.default_rng(6).standard_normal(orc.pv.size))
    orc.pv = pset.copy()
    orc.build_coarse()
    s.set_prolongation(pset)
    s.build_coarse()
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    check_apply(1e-10)

    orc.setup_basis(kmax=3, warm_start=True)
    s.setup_basis(max_iter=3, warm_start=True, fp32_basis=True)
    assert rel_max(s.get_prolongation()[2], orc.pv) <= 1e-5


@pytest.mark.parametrize("dims", [(32, 32), (40, 40), (64, 64), (80, 80), (100, 92),
                                  (176, 176), (212, 200), (256, 256)],
                         ids=["64coarse", "100coarse", "256coarse", "400coarse", "575coarse",
                              "1936coarse", "2650coarse", "4096coarse"])
def test_coarse_inverse_pivoting_nonsymmetric(torch_cuda, dims):
    # a non-symmetric operator takes the partial-pivoting Gauss-Jordan path;
    # the sizes reach every leaf form (64 to 1,024 threads with one row each,
    # then 2, 3 and 4 rows per thread up to the largest coarse system)
    cfg = _nonsymmetric(tpfa_inputs("c1", dims, 4))
    orc = oracle_setup(cfg, kmax=20)
    s, _ = gpu_setup_matrix(cfg, kmax=20)
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    v = np.random.default_rng(4).standard_normal(cfg["rp"].size - 1)
    z_ref = orc.apply(v, post=(1, 1))
    z = np.zeros_like(v)
    s.apply(v, z, post=(1, 1))
    assert rel_max(z, z_ref) <= 1e-10


# MPFA-O on perturbed grids (non-symmetric, positive off-diagonals: the
# filter acts, the coarse inverse takes the pivoting path), 16^2 coarse
# blocks with a ragged last block on each axis
MPFA_CASES = [("c2", (72, 56), 16), ("c2", (96, 80), 16)]


@pytest.mark.parametrize("case", MPFA_CASES, ids=_id)
def test_mpfa_basis_coarse_and_ilu0_apply(torch_cuda, case):
    cfg = matrix_inputs(*case)
    orc = oracle_setup(cfg)
    s, info = gpu_setup_matrix(cfg)
    _, _, pv = s.get_prolongation()
    assert rel_max(pv, orc.pv) <= 1e-12
    assert 0.0 <= info["p_min"] and info["p_max"] <= 1.0
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    v = np.random.default_rng(9).standard_normal(cfg["rp"].size - 1)
    z_ref = orc.apply(v, post=(3, 1))
    z = np.zeros_like(v)
    s.apply(v, z, post=(3, 1))
    assert rel_max(z, z_ref) <= 1e-11


@pytest.mark.parametrize("case", [("c2", (48, 40), 16), ("c2", (72, 56), 16)], ids=_id)
def test_mpfa_gmres_ilu0_solution(torch_cuda, case):
    # the i.i.d. sigma = 2 tensor field makes restarted GMRES slow near
    # 1e-12, so both sides stop at 1e-10, which leaves each within about
    # 1e-10 of the exact solution here (the direct solve agrees to 5e-11)
    cfg = matrix_inputs(*case)
    orc = oracle_setup(cfg)
    s, _ = gpu_setup_matrix(cfg)
    kw = dict(krylov="gmres", restart=30, pre=(0, 0), post=(3, 1))
    ref = orc.solve(cfg["f"], rtol=1e-10, maxit=4000, **kw)
    assert ref["status"] == 0
    u = np.zeros(cfg["rp"].size - 1)
    info = s.solve(cfg["f"], u, rtol=1e-10, max_iter=4000, **kw)
    assert info["true_rel_res"] <= 1e-10
    assert rel_max(u, ref["x"]) <= 1e-8
    # classical Gram-Schmidt twice (GPU) and modified Gram-Schmidt (oracle)
    # build the same Krylov space up to rounding: iteration counts agree to
    # a few percent
    r8 = orc.solve(cfg["f"], rtol=1e-8, maxit=4000, **kw)
    u8 = np.zeros_like(u)
    i8 = s.solve(cfg["f"], u8, rtol=1e-8, max_iter=4000, **kw)
    assert abs(i8["iters"] - r8["iters"]) <= 2 + 0.05 * r8["iters"]
    assert i8["true_rel_res"] <= 1e-8


# Q1 elasticity, 3 interleaved components, separate-displacement-component
# filter, vertex-centred supports (ragged last coarse element on y and z)
Q1_CASES = [("c3", (8, 8, 8), 4), ("c3", (12, 10, 9), 4), ("c3", (16, 16, 16), 8)]


@pytest.mark.parametrize("case", Q1_CASES, ids=_id)
def test_q1_sdc_basis_coarse_and_apply(torch_cuda, case):
    cfg = matrix_inputs(*case)
    orc = oracle_setup(cfg)
    s, info = gpu_setup_matrix(cfg)
    _, _, pv = s.get_prolongation()
    assert rel_max(pv, orc.pv) <= 1e-12
    assert 0.0 <= info["p_min"] and info["p_max"] <= 1.0
    assert info["max_rowsum_err"] <= 8 * np.finfo(float).eps
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    v = np.random.default_rng(5).standard_normal(cfg["rp"].size - 1)
    z_ref = orc.apply(v, pre=(2, 2), post=(2, 2))
    z = np.zeros_like(v)
    s.apply(v, z, pre=(2, 2), post=(2, 2))
    assert rel_max(z, z_ref) <= 1e-11


@pytest.mark.parametrize("case", Q1_CASES, ids=_id)
def test_q1_pcg_solution(torch_cuda, case):
    cfg = matrix_inputs(*case)
    orc = oracle_setup(cfg)
    s, _ = gpu_setup_matrix(cfg)
    kw = dict(pre=(2, 2), post=(2, 2))
    ref = orc.solve(cfg["f"], rtol=1e-12, maxit=3000, **kw)
    assert ref["status"] == 0
    u = np.zeros(cfg["rp"].size - 1)
    info = s.solve(cfg["f"], u, rtol=1e-12, max_iter=3000, **kw)
    assert info["true_rel_res"] <= 1e-12
    assert rel_max(u, ref["x"]) <= 1e-8
    r8 = orc.solve(cfg["f"], rtol=1e-8, maxit=3000, **kw)
    u8 = np.zeros_like(u)
    i8 = s.solve(cfg["f"], u8, rtol=1e-8, max_iter=3000, **kw)
    assert abs(i8["iters"] - r8["iters"]) <= 1
    # the FP32 form (basis, smoother) solved to 1e-12 reaches the same u
    s32, _ = gpu_setup_matrix(cfg, fp32_basis=True)
    u32 = np.zeros_like(u)
    i32 = s32.solve(cfg["f"], u32, rtol=1e-12, max_iter=3000, fp32_smoother=True, **kw)
    assert i32["true_rel_res"] <= 1e-12
    assert rel_max(u32, ref["x"]) <= 1e-8


# 2D Q1 elasticity (2 components per node, 9 node offsets): the node-block
# forms the 3D workload does not take (the two-component filter from the
# node-offset planes, R A P from the coarse rows' column lists)
def test_q1_2d_node_block_forms(torch_cuda):
    from synth.q1 import q1_elasticity
    elems, h = (24, 20), (1.0 / 24, 1.0 / 20)
    rng = np.random.default_rng(11)
    E = np.exp(rng.standard_normal(elems[0] * elems[1]))
    nnx = elems[0] + 1
    fixed = np.repeat(np.arange(nnx * (elems[1] + 1)) % nnx == 0, 2)  # the x = 0 edge
    rp, ci, a = q1_elasticity(elems, h, E, 0.3, fixed)
    f = rng.standard_normal(rp.size - 1)
    f[fixed] = 0.0
    cfg = dict(rp=rp, ci=ci, a=a, f=f, block_size=2,
               supports=synth.vector_supports(synth.vertex_supports(elems, 4), 2))
    orc = oracle_setup(cfg)
    s, info = gpu_setup_matrix(cfg)
    _, _, pv = s.get_prolongation()
    assert rel_max(pv, orc.pv) <= 1e-12
    assert info["max_rowsum_err"] <= 8 * np.finfo(float).eps
    assert rel_max(s.get_coarse_matrix(), orc.ac) <= 1e-12
    v = rng.standard_normal(rp.size - 1)
    z_ref = orc.apply(v, pre=(2, 2), post=(2, 2))
    z = np.zeros_like(v)
    s.apply(v, z, pre=(2, 2), post=(2, 2))
    assert rel_max(z, z_ref) <= 1e-11
    ref = orc.solve(f, rtol=1e-12, maxit=3000, pre=(2, 2), post=(2, 2))
    assert ref["status"] == 0
    u = np.zeros_like(f)
    out = s.solve(f, u, rtol=1e-12, max_iter=3000, pre=(2, 2), post=(2, 2))
    assert out["true_rel_res"] <= 1e-12
    assert rel_max(u, ref["x"]) <= 1e-8


@pytest.mark.parametrize("elems,h", [((12, 10, 9), (1 / 12, 1 / 10, 1 / 9)),
                                     ((12, 12), (1 / 12, 20 / 12))], ids=["3d", "2d-stretched"])
def test_q1_assembly_matches_generator(torch_cuda, elems, h):
    from synth.q1 import q1_elasticity
    from paper_1912_06934_amd import Msrsb
    d = len(elems)
    rng = np.random.default_rng(4)
    logE = 1.5 * rng.standard_normal(int(np.prod(elems)))
    n = d * int(np.prod([e + 1 for e in elems]))
    fixed = np.zeros(n, dtype=np.uint8)
    fixed[:d * (elems[0] + 1)] = 1                       # the y = 0 row / z = 0 ... first nodes
    rp, ci, a = q1_elasticity(elems, h, np.exp(logE), 0.25, fixed.astype(bool))
    s = Msrsb()
    s.assemble_q1(elems, h, 0.25, logE, fixed)
    grp, gci, ga = s.get_matrix()
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    assert np.max(np.abs(ga - a)) <= 1e-14 * np.max(np.abs(a))
    G = sp.csr_matrix((ga, gci, grp))
    assert (G - G.T).count_nonzero() == 0                # symmetric to the bit


def test_q1_adjoint_gradient_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1912_06934_amd import MsrsbQ1Solve, Q1Problem
    cfg = matrix_inputs("c3", (12, 10, 9), 4)
    sup = cfg["supports"]
    rng = np.random.default_rng(8)
    free = np.nonzero(~cfg["fixed"])[0]
    obs = np.sort(rng.choice(free, size=32, replace=False))
    data = 1e-3 * rng.standard_normal(obs.size)
    prob = Q1Problem(elems=cfg["dims"], h=cfg["h"], nu=cfg["nu"], loads=cfg["rhs"],
                     fixed=cfg["fixed"].astype(np.uint8),
                     coarse=dict(nc=sup["nc"], part=sup["part"], prp=sup["prp"], pci=sup["pci"],
                                 interior=sup["interior"]),
                     rtol=1e-12, max_iter=3000, fp32_basis=True)
    lE = torch.tensor(cfg["logE"], device="cuda", requires_grad=True)
    u = MsrsbQ1Solve.apply(lE, prob)
    ob = torch.as_tensor(obs, device="cuda")
    J = ((u[ob] - torch.as_tensor(data, device="cuda")) ** 2).sum()
    J.backward()
    g = lE.grad.cpu().numpy()
    assert prob.last_forward["solve"]["true_rel_res"] <= 1e-12
    assert prob.last_backward["solve"]["true_rel_res"] <= 1e-12
    orc = oracle_setup(cfg)
    ur = orc.solve(cfg["f"], rtol=1e-12, maxit=3000, pre=(2, 2), post=(2, 2))["x"]
    assert rel_max(u.detach().cpu().numpy(), ur) <= 1e-8
    gu = np.zeros_like(ur)
    gu[obs] = 2 * (ur[obs] - data)
    lam = orc.solve(gu, rtol=1e-12, maxit=3000, pre=(2, 2), post=(2, 2), transpose=True)["x"]
    g_ref = oracle.q1_grad(cfg["dims"], cfg["h"], cfg["nu"], cfg["logE"], cfg["fixed"], ur, lam)
    assert np.max(np.abs(g - g_ref)) <= 1e-8 * np.max(np.abs(g_ref))


def _stencil27(dims, seed):
    """A symmetric 27-point M-matrix on a 3D grid (positive random weights on
    the 26 neighbours, diagonally dominant through a Dirichlet-like shift
    on the x = 0 face): the stencil kernels' form without LDS tiling (more
    than nine diagonals)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    idx = x + nx * (y + ny * z)
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # forward half of the offsets; the mirror entries are added below
                if (dz, dy, dx) <= (0, 0, 0):
                    continue
                ok = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) &
                      (z + dz >= 0) & (z + dz < nz))
                i = idx[ok]
                j = (x + dx + nx * (y + dy + ny * (z + dz)))[ok]
                w = np.exp(0.5 * rng.standard_normal(i.size))
                rows += [i, j]
                cols += [j, i]
                vals += [-w, -w]
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    off = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    diag = -np.asarray(off.sum(axis=1)).ravel() + np.where(x == 0, 1.0, 0.0)
    A = (off + sp.diags(diag)).tocsr()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy())


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32-form"])
def test_pcg_on_27_point_stencil(torch_cuda, fp32):
    # l1-Jacobi x2 around the coarse stage on a 27-diagonal operator: the PCG
    # update runs on its own, then the untiled two-sweep kernel (FP64, or the
    # FP32 form's kernels with an FP32 basis)
    dims = (20, 18, 14)
    rp, ci, a = _stencil27(dims, 11)
    sup = synth.cell_supports(dims, 4)
    cfg = dict(rp=rp, ci=ci, a=a, supports=sup)
    f = np.random.default_rng(12).standard_normal(rp.size - 1)
    orc = oracle_setup(cfg)
    s, _ = gpu_setup_matrix(cfg, fp32_basis=fp32)
    pre = post = (2, 2)
    ref = orc.solve(f, rtol=1e-12, pre=pre, post=post)
    assert ref["status"] == 0
    u = np.zeros(rp.size - 1)
    info = s.solve(f, u, rtol=1e-12, pre=pre, post=post, fp32_smoother=fp32)
    print(f"27-point: GPU {info['iters']} / oracle {ref['iters']} iterations", flush=True)
    assert info["true_rel_res"] <= 1e-12
    assert rel_max(u, ref["x"]) <= 1e-8
    r8 = orc.solve(f, rtol=1e-8, pre=pre, post=post)
    u8 = np.zeros_like(u)
    i8 = s.solve(f, u8, rtol=1e-8, pre=pre, post=post, fp32_smoother=fp32)
    assert i8["true_rel_res"] <= 1e-8
    assert abs(i8["iters"] - r8["iters"]) <= (1 if not fp32 else 2)


def test_coarse_factor_choices(torch_cuda):
    # the automatic (Cholesky) and the pivoted Gauss-Jordan inverse of the
    # same SPD A_c both give the oracle's coarse solve; the Cholesky form is
    # refused where A_c need not be symmetric
    from paper_1912_06934_amd import MsrsbError
    cfg = tpfa_inputs("c5", (24, 20, 18), 8)
    orc = oracle_setup(cfg)
    n = cfg["rp"].size - 1
    v = np.random.default_rng(21).standard_normal(n)
    ref = orc.apply(v, pre=(2, 2), post=(2, 2))
    s, _, _ = gpu_setup_tpfa(cfg)
    out = {}
    for factor in ("auto", "pivoted", "cholesky"):
        s.build_coarse(factor=factor)
        z = np.zeros(n)
        s.apply(v, z, pre=(2, 2), post=(2, 2))
        assert rel_max(z, ref) <= 1e-11, factor
        out[factor] = z
    assert rel_max(out["pivoted"], out["cholesky"]) <= 1e-12
    with pytest.raises(MsrsbError) as e:
        s.build_coarse(restriction="msfv", factor="cholesky")
    assert e.value.code == -1
    with pytest.raises(MsrsbError) as e:
        s.build_coarse(factor=7)
    assert e.value.code == -1
    s.build_coarse(restriction="msfv", factor="pivoted")   # usable again
