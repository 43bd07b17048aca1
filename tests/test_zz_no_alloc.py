"""msrsb_apply_preconditioner_noalloc against msrsb_apply_preconditioner.

The allocation-free entry point runs the same kernels with its temporaries in
the library's static scratch array, so its output must equal the ordinary
apply's to rounding (in practice to the bit).  Two calls in a row on two
problems, the second one smaller, show that nothing left in the shared
array by the first call leaks into the second."""
import numpy as np
import pytest

import synth
from _cases import gpu_setup_tpfa, gpu_setup_matrix, matrix_inputs, tpfa_inputs

pytestmark = pytest.mark.gpu

E_ARG, E_STATE = -1, -2


def _compare(s, n, seed, **kw):
    import torch
    dev = torch.device("cuda", 0)
    v = torch.from_numpy(np.random.default_rng(seed).standard_normal(n)).to(dev)
    ref = torch.empty_like(v)
    s.apply(v, ref, **kw)                    # also forms the smoother's data
    z = torch.full_like(v, np.nan)
    s.apply_noalloc(v, z, **kw)
    torch.cuda.synchronize()
    zr, zn = ref.cpu().numpy(), z.cpu().numpy()
    assert np.all(np.isfinite(zn))
    err = float(np.max(np.abs(zn - zr)) / np.max(np.abs(zr)))
    print(f"n={n} {kw}: max rel diff {err:.2e}", flush=True)
    assert err <= 1e-14
    return err


def test_noalloc_matches_apply_two_calls():
    # first call: a 3D workload of 28,800 rows (many tiles, ragged coarse
    # blocks); second call: a smaller 2D one
    big = tpfa_inputs("c5", dims=(40, 36, 20), block=6)
    s1, _, _ = gpu_setup_tpfa(big, kmax=60)
    n1 = 40 * 36 * 20
    _compare(s1, n1, 1, pre=(2, 2), post=(2, 2))
    _compare(s1, n1, 2, pre=(2, 2), post=(2, 2), fp32_smoother=True)
    small = tpfa_inputs("c1")
    s2, _, _ = gpu_setup_tpfa(small, kmax=100)
    _compare(s2, 1024, 3, pre=(0, 0), post=(1, 1))
    _compare(s2, 1024, 4, pre=(1, 1), post=(1, 1), use_multiscale=False)


def test_noalloc_ilu0_and_repeat():
    # a non-symmetric operator with the ILU(0) post-smoother (coarse inverse by
    # Gauss-Jordan), then the larger workload again after the smaller one
    cfg = matrix_inputs("c2", dims=(48, 40), block=8)
    s, _ = gpu_setup_matrix(cfg, kmax=100)
    _compare(s, 48 * 40, 5, pre=(0, 0), post=(3, 1))
    big = tpfa_inputs("c5", dims=(24, 20, 18), block=8)
    s2, _, _ = gpu_setup_tpfa(big, kmax=100)
    _compare(s2, 24 * 20 * 18, 6, pre=(2, 2), post=(2, 2))


def test_noalloc_refuses_what_it_cannot_do():
    import torch
    from paper_1912_06934_amd import MsrsbError
    dev = torch.device("cuda", 0)
    cfg = tpfa_inputs("c1")
    s, _, _ = gpu_setup_tpfa(cfg, kmax=20)
    v = torch.ones(1024, dtype=torch.float64, device=dev)
    z = torch.empty_like(v)
    # the l1-Jacobi data do not exist yet: forming them would allocate
    with pytest.raises(MsrsbError) as e:
        s.apply_noalloc(v, z, pre=(2, 1), post=(2, 1))
    assert e.value.code == E_STATE
    # beyond the scratch limit of 262,144 rows
    cfg = synth.make_config("c4", dims=(72, 64, 64))
    from paper_1912_06934_amd import Msrsb
    s = Msrsb(device=0)
    logk = torch.from_numpy(cfg["logk"]).to(dev)
    rhs = torch.empty_like(logk)
    s.assemble_tpfa(cfg["dims"], cfg["h"], logk, cfg["bc"], rhs)
    v = torch.ones(72 * 64 * 64, dtype=torch.float64, device=dev)
    z = torch.empty_like(v)
    with pytest.raises(MsrsbError) as e:
        s.apply_noalloc(v, z, pre=(2, 1), post=(2, 1), use_multiscale=False)
    assert e.value.code == E_ARG
