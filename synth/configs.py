"""The five benchmark workloads, as seeded synthetic inputs.

Each workload is identified by a short name; ``make_config(name, dims=...)``
also builds the same recipe at a reduced size for tests.  Seeds are
1000 + workload number.

  c1  2D TPFA 32^2, log-normal k (sigma 1), 8^2 blocks, PCG + Jacobi post
  c2  2D MPFA-O 256^2, perturbed nodes, rotated 100:1 tensor, sigma 2,
      16^2 blocks, GMRES(30) + ILU(0) post
  c3  3D Q1 elasticity 64^3 elements, 3 dof per node, E log-normal sigma 1.5
      with 8-cell correlation, nu = 0.25, 8^3 coarse elements, PCG
  c4  3D TPFA 128^3, layered channelised k (sigma 2.5, 16 channels, 1000x),
      8^3 blocks, PCG + l1-Jacobi x2 pre/post; FP32 basis beside FP64
  c5  3D TPFA 96^3, log-normal k (sigma 1.5), 8^3 blocks, PCG, adjoint
      gradient of a 64-cell pressure misfit
"""
import numpy as np

from .grids import cell_supports, vertex_supports, vector_supports
from .fields import (lognormal_iid, channelised_logk, gaussian_smoothed,
                     observation_cells)

NAN = float("nan")

CONFIGS = {
    "c1": dict(kind="tpfa", dims=(32, 32), block=8, seed=1001),
    "c2": dict(kind="mpfa", dims=(256, 256), block=16, seed=1002),
    "c3": dict(kind="q1", dims=(64, 64, 64), block=8, seed=1003),
    "c4": dict(kind="tpfa", dims=(128, 128, 128), block=8, seed=1004),
    "c5": dict(kind="tpfa", dims=(96, 96, 96), block=8, seed=1005),
    # the paper's own 2D MPFA-O experiment (Sec. 3.2): 100 x 100 cells on
    # 20 m x 150 m, 400 coarse blocks of 5 x 5 cells
    "e2": dict(kind="mpfa_e2", dims=(100, 100), block=5, seed=1006),
}

# smoother codes shared with the C-ABI: 0 none, 1 Jacobi, 2 l1-Jacobi,
# 3 ILU(0), 4 symmetric Gauss-Seidel, 5 IC(0).  c2's ILU(0) runs in the
# multicolour order: in the natural order its factorisation of this rough
# non-M-matrix has a hundred non-positive pivots and restarted GMRES
# stagnates.  The paper's experiment runs Richardson and GMRES with ILU(0)
# or SGS; its recipe here is the Richardson + MsRSB + ILU(0) case.
SOLVERS = {
    "c1": dict(krylov="pcg", pre=(0, 0), post=(1, 1), ordering="natural"),
    "c2": dict(krylov="gmres", restart=30, pre=(0, 0), post=(3, 1), ordering="multicolor"),
    "c3": dict(krylov="pcg", pre=(2, 2), post=(2, 2), ordering="natural"),
    "c4": dict(krylov="pcg", pre=(2, 2), post=(2, 2), ordering="natural"),
    "c5": dict(krylov="pcg", pre=(2, 2), post=(2, 2), ordering="natural"),
    "e2": dict(krylov="richardson", pre=(0, 0), post=(3, 1), ordering="natural"),
}


def _tpfa_bc(dim):
    # p = 1 on the x = 0 face, p = 0 on the x = 1 face, no flow elsewhere
    bc = [NAN] * 6
    bc[0], bc[1] = 1.0, 0.0
    return np.array(bc, dtype=np.float64)


def make_config(name, dims=None, block=None, seed=None):
    """Build workload `name` (optionally at other dims/block/seed).

    Returns a dict with the coefficient field, grid sizes, boundary values,
    the coarse partition and support pattern, and the solver recipe."""
    base = dict(CONFIGS[name])
    dims = tuple(dims) if dims is not None else base["dims"]
    block = block if block is not None else base["block"]
    seed = seed if seed is not None else base["seed"]
    rng = np.random.default_rng(seed)
    cfg = dict(name=name, kind=base["kind"], dims=dims, block=block, seed=seed,
               dim=len(dims), omega=2.0 / 3.0, kmax=100, rtol=1e-8)
    cfg.update(SOLVERS[name])
    if base["kind"] == "tpfa":
        h = tuple(1.0 / d for d in dims) + (1.0,) * (3 - len(dims))
        if name == "c4":
            logk, chan = channelised_logk(dims, 2.5, 16, 1000.0, rng)
            cfg["channel"] = chan
        elif name == "c5":
            logk = lognormal_iid(dims, 1.5, rng)
        else:
            logk = lognormal_iid(dims, 1.0, rng)
        cfg.update(logk=logk, h=h, bc=_tpfa_bc(len(dims)), block_size=1)
        cfg["supports"] = cell_supports(dims, block)
        if name == "c5":
            n = int(np.prod(dims))
            obs = observation_cells(n, 64, rng)
            # data: the homogeneous-medium pressure 1 - x at the observation
            # cells plus N(0, 0.01^2) noise
            x = (obs % dims[0] + 0.5) / dims[0]
            cfg["obs"] = obs
            cfg["data"] = 1.0 - x + 0.01 * rng.standard_normal(obs.size)
    elif base["kind"] == "mpfa":
        from .mpfa import mpfa_case
        cfg.update(mpfa_case(dims, rng))
        cfg["block_size"] = 1
        cfg["supports"] = cell_supports(dims, block)
    elif base["kind"] == "mpfa_e2":
        from .mpfa import e2_case
        cfg.update(e2_case(dims, rng))
        cfg["block_size"] = 1
        cfg["supports"] = cell_supports(dims, block)
    elif base["kind"] == "q1":
        from .q1 import q1_case
        cfg.update(q1_case(dims, rng))
        cfg["block_size"] = 3
        cfg["supports"] = vector_supports(vertex_supports(dims, block), 3)
    return cfg
