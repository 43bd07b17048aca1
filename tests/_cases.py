"""Shared set-up of parity cases: the same seeded inputs fed to the oracle
and to the HIP library."""
import numpy as np

import oracle
import synth


def tpfa_inputs(name, dims=None, block=None, seed=None):
    cfg = synth.make_config(name, dims=dims, block=block, seed=seed)
    rp, ci, a, f = oracle.tpfa(cfg["dims"], cfg["h"], cfg["logk"], cfg["bc"])
    cfg.update(rp=rp, ci=ci, a=a, f=f)
    return cfg


def matrix_inputs(name, dims=None, block=None, seed=None):
    """Workloads whose matrix is generated as CSR (MPFA-O, Q1 elasticity)."""
    cfg = synth.make_config(name, dims=dims, block=block, seed=seed)
    rp, ci, a = cfg["matrix"]
    cfg.update(rp=rp, ci=ci, a=a, f=cfg["rhs"])
    return cfg


def oracle_setup(cfg, kmax=100, filt=True):
    m = oracle.Msrsb(cfg["rp"], cfg["ci"], cfg["a"], cfg.get("block_size", 1))
    s = cfg["supports"]
    m.set_coarse(s["nc"], s["part"], s["prp"], s["pci"], s["interior"])
    m.setup_basis(kmax=kmax, filt=filt)
    m.build_coarse()
    return m


def gpu_setup_tpfa(cfg, kmax=100, fp32_basis=False, device=0):
    """Assemble on the device from log k, then set up the preconditioner."""
    import torch
    from paper_1912_06934_amd import Msrsb
    s = Msrsb(device=device)
    dev = torch.device("cuda", device)
    logk = torch.from_numpy(np.ascontiguousarray(cfg["logk"])).to(dev)
    rhs = torch.empty_like(logk)
    s.assemble_tpfa(cfg["dims"], cfg["h"], logk, cfg["bc"], rhs)
    sup = cfg["supports"]
    s.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    binfo = s.setup_basis(max_iter=kmax, fp32_basis=fp32_basis)
    s.build_coarse()
    return s, rhs, binfo


def gpu_setup_matrix(cfg, kmax=100, fp32_basis=False, filt=True, device=0):
    from paper_1912_06934_amd import Msrsb
    s = Msrsb(device=device)
    s.set_matrix(cfg["rp"], cfg["ci"], cfg["a"], cfg.get("block_size", 1))
    sup = cfg["supports"]
    s.set_coarse(sup["nc"], sup["part"], sup["prp"], sup["pci"], sup["interior"])
    binfo = s.setup_basis(max_iter=kmax, fp32_basis=fp32_basis, filter=filt)
    s.build_coarse()
    return s, binfo


def rel_max(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))
