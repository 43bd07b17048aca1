"""Differentiation form: the solution as a differentiable function of a
log-coefficient field.

MsrsbTPFASolve: pressure p(log k) of the two-point flux system
A(k) p = f(k).  MsrsbQ1Solve: displacement u(log E) of the Q1 elasticity
system A(E) u = f (loads independent of E).  Forward assembles the system on
the device, (re)builds the MsRSB preconditioner (warm-starting the basis from
the previous one) and solves.  Backward solves the adjoint system
A^T lambda = dJ/dx with the transposed preconditioner and evaluates the
gradient kernel; no step is differentiated through the preconditioner, whose
only role is to speed up the solves.
"""
from dataclasses import dataclass, field

import numpy as np
import torch

from ._binding import Msrsb


@dataclass
class TPFAProblem:
    """Grid, boundary values and solver settings for MsrsbTPFASolve."""
    dims: tuple
    h: tuple
    bc: tuple
    coarse: dict                       # nc, part, prp, pci, interior (from a partitioner)
    krylov: str = "pcg"
    pre: tuple = (2, 2)
    post: tuple = (2, 2)
    rtol: float = 1e-8
    max_iter: int = 1000
    basis_iters: int = 100
    fp32_basis: bool = True
    fp32_smoother: bool = False
    warm_start: bool = True
    solver: Msrsb = field(default=None, repr=False)
    _coarse_set: bool = field(default=False, repr=False)
    _version: int = field(default=0, repr=False)
    last_forward: dict = field(default_factory=dict, repr=False)
    last_backward: dict = field(default_factory=dict, repr=False)

    def ensure_solver(self, device):
        if self.solver is None:
            self.solver = Msrsb(device=device)
        self.solver.set_stream(torch.cuda.current_stream(device).cuda_stream)
        return self.solver

    def solve_kw(self):
        return dict(krylov=self.krylov, rtol=self.rtol, max_iter=self.max_iter, pre=self.pre,
                    post=self.post, fp32_smoother=self.fp32_smoother)


class MsrsbTPFASolve(torch.autograd.Function):
    """p = MsrsbTPFASolve.apply(log_k, problem) with log_k a contiguous FP64
    CUDA tensor of one value per cell; p has the same shape."""

    @staticmethod
    def forward(ctx, log_k, prob):
        if not (log_k.is_cuda and log_k.dtype == torch.float64):
            raise TypeError("log_k must be a CUDA float64 tensor")
        log_k = log_k.contiguous()
        dev = log_k.device.index or 0
        s = prob.ensure_solver(dev)
        rhs = torch.empty_like(log_k)
        s.assemble_tpfa(prob.dims, prob.h, log_k, prob.bc, rhs)
        if not prob._coarse_set or s.nc is None:
            c = prob.coarse
            s.set_coarse(c["nc"], c["part"], c["prp"], c["pci"], c["interior"])
            prob._coarse_set = True
        b = s.setup_basis(max_iter=prob.basis_iters, fp32_basis=prob.fp32_basis,
                          warm_start=prob.warm_start)
        s.build_coarse()
        p = torch.zeros_like(log_k)
        info = s.solve(rhs, p, **prob.solve_kw())
        prob._version += 1
        prob.last_forward = dict(basis=b, solve=info)
        ctx.prob = prob
        ctx.version = prob._version
        ctx.save_for_backward(log_k, p)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        prob = ctx.prob
        if prob._version != ctx.version:
            raise RuntimeError("the solver was re-assembled since this forward; "
                               "run backward before the next forward on the same problem")
        log_k, p = ctx.saved_tensors
        s = prob.solver
        g = grad_p.contiguous().to(torch.float64)
        lam = torch.zeros_like(p)
        info = s.solve_transpose(g, lam, **prob.solve_kw())
        grad = torch.empty_like(log_k)
        s.tpfa_adjoint_grad(log_k, p, lam, grad)
        prob.last_backward = dict(solve=info)
        return grad, None


@dataclass
class Q1Problem:
    """Grid, material, loads, Dirichlet dofs and solver settings for
    MsrsbQ1Solve (elasticity on elems elements of sizes h, Poisson ratio
    nu)."""
    elems: tuple
    h: tuple
    nu: float
    loads: object                      # right-hand side, n values (NumPy or CUDA tensor)
    coarse: dict                       # nc, part, prp, pci, interior (per dof)
    fixed: object = None               # uint8 per dof, nonzero = fixed (or None)
    krylov: str = "pcg"
    pre: tuple = (2, 2)
    post: tuple = (2, 2)
    rtol: float = 1e-8
    max_iter: int = 1000
    basis_iters: int = 100
    fp32_basis: bool = True
    fp32_smoother: bool = False
    warm_start: bool = True
    solver: Msrsb = field(default=None, repr=False)
    _coarse_set: bool = field(default=False, repr=False)
    _version: int = field(default=0, repr=False)
    _dev: dict = field(default_factory=dict, repr=False)
    last_forward: dict = field(default_factory=dict, repr=False)
    last_backward: dict = field(default_factory=dict, repr=False)

    ensure_solver = TPFAProblem.ensure_solver
    solve_kw = TPFAProblem.solve_kw

    def device_inputs(self, device):
        """Loads and fixed flags as tensors on `device` (copied once)."""
        if self._dev.get("device") != device:
            f = torch.as_tensor(np.asarray(self.loads) if not torch.is_tensor(self.loads)
                                else self.loads, dtype=torch.float64).to(device).contiguous()
            fx = None
            if self.fixed is not None:
                fx = torch.as_tensor(np.asarray(self.fixed, dtype=np.uint8)).to(device)
            self._dev = dict(device=device, loads=f, fixed=fx)
        return self._dev["loads"], self._dev["fixed"]


class MsrsbQ1Solve(torch.autograd.Function):
    """u = MsrsbQ1Solve.apply(log_E, problem) with log_E a contiguous FP64
    CUDA tensor of one value per element; u has dim * #nodes values."""

    @staticmethod
    def forward(ctx, log_E, prob):
        if not (log_E.is_cuda and log_E.dtype == torch.float64):
            raise TypeError("log_E must be a CUDA float64 tensor")
        log_E = log_E.contiguous()
        dev = log_E.device.index or 0
        s = prob.ensure_solver(dev)
        f, fixed = prob.device_inputs(log_E.device)
        s.assemble_q1(prob.elems, prob.h, prob.nu, log_E, fixed)
        if not prob._coarse_set or s.nc is None:
            c = prob.coarse
            s.set_coarse(c["nc"], c["part"], c["prp"], c["pci"], c["interior"])
            prob._coarse_set = True
        b = s.setup_basis(max_iter=prob.basis_iters, fp32_basis=prob.fp32_basis,
                          warm_start=prob.warm_start)
        s.build_coarse()
        u = torch.zeros_like(f)
        info = s.solve(f, u, **prob.solve_kw())
        prob._version += 1
        prob.last_forward = dict(basis=b, solve=info)
        ctx.prob = prob
        ctx.version = prob._version
        ctx.save_for_backward(log_E, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        prob = ctx.prob
        if prob._version != ctx.version:
            raise RuntimeError("the solver was re-assembled since this forward; "
                               "run backward before the next forward on the same problem")
        log_E, u = ctx.saved_tensors
        s = prob.solver
        g = grad_u.contiguous().to(torch.float64)
        lam = torch.zeros_like(u)
        info = s.solve_transpose(g, lam, **prob.solve_kw())
        grad = torch.empty_like(log_E)
        s.q1_adjoint_grad(u, lam, grad)
        prob.last_backward = dict(solve=info)
        return grad, None
