"""Enhanced MsRSB preconditioning on MI355X (gfx950).

Method: Bosma, Klevtsov, Moyner, Castelletto, arXiv:1912.06934.  The
numerical work runs in the HIP library ``libmsrsb.so`` (C ABI in
``include/msrsb.h``); this package only marshals arguments:

  Msrsb                 one library context (set_matrix / assemble_tpfa,
                        set_coarse, setup_basis, build_coarse, apply, solve,
                        solve_transpose, tpfa_adjoint_grad, assemble_q1,
                        q1_adjoint_grad)
  MsrsbTPFASolve        torch.autograd.Function: log-permeability -> pressure,
                        with the hand-written adjoint in backward
  MsrsbQ1Solve          torch.autograd.Function: log Young's modulus ->
                        displacement (Q1 elasticity), likewise
"""
from ._binding import (Msrsb, MsrsbError, load, HOST, DEVICE, SMOOTH_NONE, SMOOTH_JACOBI,
                       SMOOTH_L1JACOBI, SMOOTH_ILU0, SMOOTH_SGS, SMOOTH_IC0, KRYLOV_PCG,
                       KRYLOV_GMRES, KRYLOV_RICHARDSON, KRYLOV_BICGSTAB, ORDER_NATURAL,
                       ORDER_MULTICOLOR, RESTRICT_GALERKIN, RESTRICT_MSFV, FACTOR_AUTO,
                       FACTOR_PIVOTED, FACTOR_CHOLESKY, PHASES, LIB_PATH)
from .autograd import MsrsbTPFASolve, TPFAProblem, MsrsbQ1Solve, Q1Problem

__all__ = ["Msrsb", "MsrsbError", "load", "HOST", "DEVICE", "SMOOTH_NONE", "SMOOTH_JACOBI",
           "SMOOTH_L1JACOBI", "SMOOTH_ILU0", "SMOOTH_SGS", "SMOOTH_IC0", "KRYLOV_PCG",
           "KRYLOV_GMRES", "KRYLOV_RICHARDSON", "KRYLOV_BICGSTAB", "ORDER_NATURAL",
           "ORDER_MULTICOLOR", "RESTRICT_GALERKIN", "RESTRICT_MSFV", "FACTOR_AUTO",
           "FACTOR_PIVOTED", "FACTOR_CHOLESKY", "PHASES", "LIB_PATH",
           "MsrsbTPFASolve", "TPFAProblem", "MsrsbQ1Solve", "Q1Problem"]
