"""ctypes binding of libmsrsb.so (argument marshalling only).

Every numerical step runs in the HIP library; this module converts Python
arguments (NumPy arrays, CPU or GPU torch tensors) into the plain pointers of
the C ABI declared in include/msrsb.h and turns status codes into
exceptions.  There is no fallback: without the built library nothing here
works.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsrsb.so")

HOST, DEVICE = 0, 1
SMOOTH_NONE, SMOOTH_JACOBI, SMOOTH_L1JACOBI, SMOOTH_ILU0, SMOOTH_SGS, SMOOTH_IC0 = 0, 1, 2, 3, 4, 5
KRYLOV_PCG, KRYLOV_GMRES, KRYLOV_RICHARDSON, KRYLOV_BICGSTAB = 0, 1, 2, 3
KRYLOV = {"pcg": KRYLOV_PCG, "gmres": KRYLOV_GMRES, "richardson": KRYLOV_RICHARDSON,
          "bicgstab": KRYLOV_BICGSTAB}
ORDER_NATURAL, ORDER_MULTICOLOR = 0, 1
ORDERING = {"natural": ORDER_NATURAL, "multicolor": ORDER_MULTICOLOR}
RESTRICT_GALERKIN, RESTRICT_MSFV = 0, 1
RESTRICTION = {"galerkin": RESTRICT_GALERKIN, "msfv": RESTRICT_MSFV}
FACTOR_AUTO, FACTOR_PIVOTED, FACTOR_CHOLESKY = 0, 1, 2
FACTOR = {"auto": FACTOR_AUTO, "pivoted": FACTOR_PIVOTED, "cholesky": FACTOR_CHOLESKY}
PHASES = ["filter", "init", "smooth", "rap", "factor", "solve", "solve_t", "grad", "assemble",
          "smoother_setup"]

STATUS = {0: "MSRSB_OK", -1: "MSRSB_E_ARG", -2: "MSRSB_E_STATE", -3: "MSRSB_E_HIP",
          -4: "MSRSB_E_NOMEM", -5: "MSRSB_E_BASIS_DIVERGED", -6: "MSRSB_E_COARSE_SINGULAR",
          -7: "MSRSB_E_BREAKDOWN", -8: "MSRSB_E_NOT_CONVERGED"}


class MsrsbError(RuntimeError):
    def __init__(self, code, msg, info=None):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))
        self.info = info


class BasisOpts(C.Structure):
    _fields_ = [("omega", C.c_double), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("check_every", C.c_int32), ("filter", C.c_int32), ("fp32_basis", C.c_int32),
                ("warm_start", C.c_int32)]


class BasisInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("e_it", C.c_double), ("max_rowsum_err", C.c_double),
                ("p_min", C.c_double), ("p_max", C.c_double)]


class CoarseOpts(C.Structure):
    _fields_ = [("restriction", C.c_int32), ("factor", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("krylov", C.c_int32), ("restart", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("pre_smoother", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_smoother", C.c_int32), ("post_sweeps", C.c_int32),
                ("fp32_smoother", C.c_int32), ("use_multiscale", C.c_int32),
                ("ordering", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("true_rel_res", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32)]


_P = C.c_void_p
_I32 = C.c_int32
_ST = C.c_int

# (name, restype, argtypes) for every entry point of include/msrsb.h
SIGNATURES = [
    ("msrsb_create", _ST, [C.POINTER(_P), C.c_int, _P]),
    ("msrsb_destroy", None, [_P]),
    ("msrsb_last_error", C.c_char_p, [_P]),
    ("msrsb_set_stream", _ST, [_P, _P]),
    ("msrsb_set_matrix", _ST, [_P, _I32, C.c_int64, _P, _P, _P, _I32, C.c_int]),
    ("msrsb_update_values", _ST, [_P, _P, C.c_int]),
    ("msrsb_get_matrix", _ST, [_P, _P, _P, _P, C.c_int]),
    ("msrsb_assemble_tpfa", _ST, [_P, _I32, _P, _P, _P, _P, _P, C.c_int]),
    ("msrsb_set_coarse", _ST, [_P, _I32, _P, _P, _P, _P, C.c_int]),
    ("msrsb_set_coarse_level", _ST, [_P, _I32, _I32, _P, _P, _P, _P, C.c_int]),
    ("msrsb_get_level", _ST, [_P, _I32, C.POINTER(_P)]),
    ("msrsb_setup_basis", _ST, [_P, C.POINTER(BasisOpts), C.POINTER(BasisInfo)]),
    ("msrsb_set_prolongation", _ST, [_P, _P, C.c_int]),
    ("msrsb_get_prolongation", _ST, [_P, _P, _P, _P, C.c_int]),
    ("msrsb_build_coarse", _ST, [_P, C.POINTER(CoarseOpts)]),
    ("msrsb_get_coarse_matrix", _ST, [_P, _P, C.c_int]),
    ("msrsb_apply_preconditioner", _ST, [_P, C.POINTER(SolveOpts), _P, _P, C.c_int]),
    ("msrsb_apply_preconditioner_noalloc", _ST, [_P, C.POINTER(SolveOpts), _P, _P]),
    ("msrsb_solve", _ST, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), C.c_int]),
    ("msrsb_solve_transpose", _ST,
     [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), C.c_int]),
    ("msrsb_tpfa_adjoint_grad", _ST, [_P, _P, _P, _P, _P, C.c_int]),
    ("msrsb_assemble_q1", _ST, [_P, _I32, _P, _P, C.c_double, _P, _P, C.c_int]),
    ("msrsb_q1_adjoint_grad", _ST, [_P, _P, _P, _P, C.c_int]),
    ("msrsb_get_timings", _ST, [_P, _P, _I32]),
]

_lib = None


def load():
    """Load libmsrsb.so (built by ``paper_1912_06934_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1912_06934_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _torch():
    try:
        import torch
        return torch
    except ImportError:  # pragma: no cover
        return None


def _ptr(x, dtype):
    """(pointer, where, keepalive) for a NumPy array or torch tensor of dtype."""
    if x is None:
        return None, None, None
    torch = _torch()
    if torch is not None and isinstance(x, torch.Tensor):
        tdt = {np.float64: torch.float64, np.int32: torch.int32, np.uint8: torch.uint8}[dtype]
        if x.dtype != tdt:
            raise TypeError(f"expected {tdt}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()), (DEVICE if x.is_cuda else HOST), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(C.c_void_p), HOST, a


def _where(*wheres):
    ws = {w for w in wheres if w is not None}
    if len(ws) > 1:
        raise ValueError("all buffers of one call must be on the host or all on the device")
    return ws.pop() if ws else HOST


class Msrsb:
    """One library context (one device, one stream)."""

    def __init__(self, device=0, stream=None):
        self._lib = load()
        torch = _torch()
        if stream is None and torch is not None and torch.cuda.is_available():
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        rc = self._lib.msrsb_create(C.byref(h), device, C.c_void_p(stream) if stream else None)
        if rc != 0:
            raise MsrsbError(rc, f"msrsb_create(device={device}) failed")
        self._h = h
        self._owned = True
        self.n = None
        self.nc = None
        self._levels = {}

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                self._lib.msrsb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what, info=None):
        if rc != 0:
            msg = self._lib.msrsb_last_error(self._h)
            raise MsrsbError(rc, f"{what}: {msg.decode() if msg else ''}", info)

    def set_stream(self, stream):
        self._check(self._lib.msrsb_set_stream(self._h, C.c_void_p(stream) if stream else None),
                    "set_stream")

    # -- matrix --
    def set_matrix(self, rowptr, col, val, block_size=1):
        prp, w0, k0 = _ptr(rowptr, np.int32)
        pci, w1, k1 = _ptr(col, np.int32)
        pv, w2, k2 = _ptr(val, np.float64)
        n = (len(rowptr) - 1)
        nnz = len(col)
        self._check(self._lib.msrsb_set_matrix(self._h, n, nnz, prp, pci, pv, block_size,
                                               _where(w0, w1, w2)), "set_matrix")
        self.n, self.nnz = n, nnz

    def update_values(self, val):
        pv, w, k = _ptr(val, np.float64)
        self._check(self._lib.msrsb_update_values(self._h, pv, w), "update_values")

    def get_matrix(self):
        rp = np.empty(self.n + 1, dtype=np.int32)
        rowptr_p = rp.ctypes.data_as(C.c_void_p)
        self._check(self._lib.msrsb_get_matrix(self._h, rowptr_p, None, None, HOST), "get_matrix")
        ci = np.empty(rp[-1], dtype=np.int32)
        va = np.empty(rp[-1])
        self._check(self._lib.msrsb_get_matrix(self._h, None, ci.ctypes.data_as(C.c_void_p),
                                               va.ctypes.data_as(C.c_void_p), HOST), "get_matrix")
        return rp, ci, va

    def assemble_tpfa(self, dims, h, log_k, bc, rhs_out=None):
        dim = len(dims)
        d = (C.c_int32 * 3)(*(list(dims) + [1] * (3 - dim)))
        hh = (C.c_double * 3)(*(list(h)[:3] + [1.0] * (3 - min(3, len(h)))))
        b = (C.c_double * 6)(*[float(x) for x in bc])
        pk, w0, k0 = _ptr(log_k, np.float64)
        pr, w1, k1 = _ptr(rhs_out, np.float64)
        self._check(self._lib.msrsb_assemble_tpfa(self._h, dim, d, hh, pk, b, pr, _where(w0, w1)),
                    "assemble_tpfa")
        self.n = int(np.prod(dims))
        if isinstance(rhs_out, np.ndarray) and rhs_out is not k1:
            rhs_out[...] = k1
        return rhs_out

    def assemble_q1(self, elems, h, nu, log_E, fixed=None):
        """Q1 elasticity matrix from log E per element (block size = dim)."""
        dim = len(elems)
        d = (C.c_int32 * 3)(*(list(elems) + [1] * (3 - dim)))
        hh = (C.c_double * 3)(*(list(h)[:dim] + [1.0] * (3 - dim)))
        pe, w0, k0 = _ptr(log_E, np.float64)
        pf, w1, k1 = _ptr(fixed, np.uint8)
        self._check(self._lib.msrsb_assemble_q1(self._h, dim, d, hh, float(nu), pe, pf,
                                                _where(w0, w1)), "assemble_q1")
        self.n = dim * int(np.prod([e + 1 for e in elems]))

    def q1_adjoint_grad(self, u, lam, grad):
        a = [_ptr(u, np.float64), _ptr(lam, np.float64), _ptr(grad, np.float64)]
        self._check(self._lib.msrsb_q1_adjoint_grad(self._h, a[0][0], a[1][0], a[2][0],
                                                    _where(*[x[1] for x in a])),
                    "q1_adjoint_grad")
        if isinstance(grad, np.ndarray) and grad is not a[2][2]:
            grad[...] = a[2][2]
        return grad

    # -- coarse --
    def set_coarse(self, nc, part, sup_rowptr, sup_col, interior):
        a = [_ptr(part, np.int32), _ptr(sup_rowptr, np.int32), _ptr(sup_col, np.int32),
             _ptr(interior, np.uint8)]
        self._check(self._lib.msrsb_set_coarse(self._h, int(nc), a[0][0], a[1][0], a[2][0],
                                               a[3][0], _where(*[x[1] for x in a])), "set_coarse")
        self.nc = int(nc)
        self.pnnz = len(sup_col)

    def set_coarse_level(self, level, nc, part, sup_rowptr, sup_col, interior):
        """Coarse space of level `level` >= 1 (multilevel MsRSB)."""
        a = [_ptr(part, np.int32), _ptr(sup_rowptr, np.int32), _ptr(sup_col, np.int32),
             _ptr(interior, np.uint8)]
        self._check(self._lib.msrsb_set_coarse_level(self._h, int(level), int(nc), a[0][0],
                                                     a[1][0], a[2][0], a[3][0],
                                                     _where(*[x[1] for x in a])),
                    "set_coarse_level")
        self._levels[int(level)] = (int(nc), len(sup_col))

    def level(self, level):
        """The context of level `level` (borrowed: owned by this one)."""
        h = C.c_void_p()
        self._check(self._lib.msrsb_get_level(self._h, int(level), C.byref(h)), "get_level")
        if level == 0:
            return self
        lv = Msrsb.__new__(Msrsb)
        lv._lib, lv._h, lv._owned, lv._levels = self._lib, h, False, {}
        lv.n = self.nc if level == 1 else self._levels[level - 1][0]
        lv.nc, lv.pnnz = self._levels[level]
        lv._parent = self                     # keeps the owner alive
        return lv

    def setup_basis(self, omega=2.0 / 3.0, max_iter=100, tol=-1.0, check_every=1, filter=True,
                    fp32_basis=False, warm_start=False):
        o = BasisOpts(omega, max_iter, tol, check_every, int(filter), int(fp32_basis),
                      int(warm_start))
        info = BasisInfo()
        rc = self._lib.msrsb_setup_basis(self._h, C.byref(o), C.byref(info))
        d = dict(iters=info.iters, e_it=info.e_it, max_rowsum_err=info.max_rowsum_err,
                 p_min=info.p_min, p_max=info.p_max)
        self._check(rc, "setup_basis", d)
        return d

    def set_prolongation(self, val):
        pv, w, k = _ptr(val, np.float64)
        self._check(self._lib.msrsb_set_prolongation(self._h, pv, w), "set_prolongation")

    def get_prolongation(self):
        rp = np.empty(self.n + 1, dtype=np.int32)
        ci = np.empty(self.pnnz, dtype=np.int32)
        va = np.empty(self.pnnz)
        self._check(self._lib.msrsb_get_prolongation(
            self._h, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
            va.ctypes.data_as(C.c_void_p), HOST), "get_prolongation")
        return rp, ci, va

    def build_coarse(self, restriction="galerkin", factor="auto"):
        o = CoarseOpts(RESTRICTION.get(restriction, restriction), FACTOR.get(factor, factor))
        self._check(self._lib.msrsb_build_coarse(self._h, C.byref(o)), "build_coarse")

    def get_coarse_matrix(self):
        m = np.empty((self.nc, self.nc))
        self._check(self._lib.msrsb_get_coarse_matrix(self._h, m.ctypes.data_as(C.c_void_p),
                                                      HOST), "get_coarse_matrix")
        return m

    # -- apply / solve --
    @staticmethod
    def solve_opts(krylov="pcg", restart=30, rtol=1e-8, max_iter=1000, pre=(0, 0), post=(0, 0),
                   fp32_smoother=False, use_multiscale=True, ordering="natural"):
        k = KRYLOV[krylov] if isinstance(krylov, str) else krylov
        od = ORDERING[ordering] if isinstance(ordering, str) else ordering
        return SolveOpts(k, restart, rtol, max_iter, pre[0], pre[1], post[0], post[1],
                         int(fp32_smoother), int(use_multiscale), od)

    def apply(self, v, z, **kw):
        o = self.solve_opts(**kw)
        pv, w0, k0 = _ptr(v, np.float64)
        pz, w1, k1 = _ptr(z, np.float64)
        self._check(self._lib.msrsb_apply_preconditioner(self._h, C.byref(o), pv, pz,
                                                         _where(w0, w1)), "apply")
        if isinstance(z, np.ndarray) and z is not k1:
            z[...] = k1
        return z

    def apply_noalloc(self, v, z, **kw):
        """msrsb_apply_preconditioner_noalloc: v and z are device tensors; the
        call only queues work on the context's stream."""
        o = self.solve_opts(**kw)
        pv, w0, k0 = _ptr(v, np.float64)
        pz, w1, k1 = _ptr(z, np.float64)
        if _where(w0, w1) != DEVICE:
            raise ValueError("apply_noalloc takes device tensors")
        self._check(self._lib.msrsb_apply_preconditioner_noalloc(self._h, C.byref(o), pv, pz),
                    "apply_noalloc")
        return z

    def _solve(self, fn, what, f, u, history_cap=0, **kw):
        o = self.solve_opts(**kw)
        pf, w0, k0 = _ptr(f, np.float64)
        pu, w1, k1 = _ptr(u, np.float64)
        hist = np.zeros(max(history_cap, 1))
        info = SolveInfo(0, 0.0, hist.ctypes.data_as(C.POINTER(C.c_double)), history_cap)
        rc = fn(self._h, pf, pu, C.byref(o), C.byref(info), _where(w0, w1))
        if isinstance(u, np.ndarray) and u is not k1:
            u[...] = k1
        d = dict(iters=info.iters, true_rel_res=info.true_rel_res,
                 history=hist[:min(info.iters + 1, history_cap)].copy())
        self._check(rc, what, d)
        return d

    def solve(self, f, u, **kw):
        return self._solve(self._lib.msrsb_solve, "solve", f, u, **kw)

    def solve_transpose(self, g, lam, **kw):
        return self._solve(self._lib.msrsb_solve_transpose, "solve_transpose", g, lam, **kw)

    def tpfa_adjoint_grad(self, log_k, p, lam, grad):
        a = [_ptr(log_k, np.float64), _ptr(p, np.float64), _ptr(lam, np.float64),
             _ptr(grad, np.float64)]
        self._check(self._lib.msrsb_tpfa_adjoint_grad(self._h, a[0][0], a[1][0], a[2][0],
                                                      a[3][0], _where(*[x[1] for x in a])),
                    "tpfa_adjoint_grad")
        if isinstance(grad, np.ndarray) and grad is not a[3][2]:
            grad[...] = a[3][2]
        return grad

    def timings(self):
        ms = np.zeros(len(PHASES))
        self._check(self._lib.msrsb_get_timings(self._h, ms.ctypes.data_as(C.c_void_p),
                                                len(PHASES)), "get_timings")
        return dict(zip(PHASES, ms.tolist()))
