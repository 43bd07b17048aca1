"""ctypes shim over the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the HIP path; both sides receive the same inputs from
``synth``.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_SING, E_BREAK, E_NOCONV = 0, -1, -6, -7, -8
SMOOTHERS = {"none": 0, "jacobi": 1, "l1jacobi": 2, "ilu0": 3, "sgs": 4, "ic0": 5}
ORDERINGS = {"natural": 0, "multicolor": 1}
RESTRICTIONS = {"galerkin": 0, "msfv": 1}


def build(force=True):
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_I = C.c_int
_D = C.c_double
_P = C.c_void_p


class Prec(C.Structure):
    _fields_ = [("n", _I), ("rp", _P), ("ci", _P), ("a", _P), ("nc", _I),
                ("prp", _P), ("pci", _P), ("pv", _P), ("lu", _P), ("piv", _P),
                ("lu_trans", _I), ("use_ms", _I), ("pre_kind", _I),
                ("pre_sweeps", _I), ("post_kind", _I), ("post_sweeps", _I),
                ("order", _P), ("brp", _P), ("bci", _P), ("ba", _P), ("ilu", _P),
                ("ic", _P), ("part", _P), ("next", _P)]


def _declare(L):
    L.orc_threads.argtypes = []
    L.orc_filter_jacobi.argtypes = [_I, _P, _P, _P, _I, _I, _D, _P, _P]
    L.orc_init_basis.argtypes = [_I, _P, _P, _P, _P]
    L.orc_smooth_step.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.orc_basis.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P, _I, _D, _I, _P, _P, _P]
    L.orc_rap.argtypes = [_I, _P, _P, _P, _I, _P, _P, _P, _P]
    L.orc_lu.argtypes = [_I, _P, _P]
    L.orc_lu_solve.argtypes = [_I, _P, _P, _P, _I]
    L.orc_lu_solve.restype = None
    L.orc_ilu0.argtypes = [_I, _P, _P, _P, _P]
    L.orc_ic0.argtypes = [_I, _P, _P, _P, _P]
    L.orc_color.argtypes = [_I, _P, _P, _P]
    L.orc_color_order.argtypes = [_I, _P, _I, _P]
    L.orc_color_order.restype = None
    L.orc_permute.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P]
    L.orc_richardson.argtypes = [C.POINTER(Prec), _P, _P, _D, _I, _P, _P, _P, _I]
    L.orc_bicgstab.argtypes = [C.POINTER(Prec), _P, _P, _D, _I, _P, _P, _P, _I]
    L.orc_rap_pg.argtypes = [_I, _P, _P, _P, _I, _P, _P, _P, _P, _P]
    L.orc_apply.argtypes = [C.POINTER(Prec), _P, _P]
    L.orc_pcg.argtypes = [C.POINTER(Prec), _P, _P, _D, _I, _P, _P, _P, _I]
    L.orc_gmres.argtypes = [C.POINTER(Prec), _P, _P, _I, _D, _I, _P, _P, _P, _I]
    L.orc_tpfa.argtypes = [_I, _I, _I, _I, _D, _D, _D, _P, _P, _P, _P, _P, _P]
    L.orc_tpfa_grad.argtypes = [_I, _I, _I, _I, _D, _D, _D, _P, _P, _P, _P, _P]
    L.orc_q1_grad.argtypes = [_I, _P, _P, _D, _P, _P, _P, _P, _P]


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


# ----------------------------------------------------------------------------
# step-level wrappers
# ----------------------------------------------------------------------------

def threads():
    """OpenMP threads used by the oracle's parallel loops."""
    return int(lib().orc_threads())


def filter_jacobi(rp, ci, a, bs=1, filt=True, omega=2.0 / 3.0):
    """J = I - omega Dhat^{-1} Ghat on A's pattern, and Dhat."""
    rp, ci, a = _i32(rp), _i32(ci), _f64(a)
    n = rp.size - 1
    jv = np.empty_like(a)
    dh = np.empty(n)
    _check(lib().orc_filter_jacobi(n, _p(rp), _p(ci), _p(a), bs, int(filt), omega,
                                   _p(jv), _p(dh)), "filter_jacobi")
    return jv, dh


def init_basis(prp, pci, part):
    prp, pci, part = _i32(prp), _i32(pci), _i32(part)
    pv = np.empty(pci.size)
    _check(lib().orc_init_basis(prp.size - 1, _p(prp), _p(pci), _p(part), _p(pv)),
           "init_basis")
    return pv


def smooth_step(rp, ci, jv, prp, pci, pv, interior):
    rp, ci, jv, prp, pci, pv = _i32(rp), _i32(ci), _f64(jv), _i32(prp), _i32(pci), _f64(pv)
    interior = np.ascontiguousarray(interior, dtype=np.uint8)
    out = np.empty_like(pv)
    e = C.c_double()
    _check(lib().orc_smooth_step(rp.size - 1, _p(rp), _p(ci), _p(jv), _p(prp), _p(pci),
                                 _p(pv), _p(out), _p(interior), C.byref(e)), "smooth_step")
    return out, e.value


def basis(rp, ci, jv, prp, pci, pv0, interior, kmax=100, tol=-1.0, nit=1):
    """Alg. 1 from the initial (or warm) P pv0.  Returns (P values, iterations,
    last e_it, e_it history with -1 where it was not computed)."""
    rp, ci, jv, prp, pci = _i32(rp), _i32(ci), _f64(jv), _i32(prp), _i32(pci)
    pv = np.array(pv0, dtype=np.float64, copy=True)
    interior = np.ascontiguousarray(interior, dtype=np.uint8)
    it, el = C.c_int(), C.c_double()
    hist = np.full(max(kmax, 1), -1.0)
    _check(lib().orc_basis(rp.size - 1, _p(rp), _p(ci), _p(jv), _p(prp), _p(pci), _p(pv),
                           _p(interior), kmax, tol, nit, C.byref(it), C.byref(el), _p(hist)),
           "basis")
    return pv, it.value, el.value, hist[:it.value]


def rap(rp, ci, a, nc, prp, pci, pv):
    rp, ci, a, prp, pci, pv = _i32(rp), _i32(ci), _f64(a), _i32(prp), _i32(pci), _f64(pv)
    ac = np.empty((nc, nc))
    _check(lib().orc_rap(rp.size - 1, _p(rp), _p(ci), _p(a), nc, _p(prp), _p(pci), _p(pv),
                         _p(ac)), "rap")
    return ac


def lu(ac):
    m = np.array(ac, dtype=np.float64, copy=True, order="C")
    piv = np.empty(m.shape[0], dtype=np.int32)
    _check(lib().orc_lu(m.shape[0], _p(m), _p(piv)), "lu")
    return m, piv


def lu_solve(lu_, piv, b, trans=False):
    x = np.array(b, dtype=np.float64, copy=True)
    lib().orc_lu_solve(lu_.shape[0], _p(lu_), _p(piv), _p(x), int(trans))
    return x


def ilu0(rp, ci, a):
    rp, ci, a = _i32(rp), _i32(ci), _f64(a)
    out = np.empty_like(a)
    _check(lib().orc_ilu0(rp.size - 1, _p(rp), _p(ci), _p(a), _p(out)), "ilu0")
    return out


def ic0(rp, ci, a):
    """IC(0) factor L of a symmetric matrix, on its pattern (zeros above the
    diagonal)."""
    rp, ci, a = _i32(rp), _i32(ci), _f64(a)
    out = np.empty_like(a)
    _check(lib().orc_ic0(rp.size - 1, _p(rp), _p(ci), _p(a), _p(out)), "ic0")
    return out


def color(rp, ci):
    """First-fit colouring in ascending row order on the symmetrised
    pattern: (colour per row, number of colours)."""
    rp, ci = _i32(rp), _i32(ci)
    col = np.empty(rp.size - 1, dtype=np.int32)
    nc = lib().orc_color(rp.size - 1, _p(rp), _p(ci), _p(col))
    if nc < 0:
        raise OracleError(nc, "color")
    return col, int(nc)


def sweep_order(rp, ci, ordering):
    """order[k] = k-th row visited by the triangular smoothers."""
    n = rp.size - 1
    if ORDERINGS.get(ordering, ordering) == 0:
        return np.arange(n, dtype=np.int32)
    col, ncol = color(rp, ci)
    order = np.empty(n, dtype=np.int32)
    lib().orc_color_order(n, _p(col), ncol, _p(order))
    return order


def permute(rp, ci, a, order):
    """B = Q A Q^T for the given order (CSR, columns sorted)."""
    rp, ci, a, order = _i32(rp), _i32(ci), _f64(a), _i32(order)
    brp = np.empty_like(rp)
    bci = np.empty_like(ci)
    ba = np.empty_like(a)
    _check(lib().orc_permute(rp.size - 1, _p(rp), _p(ci), _p(a), _p(order), _p(brp), _p(bci),
                             _p(ba)), "permute")
    return brp, bci, ba


def rap_pg(rp, ci, a, nc, part, prp, pci, pv):
    """Petrov-Galerkin (MsFV) coarse operator R A P with R the block indicator."""
    rp, ci, a, part = _i32(rp), _i32(ci), _f64(a), _i32(part)
    prp, pci, pv = _i32(prp), _i32(pci), _f64(pv)
    ac = np.empty((nc, nc))
    _check(lib().orc_rap_pg(rp.size - 1, _p(rp), _p(ci), _p(a), nc, _p(part), _p(prp),
                            _p(pci), _p(pv), _p(ac)), "rap_pg")
    return ac


def tpfa(dims, h, logk, bc):
    """TPFA matrix (rp, ci, val) and right-hand side for a 2D or 3D grid."""
    dim = len(dims)
    nx, ny = dims[0], dims[1]
    nz = dims[2] if dim == 3 else 1
    n = nx * ny * nz
    logk = _f64(logk)
    bc = _f64(bc)
    rp = np.empty(n + 1, dtype=np.int32)
    ci = np.empty(7 * n, dtype=np.int32)
    val = np.empty(7 * n)
    rhs = np.empty(n)
    hz = h[2] if len(h) > 2 else 1.0
    _check(lib().orc_tpfa(dim, nx, ny, nz, h[0], h[1], hz, _p(logk), _p(bc), _p(rp), _p(ci),
                          _p(val), _p(rhs)), "tpfa")
    nnz = rp[-1]
    return rp, ci[:nnz].copy(), val[:nnz].copy(), rhs


def tpfa_grad(dims, h, logk, bc, p, lam):
    dim = len(dims)
    nx, ny = dims[0], dims[1]
    nz = dims[2] if dim == 3 else 1
    g = np.empty(nx * ny * nz)
    hz = h[2] if len(h) > 2 else 1.0
    _check(lib().orc_tpfa_grad(dim, nx, ny, nz, h[0], h[1], hz, _p(_f64(logk)), _p(_f64(bc)),
                               _p(_f64(p)), _p(_f64(lam)), _p(g)), "tpfa_grad")
    return g


def q1_grad(elems, h, nu, logE, fixed, u, lam):
    """dJ/dlog E per element for Q1 elasticity, given u and the adjoint."""
    dim = len(elems)
    el = _i32(list(elems) + [1] * (3 - dim))
    hh = _f64(list(h)[:dim] + [1.0] * (3 - dim))
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    g = np.zeros(int(np.prod(elems)))
    _check(lib().orc_q1_grad(dim, _p(el), _p(hh), float(nu), _p(_f64(logE)), _p(fx),
                             _p(_f64(u)), _p(_f64(lam)), _p(g)), "q1_grad")
    return g


def transpose_csr(rp, ci, a):
    """Plain CSR transpose (columns of the result sorted ascending)."""
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    order = np.lexsort((rows, ci))
    trp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(trp, ci + 1, 1)
    trp = np.cumsum(trp).astype(np.int32)
    return trp, rows[order].astype(np.int32), np.asarray(a)[order]


# ----------------------------------------------------------------------------
# the whole method: setup (Alg. 2) and solve (Alg. 4 inside a Krylov method)
# ----------------------------------------------------------------------------

class Msrsb:
    """Oracle counterpart of the library's set_matrix / set_coarse /
    setup_basis / build_coarse / solve sequence."""

    def __init__(self, rp, ci, a, block_size=1):
        self.rp, self.ci, self.a = _i32(rp), _i32(ci), _f64(a)
        self.n = self.rp.size - 1
        self.bs = block_size
        self.pv = None
        self._fact = {}     # (ordering, kind) -> factors of B
        self._perm = {}     # ordering -> (order, B)
        self._t = None
        self.restriction = "galerkin"
        self.levels = {}    # level >= 1 -> coarse space of that level's unknowns
        self.child = None   # the next level (multilevel), built on A_c

    def set_coarse(self, nc, part, prp, pci, interior):
        self.nc = int(nc)
        self.part, self.prp, self.pci = _i32(part), _i32(prp), _i32(pci)
        self.interior = np.ascontiguousarray(interior, dtype=np.uint8)

    def set_coarse_level(self, level, nc, part, prp, pci, interior):
        """Coarse space of level `level` >= 1 (a partition of the level's
        unknowns, the coarse nodes of the level above, with its supports):
        A_c of the level above is then not factored but gets its own
        enhanced MsRSB preconditioner (multilevel)."""
        if level < 1:
            raise ValueError("level must be >= 1")
        self.levels[level] = (int(nc), _i32(part), _i32(prp), _i32(pci),
                              np.ascontiguousarray(interior, dtype=np.uint8))

    def setup_basis(self, omega=2.0 / 3.0, kmax=100, tol=-1.0, nit=1, filt=True,
                    warm_start=False):
        self._basis_opts = dict(omega=omega, kmax=kmax, tol=tol, nit=nit, filt=filt)
        self.jv, self.dhat = filter_jacobi(self.rp, self.ci, self.a, self.bs, filt, omega)
        if not warm_start or self.pv is None:
            self.pv = init_basis(self.prp, self.pci, self.part)
        self.pv, self.basis_iters, self.eit, self.eit_hist = basis(
            self.rp, self.ci, self.jv, self.prp, self.pci, self.pv, self.interior,
            kmax, tol, nit)
        return self.pv

    def build_coarse(self, restriction="galerkin"):
        """Alg. 2: R = P^T (Galerkin) or the block indicator (Petrov-Galerkin,
        MsFV), A_c = R A P, and its LU."""
        self.restriction = restriction
        if restriction == "galerkin":
            self.ac = rap(self.rp, self.ci, self.a, self.nc, self.prp, self.pci, self.pv)
        elif restriction == "msfv":
            self.ac = rap_pg(self.rp, self.ci, self.a, self.nc, self.part, self.prp, self.pci,
                             self.pv)
        else:
            raise ValueError(restriction)
        self.child = None
        if 1 in self.levels:
            # the next level: A_c as a sparse matrix (its nonzeros and the
            # diagonal), its own coarse space, basis and coarse operator
            nc = self.nc
            mask = (self.ac != 0.0) | np.eye(nc, dtype=bool)
            rows, cols = np.nonzero(mask)
            crp = np.zeros(nc + 1, dtype=np.int32)
            np.add.at(crp, rows + 1, 1)
            crp = np.cumsum(crp).astype(np.int32)
            child = Msrsb(crp, cols.astype(np.int32), self.ac[rows, cols])
            child.set_coarse(*self.levels[1])
            child.levels = {lv - 1: spec for lv, spec in self.levels.items() if lv > 1}
            child.setup_basis(**self._basis_opts)
            child.build_coarse()
            self.child = child
            self.lu, self.piv = None, None
        else:
            self.lu, self.piv = lu(self.ac)
        return self.ac

    def _order(self, ordering):
        if ordering not in self._perm:
            order = sweep_order(self.rp, self.ci, ordering)
            if ORDERINGS.get(ordering, ordering) == 0:
                self._perm[ordering] = (None, (self.rp, self.ci, self.a))
            else:
                self._perm[ordering] = (order, permute(self.rp, self.ci, self.a, order))
        return self._perm[ordering]

    def _factor(self, ordering, kind):
        key = (ordering, kind)
        if key not in self._fact:
            _, (brp, bci, ba) = self._order(ordering)
            self._fact[key] = ilu0(brp, bci, ba) if kind == 3 else ic0(brp, bci, ba)
        return self._fact[key]

    def _prec(self, pre, post, use_ms, transpose=False, ordering="natural"):
        kinds = (pre[0], post[0])
        if transpose:
            if self._t is None:
                self._t = transpose_csr(self.rp, self.ci, self.a)
            rp, ci, a = self._t
            pre, post = post, pre
            if self.restriction != "galerkin" and use_ms:
                raise OracleError(E_ARG, "transposed Petrov-Galerkin preconditioner")
        else:
            rp, ci, a = self.rp, self.ci, self.a
        order, brp, bci, ba, ilu, ic = None, None, None, None, None, None
        if any(k >= 3 for k in kinds):
            if transpose:
                raise OracleError(E_ARG, "transposed triangular smoother")
            order, (brp, bci, ba) = self._order(ordering)
            if 3 in kinds:
                ilu = self._factor(ordering, 3)
            if 5 in kinds:
                ic = self._factor(ordering, 5)
        part = self.part if self.restriction == "msfv" else None
        nxt = None
        keep = [rp, ci, a, order, brp, bci, ba, ilu, ic, part]
        if self.child is not None and use_ms:
            # the next level's two-stage preconditioner with the same smoothers
            cm, ckeep = self.child._prec(pre if not transpose else post,
                                         post if not transpose else pre, True, transpose,
                                         ordering)
            keep += [cm, ckeep]
            nxt = C.cast(C.pointer(cm), C.c_void_p)
        m = Prec(self.n, _p(rp), _p(ci), _p(a), self.nc, _p(self.prp), _p(self.pci),
                 _p(self.pv), _p(self.lu), _p(self.piv), int(transpose), int(use_ms),
                 pre[0], pre[1], post[0], post[1], _p(order), _p(brp), _p(bci), _p(ba),
                 _p(ilu), _p(ic), _p(part), nxt)
        return m, keep

    def apply(self, v, pre=(0, 0), post=(0, 0), use_ms=True, transpose=False,
              ordering="natural"):
        m, keep = self._prec(pre, post, use_ms, transpose, ordering)
        z = np.empty(self.n)
        v = _f64(v)
        _check(lib().orc_apply(C.byref(m), _p(v), _p(z)), "apply")
        return z

    def solve(self, f, x0=None, krylov="pcg", restart=30, rtol=1e-8, maxit=1000,
              pre=(0, 0), post=(0, 0), use_ms=True, transpose=False, hist_cap=0,
              ordering="natural"):
        m, keep = self._prec(pre, post, use_ms, transpose, ordering)
        f = _f64(f)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it, tr = C.c_int(), C.c_double()
        hist = np.zeros(max(hist_cap, 1))
        if krylov == "pcg":
            rc = lib().orc_pcg(C.byref(m), _p(f), _p(x), rtol, maxit, C.byref(it),
                               C.byref(tr), _p(hist), hist_cap)
        elif krylov == "gmres":
            rc = lib().orc_gmres(C.byref(m), _p(f), _p(x), restart, rtol, maxit, C.byref(it),
                                 C.byref(tr), _p(hist), hist_cap)
        elif krylov == "richardson":
            rc = lib().orc_richardson(C.byref(m), _p(f), _p(x), rtol, maxit, C.byref(it),
                                      C.byref(tr), _p(hist), hist_cap)
        elif krylov == "bicgstab":
            rc = lib().orc_bicgstab(C.byref(m), _p(f), _p(x), rtol, maxit, C.byref(it),
                                    C.byref(tr), _p(hist), hist_cap)
        else:
            raise ValueError(krylov)
        return dict(x=x, iters=it.value, true_rel=tr.value, status=rc,
                    hist=hist[:min(it.value + 1, hist_cap)])
