"""ctypes view of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and this package never
imports the product.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB, build

ILU0, MILU0, ILUT = 0, 1, 2
BJ, SCHUR, RAP = 0, 1, 2
PIVOT_ERROR, PIVOT_PERTURB = 0, 1
OK, NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_CSR, ERR_ZERO_PIVOT, ERR_OOM, ERR_BREAKDOWN = -1, -2, -3, -4, -6

X = dict(perm=0, iperm=1, iface=2, offsets=3, LB=10, UB=13, DB=16, Z=17, W=20, LS=23, US=26, DS=29,
         Coff=30, lev_LB=40, lev_UB=41, lev_LS=42, lev_US=43, Stilde=50)


_CSR_BLOCKS = ("LB", "UB", "Z", "W", "LS", "US", "Coff", "Stilde")


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("interior_fact", C.c_int32), ("interface_fact", C.c_int32),
                ("droptol", C.c_double), ("lfil", C.c_int32), ("inner_iters", C.c_int32),
                ("inner_rtol", C.c_double), ("pivot_mode", C.c_int32), ("pivot_tol", C.c_double),
                ("smooth_fact", C.c_int32)]


class _Res(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("final_relres", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_validate.argtypes = [vp]
        L.orc_classify.argtypes = [vp, vp, i32, vp]
        L.orc_permutation.argtypes = [i64, vp, i32, vp, vp, vp, vp]
        L.orc_spmv.argtypes = [vp, vp, vp]
        L.orc_spmv.restype = None
        L.orc_residual.argtypes = [vp, vp, vp, vp]
        L.orc_residual.restype = None
        L.orc_levels.argtypes = [i64, vp, vp, C.c_int, i64, i64, vp]
        L.orc_levels.restype = None
        L.orc_factor.argtypes = [vp, i64, i32, d, i32, i32, d, C.POINTER(vp), C.POINTER(i64)]
        L.orc_fact_get.argtypes = [vp, C.c_int, C.c_int, C.POINTER(vp), C.POINTER(i64)]
        L.orc_fact_free.argtypes = [vp]
        L.orc_fact_free.restype = None
        L.orc_setup.argtypes = [vp, vp, i32, vp, C.POINTER(vp), C.POINTER(i64)]
        L.orc_apply.argtypes = [vp, vp, vp]
        L.orc_apply.restype = None
        L.orc_rap_matvec.argtypes = [vp, vp, vp]
        L.orc_rap_matvec.restype = None
        L.orc_fgmres.argtypes = [vp, vp, vp, vp, d, i32, i32, vp, vp]
        L.orc_gmres.argtypes = [vp, vp, vp, vp, d, i32, i32, vp, vp]
        L.orc_free.argtypes = [vp]
        L.orc_free.restype = None
        L.orc_export.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle error {code} {msg}")
        self.code = code


@dataclass
class Options:
    method: int = BJ
    interior_fact: int = ILU0
    interface_fact: int = ILU0
    droptol: float = 0.0
    lfil: int = -1
    inner_iters: int = 3
    inner_rtol: float = 0.0
    pivot_mode: int = PIVOT_ERROR
    pivot_tol: float = 0.0
    smooth_fact: int = ILU0

    def c(self):
        return _Opts(self.method, self.interior_fact, self.interface_fact, self.droptol, self.lfil,
                     self.inner_iters, self.inner_rtol, self.pivot_mode, self.pivot_tol, self.smooth_fact)


class _Mat:
    """Keeps contiguous copies alive for the lifetime of the C view."""

    def __init__(self, A):
        self.rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
        self.ci = np.ascontiguousarray(A.col, dtype=np.int32)
        self.v = np.ascontiguousarray(A.val, dtype=np.float64)
        self.n = int(A.n)
        self.c = _CSR(self.n, _p(self.rp), _p(self.ci), _p(self.v))

    @property
    def ref(self):
        return C.byref(self.c)


def validate(A) -> int:
    m = _Mat(A)
    return lib().orc_validate(m.ref)


def spmv(A, x):
    m = _Mat(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(m.n)
    lib().orc_spmv(m.ref, _p(x), _p(y))
    return y


def residual(A, b, x):
    m = _Mat(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = np.empty(m.n)
    lib().orc_residual(m.ref, _p(b), _p(x), _p(r))
    return r


def classify(A, part, nparts):
    m = _Mat(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    out = np.empty(m.n, dtype=np.uint8)
    rc = lib().orc_classify(m.ref, _p(part), nparts, _p(out))
    if rc:
        raise OracleError(rc)
    return out


def permutation(n, part, nparts, iface):
    part = np.ascontiguousarray(part, dtype=np.int32)
    iface = np.ascontiguousarray(iface, dtype=np.uint8)
    perm = np.empty(n, np.int32)
    iperm = np.empty(n, np.int32)
    off = np.empty(2 * nparts + 2, np.int64)
    rc = lib().orc_permutation(n, _p(part), nparts, _p(iface), _p(perm), _p(iperm), _p(off))
    if rc:
        raise OracleError(rc)
    return perm, iperm, off


def levels(rp, ci, lower, lo=0, hi=None):
    rp = np.ascontiguousarray(rp, np.int64)
    ci = np.ascontiguousarray(ci, np.int32)
    n = len(rp) - 1
    hi = n if hi is None else hi
    out = np.empty(n, np.int32)
    lib().orc_levels(n, _p(rp), _p(ci), 1 if lower else 0, lo, hi, _p(out))
    return out


def _copy(ptr, length, dtype):
    if length == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    buf = (C.c_char * (length * np.dtype(dtype).itemsize)).from_address(ptr)
    return np.frombuffer(buf, dtype=dtype).copy()


def factor(M, nfull=None, method=ILU0, droptol=0.0, lfil=-1, pivot_mode=PIVOT_ERROR, pivot_tol=0.0):
    """Row-wise factor of M: rows < nfull full ILU rows, rows >= nfull partial.

    Returns dict with L, U, R as (row_ptr, col, val) and D.
    """
    m = _Mat(M)
    nfull = m.n if nfull is None else nfull
    h = C.c_void_p()
    bad = C.c_int64(-1)
    rc = lib().orc_factor(m.ref, nfull, method, droptol, lfil, pivot_mode, pivot_tol, C.byref(h), C.byref(bad))
    if rc:
        raise OracleError(rc, f"row {bad.value}")
    out = {}
    try:
        for name, part in (("L", 0), ("U", 1), ("R", 2)):
            arrs = []
            for field, dt in ((0, np.int64), (1, np.int32), (2, np.float64)):
                ptr, ln = C.c_void_p(), C.c_int64()
                lib().orc_fact_get(h, part, field, C.byref(ptr), C.byref(ln))
                arrs.append(_copy(ptr.value, ln.value, dt))
            out[name] = tuple(arrs)
        ptr, ln = C.c_void_p(), C.c_int64()
        lib().orc_fact_get(h, 3, 2, C.byref(ptr), C.byref(ln))
        out["D"] = _copy(ptr.value, ln.value, np.float64)
    finally:
        lib().orc_fact_free(h)
    return out


class Precond:
    """Oracle preconditioner; same call shapes as the product on host arrays."""

    def __init__(self, A, part=None, nparts=1, opts: Options | None = None, **kw):
        self.opts = opts or Options(**kw)
        self._m = _Mat(A)
        self.n = self._m.n
        self._part = None if part is None else np.ascontiguousarray(part, np.int32)
        self.nparts = nparts
        h = C.c_void_p()
        bad = C.c_int64(-1)
        o = self.opts.c()
        rc = lib().orc_setup(self._m.ref, _p(self._part), nparts, C.byref(o), C.byref(h), C.byref(bad))
        if rc:
            raise OracleError(rc, f"row {bad.value}")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def apply(self, r):
        r = np.ascontiguousarray(r, np.float64)
        z = np.empty(self.n)
        lib().orc_apply(self._h, _p(r), _p(z))
        return z

    def rap_matvec(self, v):
        """R A P v on the interface unknowns (multiplicative method only)."""
        v = np.ascontiguousarray(v, np.float64)
        out = np.empty(v.size)
        lib().orc_rap_matvec(self._h, _p(v), _p(out))
        return out

    def export(self, what):
        code = X[what] if isinstance(what, str) else what
        ptr, ln = C.c_void_p(), C.c_int64()
        rc = lib().orc_export(self._h, code, C.byref(ptr), C.byref(ln))
        if rc:
            raise OracleError(rc)
        if code in (X["perm"], X["iperm"], X["lev_LB"], X["lev_UB"], X["lev_LS"], X["lev_US"]):
            return _copy(ptr.value, ln.value, np.int32)
        if code == X["iface"]:
            return _copy(ptr.value, ln.value, np.uint8)
        if code == X["offsets"]:
            return _copy(ptr.value, ln.value, np.int64)
        if code in (X["DB"], X["DS"]):
            return _copy(ptr.value, ln.value, np.float64)
        base = max(v for k, v in X.items() if v <= code and k in _CSR_BLOCKS)
        return _copy(ptr.value, ln.value, (np.int64, np.int32, np.float64)[code - base])

    def csr(self, name):
        b = X[name]
        return self.export(b), self.export(b + 1), self.export(b + 2)


def fgmres(A, P: Precond, b, x0=None, rtol=1e-8, restart=30, maxit=1000, history=False):
    """Flexible GMRES(restart), right preconditioned (Section 4.1)."""
    return _krylov(lib().orc_fgmres, A, P, b, x0, rtol, restart, maxit, history)


def gmres(A, P: Precond, b, x0=None, rtol=1e-8, restart=20, maxit=1000, history=False):
    """GMRES(restart), right preconditioned with the fixed P (the batched systems)."""
    return _krylov(lib().orc_gmres, A, P, b, x0, rtol, restart, maxit, history)


def _krylov(fn, A, P, b, x0, rtol, restart, maxit, history):
    m = _Mat(A)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(m.n) if x0 is None else np.array(x0, dtype=np.float64)
    res = _Res()
    hist = np.full(maxit + 1, np.nan) if history else None
    rc = fn(m.ref, P._h, _p(b), _p(x), rtol, restart, maxit, C.byref(res), _p(hist))
    if rc < 0:
        raise OracleError(rc)
    out = dict(x=x, iterations=res.iterations, converged=bool(res.converged), relres=res.final_relres, rc=rc)
    if history:
        out["history"] = hist[: res.iterations + 1]
    return out
