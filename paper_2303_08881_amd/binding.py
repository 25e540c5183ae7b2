"""ctypes binding of the C ABI in include/schurilu.h.

Names follow the C entry points: ``setup`` -> ilu_setup, ``Precond.apply`` ->
ilu_apply, ``Precond.rap_matvec`` -> ilu_rap_matvec, ``fgmres`` -> fgmres_solve, ``spmv`` -> csr_spmv,
``Precond.export`` -> ilu_export.  Tensors must live on the current HIP
device; the current torch stream is passed to every call.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libschurilu.so")

BJ, SCHUR, RAP = 0, 1, 2
ILU0, MILU0, ILUT = 0, 1, 2
PIVOT_ERROR, PIVOT_PERTURB = 0, 1
TRSV_AUTO, TRSV_LEVELS, TRSV_BLOCK = 0, 1, 2
PREC_F64, PREC_F32, PREC_F16 = 0, 1, 2
ARNOLDI_AUTO, ARNOLDI_PER_PASS = 0, 1
OK, NOT_CONVERGED = 0, 1

EXPORT = dict(perm=(0, np.int32), iperm=(1, np.int32), iface=(2, np.uint8), offsets=(3, np.int64),
              DB=(16, np.float64), DS=(29, np.float64), lev_LB=(40, np.int32), lev_UB=(41, np.int32),
              lev_LS=(42, np.int32), lev_US=(43, np.int32), schedule=(44, np.int32))
# kernel classes of ilu_kernel_timing / ilu_kernel_stats (bit k = class k)
KERNEL_ALL = (1 << 7) - 1
_CSR_CODES = dict(LB=10, UB=13, Z=17, W=20, LS=23, US=26, Coff=30)
_FIELD_T = (np.int64, np.int32, np.float64)


class SchurILUError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("d_row_ptr", C.c_void_p), ("d_col", C.c_void_p),
                ("d_val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("interior_fact", C.c_int32), ("interface_fact", C.c_int32),
                ("droptol", C.c_double), ("lfil", C.c_int32), ("inner_iters", C.c_int32),
                ("inner_rtol", C.c_double), ("pivot_mode", C.c_int32), ("pivot_tol", C.c_double),
                ("trsv_mode", C.c_int32), ("factor_prec", C.c_int32), ("smooth_fact", C.c_int32),
                ("arnoldi_mode", C.c_int32), ("block_split", C.c_int32)]


class _Req(C.Structure):
    _fields_ = [("ticket", C.c_int64), ("matrix_id", C.c_int64), ("status", C.c_int32), ("iterations", C.c_int32),
                ("final_relres", C.c_double), ("cache_hit", C.c_int32), ("slot", C.c_int32),
                ("submit_us", C.c_double), ("start_us", C.c_double), ("done_us", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


class _Res(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("final_relres", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


_lib = None


def lib():
    """Load libschurilu.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SchurILUError(-5, f"{LIB_PATH} not found: build it with paper_2303_08881_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ilu_default_options.argtypes = [vp]
        L.ilu_default_options.restype = None
        L.ilu_setup.argtypes = [vp, vp, i32, vp, vp, C.POINTER(vp)]
        L.ilu_apply.argtypes = [vp, vp, vp, vp]
        L.ilu_rap_matvec.argtypes = [vp, vp, vp, vp]
        L.fgmres_solve.argtypes = [vp, vp, vp, vp, d, i32, i32, vp, vp, vp]
        L.csr_spmv.argtypes = [vp, vp, vp, vp]
        L.ilu_destroy.argtypes = [vp]
        L.ilu_destroy.restype = None
        L.ilu_memory_trim.argtypes = []
        L.ilu_memory_trim.restype = None
        L.ilu_last_error.argtypes = []
        L.ilu_last_error.restype = C.c_char_p
        L.ilu_export.argtypes = [vp, i32, vp, C.POINTER(i64)]
        L.ilu_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
        L.ilu_kernel_timing.argtypes = [i32]
        L.ilu_kernel_timing.restype = None
        L.ilu_kernel_stats.argtypes = [i32, C.POINTER(d), C.POINTER(i64), C.POINTER(d), i32]
        L.ilu_batch_setup.argtypes = [vp, vp, i32, i32, vp, C.POINTER(vp)]
        L.ilu_batch_solve.argtypes = [vp, vp, vp, vp, d, i32, i32, vp]
        L.ilu_batch_results.argtypes = [vp, vp, vp, vp, vp]
        L.ilu_batch_schedule.argtypes = [vp, i32, i32, i32]
        L.ilu_batch_tune.argtypes = [vp, vp, vp, vp, d, i32, i32, vp, C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i32), C.POINTER(d)]
        L.ilu_batch_capture.argtypes = [vp, vp, vp, vp, d, i32, i32, vp]
        L.ilu_batch_replay.argtypes = [vp, vp]
        L.ilu_batch_export.argtypes = [vp, i32, vp, C.POINTER(i64)]
        L.ilu_server_create.argtypes = [i32, i64, vp, C.POINTER(vp)]
        L.ilu_server_submit.argtypes = [vp, i64, vp, vp, i32, vp, vp, d, i32, i32, C.POINTER(i64)]
        L.ilu_server_wait.argtypes = [vp, i64, vp]
        L.ilu_server_stats.argtypes = [vp, vp, i32]
        L.ilu_server_destroy.argtypes = [vp]
        L.ilu_server_destroy.restype = None
        L.ilu_batch_destroy.argtypes = [vp]
        L.ilu_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_not_converged):
        raise SchurILUError(rc, lib().ilu_last_error().decode())
    return rc


def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t is not None else 0)


class DeviceCSR:
    """CSR matrix resident in device memory (torch tensors)."""

    def __init__(self, n, row_ptr, col, val):
        self.n = int(n)
        self.row_ptr, self.col, self.val = row_ptr, col, val
        self.nnz = int(col.numel())
        self._c = _CSR(self.n, self.nnz, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())

    @staticmethod
    def from_host(A, device="cuda"):
        torch = _torch()
        rp = torch.as_tensor(np.asarray(A.row_ptr, dtype=np.int64)).to(device)
        ci = torch.as_tensor(np.asarray(A.col, dtype=np.int32)).to(device)
        v = torch.as_tensor(np.asarray(A.val, dtype=np.float64)).to(device)
        return DeviceCSR(A.n, rp, ci, v)

    @property
    def ref(self):
        return C.byref(self._c)


def _options(method=BJ, interior_fact=ILU0, interface_fact=ILU0, droptol=0.0, lfil=-1, inner_iters=3,
             inner_rtol=0.0, pivot_mode=PIVOT_ERROR, pivot_tol=0.0, trsv_mode=TRSV_AUTO, factor_prec=PREC_F64,
             smooth_fact=ILU0, arnoldi_mode=ARNOLDI_AUTO, block_split=0):
    return _Opts(method, interior_fact, interface_fact, droptol, lfil, inner_iters, inner_rtol, pivot_mode,
                 pivot_tol, trsv_mode, factor_prec, smooth_fact, arnoldi_mode, block_split)


# Every live handle, so that the exit hook below can release them while the
# HIP runtime (and any profiler attached to it) is still up.
_live: "weakref.WeakSet[Precond]" = weakref.WeakSet()
_live_batches: "weakref.WeakSet[Batch]" = weakref.WeakSet()
_live_servers: "weakref.WeakSet[Server]" = weakref.WeakSet()


@atexit.register
def _release_at_exit():
    """Destroy live handles and return the library's cached device blocks before
    interpreter teardown, so no HIP call runs from a finaliser after the
    runtime's own exit handlers."""
    if _lib is None:
        return
    for p in list(_live_servers) + list(_live) + list(_live_batches):
        p.close()
    _lib.ilu_kernel_timing(0)
    _lib.ilu_memory_trim()


class Precond:
    """Handle returned by ilu_setup; owns the device memory of the preconditioner."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n
        _live.add(self)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ilu_destroy(self._h)
        self._h = None

    def apply(self, r, z=None):
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        _check(lib().ilu_apply(self._h, _ptr(r), _ptr(z), _stream()))
        return z

    def rap_matvec(self, v, out=None):
        """ilu_rap_matvec: out = R A P v (RAP handles; interface numbering, length n_S)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(v)
        _check(lib().ilu_rap_matvec(self._h, _ptr(v), _ptr(out), _stream()))
        return out

    def info(self):
        n, nB, nS, npart = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().ilu_info(self._h, C.byref(n), C.byref(nB), C.byref(nS), C.byref(npart)))
        return dict(n=n.value, nB=nB.value, nS=nS.value, nparts=npart.value)

    def _export(self, code, dtype):
        ln = C.c_int64(0)
        _check(lib().ilu_export(self._h, code, None, C.byref(ln)))
        out = np.zeros(ln.value, dtype=dtype)
        _check(lib().ilu_export(self._h, code, out.ctypes.data_as(C.c_void_p), C.byref(ln)))
        return out

    def export(self, name):
        """Copy an internal array to host: perm, iperm, iface, offsets, DB, DS, lev_*."""
        code, dt = EXPORT[name]
        return self._export(code, dt)

    def csr(self, name):
        """(row_ptr, col, val) of LB, UB, Z, W, LS, US or Coff."""
        base = _CSR_CODES[name]
        return tuple(self._export(base + k, _FIELD_T[k]) for k in range(3))


def setup(A: DeviceCSR, part=None, nparts=1, **opts) -> Precond:
    """ilu_setup: build the preconditioner of A on the device."""
    h = C.c_void_p()
    o = _options(**opts)
    torch = _torch()
    if part is not None and not (isinstance(part, torch.Tensor) and part.is_cuda):
        part = torch.as_tensor(np.asarray(part, dtype=np.int32)).to(A.val.device)
    pp = C.c_void_p(part.data_ptr()) if part is not None else C.c_void_p(0)
    _check(lib().ilu_setup(A.ref, pp, int(nparts), C.byref(o), _stream(), C.byref(h)))
    return Precond(h, A.n)


def fgmres(A: DeviceCSR, P: Precond, b, x0=None, rtol=1e-8, restart=30, maxit=1000, history=False, x=None):
    """fgmres_solve: right-preconditioned FGMRES(restart); returns a dict.  A given x holds x0 on entry (unless x0
    is passed too) and receives the solution."""
    return _fgmres(lib().fgmres_solve, A, P, b, x0, rtol, restart, maxit, history, x)


def _fgmres(fn, A, P, b, x0, rtol, restart, maxit, history, x):
    torch = _torch()
    if x is None:
        x = torch.zeros_like(b) if x0 is None else x0.clone()
    elif x0 is not None:
        x.copy_(x0)
    res = _Res()
    hist = np.full(maxit + 1, np.nan) if history else None
    hp = hist.ctypes.data_as(C.c_void_p) if history else None
    rc = fn(A.ref, P._h, _ptr(b), _ptr(x), float(rtol), int(restart), int(maxit), _stream(), C.byref(res), hp)
    _check(rc, allow_not_converged=True)
    out = dict(x=x, iterations=res.iterations, converged=bool(res.converged), relres=res.final_relres,
               setup_ms=res.setup_ms, solve_ms=res.solve_ms, rc=rc)
    if history:
        out["history"] = hist[: res.iterations + 1]
    return out


def spmv(A: DeviceCSR, x, y=None):
    """csr_spmv: y = A x."""
    torch = _torch()
    if y is None:
        y = torch.empty_like(x)
    _check(lib().csr_spmv(A.ref, _ptr(x), _ptr(y), _stream()))
    return y


class Batch:
    """Handle of ilu_batch_setup: many independent systems, ILU(0) + GMRES(m) each, solved in one persistent
    launch.  Arguments of solve / tune / capture are device tensors on the setup's pattern."""

    def __init__(self, handle, n, nnz, nsys):
        self._h = handle
        self.n, self.nnz, self.nsys = n, nnz, nsys
        _live_batches.add(self)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ilu_batch_destroy(self._h)
        self._h = None

    def solve(self, val, b, x, rtol=1e-8, restart=20, maxit=1000):
        """ilu_batch_solve: enqueue the factor + solve launch (x: initial guess in, solution out)."""
        _check(lib().ilu_batch_solve(self._h, _ptr(val), _ptr(b), _ptr(x), float(rtol), int(restart), int(maxit),
                                     _stream()))

    def results(self):
        """ilu_batch_results: (iterations, relres, status) per system, after the stream has finished."""
        it = np.zeros(self.nsys, np.int32)
        rr = np.zeros(self.nsys, np.float64)
        st = np.zeros(self.nsys, np.int32)
        _check(lib().ilu_batch_results(self._h, it.ctypes.data_as(C.c_void_p), rr.ctypes.data_as(C.c_void_p),
                                       st.ctypes.data_as(C.c_void_p), _stream()))
        return it, rr, st

    def schedule(self, merge, wpc, threads=256):
        _check(lib().ilu_batch_schedule(self._h, int(merge), int(wpc), int(threads)))

    def tune(self, val, b, x, rtol=1e-8, restart=20, maxit=1000):
        """ilu_batch_tune: time every candidate schedule, keep the fastest; returns (merge, wpc, threads, ms)."""
        mg, w, th, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().ilu_batch_tune(self._h, _ptr(val), _ptr(b), _ptr(x), float(rtol), int(restart), int(maxit),
                                    _stream(), C.byref(mg), C.byref(w), C.byref(th), C.byref(ms)))
        return mg.value, w.value, th.value, ms.value

    def capture(self, val, b, x, rtol=1e-8, restart=20, maxit=1000):
        """ilu_batch_capture on the current (non-default) stream."""
        _check(lib().ilu_batch_capture(self._h, _ptr(val), _ptr(b), _ptr(x), float(rtol), int(restart),
                                       int(maxit), _stream()))

    def replay(self):
        _check(lib().ilu_batch_replay(self._h, _stream()))

    def export(self, what):
        """'lu' factor values, 'lev_L' / 'lev_U' row levels, 'schedule' [E, merge, wpc, grid, threads]."""
        code, dt = dict(lu=(0, np.float64), lev_L=(1, np.int32), lev_U=(2, np.int32), schedule=(3, np.int32))[what]
        ln = C.c_int64(0)
        _check(lib().ilu_batch_export(self._h, code, None, C.byref(ln)))
        out = np.zeros(ln.value, dtype=dt)
        _check(lib().ilu_batch_export(self._h, code, out.ctypes.data_as(C.c_void_p), C.byref(ln)))
        return out


def batch_setup(A: DeviceCSR, sys_row, restart=20) -> Batch:
    """ilu_batch_setup: A block diagonal (global columns), sys_row the first row of each system (host, nsys+1)."""
    sr = np.ascontiguousarray(sys_row, dtype=np.int64)
    h = C.c_void_p()
    _check(lib().ilu_batch_setup(A.ref, sr.ctypes.data_as(C.c_void_p), int(len(sr) - 1), int(restart), _stream(),
                                 C.byref(h)))
    return Batch(h, A.n, A.nnz, len(sr) - 1)


def memory_trim():
    """ilu_memory_trim: free the library's cached device blocks."""
    lib().ilu_memory_trim()


SERVER_STATS = ("bytes", "peak_bytes", "resident", "hits", "misses", "evictions", "queued", "running", "budget")


class Server:
    """Handle of ilu_server_create: `slots` workers with their own streams, resident factors per matrix id, admission
    by a device-memory budget.  Every request is one fgmres_solve with the server's options."""

    def __init__(self, slots=4, budget_bytes=16 << 30, **opts):
        h = C.c_void_p()
        o = _options(**opts)
        _check(lib().ilu_server_create(int(slots), int(budget_bytes), C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> the device tensors a queued or running request reads
        _live_servers.add(self)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ilu_server_destroy(self._h)
        self._h = None
        self._keep = {}

    def submit(self, matrix_id, b, x, A: DeviceCSR | None = None, part=None, nparts=1, rtol=1e-8, restart=50,
               maxit=1000, sync=True) -> int:
        """ilu_server_submit; returns the ticket.  A is needed only for an id that is not resident.  With sync the
        current stream is synchronised first, so the server's streams see b and x as written."""
        torch = _torch()
        if sync:
            torch.cuda.current_stream().synchronize()
        keep = [b, x]
        aref = None
        pp = C.c_void_p(0)
        if A is not None:
            aref = A.ref
            keep.append(A)
            if part is not None:
                if not (isinstance(part, torch.Tensor) and part.is_cuda):
                    part = torch.as_tensor(np.asarray(part, dtype=np.int32)).to(A.val.device)
                    torch.cuda.current_stream().synchronize()
                keep.append(part)
                pp = C.c_void_p(part.data_ptr())
        t = C.c_int64()
        _check(lib().ilu_server_submit(self._h, int(matrix_id), aref, pp, int(nparts), _ptr(b), _ptr(x), float(rtol),
                                       int(restart), int(maxit), C.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def wait(self, ticket=-1) -> dict:
        """ilu_server_wait: the record of `ticket` (or of the next request to complete) as a dict."""
        r = _Req()
        _check(lib().ilu_server_wait(self._h, int(ticket), C.byref(r)))
        self._keep.pop(r.ticket, None)
        out = {f: getattr(r, f) for f, _ in _Req._fields_}
        if r.status < 0:
            out["error"] = lib().ilu_last_error().decode()
        return out

    def stats(self) -> dict:
        v = np.zeros(len(SERVER_STATS), dtype=np.int64)
        _check(lib().ilu_server_stats(self._h, v.ctypes.data_as(C.c_void_p), len(SERVER_STATS)))
        return dict(zip(SERVER_STATS, (int(x) for x in v)))
