"""mgk: AMG-preconditioned Krylov solver for block-structured Stokes systems on MI355X.

A thin ctypes binding over ``libmgk.so`` (declared in ``include/mgk.h``).  This
module only marshals arguments: every step of setup and solve runs in the native
library (host setup in C++, solve phase in HIP kernels for gfx950).  PyTorch
supplies device memory and streams.  There is no fallback: if the native
library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgk.so")

MGK_OK, MGK_NOT_CONVERGED = 0, 1
AMG_SPAI0, AMG_JACOBI, SCHUR, ILU = 0, 1, 2, 3
F64, F32, BF16 = 0, 1, 2
BICGSTAB, FGMRES, IDRS = 0, 1, 2
SMOOTHED_AGGREGATION, PLAIN_AGGREGATION = 0, 1
STORAGE = {"f64": F64, "f32": F32, "bf16": BF16}


class MgkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgk error {code}: {msg}")
        self.code = code


class _Bsr(C.Structure):
    _fields_ = [("n_brows", C.c_int32), ("block", C.c_int32), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("krylov", C.c_int32), ("fgmres_m", C.c_int32), ("maxiter", C.c_int32),
                ("max_restarts", C.c_int32), ("hier", C.c_int32), ("coarse_enough", C.c_int32),
                ("max_levels", C.c_int32), ("block_spai0", C.c_int32),
                ("eps_strong", C.c_double), ("jacobi_omega", C.c_double),
                ("keep_host", C.c_int32), ("enable_transpose", C.c_int32),
                ("time_spmv", C.c_int32), ("force_tile", C.c_int32),
                ("coarsening", C.c_int32), ("schur_approx", C.c_int32),
                ("schur_spai0", C.c_int32), ("schur_lower", C.c_int32), ("idr_s", C.c_int32),
                ("ilu_level", C.c_int32), ("ilu_sweeps", C.c_int32), ("ilu_smoother", C.c_int32),
                ("schur_scalar_u", C.c_int32), ("ilu_kind", C.c_int32),
                ("ilut_p", C.c_double), ("ilut_tau", C.c_double), ("layout", C.c_int32),
                ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("levels", C.c_int32), ("restarts", C.c_int32),
                ("status", C.c_int32), ("rel_resid", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("device_bytes", C.c_int64),
                ("spmv_ms", C.c_double), ("spmv_calls", C.c_int32), ("outer_tile", C.c_int32),
                ("precond_ms", C.c_double), ("precond_calls", C.c_int32),
                ("outer_dia", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelDesc(C.Structure):
    _fields_ = [("n_brows", C.c_int32), ("block", C.c_int32), ("nnzb", C.c_int64),
                ("n_agg", C.c_int32), ("dia", C.c_int32), ("p_nnzb", C.c_int64),
                ("r_nnzb", C.c_int64), ("omega", C.c_double)]


EXPORTS = ["mgk_params_default", "mgk_stokes_sizes", "mgk_stokes_assemble", "mgk_csr_to_bsr",
           "mgk_setup", "mgk_setup_host", "mgk_solve", "mgk_solve_noalloc",
           "mgk_solve_transposed", "mgk_solve_multi",
           "mgk_batch_setup", "mgk_batch_solve", "mgk_spmv", "mgk_precond_apply", "mgk_set_timing",
           "mgk_level_count", "mgk_level_info", "mgk_level_export", "mgk_ilu_info",
           "mgk_ilu_export", "mgk_theta_grad", "mgk_bsr_grad", "mgk_destroy", "mgk_last_error"]

_lib = None


def lib():
    """Load libmgk.so (built by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.mgk_last_error.restype = C.c_char_p
    L.mgk_params_default.argtypes = [C.POINTER(Params)]
    L.mgk_stokes_sizes.argtypes = [I32, C.POINTER(I32), C.POINTER(I64)]
    L.mgk_stokes_assemble.argtypes = [I32, P, P, P, P]
    L.mgk_csr_to_bsr.argtypes = [I32, P, P, P, I32, P, P, P, C.POINTER(I64)]
    L.mgk_setup.argtypes = [C.POINTER(_Bsr), I32, I32, C.POINTER(Params), P, C.POINTER(P)]
    L.mgk_setup_host.argtypes = [C.POINTER(_Bsr), I32, I32, C.POINTER(Params), C.POINTER(P)]
    L.mgk_solve.argtypes = [P, P, P, D, C.POINTER(Info)]
    L.mgk_solve_noalloc.argtypes = [P, P, P, D, C.POINTER(Info)]
    L.mgk_ilu_info.argtypes = [P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I64)]
    L.mgk_ilu_export.argtypes = [P, I32, P, P, P]
    L.mgk_solve_transposed.argtypes = [P, P, P, D, C.POINTER(Info)]
    L.mgk_solve_multi.argtypes = [P, I32, P, P, D, P]
    L.mgk_batch_setup.argtypes = [I32, P, I32, I32, C.POINTER(Params), P, C.POINTER(P)]
    L.mgk_batch_solve.argtypes = [P, P, P, D, P]
    L.mgk_spmv.argtypes = [P, I32, I32, I32, P, P]
    L.mgk_precond_apply.argtypes = [P, P, P, I32]
    L.mgk_set_timing.argtypes = [P, I32]
    L.mgk_level_count.argtypes = [P, I32]
    L.mgk_level_info.argtypes = [P, I32, I32, C.POINTER(LevelDesc)]
    L.mgk_level_export.argtypes = [P, I32, I32, I32, P, P, P, P]
    L.mgk_theta_grad.argtypes = [I32, P, P, P, P]
    L.mgk_bsr_grad.argtypes = [P, P, P, P]
    L.mgk_destroy.argtypes = [P]
    _lib = L
    return L


def _err(code):
    raise MgkError(code, lib().mgk_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype=None, numel=None):
    """Device pointer of a contiguous CUDA tensor, with dtype/size checks."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def default_params(**kw) -> Params:
    p = Params()
    lib().mgk_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "hier" and isinstance(v, str):
            v = STORAGE[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def stokes_bsr(n: int, theta: np.ndarray | None = None):
    """Host BSR (rowptr, col, val[nnzb,4,4]) of the synthetic FD Stokes system on n^3 nodes."""
    L = lib()
    nbr, nnzb = C.c_int32(), C.c_int64()
    rc = L.mgk_stokes_sizes(n, C.byref(nbr), C.byref(nnzb))
    if rc:
        _err(rc)
    ptr = np.empty(nbr.value + 1, np.int32)
    col = np.empty(nnzb.value, np.int32)
    val = np.empty((nnzb.value, 4, 4), np.float64)
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    if th is not None and th.size != (n - 1) ** 3:
        raise ValueError("theta needs (n-1)^3 values")
    rc = L.mgk_stokes_assemble(n, None if th is None else _np_ptr(th), _np_ptr(ptr), _np_ptr(col),
                               _np_ptr(val))
    if rc:
        _err(rc)
    return ptr, col, val


def csr_to_bsr(ptr, col, val, b: int):
    L = lib()
    ptr = np.ascontiguousarray(ptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    nrows = ptr.size - 1
    nnzb = C.c_int64()
    rc = L.mgk_csr_to_bsr(nrows, _np_ptr(ptr), _np_ptr(col), _np_ptr(val), b, None, None, None,
                          C.byref(nnzb))
    if rc:
        _err(rc)
    bptr = np.empty(nrows // b + 1, np.int32)
    bcol = np.empty(nnzb.value, np.int32)
    bval = np.empty((nnzb.value, b, b), np.float64)
    rc = L.mgk_csr_to_bsr(nrows, _np_ptr(ptr), _np_ptr(col), _np_ptr(val), b, _np_ptr(bptr),
                          _np_ptr(bcol), _np_ptr(bval), C.byref(nnzb))
    if rc:
        _err(rc)
    return bptr, bcol, bval


def theta_grad(n: int, lam, x, g, stream=None):
    import torch
    N = 4 * n ** 3
    rc = lib().mgk_theta_grad(n, _dev_ptr(lam, torch.float64, N), _dev_ptr(x, torch.float64, N),
                              _dev_ptr(g, torch.float64, (n - 1) ** 3), _stream_handle(stream))
    if rc:
        _err(rc)


class Solver:
    """setup(A in BSR, block size, preconditioner kind) then solve(b, x, rtol)."""

    def __init__(self, rowptr, col, val, block: int, kind: int = AMG_SPAI0, stream=None,
                 host_only: bool = False, **params):
        L = lib()
        self._ptr = np.ascontiguousarray(rowptr, np.int32)
        self._col = np.ascontiguousarray(col, np.int32)
        self._val = np.ascontiguousarray(val, np.float64).reshape(-1)
        self.block = block
        self.n_brows = self._ptr.size - 1
        self.n = self.n_brows * block
        self.params = default_params(**params)
        A = _Bsr(self.n_brows, block, _np_ptr(self._ptr).value, _np_ptr(self._col).value,
                 _np_ptr(self._val).value)
        h = C.c_void_p()
        self._stream = stream
        if host_only:
            rc = L.mgk_setup_host(C.byref(A), block, kind, C.byref(self.params), C.byref(h))
        else:
            rc = L.mgk_setup(C.byref(A), block, kind, C.byref(self.params),
                             _stream_handle(stream), C.byref(h))
        if rc:
            _err(rc)
        self._h = h
        # setup deep-copies the matrix; drop the host arrays unless export is wanted
        if not self.params.keep_host and not host_only:
            self._ptr = self._col = self._val = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.mgk_destroy(self._h)
            self._h = C.c_void_p()

    __del__ = close

    def _solve(self, fn, b, x, rtol):
        import torch
        info = Info()
        rc = fn(self._h, _dev_ptr(b, torch.float64, self.n), _dev_ptr(x, torch.float64, self.n),
                rtol, C.byref(info))
        if rc < 0:
            _err(rc)
        return info.as_dict()

    def solve(self, b, x, rtol: float = 1e-8) -> dict:
        """x (in: initial guess, out: solution); returns the info record."""
        return self._solve(lib().mgk_solve, b, x, rtol)

    def set_timing(self, mask: int):
        """Timing events of later solves: mask & the setup's time_spmv (0 turns them off)."""
        rc = lib().mgk_set_timing(self._h, int(mask))
        if rc:
            _err(rc)

    def solve_noalloc(self, b, x, rtol: float = 1e-8) -> dict:
        """solve() with the Krylov workspace in the library's static device array: the
        call allocates no device memory (BiCGStab solvers of at most 524288 unknowns)."""
        return self._solve(lib().mgk_solve_noalloc, b, x, rtol)

    def solve_multi(self, B, X, rtol: float = 1e-8) -> list:
        """K <= 32 right-hand sides together: B, X are [n, K] (right-hand sides fastest);
        X holds the initial guesses.  Returns one info record per column."""
        import torch
        if B.dim() != 2 or B.shape[0] != self.n or X.shape != B.shape:
            raise ValueError("B and X must both be [n, K]")
        K = B.shape[1]
        infos = (Info * K)()
        rc = lib().mgk_solve_multi(self._h, K, _dev_ptr(B, torch.float64),
                                   _dev_ptr(X, torch.float64), rtol, infos)
        if rc < 0:
            _err(rc)
        return [i.as_dict() for i in infos]

    def solve_transposed(self, g, lam, rtol: float = 1e-8) -> dict:
        return self._solve(lib().mgk_solve_transposed, g, lam, rtol)

    def spmv(self, x, y, level: int = -1, which: int = 0, hier: int = 0):
        rc = lib().mgk_spmv(self._h, hier, level, which, _dev_ptr(x), _dev_ptr(y))
        if rc:
            _err(rc)

    def precond(self, r, z, transposed: bool = False):
        import torch
        rc = lib().mgk_precond_apply(self._h, _dev_ptr(r, torch.float64, self.n),
                                     _dev_ptr(z, torch.float64, self.n), int(transposed))
        if rc:
            _err(rc)

    def bsr_grad(self, lam, x, gval):
        import torch
        rc = lib().mgk_bsr_grad(self._h, _dev_ptr(lam, torch.float64, self.n),
                                _dev_ptr(x, torch.float64, self.n), _dev_ptr(gval, torch.float64))
        if rc:
            _err(rc)

    def nlevels(self, hier: int = 0) -> int:
        return lib().mgk_level_count(self._h, hier)

    def level_info(self, level: int, hier: int = 0) -> dict:
        d = LevelDesc()
        rc = lib().mgk_level_info(self._h, hier, level, C.byref(d))
        if rc:
            _err(rc)
        return {k: getattr(d, k) for k, _ in d._fields_}

    def ilu_export(self):
        """Host FP64 block ILU factors: (L, U) as (rowptr, col, val[nnzb, b, b]) and Dinv."""
        L = lib()
        nb = C.c_int32()
        ln, un = C.c_int64(), C.c_int64()
        rc = L.mgk_ilu_info(self._h, C.byref(nb), C.byref(ln), C.byref(un))
        if rc:
            _err(rc)
        b = self.block
        out = []
        for which, nz in ((0, ln.value), (1, un.value)):
            ptr = np.zeros(nb.value + 1, np.int32)
            col = np.zeros(max(nz, 1), np.int32)
            val = np.zeros(max(nz, 1) * b * b, np.float64)
            rc = L.mgk_ilu_export(self._h, which, _np_ptr(ptr), _np_ptr(col), _np_ptr(val))
            if rc:
                _err(rc)
            out.append((ptr, col[:nz], val[:nz * b * b].reshape(nz, b, b)))
        dinv = np.zeros(nb.value * b * b, np.float64)
        rc = L.mgk_ilu_export(self._h, 2, None, None, _np_ptr(dinv))
        if rc:
            _err(rc)
        return out[0], out[1], dinv.reshape(nb.value, b, b)

    def level_smoother(self, level: int, hier: int = 0):
        """Host FP64 copy of the smoother blocks M_l, (n_brows, b, b)."""
        d = self.level_info(level, hier)
        b, nb = d["block"], d["n_brows"]
        val = np.zeros(max(nb, 1) * b * b, np.float64)
        rc = lib().mgk_level_export(self._h, hier, level, 3, None, None, _np_ptr(val), None)
        if rc:
            _err(rc)
        return val[:nb * b * b].reshape(nb, b, b)

    def level_export(self, level: int, which: int = 0, hier: int = 0):
        """Host FP64 copy (rowptr, col, val) of A_l (0), P_l (1) or R_l (2), plus aggregates."""
        d = self.level_info(level, hier)
        b = d["block"]
        nb = d["n_brows"]
        if which == 0:
            rows, nnz, cb = nb, d["nnzb"], b
        elif which == 1:
            rows, nnz, cb = nb, d["p_nnzb"], b
        else:
            rows, nnz, cb = d["n_agg"], d["r_nnzb"], b
        ptr = np.zeros(rows + 1, np.int32)
        col = np.zeros(max(nnz, 1), np.int32)
        val = np.zeros(max(nnz, 1) * b * cb, np.float64)
        agg = np.zeros(max(nb, 1), np.int32)
        rc = lib().mgk_level_export(self._h, hier, level, which, _np_ptr(ptr), _np_ptr(col),
                                    _np_ptr(val), _np_ptr(agg))
        if rc:
            _err(rc)
        return ptr, col[:nnz], val[:nnz * b * cb].reshape(nnz, b, cb), agg[:nb]


class BatchSolver:
    """Several independent systems of uneven size behind one solver: every stage of the
    lockstep BiCGStab solve is one launch over all systems (mgk_batch_setup/solve)."""

    def __init__(self, systems, block: int, kind: int = AMG_SPAI0, stream=None, **params):
        L = lib()
        self._keep = []
        structs = []
        self.sizes = []
        for ptr, col, val in systems:
            ptr = np.ascontiguousarray(ptr, np.int32)
            col = np.ascontiguousarray(col, np.int32)
            val = np.ascontiguousarray(val, np.float64).reshape(-1)
            self._keep += [ptr, col, val]
            structs.append(_Bsr(ptr.size - 1, block, _np_ptr(ptr).value, _np_ptr(col).value,
                                _np_ptr(val).value))
            self.sizes.append((ptr.size - 1) * block)
        self._structs = (_Bsr * len(structs))(*structs)
        ptrs = (C.c_void_p * len(structs))(*[C.addressof(self._structs[i])
                                               for i in range(len(structs))])
        self._ptrs = ptrs
        self.params = default_params(**params)
        h = C.c_void_p()
        rc = L.mgk_batch_setup(len(structs), C.cast(ptrs, C.c_void_p), block, kind,
                               C.byref(self.params), _stream_handle(stream), C.byref(h))
        if rc:
            _err(rc)
        self._h = h
        self._keep = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.mgk_destroy(self._h)
            self._h = C.c_void_p()

    __del__ = close

    def solve(self, bs, xs, rtol: float = 1e-8) -> list:
        import torch
        n = len(self.sizes)
        if len(bs) != n or len(xs) != n:
            raise ValueError("one right-hand side and one solution vector per system")
        bp = (C.c_void_p * n)(*[_dev_ptr(b, torch.float64, m).value for b, m in zip(bs, self.sizes)])
        xp = (C.c_void_p * n)(*[_dev_ptr(x, torch.float64, m).value for x, m in zip(xs, self.sizes)])
        infos = (Info * n)()
        rc = lib().mgk_batch_solve(self._h, C.cast(bp, C.c_void_p), C.cast(xp, C.c_void_p),
                                   rtol, infos)
        if rc < 0:
            _err(rc)
        return [i.as_dict() for i in infos]
