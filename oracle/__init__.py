"""Plain FP64 CPU oracle of the AMG-preconditioned Krylov Stokes solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

The C++ sources next to this file hold the arithmetic (scalar CSR, FP64,
``-ffp-contract=off``); this module only compiles them and marshals numpy
arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
SOURCES = ["csr.cpp", "stokes.cpp", "amg.cpp", "krylov.cpp", "ilu.cpp", "capi.cpp"]

KIND_AMG, KIND_SCHUR, KIND_IDENTITY, KIND_ILU = 0, 1, 2, 3
SPAI0_BLOCK, JACOBI, SPAI0_SCALAR, ILU0, ILUT = 0, 1, 2, 3, 4
BICGSTAB, FGMRES, IDRS = 0, 1, 2
SMOOTHED, PLAIN = 0, 1


def build(verbose: bool = False) -> str:
    """Compile liborc.so with g++ (FP64, no FMA contraction, OpenMP SpMV)."""
    cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("krylov", C.c_int32), ("fgmres_m", C.c_int32), ("maxiter", C.c_int32),
                ("max_restarts", C.c_int32), ("eps_strong", C.c_double),
                ("coarse_enough", C.c_int32), ("max_levels", C.c_int32),
                ("smoother", C.c_int32), ("kind", C.c_int32), ("jacobi_omega", C.c_double),
                ("coarsening", C.c_int32), ("schur_approx", C.c_int32),
                ("schur_spai0", C.c_int32), ("schur_lower", C.c_int32), ("idr_s", C.c_int32),
                ("ilu_level", C.c_int32), ("ilu_sweeps", C.c_int32),
                ("schur_scalar_u", C.c_int32), ("ilu_kind", C.c_int32),
                ("ilut_p", C.c_double), ("ilut_tau", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("pad", C.c_int32), ("rel_resid", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_last_error.restype = C.c_char_p
        L.orc_stokes_nnz.restype = C.c_int64
        L.orc_stokes_nnz.argtypes = [C.c_int]
        L.orc_stokes_assemble.argtypes = [C.c_int, P, P, P, P]
        L.orc_theta_grad.argtypes = [C.c_int, P, P, P]
        L.orc_spmv.argtypes = [C.c_int64, C.c_int64, P, P, P, P, P]
        L.orc_setup.restype = P
        L.orc_setup.argtypes = [C.c_int64, P, P, P, C.c_int, C.POINTER(_Params)]
        L.orc_free.argtypes = [P]
        L.orc_nlevels.argtypes = [P, C.c_int]
        L.orc_level_sizes.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_level_get.argtypes = [P, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_level_agg.argtypes = [P, C.c_int, C.c_int, P, C.POINTER(C.c_double)]
        L.orc_level_smoother.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_precond.argtypes = [P, P, P, C.c_int]
        L.orc_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.POINTER(_Info)]
        L.orc_idr_shadow.argtypes = [C.c_int64, C.c_int, P]
        L.orc_ilu_factor.argtypes = [P, P, P, P]
        L.orc_ilu_factor.restype = C.c_int64
        L.orc_ilu_dinv.argtypes = [P, P]
        L.orc_ilu_dinv.restype = None
        L.orc_idr_shadow.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.restype = C.c_int
        L.orc_set_limits.argtypes = [P, C.c_int, C.c_int]
        L.orc_set_limits.restype = None
        L.orc_gather_block_row.argtypes = [C.c_int64, P, P, P, C.c_int, C.c_int64, P, P,
                                           C.c_int32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def stokes_matrix(n: int, theta: np.ndarray | None = None) -> sp.csr_matrix:
    """Scalar CSR of the stabilized FD Stokes operator on n^3 nodes."""
    L = lib()
    nr = 4 * n ** 3
    nnz = L.orc_stokes_nnz(n)
    ptr = np.empty(nr + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    th = None if theta is None else _f64(theta)
    if th is not None and th.size != (n - 1) ** 3:
        raise ValueError("theta needs (n-1)^3 cell values")
    rc = L.orc_stokes_assemble(n, None if th is None else _p(th), _p(ptr), _p(col), _p(val))
    if rc:
        raise ValueError("oracle assembly failed")
    return sp.csr_matrix((val, col, ptr), shape=(nr, nr))


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (sparse products)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return lib().orc_max_threads()


def theta_gradient(n: int, lam: np.ndarray, x: np.ndarray) -> np.ndarray:
    g = np.empty((n - 1) ** 3, np.float64)
    lam, x = _f64(lam), _f64(x)
    lib().orc_theta_grad(n, _p(lam), _p(x), _p(g))
    return g


def idr_shadow(n: int, s: int) -> np.ndarray:
    """The n x s IDR(s) shadow space (columns orthonormal), as an (n, s) array."""
    out = np.zeros(n * s, np.float64)
    lib().orc_idr_shadow(n, s, _p(out))
    return out.reshape(s, n).T.copy()


def gather_block_row(A: sp.csr_matrix, b: int, i: int):
    """Block columns and dense b x b blocks of node row i (the oracle's node view)."""
    ptr = np.ascontiguousarray(A.indptr, np.int64)
    col = np.ascontiguousarray(A.indices, np.int32)
    val = _f64(A.data)
    cap = A.shape[1] // b
    cols = np.zeros(cap, np.int32)
    vals = np.zeros(cap * b * b, np.float64)
    m = lib().orc_gather_block_row(A.shape[0], _p(ptr), _p(col), _p(val), b, i, _p(cols),
                                   _p(vals), cap)
    return cols[:m], vals[:m * b * b].reshape(m, b, b)


def spmv(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    ptr = np.ascontiguousarray(A.indptr, np.int64)
    col = np.ascontiguousarray(A.indices, np.int32)
    val = _f64(A.data)
    x = _f64(x)
    y = np.empty(A.shape[0], np.float64)
    lib().orc_spmv(A.shape[0], A.shape[1], _p(ptr), _p(col), _p(val), _p(x), _p(y))
    return y


class Solver:
    """Oracle setup + solve.  kind: KIND_AMG (monolithic SA-AMG), KIND_SCHUR
    (pressure correction, interleaved 4-component unknowns), KIND_IDENTITY."""

    def __init__(self, A: sp.csr_matrix, block: int, kind: int = KIND_AMG,
                 krylov: int = BICGSTAB, smoother: int = SPAI0_BLOCK,
                 eps_strong: float = 0.08, coarse_enough: int = 3000, max_levels: int = 20,
                 maxiter: int = 1000, fgmres_m: int = 30, max_restarts: int = 5,
                 jacobi_omega: float = 2.0 / 3.0, coarsening: int = SMOOTHED,
                 schur_approx: int = 0, schur_spai0: int = 0, schur_lower: int = 0,
                 idr_s: int = 5, ilu_level: int = 0, ilu_sweeps: int = 2,
                 schur_scalar_u: int = 0, ilu_kind: int = 0, ilut_p: float = 2.0,
                 ilut_tau: float = 1e-2):
        A = sp.csr_matrix(A)
        A.sort_indices()
        self.n = A.shape[0]
        self._keep = (np.ascontiguousarray(A.indptr, np.int64),
                      np.ascontiguousarray(A.indices, np.int32), _f64(A.data))
        self.prm = _Params(krylov, fgmres_m, maxiter, max_restarts, eps_strong, coarse_enough,
                           max_levels, smoother, kind, jacobi_omega, coarsening, schur_approx,
                           schur_spai0, schur_lower, idr_s, ilu_level, ilu_sweeps,
                           schur_scalar_u, ilu_kind, ilut_p, ilut_tau)
        self.block = block
        L = lib()
        h = L.orc_setup(self.n, *(_p(a) for a in self._keep), block, C.byref(self.prm))
        if not h:
            raise RuntimeError(L.orc_last_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def set_limits(self, maxiter: int, max_restarts: int) -> None:
        """Change the iteration limits of later solves (setup is unchanged)."""
        lib().orc_set_limits(self._h, int(maxiter), int(max_restarts))

    def ilu_factor(self) -> sp.csr_matrix:
        """Combined block ILU factor (L strictly lower with unit diagonal implied, U on and
        above the diagonal) as scalar CSR."""
        L = lib()
        nz = L.orc_ilu_factor(self._h, None, None, None)
        ptr = np.zeros(self.n + 1, np.int64)
        col = np.zeros(max(nz, 1), np.int32)
        val = np.zeros(max(nz, 1), np.float64)
        L.orc_ilu_factor(self._h, _p(ptr), _p(col), _p(val))
        return sp.csr_matrix((val[:nz], col[:nz], ptr), shape=(self.n, self.n))

    def ilu_dinv(self) -> np.ndarray:
        """Inverses of the ILU pivot blocks, (n / b, b, b)."""
        out = np.zeros(self.n * self.block, np.float64)
        lib().orc_ilu_dinv(self._h, _p(out))
        return out.reshape(self.n // self.block, self.block, self.block)

    def nlevels(self, which: int = 0) -> int:
        return lib().orc_nlevels(self._h, which)

    def level(self, l: int, which: int = 0) -> dict:
        """Copies of level l: A, P, R (scipy CSR), aggregates, omega, smoother blocks."""
        L = lib()
        sz = np.zeros(8, np.int64)
        if L.orc_level_sizes(self._h, which, l, _p(sz)):
            raise IndexError(l)
        nr, annz, pnc, pnnz, rnnz, nagg, b = (int(v) for v in sz[:7])
        out = {"n_agg": nagg, "block": b}

        def get(mat, rows, cols, nnz):
            ptr = np.zeros(rows + 1, np.int64)
            col = np.zeros(max(nnz, 1), np.int32)
            val = np.zeros(max(nnz, 1), np.float64)
            L.orc_level_get(self._h, which, l, mat, _p(ptr), _p(col), _p(val))
            return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(rows, cols))

        out["A"] = get(0, nr, nr, annz)
        if pnnz or pnc:
            out["P"] = get(1, nr, pnc, pnnz)
            out["R"] = get(2, pnc, nr, rnnz)
        agg = np.zeros(nr // b, np.int32)
        om = C.c_double(0)
        L.orc_level_agg(self._h, which, l, _p(agg), C.byref(om))
        out["agg"] = agg
        out["omega"] = om.value
        if pnnz or pnc:
            M = np.zeros((nr // b) * b * b, np.float64)
            L.orc_level_smoother(self._h, which, l, _p(M))
            out["M"] = M.reshape(nr // b, b, b)
        return out

    def precond(self, r: np.ndarray, transposed: bool = False) -> np.ndarray:
        r = _f64(r)
        z = np.zeros(self.n, np.float64)
        if lib().orc_precond(self._h, _p(r), _p(z), int(transposed)):
            raise RuntimeError(lib().orc_last_error().decode())
        return z

    def solve(self, b: np.ndarray, tol: float = 1e-8, x0: np.ndarray | None = None,
              transposed: bool = False):
        b = _f64(b)
        x = np.zeros(self.n, np.float64) if x0 is None else _f64(x0).copy()
        info = _Info()
        rc = lib().orc_solve(self._h, _p(b), _p(x), tol, int(transposed), C.byref(info))
        if rc < 0:
            raise RuntimeError(lib().orc_last_error().decode())
        return x, {"iters": info.iters, "restarts": info.restarts,
                   "converged": bool(info.converged), "rel_resid": info.rel_resid}
