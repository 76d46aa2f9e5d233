"""Seeded synthetic inputs for the stabilized finite-difference Stokes workloads.

This module is shared by the oracle tests and the GPU path.  It holds no solver
arithmetic: it only draws the random fields and evaluates the manufactured
solution that define each problem.  Matrices are assembled separately by each
side from these inputs.

Grid: n^3 nodes on the unit cube, x = (i, j, k) h with h = 1/(n-1); node id
g = i + n (j + n k); unknown 4 g + c with c = 0, 1, 2 velocity and c = 3
pressure.  Cells e = i + (n-1) (j + (n-1) k).  The paper's weak-Galerkin test
matrices are not available; these synthetic systems stand in for them at sizes
spanning its 8K to 9.4M unknowns.
"""
from __future__ import annotations

import numpy as np

# Workloads (grid nodes per side, seeds).  Names describe the problem.
WORKLOADS = {
    "cube16_mms": dict(n=16, rhs="mms"),
    "cube96_mms_noise": dict(n=96, rhs="mms+noise", noise_var=1e-3, seed=2),
    "cube64_lognormal_schur": dict(n=64, rhs="Axstar", sigma=1.0, seed=3),
    "cube64_forces_32rhs": dict(n=64, rhs="forces", nrhs=32, seed=4),
    "multi8_lognormal": dict(ns=[24, 32, 40, 48, 48, 56, 64, 64], sigma=0.5, seed=40),
    "cube48_adjoint": dict(n=48, sigma=0.5, seed=5, ref_seed=50, fd_seed=51, fd_cells=20),
}


def node_coords(n: int) -> np.ndarray:
    """(n^3, 3) coordinates of every node in node-id order."""
    t = np.arange(n, dtype=np.float64) / (n - 1)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def interior_nodes(n: int) -> np.ndarray:
    """Boolean mask over node ids: True for nodes with no index at 0 or n-1."""
    i = np.arange(n)
    inner = (i > 0) & (i < n - 1)
    k, j, ii = np.meshgrid(inner, inner, inner, indexing="ij")
    return (k & j & ii).ravel()


def theta_field(n: int, sigma: float, seed: int) -> np.ndarray:
    """Per-cell viscosity exp(N(0, sigma^2)), (n-1)^3 values."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(0.0, sigma, size=(n - 1) ** 3))


def mms_solution(n: int) -> np.ndarray:
    """Nodal u* = (sin x cos y, -cos x sin y, 0), p* = x + y - 1, interleaved."""
    X = node_coords(n)
    x, y = X[:, 0], X[:, 1]
    out = np.empty((n ** 3, 4))
    out[:, 0] = np.sin(x) * np.cos(y)
    out[:, 1] = -np.cos(x) * np.sin(y)
    out[:, 2] = 0.0
    out[:, 3] = x + y - 1.0
    return out.ravel()


def mms_rhs(n: int) -> np.ndarray:
    """Right-hand side of the manufactured problem with mu = 1.

    Interior velocity rows: f = (2 sin x cos y + 1, -2 cos x sin y + 1, 0);
    interior pressure rows: 0; boundary rows: the exact u*, p* values."""
    X = node_coords(n)
    x, y = X[:, 0], X[:, 1]
    f = np.zeros((n ** 3, 4))
    f[:, 0] = 2.0 * np.sin(x) * np.cos(y) + 1.0
    f[:, 1] = -2.0 * np.cos(x) * np.sin(y) + 1.0
    bnd = ~interior_nodes(n)
    f[bnd] = mms_solution(n).reshape(-1, 4)[bnd]
    return f.ravel()


def interior_noise(n: int, var: float, seed: int) -> np.ndarray:
    """N(0, var) on every unknown of an interior node, 0 on boundary nodes."""
    rng = np.random.default_rng(seed)
    e = rng.normal(0.0, np.sqrt(var), size=(n ** 3, 4))
    e[~interior_nodes(n)] = 0.0
    return e.ravel()


def body_forces(n: int, nrhs: int, seed: int) -> np.ndarray:
    """(4 n^3, nrhs) right-hand sides: U[-1, 1] on interior velocity rows, else 0.
    Stored RHS-fastest (row-major), the layout of the multi-RHS solve."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1.0, 1.0, size=(n ** 3, 4, nrhs))
    F[:, 3, :] = 0.0
    F[~interior_nodes(n)] = 0.0
    return F.reshape(4 * n ** 3, nrhs)


def fd_cells(n: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice((n - 1) ** 3, count, replace=False)


def c2_rhs(n: int = 96, var: float = 1e-3, seed: int = 2) -> np.ndarray:
    return mms_rhs(n) + interior_noise(n, var, seed)
