"""Parity at the full workload sizes, in the configuration bench.py times.

96^3 monolithic (mixed FP32 hierarchy, BiCGStab), 64^3 Schur pressure correction (BF16
hierarchy, FGMRES(30)), 48^3 adjoint gradient, 64^3 with 32 right-hand sides in one lockstep
solve, and the eight 24^3 ... 64^3 systems in one batched solve.  The residual of every GPU solution is
evaluated with the oracle's own FP64 SpMV; solutions are compared with the oracle's FP64
solve; the gradient with the oracle's gradient over all cells and with central finite
differences on 20 seeded cells.
"""
import numpy as np
import pytest

import oracle
import stokes_synth as S

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(300)]

import paper_2006_06052_amd as mgk  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def solver(ptr, col, val, **kw):
    return mgk.Solver(ptr, col, val, 4, kw.pop("kind", mgk.AMG_SPAI0),
                      stream=torch.cuda.current_stream(), **kw)


@pytest.fixture(scope="module")
def cube96():
    """The 96^3 headline system (manufactured RHS plus noise) and the oracle's FP64 solve."""
    n = 96
    say("cube96: assembling")
    ptr, col, val = mgk.stokes_bsr(n)
    b = S.c2_rhs(n)
    A = oracle.stokes_matrix(n)
    say("cube96: oracle solve")
    xo, oi = oracle.Solver(A, 4).solve(b, 1e-11)
    say("cube96 oracle", oi)
    return (ptr, col, val), A, b, xo


def scalar_csr(ptr, col, val):
    """Scalar CSR (nonzero entries) of a 4x4 BSR matrix: the input of the scalar arm."""
    import scipy.sparse as sp
    nb = len(ptr) - 1
    rows = np.repeat(np.arange(nb), np.diff(ptr))
    r = (4 * rows[:, None, None] + np.arange(4)[None, :, None]) * np.ones((1, 1, 4), np.int64)
    c = (4 * col[:, None, None] + np.arange(4)[None, None, :]) * np.ones((1, 4, 1), np.int64)
    keep = val != 0.0
    M = sp.csr_matrix((val[keep], (r[keep], c[keep])), shape=(4 * nb, 4 * nb))
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data


# every solve the benchmark times on the 96^3 system: the FP32 (headline), FP64 and BF16
# hierarchies and the scalar FP64 arm under BiCGStab, and IDR(5) and plain aggregation with
# the FP32 hierarchy
ARMS96 = {
    "bsr_f32": dict(hier="f32"),
    "bsr_f64": dict(hier="f64"),
    "bsr_bf16": dict(hier="bf16"),
    "csr_f64": dict(hier="f64", scalar=True),
    "idrs5_f32": dict(hier="f32", krylov="idrs", idr_s=5),
    "plain_f32": dict(hier="f32", coarsening="plain"),
}


@pytest.mark.parametrize("arm", list(ARMS96))
def test_cube96_arms_vs_oracle(cube96, arm):
    (ptr, col, val), A, b, xo = cube96
    kw = dict(ARMS96[arm])
    say("cube96 arm", arm, kw)
    hier = {"f64": mgk.F64, "f32": mgk.F32, "bf16": mgk.BF16}[kw.pop("hier")]
    if kw.pop("krylov", None) == "idrs":
        kw["krylov"] = mgk.IDRS
    if kw.pop("coarsening", None) == "plain":
        kw["coarsening"] = mgk.PLAIN_AGGREGATION
    if kw.pop("scalar", False):
        bp, bc, bv = mgk.csr_to_bsr(*scalar_csr(ptr, col, val), 1)
        s = mgk.Solver(bp, bc, bv, 1, mgk.AMG_SPAI0, stream=torch.cuda.current_stream(),
                       hier=hier, **kw)
    else:
        s = solver(ptr, col, val, hier=hier, **kw)
    dx = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("cube96 gpu", arm, info)
    x = dx.cpu().numpy()
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    assert info["status"] == 0 and res <= 1e-8, res
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


def test_cube64_schur_bf16_vs_oracle():
    n = 64
    th = S.theta_field(n, 1.0, 3)
    ptr, col, val = mgk.stokes_bsr(n, th)
    A = oracle.stokes_matrix(n, th)
    b = oracle.spmv(A, S.mms_solution(n))
    s = solver(ptr, col, val, kind=mgk.SCHUR, hier=mgk.BF16, krylov=mgk.FGMRES)
    dx = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("cube64 schur gpu", info)
    x = dx.cpu().numpy()
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    assert info["status"] == 0 and res <= 1e-8, res
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES)
    xo, oi = so.solve(b, 1e-11)
    say("cube64 schur oracle", oi)
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


def test_cube48_adjoint_gradient():
    n = 48
    th = S.theta_field(n, 0.5, 5)
    thr = S.theta_field(n, 0.5, 50)
    b = S.mms_rhs(n)
    # target from the reference viscosity
    pr, cr, vr = mgk.stokes_bsr(n, thr)
    s_ref = solver(pr, cr, vr, hier=mgk.F64)
    dxt = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    s_ref.solve(dev(b), dxt, 1e-12)
    ptr, col, val = mgk.stokes_bsr(n, th)
    s = solver(ptr, col, val, hier=mgk.F32, enable_transpose=1)
    dx = torch.zeros_like(dxt)
    s.solve(dev(b), dx, 1e-10)
    dlam = torch.zeros_like(dx)
    info = s.solve_transposed(dx - dxt, dlam, 1e-10)
    say("adjoint", info)
    g = torch.empty((n - 1) ** 3, dtype=torch.float64, device=DEV)
    mgk.theta_grad(n, dlam, dx, g)
    g = g.cpu().numpy()
    # oracle gradient over all cells (FP64 forward and adjoint at rtol 1e-12)
    A = oracle.stokes_matrix(n, th)
    so = oracle.Solver(A, 4)
    xo, _ = so.solve(b, 1e-12)
    xto, _ = oracle.Solver(oracle.stokes_matrix(n, thr), 4).solve(b, 1e-12)
    lo, _ = so.solve(xo - xto, 1e-12, transposed=True)
    go = oracle.theta_gradient(n, lo, xo)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    say("gradient vs oracle", rel)
    assert rel <= 1e-6
    # central differences (step 1e-6) on 20 seeded cells.  x(theta +- d) is obtained from the
    # base solution by one defect-correction solve, A(theta +- d) c = b - A(theta +- d) x,
    # x(theta +- d) = x + c, with an FP64 hierarchy: the correction is small, so a relative
    # tolerance of 1e-10 on it gives x(theta +- d) to about 1e-16 of ||x||.
    cells = S.fd_cells(n, 20, 51)
    xb = dx.clone()

    def correction(t):
        p_, c_, v_ = mgk.stokes_bsr(n, t)
        sf = solver(p_, c_, v_, hier=mgk.F64)
        ax = torch.empty_like(xb)
        sf.spmv(xb, ax)
        r = dev(b) - ax
        c = torch.zeros_like(xb)
        inf = sf.solve(r, c, 1e-10)
        assert inf["status"] == 0, inf
        return c

    # (L(t+) - L(t-)) / 2d with L = ||x - x_t||^2 / 2, written as
    # (x+ - x-) . (x+ + x- - 2 x_t) / (4 d) so that the difference is not lost to cancellation
    fd = []
    for e in cells:
        d = np.zeros_like(th)
        d[e] = 1e-6
        cp, cm = correction(th + d), correction(th - d)
        fd.append(float(torch.dot(cp - cm, cp + cm + 2.0 * (xb - dxt))) / 4e-6)
    fd = np.array(fd)
    relfd = np.linalg.norm(g[cells] - fd) / np.linalg.norm(fd)
    say("gradient vs central FD", relfd)
    assert relfd <= 1e-6


# Random interior body forces excite the slow modes of the 64^3 operator: at rtol 1e-8 a
# column's solution error lands anywhere up to about 1.5e-6 (1.49e-6 measured for column 0),
# depending on how far below 1e-8 its last iteration takes the residual.  The benchmark
# therefore solves this workload to rtol 1e-9, where both bars hold on the same solve.
MULTI64_RTOL = 1e-9


def test_cube64_32rhs_lockstep_vs_oracle():
    """The solve the benchmark times (rtol 1e-9): all 32 columns meet ||b - A x|| <= 1e-8 ||b||
    (oracle SpMV); columns 0, 9, 17 and 31 match oracle solves to 1e-6."""
    n, K = 64, 32
    ptr, col, val = mgk.stokes_bsr(n)
    Bm = S.body_forces(n, K, 4)
    s = solver(ptr, col, val, hier=mgk.F32)
    dB = dev(Bm)
    dX = torch.zeros_like(dB)
    infos = s.solve_multi(dB, dX, MULTI64_RTOL)
    X = dX.cpu().numpy()
    say("multi64", [i["iters"] for i in infos])
    A = oracle.stokes_matrix(n)
    AX = np.column_stack([oracle.spmv(A, np.ascontiguousarray(X[:, k])) for k in range(K)])
    res = np.linalg.norm(Bm - AX, axis=0) / np.linalg.norm(Bm, axis=0)
    assert all(i["status"] == 0 for i in infos) and res.max() <= MULTI64_RTOL, res.max()
    so = oracle.Solver(A, 4)
    for k in (0, 9, 17, 31):
        xo, _ = so.solve(np.ascontiguousarray(Bm[:, k]), 1e-11)
        err = np.linalg.norm(X[:, k] - xo) / np.linalg.norm(xo)
        say("multi64 column", k, "error", err)
        assert err <= 1e-6, (k, err)


def test_batch_eight_systems_vs_oracle():
    """The eight log-normal systems (24^3 ... 64^3) in one batched solve: every system meets
    1e-8 (oracle SpMV); the 24^3 and one 64^3 system match oracle solves."""
    ns = [24, 32, 40, 48, 48, 56, 64, 64]
    systems, bs, As = [], [], []
    for k, n in enumerate(ns):
        th = S.theta_field(n, 0.5, 40 + k)
        systems.append(mgk.stokes_bsr(n, th))
        A = oracle.stokes_matrix(n, th)
        As.append(A)
        bs.append(oracle.spmv(A, S.mms_solution(n)))
    bsol = mgk.BatchSolver(systems, 4, mgk.AMG_SPAI0, stream=torch.cuda.current_stream(),
                           hier=mgk.F32)
    db = [dev(b) for b in bs]
    xs = [torch.zeros_like(b) for b in db]
    infos = bsol.solve(db, xs, 1e-8)
    say("batch8", [i["iters"] for i in infos])
    for k, (A, b, x) in enumerate(zip(As, bs, xs)):
        xk = x.cpu().numpy()
        assert infos[k]["status"] == 0
        assert np.linalg.norm(b - oracle.spmv(A, xk)) <= 1e-8 * np.linalg.norm(b), k
        if k in (0, 6):
            xo, _ = oracle.Solver(A, 4).solve(b, 1e-11)
            assert np.linalg.norm(xk - xo) <= 1e-6 * np.linalg.norm(xo), k


# the paper's Schur configuration on the 64^3 log-normal system, as the benchmark times it:
# IDR(5), plain-aggregation velocity AMG (scalar or 3x3-block values), pressure step one
# SPAI(0) application of the diagonal Schur approximation, and the velocity AMG smoothed by
# block ILUT(2, 0.01) (the paper's smoother) or block ILU(0)
PAPER_SCHUR64 = {
    "scalar_f64": dict(hier="f64", schur_scalar_u=1),
    "f64": dict(hier="f64"),
    "f32": dict(hier="f32"),
    "bf16": dict(hier="bf16"),
    "ilut_f64": dict(hier="f64", ilu_smoother=1, ilu_kind=1, ilu_sweeps=2),
    "ilut_f32": dict(hier="f32", ilu_smoother=1, ilu_kind=1, ilu_sweeps=2),
    "ilu_f64": dict(hier="f64", ilu_smoother=1, ilu_sweeps=2),
    "ilu_f32": dict(hier="f32", ilu_smoother=1, ilu_sweeps=2),
}


@pytest.fixture(scope="module")
def cube64_lognormal():
    n = 64
    th = S.theta_field(n, 1.0, 3)
    A = oracle.stokes_matrix(n, th)
    xs = S.mms_solution(n)
    return mgk.stokes_bsr(n, th), A, oracle.spmv(A, xs), xs


# The log-normal viscosity (sigma = 1, spanning about e^(+-4)) amplifies the residual into
# the solution: at rtol 1e-8 the solution error is about 1e-6 (1.08e-6 measured for the FP32
# arm).  The benchmark therefore solves this workload to rtol 1e-9, where both bars hold on
# the same solve.
PAPER_SCHUR64_RTOL = 1e-9


@pytest.mark.parametrize("arm", list(PAPER_SCHUR64))
def test_cube64_paper_schur_idrs(cube64_lognormal, arm):
    """b = A x* (x* the manufactured nodal values), so x* is the exact solution.  The solve
    the benchmark times (rtol 1e-9) must meet both bars: ||b - A x|| <= 1e-8 ||b|| (by the
    oracle's SpMV) and ||x - x*|| <= 1e-6 ||x*||."""
    (ptr, col, val), A, b, xs = cube64_lognormal
    kw = dict(PAPER_SCHUR64[arm])
    hier = {"f64": mgk.F64, "f32": mgk.F32, "bf16": mgk.BF16}[kw.pop("hier")]
    say("paper_schur64", arm)
    s = solver(ptr, col, val, kind=mgk.SCHUR, hier=hier, krylov=mgk.IDRS, idr_s=5,
               coarsening=mgk.PLAIN_AGGREGATION, schur_approx=1, schur_spai0=1, **kw)
    dx = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, PAPER_SCHUR64_RTOL)
    say("paper_schur64 gpu", arm, info)
    x = dx.cpu().numpy()
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    say("paper_schur64 residual", res, "error", err)
    assert info["status"] == 0 and res <= PAPER_SCHUR64_RTOL, res
    assert err <= 1e-6, err


@pytest.fixture(scope="module")
def cube48_noise():
    n = 48
    A = oracle.stokes_matrix(n)
    b = S.c2_rhs(n)
    xo, oi = oracle.Solver(A, 4).solve(b, 1e-11)
    say("cube48 oracle", oi)
    return mgk.stokes_bsr(n), A, b, xo


@pytest.mark.parametrize("arm", ["ilu1_f64", "ilu1_f32", "amg_f32"])
def test_cube48_idrs_ilu1(cube48_noise, arm):
    """IDR(5) with block ILU(1) (3 Jacobi sweeps per factor) and with the FP32 AMG on the
    48^3 manufactured-plus-noise system, against the oracle's FP64 solve."""
    (ptr, col, val), A, b, xo = cube48_noise
    kind, kw = {"ilu1_f64": (mgk.ILU, dict(ilu_level=1, ilu_sweeps=3)),
                "ilu1_f32": (mgk.ILU, dict(ilu_level=1, ilu_sweeps=3, hier=mgk.F32)),
                "amg_f32": (mgk.AMG_SPAI0, dict(hier=mgk.F32))}[arm]
    s = solver(ptr, col, val, kind=kind, krylov=mgk.IDRS, idr_s=5, maxiter=4000, **kw)
    dx = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("ilu48 gpu", arm, info)
    x = dx.cpu().numpy()
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    assert info["status"] == 0 and res <= 1e-8, res
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


def test_batch_32_small_systems():
    """The 32 small log-normal systems (12^3 ... 22^3 nodes) in one batched solve, as the
    benchmark times them: b_k = A_k x*, so every system's exact solution is x*."""
    ns = [12 + (k % 6) * 2 for k in range(32)]
    systems, bs, As, xs_ = [], [], [], []
    for k, n in enumerate(ns):
        th = S.theta_field(n, 0.5, 100 + k)
        systems.append(mgk.stokes_bsr(n, th))
        A = oracle.stokes_matrix(n, th)
        As.append(A)
        xs_.append(S.mms_solution(n))
        bs.append(oracle.spmv(A, xs_[-1]))
    bsol = mgk.BatchSolver(systems, 4, mgk.AMG_SPAI0, stream=torch.cuda.current_stream(),
                           hier=mgk.F32, coarse_enough=500)
    db = [dev(b) for b in bs]
    xs = [torch.zeros_like(b) for b in db]
    infos = bsol.solve(db, xs, 1e-8)
    say("batch32small", [i["iters"] for i in infos])
    for k, (A, b, x, xe) in enumerate(zip(As, bs, xs, xs_)):
        xk = x.cpu().numpy()
        assert infos[k]["status"] == 0, k
        assert np.linalg.norm(b - oracle.spmv(A, xk)) <= 1e-8 * np.linalg.norm(b), k
        assert np.linalg.norm(xk - xe) <= 1e-6 * np.linalg.norm(xe), k
