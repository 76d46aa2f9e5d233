"""GPU parity of the solver variants: plain aggregation, IDR(s), the Schur
pressure-correction options (diagonal approximation of the pressure operator,
SPAI(0) pressure step, lower factorization), and the block ILU(k) preconditioner
with Jacobi-iterated triangular solves, against the FP64 CPU oracle.

Bars as for the other parity tests: ||b - A x|| / ||b|| <= 1e-8 with the oracle's
SpMV, and agreement with the oracle's FP64 solve (rtol 1e-12) to 1e-6 relative.
"""
import numpy as np
import pytest

import oracle
import stokes_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2006_06052_amd as mgk  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(n, sigma=None, seed=1):
    th = None if sigma is None else S.theta_field(n, sigma, seed)
    ptr, col, val = mgk.stokes_bsr(n, th)
    return th, (ptr, col, val), oracle.stokes_matrix(n, th)


def gpu_solver(bsr, kind=mgk.AMG_SPAI0, **kw):
    return mgk.Solver(*bsr, 4, kind, stream=torch.cuda.current_stream(), **kw)


def check_solution(A, b, x, xo, tol=1e-8, err=1e-6):
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    e = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert res <= tol, res
    assert e <= err, e
    return res, e


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_plain_aggregation_solve(storage):
    n = 16
    th, bsr, A = problem(n, 0.5, 11)
    b = oracle.spmv(A, S.mms_solution(n))
    s = gpu_solver(bsr, hier=storage, coarse_enough=300, coarsening=mgk.PLAIN_AGGREGATION)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    so = oracle.Solver(A, 4, coarse_enough=300, coarsening=oracle.PLAIN)
    xo, oi = so.solve(b, 1e-12)
    say("plain", storage, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)
    if storage == "f64":
        # same hierarchy, same method: the V-cycle agrees with the oracle's
        r = np.random.default_rng(2).normal(size=A.shape[0])
        dz = torch.empty_like(dx)
        s.precond(dev(r), dz)
        zo = so.precond(r)
        assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)


@pytest.mark.parametrize("s_dim,storage", [(1, "f64"), (5, "f64"), (8, "f64"), (5, "f32"),
                                           (5, "bf16")])
def test_idrs_solve(s_dim, storage):
    """IDR(s) against the oracle's IDR(s) solve (same shadow space); with the FP64
    hierarchy the two runs are the same method and take about the same number of
    products with A."""
    n = 16
    th, bsr, A = problem(n, 0.5, 12)
    b = oracle.spmv(A, S.mms_solution(n))
    s = gpu_solver(bsr, hier=storage, coarse_enough=300, krylov=mgk.IDRS, idr_s=s_dim)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    so = oracle.Solver(A, 4, coarse_enough=300, krylov=oracle.IDRS, idr_s=s_dim)
    xo, oi = so.solve(b, 1e-12)
    xo8, oi8 = so.solve(b, 1e-8)
    say("idrs", s_dim, storage, info, oi8["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)
    if storage == "f64":
        assert abs(info["iters"] - oi8["iters"]) <= max(3, oi8["iters"] // 10)


def test_idrs_transposed_and_edge_cases():
    n = 10
    th, bsr, A = problem(n, 0.5, 13)
    s = gpu_solver(bsr, coarse_enough=200, krylov=mgk.IDRS, enable_transpose=1)
    g = np.random.default_rng(3).normal(size=A.shape[0])
    dl = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve_transposed(dev(g), dl, 1e-9)
    lo, _ = oracle.Solver(A, 4, coarse_enough=200, krylov=oracle.IDRS).solve(g, 1e-12,
                                                                                transposed=True)
    assert info["status"] == 0
    At = A.T.tocsr()
    check_solution(At, g, dl.cpu().numpy(), lo, tol=1e-9)
    # zero right-hand side, and an iteration cap
    z = torch.zeros_like(dl)
    x = torch.ones_like(dl)
    info = s.solve(z, x, 1e-8)
    assert info["status"] == 0 and info["iters"] == 0 and not torch.any(x)
    s1 = gpu_solver(bsr, coarse_enough=200, krylov=mgk.IDRS, maxiter=3, max_restarts=0)
    x = torch.zeros_like(dl)
    info = s1.solve(dev(S.mms_rhs(n)), x, 1e-12)
    assert info["status"] == mgk.MGK_NOT_CONVERGED and info["iters"] == 3


@pytest.mark.parametrize("approx,spai0,lower", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0),
                                                (1, 1, 1)])
def test_schur_variants_match_oracle(approx, spai0, lower):
    """Schur preconditioner options: the FP64 application agrees with the oracle's, and
    FGMRES solves reach the oracle's solution."""
    n = 14
    th, bsr, A = problem(n, 1.0, 3)
    b = oracle.spmv(A, S.mms_solution(n))
    kw = dict(schur_approx=approx, schur_spai0=spai0, schur_lower=lower, coarse_enough=200)
    s = gpu_solver(bsr, mgk.SCHUR, krylov=mgk.FGMRES, **kw)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES, **kw)
    r = np.random.default_rng(4).normal(size=A.shape[0])
    dz = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    s.precond(dev(r), dz)
    zo = so.precond(r)
    assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    dx = torch.zeros_like(dz)
    info = s.solve(dev(b), dx, 1e-8)
    xo, oi = so.solve(b, 1e-12)
    say("schur variant", kw, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_paper_schur_configuration_idrs(storage):
    """The paper's Schur configuration on the GPU: IDR(5) outer solver; velocity AMG with
    plain aggregation on the 3x3 blocks; pressure step one SPAI(0) application of the
    diagonal approximation of the Schur complement; full factorization; FP64 or BF16
    hierarchy values."""
    n = 16
    th, bsr, A = problem(n, 1.0, 14)
    b = oracle.spmv(A, S.mms_solution(n))
    kw = dict(schur_approx=1, schur_spai0=1, coarse_enough=300)
    s = gpu_solver(bsr, mgk.SCHUR, krylov=mgk.IDRS, idr_s=5, hier=storage,
                   coarsening=mgk.PLAIN_AGGREGATION, **kw)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.IDRS, idr_s=5,
                       coarsening=oracle.PLAIN, **kw)
    xo, oi = so.solve(b, 1e-12)
    say("paper schur", storage, info, oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("level,sweeps", [(0, 2), (1, 3), (1, 0)])
def test_ilu_application_matches_oracle(level, sweeps):
    """Block ILU(k) with Jacobi-iterated triangular solves: the FP64 application agrees
    with the oracle's to rounding."""
    n = 10
    th, bsr, A = problem(n, 0.5, 15)
    kw = dict(ilu_level=level, ilu_sweeps=sweeps)
    s = gpu_solver(bsr, mgk.ILU, **kw)
    so = oracle.Solver(A, 4, kind=oracle.KIND_ILU, **kw)
    r = np.random.default_rng(5).normal(size=A.shape[0])
    dz = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    s.precond(dev(r), dz)
    zo = so.precond(r)
    assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-12 * np.linalg.norm(zo)
    with pytest.raises(mgk.MgkError):
        s.precond(dev(r), dz, transposed=True)


@pytest.mark.parametrize("storage,krylov", [("f64", "idrs"), ("f32", "idrs"), ("bf16", "idrs"),
                                            ("f64", "bicgstab")])
def test_paper_monolithic_ilu_configuration(storage, krylov):
    """The paper's monolithic configuration, IDR(5) preconditioned with ILU(1), and
    BiCGStab with ILU(1), on a small system (ILU alone does not scale with size)."""
    n = 10
    th, bsr, A = problem(n, 0.5, 16)
    b = oracle.spmv(A, S.mms_solution(n))
    kr = {"idrs": (mgk.IDRS, oracle.IDRS), "bicgstab": (mgk.BICGSTAB, oracle.BICGSTAB)}[krylov]
    kw = dict(ilu_level=1, ilu_sweeps=3)
    s = gpu_solver(bsr, mgk.ILU, hier=storage, krylov=kr[0], idr_s=5, **kw)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    so = oracle.Solver(A, 4, kind=oracle.KIND_ILU, krylov=kr[1], idr_s=5, **kw)
    xo, oi = so.solve(b, 1e-12)
    say("ilu", storage, krylov, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)
    B = torch.zeros((A.shape[0], 2), dtype=torch.float64, device=DEV)
    with pytest.raises(mgk.MgkError):
        s.solve_multi(B, torch.zeros_like(B), 1e-8)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_amg_with_ilu0_smoother(storage):
    """Every AMG level smoothed with block ILU(0) (2 Jacobi sweeps per factor): the FP64
    V-cycle agrees with the oracle's, and solves reach the oracle's solution."""
    n = 12
    th, bsr, A = problem(n, 0.5, 17)
    b = oracle.spmv(A, S.mms_solution(n))
    s = gpu_solver(bsr, hier=storage, coarse_enough=300, ilu_smoother=1, ilu_sweeps=2)
    so = oracle.Solver(A, 4, coarse_enough=300, smoother=oracle.ILU0, ilu_sweeps=2)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    if storage == "f64":
        r = np.random.default_rng(6).normal(size=A.shape[0])
        s.precond(dev(r), dx)
        zo = so.precond(r)
        assert np.linalg.norm(dx.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
        dx.zero_()
    info = s.solve(dev(b), dx, 1e-8)
    xo, oi = so.solve(b, 1e-12)
    say("ilu smoother", storage, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)
    with pytest.raises(mgk.MgkError):
        gpu_solver(bsr, ilu_smoother=1, enable_transpose=1)
    B = torch.zeros((A.shape[0], 2), dtype=torch.float64, device=DEV)
    with pytest.raises(mgk.MgkError):
        s.solve_multi(B, torch.zeros_like(B), 1e-8)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_paper_v2_shape_schur_ilu_smoothed(storage):
    """The paper's Schur variant shape: IDR(5); velocity AMG with plain aggregation and
    ILU smoothing (block ILU(0) in place of ILUT) on the 3x3 blocks; SPAI(0) pressure
    step on the diagonal Schur approximation; FP64 or FP32 hierarchy (V3 / V4)."""
    n = 14
    th, bsr, A = problem(n, 1.0, 18)
    b = oracle.spmv(A, S.mms_solution(n))
    kw = dict(schur_approx=1, schur_spai0=1, coarse_enough=300, ilu_sweeps=2)
    s = gpu_solver(bsr, mgk.SCHUR, krylov=mgk.IDRS, idr_s=5, hier=storage, ilu_smoother=1,
                   coarsening=mgk.PLAIN_AGGREGATION, **kw)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.IDRS, idr_s=5,
                       smoother=oracle.ILU0, coarsening=oracle.PLAIN, **kw)
    xo, oi = so.solve(b, 1e-12)
    say("paper v2 shape", storage, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("p,tau,sweeps", [(2.0, 1e-2, 2), (1.0, 5e-2, 3), (3.0, 1e-3, 0)])
def test_ilut_application_matches_oracle(p, tau, sweeps):
    """Block ILUT(p, tau) as the monolithic preconditioner: the FP64 application (Jacobi
    sweeps on the threshold factors) agrees with the oracle's to rounding."""
    n = 10
    th, bsr, A = problem(n, 0.5, 25)
    s = gpu_solver(bsr, mgk.ILU, ilu_kind=1, ilut_p=p, ilut_tau=tau, ilu_sweeps=sweeps)
    so = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_kind=1, ilut_p=p, ilut_tau=tau,
                       ilu_sweeps=sweeps)
    r = np.random.default_rng(8).normal(size=A.shape[0])
    dz = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    s.precond(dev(r), dz)
    zo = so.precond(r)
    assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-12 * np.linalg.norm(zo)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_paper_schur_ilut_smoothed(storage):
    """The paper's Schur configuration (listings V2-V4): IDR(5); velocity AMG with plain
    aggregation smoothed by block ILUT(2, 0.01) on the 3x3 blocks; SPAI(0) pressure step on
    the diagonal Schur approximation.  The FP64 preconditioner application agrees with the
    oracle's; FP64, FP32 and BF16 hierarchies solve to the oracle's solution."""
    n = 14
    th, bsr, A = problem(n, 1.0, 18)
    b = oracle.spmv(A, S.mms_solution(n))
    kw = dict(schur_approx=1, schur_spai0=1, coarse_enough=300, ilu_sweeps=2)
    s = gpu_solver(bsr, mgk.SCHUR, krylov=mgk.IDRS, idr_s=5, hier=storage, ilu_smoother=1,
                   ilu_kind=1, coarsening=mgk.PLAIN_AGGREGATION, **kw)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.IDRS, idr_s=5,
                       smoother=oracle.ILUT, coarsening=oracle.PLAIN, **kw)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    if storage == "f64":
        r = np.random.default_rng(10).normal(size=A.shape[0])
        s.precond(dev(r), dx)
        zo = so.precond(r)
        assert np.linalg.norm(dx.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
        dx.zero_()
    info = s.solve(dev(b), dx, 1e-8)
    xo, oi = so.solve(b, 1e-12)
    say("paper schur ilut", storage, info["iters"], oi["iters"])
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_amg_with_ilut_smoother(storage):
    """Monolithic AMG with every level smoothed by block ILUT: FP64 V-cycle vs oracle,
    solves vs the oracle's solution."""
    n = 12
    th, bsr, A = problem(n, 0.5, 26)
    b = oracle.spmv(A, S.mms_solution(n))
    s = gpu_solver(bsr, hier=storage, coarse_enough=300, ilu_smoother=1, ilu_kind=1,
                   ilu_sweeps=2)
    so = oracle.Solver(A, 4, coarse_enough=300, smoother=oracle.ILUT, ilu_sweeps=2)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    if storage == "f64":
        r = np.random.default_rng(11).normal(size=A.shape[0])
        s.precond(dev(r), dx)
        zo = so.precond(r)
        assert np.linalg.norm(dx.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
        dx.zero_()
    info = s.solve(dev(b), dx, 1e-8)
    xo, _ = so.solve(b, 1e-12)
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_schur_scalar_velocity_amg(storage):
    """Schur preconditioner with the velocity AMG on scalar values: agrees with the oracle
    (and, for this decoupled velocity operator, with the 3x3-block AMG)."""
    n = 14
    th, bsr, A = problem(n, 1.0, 19)
    b = oracle.spmv(A, S.mms_solution(n))
    kw = dict(coarse_enough=200, schur_scalar_u=1)
    s = gpu_solver(bsr, mgk.SCHUR, krylov=mgk.FGMRES, hier=storage, **kw)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES, **kw)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    if storage == "f64":
        r = np.random.default_rng(7).normal(size=A.shape[0])
        s.precond(dev(r), dx)
        zo = so.precond(r)
        assert np.linalg.norm(dx.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
        dx.zero_()
    info = s.solve(dev(b), dx, 1e-8)
    xo, _ = so.solve(b, 1e-12)
    assert info["status"] == 0
    check_solution(A, b, dx.cpu().numpy(), xo)
