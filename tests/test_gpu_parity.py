"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 products within gamma_k * sum|a||x| of the oracle; solves reach
||b - A x|| / ||b|| <= 1e-8 (checked with the oracle's own SpMV) and agree with the
oracle's FP64 solve (rtol 1e-12) to 1e-6 relative; repeated runs are bitwise equal.
"""
import numpy as np
import pytest

import oracle
import stokes_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2006_06052_amd as mgk  # noqa: E402

EPS = np.finfo(np.float64).eps
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(n, sigma=None, seed=1):
    th = None if sigma is None else S.theta_field(n, sigma, seed)
    ptr, col, val = mgk.stokes_bsr(n, th)
    return th, (ptr, col, val), oracle.stokes_matrix(n, th)


def gpu_solver(bsr, block=4, kind=mgk.AMG_SPAI0, **kw):
    stream = torch.cuda.current_stream()
    return mgk.Solver(*bsr, block, kind, stream=stream, **kw)


def check_solution(A, b, x, xo, tol=1e-8, err=1e-6):
    res = np.linalg.norm(b - oracle.spmv(A, x)) / np.linalg.norm(b)
    e = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert res <= tol, res
    assert e <= err, e
    return res, e


# ------------------------------------------------------------------ kernels

@pytest.mark.parametrize("n,sigma", [(16, None), (21, 1.0)])
def test_outer_spmv_matches_oracle_and_is_deterministic(n, sigma):
    say("spmv", n, sigma)
    th, bsr, A = problem(n, sigma)
    s = gpu_solver(bsr, coarse_enough=500)
    x = np.random.default_rng(0).normal(size=A.shape[0])
    dx = dev(x)
    dy = torch.empty_like(dx)
    s.spmv(dx, dy)
    y1 = dy.cpu().numpy()
    s.spmv(dx, dy)
    assert np.array_equal(y1, dy.cpu().numpy())
    yo = oracle.spmv(A, x)
    bound = 16 * EPS * (abs(A) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(y1 - yo) <= bound)


def test_transposed_spmv_is_adjoint():
    n = 13
    th, bsr, A = problem(n, 0.5)
    s = gpu_solver(bsr, coarse_enough=500, enable_transpose=1)
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    dy = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    s.spmv(dev(x), dy, level=-1, which=3)
    aty = dy.cpu().numpy()
    ref = A.T @ x
    assert np.allclose(aty, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    s.spmv(dev(x), dy)
    Ax = dy.cpu().numpy()
    s.spmv(dev(y), dy, level=-1, which=3)
    lhs, rhs = y @ Ax, dy.cpu().numpy() @ x
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(y) @ (abs(A) @ np.abs(x)))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_level_operators_match_rounded_oracle(storage):
    """A_l, P_l, R_l of the uploaded hierarchy against the oracle's level matrices with
    values rounded to the storage precision, vectors in the hierarchy precision."""
    n = 14
    th, bsr, A = problem(n, 0.5, 3)
    s = gpu_solver(bsr, coarse_enough=200, hier=storage)
    so = oracle.Solver(A, 4, coarse_enough=200)
    vdt = torch.float64 if storage == "f64" else torch.float32
    rng = np.random.default_rng(2)
    for l in range(s.nlevels() - 1):
        L = so.level(l)
        for which, key in ((0, "A"), (1, "P"), (2, "R")):
            M = L[key].copy()
            if storage == "f32":
                M.data = M.data.astype(np.float32).astype(np.float64)
            elif storage == "bf16":
                M.data = torch.from_numpy(M.data).to(torch.bfloat16).to(torch.float64).numpy()
            x = rng.normal(size=M.shape[1])
            if storage != "f64":
                x = x.astype(np.float32).astype(np.float64)
            dx = torch.from_numpy(x).to(vdt).to(DEV)
            dy = torch.empty(M.shape[0], dtype=vdt, device=DEV)
            say("level", l, key, storage)
            s.spmv(dx, dy, level=l, which=which)
            y = dy.double().cpu().numpy()
            ref = M @ x
            unit = EPS if storage == "f64" else np.finfo(np.float32).eps
            bound = 64 * unit * (abs(M) @ np.abs(x)) + 1e-30
            assert np.all(np.abs(y - ref) <= bound), (l, key)


def test_vcycle_matches_oracle_fp64():
    """With the bit-identical hierarchy, one FP64 V-cycle on the GPU equals the oracle's
    up to summation order."""
    n = 16
    th, bsr, A = problem(n, 0.5, 4)
    s = gpu_solver(bsr, coarse_enough=300, enable_transpose=1)
    so = oracle.Solver(A, 4, coarse_enough=300)
    r = np.random.default_rng(3).normal(size=A.shape[0])
    dz = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    for tr in (False, True):
        say("vcycle transposed", tr)
        s.precond(dev(r), dz, transposed=tr)
        z = dz.cpu().numpy()
        zo = so.precond(r, transposed=tr)
        assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)


SMOOTHERS = {"jacobi": (mgk.AMG_JACOBI, dict(), oracle.JACOBI),
             "spai0_scalar": (mgk.AMG_SPAI0, dict(block_spai0=0), oracle.SPAI0_SCALAR)}


@pytest.mark.parametrize("smoother", list(SMOOTHERS))
def test_other_smoothers_vcycle_and_solve(smoother):
    """Damped block Jacobi (omega_J = 2/3) and scalar-row SPAI(0) on every level: the FP64
    V-cycle (forward and transposed) against the oracle's at 1e-10, then solves with the
    FP64 and FP32 hierarchies against the oracle's FP64 solution."""
    kind, kw, osm = SMOOTHERS[smoother]
    n = 14
    th, bsr, A = problem(n, 0.5, 8)
    so = oracle.Solver(A, 4, smoother=osm, coarse_enough=300)
    s = gpu_solver(bsr, kind=kind, coarse_enough=300, enable_transpose=1, **kw)
    assert s.nlevels() >= 3
    r = np.random.default_rng(9).normal(size=A.shape[0])
    dz = torch.empty(A.shape[0], dtype=torch.float64, device=DEV)
    for tr in (False, True):
        say("smoother", smoother, "transposed", tr)
        s.precond(dev(r), dz, transposed=tr)
        zo = so.precond(r, transposed=tr)
        assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)
    b = S.mms_rhs(n)
    xo, _ = so.solve(b, 1e-12)
    for storage in ("f64", "f32"):
        s2 = gpu_solver(bsr, kind=kind, coarse_enough=300, hier=storage, **kw)
        dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
        info = s2.solve(dev(b), dx, 1e-8)
        say("smoother solve", smoother, storage, info)
        assert info["status"] == 0
        check_solution(A, b, dx.cpu().numpy(), xo)


# ------------------------------------------------------------------ solves

@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_c1_monolithic_bicgstab(storage):
    """16^3 manufactured problem, SA-AMG + SPAI0 V(1,1), BiCGStab to 1e-8."""
    n = 16
    th, bsr, A = problem(n)
    b = S.mms_rhs(n)
    s = gpu_solver(bsr, hier=storage)
    db, dx = dev(b), torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(db, dx, 1e-8)
    say("c1", storage, info)
    x = dx.cpu().numpy()
    xo, oi = oracle.Solver(A, 4).solve(b, 1e-12)
    check_solution(A, b, x, xo)
    assert info["status"] == 0 and info["rel_resid"] <= 1e-8
    # the mixed-precision preconditioner must not cost more than ~10% extra iterations
    _, o8 = oracle.Solver(A, 4).solve(b, 1e-8)
    assert info["iters"] <= int(np.ceil(1.1 * o8["iters"])) + 1, (info["iters"], o8["iters"])
    # determinism: a second solve from zero is bitwise identical
    dx2 = torch.zeros_like(dx)
    s.solve(db, dx2, 1e-8)
    assert torch.equal(dx, dx2)


def test_monolithic_lognormal_fgmres():
    n = 18
    th, bsr, A = problem(n, 1.0, 5)
    xs = S.mms_solution(n)
    b = oracle.spmv(A, xs)
    s = gpu_solver(bsr, hier="f32", krylov=mgk.FGMRES)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("fgmres mono", info)
    xo, _ = oracle.Solver(A, 4).solve(b, 1e-12)
    check_solution(A, b, dx.cpu().numpy(), xo)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_schur_fgmres(storage):
    """Schur pressure correction (3x3 velocity AMG, scalar pressure AMG on
    C - B_lo diag(A_uu)^-1 B_up) under FGMRES(30)."""
    n = 18
    th, bsr, A = problem(n, 1.0, 3)
    xs = S.mms_solution(n)
    b = oracle.spmv(A, xs)
    s = gpu_solver(bsr, kind=mgk.SCHUR, hier=storage, krylov=mgk.FGMRES)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("schur", storage, info)
    so = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES)
    xo, _ = so.solve(b, 1e-12)
    check_solution(A, b, dx.cpu().numpy(), xo)
    # the FP64 Schur preconditioner application matches the oracle's
    if storage == "f64":
        r = np.random.default_rng(4).normal(size=A.shape[0])
        dz = torch.empty_like(dx)
        s.precond(dev(r), dz)
        zo = so.precond(r)
        assert np.linalg.norm(dz.cpu().numpy() - zo) <= 1e-10 * np.linalg.norm(zo)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_schur_diagonal_layout_3x3(storage):
    """The Schur preconditioner's 3x3 velocity operators (7 block diagonals; Dirichlet rows
    hold only the diagonal block) read in the diagonal layout give bitwise the BSR results:
    preconditioner application and FGMRES solve."""
    n = 14
    th, bsr, A = problem(n, 1.0, 3)
    b = dev(oracle.spmv(A, S.mms_solution(n)))
    r = dev(np.random.default_rng(4).normal(size=A.shape[0]))
    outs = []
    for layout in (2, 1):
        s = gpu_solver(bsr, kind=mgk.SCHUR, hier=storage, krylov=mgk.FGMRES, layout=layout)
        assert s.level_info(0)["block"] == 3
        assert s.level_info(0)["dia"] == (7 if layout == 2 else 0)
        z = torch.empty_like(b)
        s.precond(r, z)
        x = torch.zeros_like(b)
        info = s.solve(b, x, 1e-8)
        assert info["status"] == 0
        outs.append((z.cpu().numpy(), x.cpu().numpy(), info["iters"]))
    for a, c in zip(outs[0], outs[1]):
        assert np.array_equal(a, c)


def test_scalar_csr_arm():
    """The same system as scalar CSR (block size 1) through the whole solver."""
    n = 12
    th, bsr, A = problem(n)
    b = S.mms_rhs(n)
    bptr, bcol, bval = mgk.csr_to_bsr(A.indptr, A.indices, A.data, 1)
    s = gpu_solver((bptr, bcol, bval), block=1, hier="f32")
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    info = s.solve(dev(b), dx, 1e-8)
    say("scalar", info)
    xo, _ = oracle.Solver(A, 1).solve(b, 1e-12)
    check_solution(A, b, dx.cpu().numpy(), xo)


def test_adjoint_and_gradients():
    n = 12
    th, bsr, A = problem(n, 0.5, 5)
    b = S.mms_rhs(n)
    s = gpu_solver(bsr, hier="f32", enable_transpose=1)
    dx = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    s.solve(dev(b), dx, 1e-10)
    x = dx.cpu().numpy()
    g = x - S.mms_solution(n)
    dl = torch.zeros_like(dx)
    info = s.solve_transposed(dev(g), dl, 1e-10)
    say("adjoint", info)
    lam = dl.cpu().numpy()
    assert np.linalg.norm(g - A.T @ lam) <= 1e-10 * np.linalg.norm(g)
    so = oracle.Solver(A, 4)
    lo, _ = so.solve(g, 1e-13, transposed=True)
    assert np.linalg.norm(lam - lo) <= 1e-6 * np.linalg.norm(lo)
    # per-cell gradient kernel against the oracle's formula on the same inputs
    dg = torch.empty((n - 1) ** 3, dtype=torch.float64, device=DEV)
    mgk.theta_grad(n, dl, dx, dg)
    go = oracle.theta_gradient(n, lam, x)
    assert np.allclose(dg.cpu().numpy(), go, rtol=1e-12, atol=1e-12 * np.abs(go).max())
    # block-pattern gradient -lambda_I x_J^T
    ptr, col, val = bsr
    dG = torch.empty(val.size, dtype=torch.float64, device=DEV)
    s.bsr_grad(dl, dx, dG)
    G = dG.cpu().numpy().reshape(-1, 4, 4)
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    ref = -lam.reshape(-1, 4)[rows][:, :, None] * x.reshape(-1, 4)[col][:, None, :]
    assert np.array_equal(G, ref)


def test_edge_cases():
    n = 8
    th, bsr, A = problem(n)
    s = gpu_solver(bsr, coarse_enough=100, maxiter=1, max_restarts=0)
    z = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    x = torch.ones_like(z)
    info = s.solve(z, x, 1e-8)
    assert info["status"] == 0 and info["iters"] == 0 and not torch.any(x)
    b = dev(S.mms_rhs(n))
    x = torch.zeros_like(b)
    info = s.solve(b, x, 1e-12)
    assert info["status"] == mgk.MGK_NOT_CONVERGED and info["iters"] == 1
    # warm start from the exact discrete solution converges immediately
    s2 = gpu_solver(bsr, coarse_enough=100)
    xs = S.mms_solution(n)
    bx = dev(oracle.spmv(A, xs))
    x = dev(xs)
    info = s2.solve(bx, x, 1e-8)
    assert info["status"] == 0 and info["iters"] == 0
    with pytest.raises(mgk.MgkError):
        s2.solve_transposed(bx, x, 1e-8)   # set up without transpose indices
    with pytest.raises(TypeError):
        s2.solve(bx.float(), x, 1e-8)


def test_timing_switch_leaves_results_bitwise_equal():
    """mgk_set_timing turns the solve's timing events off and on again; the iterates do not
    depend on it (the events only mark points on the stream)."""
    n = 12
    th, bsr, A = problem(n, 1.0, 3)
    b = dev(S.c2_rhs(n, 1e-3, 5))
    s = gpu_solver(bsr, coarse_enough=300, hier=mgk.F32, time_spmv=3)
    xs = []
    for mask in (3, 0, 1, 2, 3):
        s.set_timing(mask)
        x = torch.zeros_like(b)
        info = s.solve(b, x, 1e-8)
        assert info["status"] == 0
        assert (info["spmv_calls"] > 0) == bool(mask & 1), (mask, info["spmv_calls"])
        assert (info["precond_calls"] > 0) == bool(mask & 2), (mask, info["precond_calls"])
        xs.append(x)
    for x in xs[1:]:
        assert torch.equal(x, xs[0])
    with pytest.raises(mgk.MgkError):
        s.set_timing(4)
    # bits not set at setup stay off
    s0 = gpu_solver(bsr, coarse_enough=300, hier=mgk.F32)
    s0.set_timing(3)
    x = torch.zeros_like(b)
    info = s0.solve(b, x, 1e-8)
    assert info["spmv_calls"] == 0 and info["precond_calls"] == 0
    assert torch.equal(x, xs[0])


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_results_independent_of_kernel_tile(storage):
    """Every engine tile sums in the same fixed order, so SpMV and whole solves are bitwise
    identical whatever tile the autotuner (or force_tile) selects."""
    n = 14
    th, bsr, A = problem(n, 0.5, 8)
    b = dev(S.mms_rhs(n))
    x0 = dev(np.random.default_rng(9).normal(size=A.shape[0]))
    outs = []
    # 10000*RPL + 100*S + U; the RPL 2 / 4 tiles are the wide lanes of 4x4 blocks (every
    # storage, the FP64 outer operator and its fused dots included)
    for tile in (0, 108, 202, 204, 402, 404, 804, 1602, 20204, 20402, 20404, 20802, 21602,
                 40402, 40801, 41601):
        say("tile", storage, tile)
        s = gpu_solver(bsr, hier=storage, coarse_enough=200, force_tile=tile)
        y = torch.empty_like(b)
        s.spmv(x0, y)
        x = torch.zeros_like(b)
        info = s.solve(b, x, 1e-8)
        outs.append((y.cpu().numpy(), x.cpu().numpy(), info["iters"]))
    for y, x, it in outs[1:]:
        assert np.array_equal(y, outs[0][0])
        assert np.array_equal(x, outs[0][1]) and it == outs[0][2]
    with pytest.raises(mgk.MgkError):
        gpu_solver(bsr, hier=storage, force_tile=303)
    with pytest.raises(mgk.MgkError):
        gpu_solver(bsr, hier=storage, force_tile=30402)   # no 3-row lanes of 4x4 blocks


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_diagonal_layout_matches_bsr_bitwise(storage):
    """The fine operator of the Stokes system has 7 block diagonals, so it can be read in
    the diagonal-offset layout.  Its rows are either full (same products in the same order
    as BSR) or a lone diagonal block (the padding adds exact +0), so SpMV, V-cycle and
    whole solves are bitwise those of the BSR layout.  At 14^3 the Dirichlet rows pad the
    layout by 46%, so the automatic choice keeps BSR and layout 2 forces the diagonals."""
    n = 14
    th, bsr, A = problem(n, 0.5, 8)
    b = dev(S.mms_rhs(n))
    x0 = dev(np.random.default_rng(9).normal(size=A.shape[0]))
    outs = []
    for layout, k in ((2, 7), (1, 0), (0, 0)):
        say("layout", storage, layout)
        s = gpu_solver(bsr, hier=storage, coarse_enough=200, layout=layout)
        assert s.level_info(0)["dia"] == k
        y = torch.empty_like(b)
        s.spmv(x0, y)
        z = torch.empty_like(b)
        s.precond(x0, z)
        x = torch.zeros_like(b)
        info = s.solve(b, x, 1e-8)
        assert info["outer_dia"] == k
        outs.append((y.cpu().numpy(), z.cpu().numpy(), x.cpu().numpy(), info["iters"]))
    for o in outs[1:]:
        for a, c in zip(outs[0], o):
            assert np.array_equal(a, c)


def test_diagonal_layout_chosen_at_scale():
    """At 40^3 the boundary rows pad the 7 diagonals by 14%: the automatic choice reads the
    fine operator (outer and hierarchy level 0) in the diagonal layout, aggregated levels
    in BSR."""
    ptr, col, val = mgk.stokes_bsr(40)
    s = gpu_solver((ptr, col, val), hier="f32", coarse_enough=2000)
    assert s.level_info(0)["dia"] == 7
    assert all(s.level_info(l)["dia"] == 0 for l in range(1, s.nlevels()))
    b = torch.ones(4 * 40 ** 3, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    info = s.solve(b, x, 1e-8)
    assert info["outer_dia"] == 7 and info["rel_resid"] <= 1e-8


def drop_mirrored_pairs(bsr, seed):
    """The BSR operator with about 4% of its off-diagonal blocks dropped in mirrored pairs
    (every block diagonal keeps some blocks, so the diagonal layout still has 7 slots)."""
    ptr, col, val = bsr
    rng = np.random.default_rng(seed)
    nbr = ptr.size - 1
    keep = np.ones(col.size, bool)
    rows = np.repeat(np.arange(nbr), np.diff(ptr))
    pos = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(rows, col))}
    for k in np.flatnonzero(rng.random(col.size) < 0.02):
        i, j = int(rows[k]), int(col[k])
        if i != j and (j, i) in pos:
            keep[k] = keep[pos[(j, i)]] = False
    nptr = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=nbr))]).astype(np.int32)
    assert 0.94 * col.size < keep.sum() < 0.98 * col.size
    return nptr, col[keep].copy(), val[keep].copy()


def test_diagonal_layout_with_partial_rows():
    """Rows with some diagonals missing are padded with zero blocks, which moves products
    between summation stripes: SpMV stays within the FP64 bound of the oracle, and a few
    solver iterations agree with the BSR layout to rounding."""
    n = 12
    th, bsr, A0 = problem(n, 0.5, 4)
    pbsr = drop_mirrored_pairs(bsr, 5)
    import scipy.sparse as sp
    A = sp.bsr_matrix((pbsr[2], pbsr[1], pbsr[0]), shape=A0.shape).tocsr()
    x = np.random.default_rng(1).normal(size=A.shape[0])
    b = dev(A @ np.ones(A.shape[0]))
    res = []
    for layout in (2, 1):
        say("partial rows, layout", layout)
        s = gpu_solver(pbsr, coarse_enough=200, layout=layout, maxiter=4)
        assert s.level_info(0)["dia"] == (7 if layout == 2 else 0)
        dy = torch.empty_like(b)
        s.spmv(dev(x), dy)
        y = dy.cpu().numpy()
        bound = 16 * EPS * (abs(A) @ np.abs(x)) + 1e-300
        assert np.all(np.abs(y - A @ x) <= bound)
        z = torch.empty_like(b)
        s.precond(dev(x), z)
        xs = torch.zeros_like(b)
        s.solve(b, xs, 1e-14)
        res.append((z.cpu().numpy(), xs.cpu().numpy()))
    for a, c in zip(res[0], res[1]):
        assert np.linalg.norm(a - c) <= 1e-10 * np.linalg.norm(c)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_cached_and_streamed_value_loads_agree(storage, monkeypatch):
    """Value loads are streamed or cached by operator precision; the arithmetic is the same,
    so SpMV, V-cycle and solves are bitwise identical whichever load every operator uses."""
    n = 14
    th, bsr, A = problem(n, 0.5, 8)
    b = dev(S.mms_rhs(n))
    x0 = dev(np.random.default_rng(9).normal(size=A.shape[0]))
    outs = []
    for mode in ("0", "1", "2", "4", "8", "15"):
        monkeypatch.setenv("MGK_CACHED_LOADS", mode)
        s = gpu_solver(bsr, hier=storage, coarse_enough=200)
        y = torch.empty_like(b)
        s.spmv(x0, y)
        z = torch.empty_like(b)
        s.precond(x0, z)
        x = torch.zeros_like(b)
        info = s.solve(b, x, 1e-8)
        outs.append((y.cpu().numpy(), z.cpu().numpy(), x.cpu().numpy(), info["iters"]))
    for o in outs[1:]:
        for a, c in zip(outs[0], o):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("storage", ["f64", "bf16"])
def test_batch_diagonal_layout_bitwise(storage):
    """The grouped kernels read every system's fine operator (outer and hierarchy level 0)
    in its diagonal layout, with row masks for the Dirichlet rows (the 10^3 system pads its
    7 diagonals by 58%): a batched solve is bitwise the one with every operator in BSR."""
    ns = [10, 13, 16]
    probs = [problem(n, 0.5, 70 + k) for k, n in enumerate(ns)]
    bs = [dev(oracle.spmv(A, S.mms_solution(n))) for n, (_, _, A) in zip(ns, probs)]
    outs = []
    for layout in (0, 1):
        say("batch layout", storage, layout)
        bsol = mgk.BatchSolver([p[1] for p in probs], 4, mgk.AMG_SPAI0,
                               stream=torch.cuda.current_stream(), hier=storage,
                               coarse_enough=300, layout=layout)
        xs = [torch.zeros_like(b) for b in bs]
        infos = bsol.solve(bs, xs, 1e-8)
        assert all(i["status"] == 0 for i in infos)
        outs.append(([x.cpu().numpy() for x in xs], [i["iters"] for i in infos]))
    assert outs[0][1] == outs[1][1]
    for a, c in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, c)


def test_cached_and_streamed_loads_agree_in_batches(monkeypatch):
    """The grouped batch kernels take the same load policy: a batched solve is bitwise the
    same with every operator streamed and every operator cached."""
    ns = [10, 13]
    probs = [problem(n, 0.5, 60 + k) for k, n in enumerate(ns)]
    bs = [dev(oracle.spmv(A, S.mms_solution(n))) for n, (_, _, A) in zip(ns, probs)]
    outs = []
    for mode in ("0", "15"):
        monkeypatch.setenv("MGK_CACHED_LOADS", mode)
        bsol = mgk.BatchSolver([p[1] for p in probs], 4, mgk.AMG_SPAI0,
                               stream=torch.cuda.current_stream(), hier="bf16",
                               coarse_enough=300)
        xs = [torch.zeros_like(b) for b in bs]
        infos = bsol.solve(bs, xs, 1e-8)
        outs.append(([x.cpu().numpy() for x in xs], [i["iters"] for i in infos]))
    assert outs[0][1] == outs[1][1]
    for a, c in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_multi_rhs_lockstep(storage):
    """K right-hand sides in one lockstep solve: every column meets the tolerance (oracle
    SpMV), agrees with the oracle's solve of that column, and a zero column stays zero."""
    n = 14
    th, bsr, A = problem(n, 0.5, 21)
    K = 9
    Bm = S.body_forces(n, K, 4)
    Bm[:, 3] = 0.0                        # a zero right-hand side
    Bm[:, 5] = S.mms_rhs(n)               # a manufactured one
    s = gpu_solver(bsr, hier=storage)
    dB = dev(Bm)
    dX = torch.zeros_like(dB)
    infos = s.solve_multi(dB, dX, 1e-8)
    say("multi", storage, [i["iters"] for i in infos])
    X = dX.cpu().numpy()
    assert not np.any(X[:, 3]) and infos[3]["iters"] == 0
    so = oracle.Solver(A, 4)
    for k in range(K):
        if k == 3:
            continue
        assert infos[k]["status"] == 0
        b = Bm[:, k]
        res = np.linalg.norm(b - oracle.spmv(A, X[:, k])) / np.linalg.norm(b)
        assert res <= 1e-8, (k, res)
        xo, _ = so.solve(b, 1e-12)
        assert np.linalg.norm(X[:, k] - xo) <= 1e-6 * np.linalg.norm(xo), k
    # a column of the lockstep solve equals the same system solved alone (tolerance level)
    x1 = torch.zeros(A.shape[0], dtype=torch.float64, device=DEV)
    s.solve(dev(np.ascontiguousarray(Bm[:, 5])), x1, 1e-8)
    assert np.linalg.norm(x1.cpu().numpy() - X[:, 5]) <= 1e-6 * np.linalg.norm(X[:, 5])
    with pytest.raises(mgk.MgkError):
        s.solve_multi(torch.zeros((A.shape[0], 33), dtype=torch.float64, device=DEV),
                      torch.zeros((A.shape[0], 33), dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_multi_rhs_diagonal_layout_bitwise(storage):
    """The multi-RHS kernels read a diagonal-layout operator (the outer FP64 operator and
    hierarchy level 0) with the same ascending per-row sums as the walk over its BSR rows,
    skipping the slots a row does not store, so lockstep solves are bitwise the same in
    both layouts: on the Stokes operator (a full solve, every column checked by oracle
    SpMV) and on one with about 4% of its off-diagonal blocks dropped (five iterations).
    13^3 leaves a ragged last workgroup (2197 block rows) and 9 columns leave lanes idle."""
    n, K = 13, 9
    th, bsr, A = problem(n, 0.5, 22)
    Bm = S.body_forces(n, K, 4)
    Bm[:, 3] = 0.0
    dB = dev(Bm)
    full = None
    for op, maxiter in ((bsr, 1000), (drop_mirrored_pairs(bsr, 6), 5)):
        outs = []
        for layout in (2, 1):
            say("multi layout", storage, layout, maxiter)
            s = gpu_solver(op, hier=storage, coarse_enough=200, layout=layout, maxiter=maxiter)
            assert s.level_info(0)["dia"] == (7 if layout == 2 else 0)
            dX = torch.zeros_like(dB)
            infos = s.solve_multi(dB, dX, 1e-8)
            outs.append((dX.cpu().numpy(), [i["iters"] for i in infos]))
        assert outs[0][1] == outs[1][1]
        assert np.array_equal(outs[0][0], outs[1][0])
        full = outs[0][0] if full is None else full
    assert not np.any(full[:, 3])
    for k in range(K):
        if k != 3:
            b = Bm[:, k]
            res = np.linalg.norm(b - oracle.spmv(A, full[:, k])) / np.linalg.norm(b)
            assert res <= 1e-8, (k, res)


def leading_block(bsr, m):
    """The leading m x m block rows and columns of a BSR operator."""
    ptr, col, val = bsr
    rows = np.repeat(np.arange(ptr.size - 1), np.diff(ptr))
    keep = (rows < m) & (col < m)
    nptr = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=m)[:m])])
    return nptr.astype(np.int32), col[keep].copy(), val[keep].copy()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_multi_rhs_plane_tiled_order_bitwise(storage):
    """At 36^3 the largest diagonal offset (a grid plane, 1296 block rows) makes the
    multi-RHS kernels take their 8-row blocks plane by plane in 8 tiles of 21 blocks, the
    last tile of each plane with holes (8 x 21 > 162).  The schedule changes no sum, so
    lockstep iterations are bitwise those of the BSR layout's linear order; also on the
    leading 46,556 block rows (a partial last plane and a ragged last block)."""
    n, K = 36, 5
    th, bsr, A = problem(n, 0.5, 23)
    nb = A.shape[0] // 4
    for op in (bsr, leading_block(bsr, nb - 100)):
        m = op[0].size - 1
        Bm = S.body_forces(n, K, 4)[: 4 * m]
        dB = dev(Bm)
        outs = []
        for layout in (2, 1):
            say("tiled order", storage, m, layout)
            s = gpu_solver(op, hier=storage, layout=layout, maxiter=3)
            assert s.level_info(0)["dia"] == (7 if layout == 2 else 0)
            dX = torch.zeros_like(dB)
            infos = s.solve_multi(dB, dX, 1e-8)
            outs.append((dX.cpu().numpy(), [i["iters"] for i in infos]))
        assert outs[0][1] == outs[1][1]
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.all(np.isfinite(outs[0][0])) and np.any(outs[0][0])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_uneven_systems(storage):
    """Uneven systems in one batch: each meets 1e-8 (oracle SpMV), agrees with its own
    oracle solve, and with the same system solved alone on the GPU (to the tolerance: the
    batched dot products use a different, fixed, reduction partition)."""
    ns = [10, 13, 16, 12]
    probs = [problem(n, 0.5, 40 + k) for k, n in enumerate(ns)]
    bs = [dev(oracle.spmv(A, S.mms_solution(n))) for n, (_, _, A) in zip(ns, probs)]
    bsol = mgk.BatchSolver([p[1] for p in probs], 4, mgk.AMG_SPAI0,
                           stream=torch.cuda.current_stream(), hier=storage, coarse_enough=300)
    xs = [torch.zeros_like(b) for b in bs]
    infos = bsol.solve(bs, xs, 1e-8)
    say("batch", storage, [i["iters"] for i in infos])
    for k, (n, (th, bsr, A)) in enumerate(zip(ns, probs)):
        b = bs[k].cpu().numpy()
        x = xs[k].cpu().numpy()
        assert infos[k]["status"] == 0
        assert np.linalg.norm(b - oracle.spmv(A, x)) <= 1e-8 * np.linalg.norm(b)
        xo, _ = oracle.Solver(A, 4, coarse_enough=300).solve(b, 1e-12)
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
        s1 = gpu_solver(bsr, hier=storage, coarse_enough=300)
        x1 = torch.zeros_like(bs[k])
        i1 = s1.solve(bs[k], x1, 1e-8)
        assert abs(i1["iters"] - infos[k]["iters"]) <= max(2, infos[k]["iters"] // 10)
        assert torch.linalg.norm(x1 - xs[k]) <= 1e-6 * torch.linalg.norm(x1), k


def test_autograd_functions():
    """torch.autograd through the solve: d/dtheta against the oracle gradient formula on the
    oracle's own solves, d/db = lambda, and the block-value gradient -lambda x^T."""
    from paper_2006_06052_amd.autograd import bsr_solve, stokes_solve
    n = 10
    th = S.theta_field(n, 0.5, 60)
    thr = S.theta_field(n, 0.5, 61)
    b = S.mms_rhs(n)
    A, Ar = oracle.stokes_matrix(n, th), oracle.stokes_matrix(n, thr)
    xt, _ = oracle.Solver(Ar, 4, coarse_enough=300).solve(b, 1e-13)
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    db = dev(b).requires_grad_(True)
    x = stokes_solve(theta, db, n, hier=mgk.F32, coarse_enough=300)
    loss = 0.5 * torch.sum((x - dev(xt)) ** 2)
    loss.backward()
    so = oracle.Solver(A, 4, coarse_enough=300)
    xo, _ = so.solve(b, 1e-13)
    lo, _ = so.solve(xo - xt, 1e-13, transposed=True)
    go = oracle.theta_gradient(n, lo, xo)
    g = theta.grad.numpy()
    assert np.linalg.norm(g - go) <= 1e-6 * np.linalg.norm(go)
    assert np.linalg.norm(db.grad.cpu().numpy() - lo) <= 1e-6 * np.linalg.norm(lo)
    # gradient with respect to the stored block values
    ptr, col, val = mgk.stokes_bsr(n, th)
    vals = torch.tensor(val, dtype=torch.float64, requires_grad=True)
    x2 = bsr_solve(ptr, col, vals, dev(b), 4, hier=mgk.F32, coarse_enough=300)
    (0.5 * torch.sum((x2 - dev(xt)) ** 2)).backward()
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    ref = -lo.reshape(-1, 4)[rows][:, :, None] * xo.reshape(-1, 4)[col][:, None, :]
    assert np.linalg.norm(vals.grad.numpy() - ref) <= 1e-6 * np.linalg.norm(ref)
