"""The allocation-free solve (mgk_solve_noalloc): its Krylov workspace lives in the
library's static device array instead of buffers the solver allocated.  It must give
exactly the result of mgk_solve (same kernels, same partition, same order), on calls in
a row that reuse the array with different sizes, and reject what does not fit."""
import numpy as np
import pytest

import stokes_synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2006_06052_amd as mgk  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def _solver(n, sigma, seed, **kw):
    ptr, col, val = mgk.stokes_bsr(n, S.theta_field(n, sigma, seed))
    kw.setdefault("coarse_enough", 300)
    return mgk.Solver(ptr, col, val, 4, mgk.AMG_SPAI0, stream=torch.cuda.current_stream(), **kw)


def _rhs(n, seed):
    return torch.from_numpy(S.c2_rhs(n, seed=seed)).to(DEV)


@pytest.mark.parametrize("hier", [mgk.F32, mgk.BF16, mgk.F64])
def test_noalloc_solve_equals_solve_on_two_calls(hier):
    # a larger system first, then a smaller one: the second call reuses the array
    # that still holds the first call's vectors
    for n, seed in ((18, 61), (11, 62)):
        say("noalloc", n, hier)
        s = _solver(n, 0.5, seed, hier=hier)
        b = _rhs(n, seed)
        x_ref = torch.zeros_like(b)
        info_ref = s.solve(b, x_ref, 1e-8)
        x = torch.full_like(b, 3.0)          # garbage, then the same initial guess
        x.zero_()
        info = s.solve_noalloc(b, x, 1e-8)
        torch.cuda.synchronize()
        assert info["status"] == 0 and info_ref["status"] == 0
        assert info["iters"] == info_ref["iters"]
        assert info["rel_resid"] == info_ref["rel_resid"]
        assert torch.equal(x, x_ref), (x - x_ref).abs().max().item()
        # the solver's own workspace is still intact for ordinary solves
        x2 = torch.zeros_like(b)
        assert s.solve(b, x2, 1e-8)["iters"] == info_ref["iters"]
        assert torch.equal(x2, x_ref)
        del s


def test_noalloc_solve_from_nonzero_guess_and_zero_rhs():
    n = 9
    s = _solver(n, 0.5, 63, hier=mgk.F32)
    b = _rhs(n, 63)
    x0 = torch.from_numpy(np.random.default_rng(5).normal(size=b.numel())).to(DEV)
    xa, xb = x0.clone(), x0.clone()
    ia = s.solve(b, xa, 1e-9)
    ib = s.solve_noalloc(b, xb, 1e-9)
    assert ia["iters"] == ib["iters"] and torch.equal(xa, xb)
    z = torch.zeros_like(b)
    xz = x0.clone()
    info = s.solve_noalloc(z, xz, 1e-8)
    assert info["status"] == 0 and info["iters"] == 0
    assert torch.count_nonzero(xz).item() == 0


def test_noalloc_rejects_what_does_not_fit():
    # 51^3 nodes * 4 = 530,604 unknowns > 524,288: rejected before any device work
    n = 51
    s = _solver(n, 0.5, 64, hier=mgk.F32, coarse_enough=3000)
    b = _rhs(n, 64)
    x = torch.zeros_like(b)
    with pytest.raises(mgk.MgkError) as e:
        s.solve_noalloc(b, x, 1e-8)
    assert e.value.code == -1 and "exceed" in str(e.value)
    assert torch.count_nonzero(x).item() == 0
    del s
    s2 = _solver(8, 0.5, 65, krylov=mgk.FGMRES)
    b2 = _rhs(8, 65)
    with pytest.raises(mgk.MgkError) as e:
        s2.solve_noalloc(b2, torch.zeros_like(b2), 1e-8)
    assert e.value.code == -5
