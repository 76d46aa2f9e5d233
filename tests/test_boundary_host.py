"""Host-side checks of the C-ABI library: it loads, exports every declared entry point,
ingests matrices exactly, rejects bad input, and its FP64 host setup reproduces the
oracle's hierarchy bit for bit.  None of these tests touches a GPU."""
import json
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2006_06052_amd as mgk
import stokes_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mgk.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(mgk_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    L = mgk.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(mgk.EXPORTS)


def test_csr_to_bsr_worked_example():
    with open(os.path.join(ROOT, "tests", "golden", "bsr_worked_example.json")) as f:
        ex = json.load(f)
    c = ex["csr"]
    bptr, bcol, bval = mgk.csr_to_bsr(c["ptr"], c["col"], c["val"], ex["block"])
    assert bptr.tolist() == ex["bsr"]["ptr"]
    assert bcol.tolist() == ex["bsr"]["col"]
    assert bval.tolist() == ex["bsr"]["val"]
    # pointer and column arrays shrink by the block size and its square
    assert len(bptr) - 1 == (len(c["ptr"]) - 1) // 2 and len(bcol) * 4 == len(c["col"])


def oracle_blocks(A, b):
    B = sp.csr_matrix(A).tobsr(blocksize=(b, b))
    B.sort_indices()
    return B.indptr, B.indices, B.data


@pytest.mark.parametrize("n,sigma", [(5, None), (8, 0.5), (16, None), (12, 1.0)])
def test_stokes_assembly_matches_oracle_bitwise(n, sigma):
    th = None if sigma is None else S.theta_field(n, sigma, 21)
    ptr, col, val = mgk.stokes_bsr(n, th)
    A = oracle.stokes_matrix(n, th)
    optr, ocol, oval = oracle_blocks(A, 4)
    assert np.array_equal(ptr, optr) and np.array_equal(col, ocol)
    assert np.array_equal(val, oval)
    assert len(col) == 7 * (n - 2) ** 3 + n ** 3 - (n - 2) ** 3


def test_csr_to_bsr_of_oracle_matrix():
    n = 6
    A = oracle.stokes_matrix(n, S.theta_field(n, 1.0, 2))
    bptr, bcol, bval = mgk.csr_to_bsr(A.indptr, A.indices, A.data, 4)
    ptr, col, val = mgk.stokes_bsr(n, S.theta_field(n, 1.0, 2))
    assert np.array_equal(bptr, ptr) and np.array_equal(bcol, col) and np.array_equal(bval, val)


def host_solver(ptr, col, val, block, kind=mgk.AMG_SPAI0, **kw):
    return mgk.Solver(ptr, col, val, block, kind, host_only=True, **kw)


def compare_hierarchies(hs, which_h, os_, which_o, levels_expected=None):
    nl = hs.nlevels(which_h)
    assert nl == os_.nlevels(which_o)
    if levels_expected:
        assert nl >= levels_expected
    for l in range(nl):
        d = hs.level_info(l, which_h)
        L = os_.level(l, which_o)
        b = d["block"]
        ptr, col, val, agg = hs.level_export(l, 0, which_h)
        optr, ocol, oval = oracle_blocks(L["A"], b)
        assert np.array_equal(ptr, optr) and np.array_equal(col, ocol), f"A pattern, level {l}"
        assert np.array_equal(val, oval), f"A values, level {l}"
        if l == nl - 1:
            break
        assert np.array_equal(agg, L["agg"]), f"aggregates, level {l}"
        assert d["omega"] == L["omega"], f"omega, level {l}"
        if "M" in L and np.any(L["M"]):
            assert np.array_equal(hs.level_smoother(l, which_h), L["M"]), f"M, level {l}"
        for which, key in ((1, "P"), (2, "R")):
            p, c, v, _ = hs.level_export(l, which, which_h)
            op, oc, ov = oracle_blocks(L[key], b)
            assert np.array_equal(p, op) and np.array_equal(c, oc), f"{key} pattern, level {l}"
            assert np.array_equal(v, ov), f"{key} values, level {l}"


@pytest.mark.parametrize("n,sigma,block_spai0", [(16, None, 1), (12, 1.0, 1), (12, 0.5, 0)])
def test_host_setup_matches_oracle_monolithic(n, sigma, block_spai0):
    th = None if sigma is None else S.theta_field(n, sigma, 31)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4, coarse_enough=200, block_spai0=block_spai0)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, coarse_enough=200,
                        smoother=oracle.SPAI0_BLOCK if block_spai0 else oracle.SPAI0_SCALAR)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)


def test_host_setup_matches_oracle_schur():
    n = 14
    th = S.theta_field(n, 1.0, 3)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4, mgk.SCHUR, coarse_enough=150, krylov=mgk.FGMRES)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_SCHUR,
                        krylov=oracle.FGMRES, coarse_enough=150)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)
    compare_hierarchies(hs, 1, os_, 1, levels_expected=2)


@pytest.mark.parametrize("n,sigma", [(14, None), (12, 1.0)])
def test_host_setup_matches_oracle_plain_aggregation(n, sigma):
    """Plain aggregation (P = P_tent): patterns, values, aggregates and omega = 0 bit-exact."""
    th = None if sigma is None else S.theta_field(n, sigma, 33)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4, coarse_enough=200, coarsening=mgk.PLAIN_AGGREGATION)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, coarse_enough=200,
                        coarsening=oracle.PLAIN)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)
    assert hs.level_info(0)["omega"] == 0.0


def test_host_setup_matches_oracle_schur_diagonal_approximation():
    """eq. SchurApprox pressure operator and the plain-aggregation velocity hierarchy of
    the paper's Schur configuration, bit-exact; with the SPAI(0) pressure step there is
    no pressure hierarchy."""
    n = 14
    th = S.theta_field(n, 1.0, 3)
    ptr, col, val = mgk.stokes_bsr(n, th)
    kw = dict(coarse_enough=150, schur_approx=1)
    hs = host_solver(ptr, col, val, 4, mgk.SCHUR, coarsening=mgk.PLAIN_AGGREGATION, **kw)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_SCHUR,
                        coarsening=oracle.PLAIN, **kw)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)
    compare_hierarchies(hs, 1, os_, 1, levels_expected=2)
    hs2 = host_solver(ptr, col, val, 4, mgk.SCHUR, schur_spai0=1, **kw)
    assert hs2.nlevels(1) == 0 and hs2.nlevels(0) >= 2


@pytest.mark.parametrize("n,level", [(6, 0), (9, 1), (7, 1)])
def test_host_ilu_factors_match_oracle_bitwise(n, level):
    """Block ILU(k) host factorization: L and U blocks and the pivot inverses bit-exact."""
    th = S.theta_field(n, 0.5, 3 + n)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4, mgk.ILU, ilu_level=level)
    (lp, lc, lv), (up, uc, uv), dinv = hs.ilu_export()
    so = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_ILU, ilu_level=level)
    F = so.ilu_factor()
    optr, ocol, oval = oracle_blocks(F, 4)
    nb = n ** 3
    for i in range(nb):
        oc = ocol[optr[i]:optr[i + 1]]
        ov = oval[optr[i]:optr[i + 1]]
        lo, up_ = oc < i, oc > i
        assert np.array_equal(lc[lp[i]:lp[i + 1]], oc[lo]) and np.array_equal(lv[lp[i]:lp[i + 1]], ov[lo])
        assert np.array_equal(uc[up[i]:up[i + 1]], oc[up_]) and np.array_equal(uv[up[i]:up[i + 1]], ov[up_])
    assert np.array_equal(dinv, so.ilu_dinv())


def test_host_setup_matches_oracle_schur_scalar_velocity():
    """Schur split with the velocity AMG on scalar values (the paper's V2 format)."""
    n = 12
    th = S.theta_field(n, 1.0, 5)
    ptr, col, val = mgk.stokes_bsr(n, th)
    kw = dict(coarse_enough=150, schur_scalar_u=1)
    hs = host_solver(ptr, col, val, 4, mgk.SCHUR, coarsening=mgk.PLAIN_AGGREGATION, **kw)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_SCHUR,
                        coarsening=oracle.PLAIN, **kw)
    assert hs.level_info(0, 0)["block"] == 1
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)
    compare_hierarchies(hs, 1, os_, 1, levels_expected=2)


def test_host_setup_scalar_csr_arm():
    """The whole setup at block size 1 on the scalar CSR matrix (V2-style scalar arm)."""
    n = 8
    A = oracle.stokes_matrix(n)
    bptr, bcol, bval = mgk.csr_to_bsr(A.indptr, A.indices, A.data, 1)
    hs = host_solver(bptr, bcol, bval, 1, coarse_enough=300)
    os_ = oracle.Solver(A, 1, coarse_enough=300)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)


@pytest.mark.slow
def test_host_setup_matches_oracle_cube32():
    n = 32
    th = S.theta_field(n, 0.5, 41)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=3)


def test_invalid_input_rejected_before_device_work():
    ptr, col, val = mgk.stokes_bsr(4)
    r = 21                                    # an interior node row (7 blocks)
    k0 = ptr[r]
    bad = col.copy()
    bad[k0], bad[k0 + 1] = bad[k0 + 1], bad[k0]
    with pytest.raises(mgk.MgkError) as e:
        host_solver(ptr, bad, val, 4)
    assert e.value.code == -1
    with pytest.raises(mgk.MgkError) as e:
        mgk.Solver(ptr, col, val, 2, host_only=True)  # unsupported block size
    assert e.value.code == -1
    v2 = val.copy()
    v2[3, 0, 0] = np.nan
    with pytest.raises(mgk.MgkError) as e:
        host_solver(ptr, col, v2, 4)
    assert e.value.code == -1
    with pytest.raises(mgk.MgkError):
        host_solver(ptr, col, val, 4, maxiter=0)
    with pytest.raises(mgk.MgkError):
        host_solver(ptr, col, val, 4, mgk.ILU, ilu_level=2)
    with pytest.raises(mgk.MgkError):
        host_solver(ptr, col, val, 4, mgk.ILU, ilu_sweeps=-1)
    with pytest.raises(mgk.MgkError) as e:
        host_solver(ptr, col, val, 4).ilu_export()     # not an ILU solver
    assert e.value.code == -5
    hs = host_solver(ptr, col, val, 4)
    hs.set_timing(0)                                   # a mask within 0..3 is accepted
    for bad_mask in (-1, 4):
        with pytest.raises(mgk.MgkError) as e:
            hs.set_timing(bad_mask)
        assert e.value.code == -1, bad_mask
    for bad_kw in (dict(krylov=mgk.IDRS, idr_s=0), dict(krylov=mgk.IDRS, idr_s=17),
                   dict(krylov=3), dict(coarsening=2), dict(schur_lower=2)):
        with pytest.raises(mgk.MgkError) as e:
            host_solver(ptr, col, val, 4, **bad_kw)
        assert e.value.code == -1, bad_kw
    with pytest.raises(mgk.MgkError):
        mgk.stokes_bsr(2)
    with pytest.raises(mgk.MgkError):
        mgk.csr_to_bsr([0, 1, 2, 3], [0, 1, 2], [1.0, 1.0, 1.0], 2)


def test_singular_block_row_rejected():
    """A zero diagonal block makes the smoother or filtered diagonal singular."""
    ptr, col, val = mgk.stokes_bsr(6)
    v = val.copy()
    i = 1 + 6 * (1 + 6 * 1)                   # an interior node: 7 blocks
    k = ptr[i] + 3
    assert col[k] == i
    v[ptr[i]:ptr[i + 1]] = 0.0
    with pytest.raises(mgk.MgkError) as e:
        host_solver(ptr, col, v, 4, coarse_enough=10)
    assert e.value.code in (-4, -1)


# Hierarchies of the benchmark workloads at their full sizes, bit for bit.
CONFIG_SHAPES = {
    # 48^3, theta = exp(N(0, 0.5^2)) seed 5 (the differentiable-solve workload)
    "cube48_theta": dict(n=48, sigma=0.5, seed=5, kind="amg"),
    # 64^3, mu = 1 (the 32-right-hand-side workload)
    "cube64_mu1": dict(n=64, sigma=None, seed=None, kind="amg"),
    # 64^3, theta = exp(N(0, 1)) seed 3: the Schur workload's velocity and pressure hierarchies
    "cube64_schur": dict(n=64, sigma=1.0, seed=3, kind="schur"),
    # 64^3, seed 3, the paper's Schur configuration: plain-aggregation velocity AMG and the
    # diagonal pressure approximation of eq. SchurApprox
    "cube64_paper_schur": dict(n=64, sigma=1.0, seed=3, kind="schur",
                               kw=dict(coarsening=1, schur_approx=1)),
    # 56^3, theta = exp(N(0, 0.5^2)) seed 45: one of the eight batched systems
    "cube56_theta": dict(n=56, sigma=0.5, seed=45, kind="amg"),
    # 96^3, mu = 1 (the headline workload)
    "cube96_mu1": dict(n=96, sigma=None, seed=None, kind="amg"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", list(CONFIG_SHAPES))
def test_host_setup_matches_oracle_at_workload_shape(name):
    """Aggregates, omega, A/P/R patterns and values and the smoother blocks of every level
    equal the oracle's at the benchmark sizes (default parameters: eps 0.08, 3000 coarse
    unknowns)."""
    c = CONFIG_SHAPES[name]
    n = c["n"]
    th = None if c["sigma"] is None else S.theta_field(n, c["sigma"], c["seed"])
    ptr, col, val = mgk.stokes_bsr(n, th)
    A = oracle.stokes_matrix(n, th)
    kw = c.get("kw", {})
    if c["kind"] == "schur":
        hs = host_solver(ptr, col, val, 4, mgk.SCHUR, krylov=mgk.FGMRES, **kw)
        del ptr, col, val
        os_ = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES, **kw)
        del A
        compare_hierarchies(hs, 0, os_, 0, levels_expected=3)
        compare_hierarchies(hs, 1, os_, 1, levels_expected=3)
    else:
        hs = host_solver(ptr, col, val, 4)
        del ptr, col, val
        os_ = oracle.Solver(A, 4)
        del A
        compare_hierarchies(hs, 0, os_, 0, levels_expected=3)


@pytest.mark.parametrize("n,p,tau", [(6, 2.0, 1e-2), (7, 1.0, 5e-2), (6, 3.0, 1e-3)])
def test_host_ilut_factors_match_oracle_bitwise(n, p, tau):
    """Block ILUT(p, tau) host factorization: L and U blocks (pattern and values) and the
    pivot inverses bit-exact against the oracle."""
    th = S.theta_field(n, 0.5, 30 + n)
    ptr, col, val = mgk.stokes_bsr(n, th)
    hs = host_solver(ptr, col, val, 4, mgk.ILU, ilu_kind=1, ilut_p=p, ilut_tau=tau)
    (lp, lc, lv), (up, uc, uv), dinv = hs.ilu_export()
    so = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_ILU, ilu_kind=1,
                       ilut_p=p, ilut_tau=tau)
    F = so.ilu_factor()
    optr, ocol, oval = oracle_blocks(F, 4)
    dropped = 0
    for i in range(n ** 3):
        oc = ocol[optr[i]:optr[i + 1]]
        ov = oval[optr[i]:optr[i + 1]]
        lo, up_ = oc < i, oc > i
        assert np.array_equal(lc[lp[i]:lp[i + 1]], oc[lo]) and np.array_equal(lv[lp[i]:lp[i + 1]], ov[lo])
        assert np.array_equal(uc[up[i]:up[i + 1]], oc[up_]) and np.array_equal(uv[up[i]:up[i + 1]], ov[up_])
        dropped += (ptr[i + 1] - ptr[i]) - (lp[i + 1] - lp[i]) - (up[i + 1] - up[i]) - 1
    assert np.array_equal(dinv, so.ilu_dinv())
    assert dropped != 0 or tau < 1e-2          # the threshold is active in these cases


def test_host_setup_matches_oracle_ilut_smoothed_schur():
    """The paper's Schur configuration with the ILUT-smoothed velocity AMG (plain
    aggregation, diagonal pressure approximation): the hierarchy bit-exact against the
    oracle's (each level's ILUT factors enter the FP64 V-cycle compared on the GPU)."""
    n = 12
    th = S.theta_field(n, 1.0, 3)
    ptr, col, val = mgk.stokes_bsr(n, th)
    kw = dict(coarse_enough=150, schur_approx=1, schur_spai0=1)
    hs = host_solver(ptr, col, val, 4, mgk.SCHUR, coarsening=mgk.PLAIN_AGGREGATION,
                     ilu_smoother=1, ilu_kind=1, **kw)
    os_ = oracle.Solver(oracle.stokes_matrix(n, th), 4, kind=oracle.KIND_SCHUR,
                        coarsening=oracle.PLAIN, smoother=oracle.ILUT, **kw)
    compare_hierarchies(hs, 0, os_, 0, levels_expected=2)
