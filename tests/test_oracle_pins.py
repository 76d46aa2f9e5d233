"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test fixes one part of the oracle with something other than the oracle
itself: closed forms, hand-derived small cases, brute-force dense algebra,
invariants and the paper's own worked values.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import stokes_synth as S


def dense(M):
    return np.asarray(M.todense())


# ---------------------------------------------------------------- assembly

def test_assembly_counts_and_structure():
    n = 6
    A = oracle.stokes_matrix(n)
    ni = (n - 2) ** 3
    assert A.nnz == 40 * ni + 4 * (n ** 3 - ni)
    interior = S.interior_nodes(n)
    rows = np.diff(A.indptr).reshape(-1, 4)
    assert np.all(rows[interior] == [9, 9, 9, 13])
    assert np.all(rows[~interior] == 1)
    # boundary rows are identity rows
    D = dense(A)
    for g in np.flatnonzero(~interior):
        for c in range(4):
            r = 4 * g + c
            assert D[r, r] == 1.0 and np.count_nonzero(D[r]) == 1


def test_assembly_interior_blocks_symmetric_with_viscosity():
    """Interior-interior blocks satisfy A_gh = A_hg^T (symmetric indefinite interior,
    Section 3); boundary columns make the full matrix nonsymmetric."""
    n = 7
    th = S.theta_field(n, 0.5, 11)
    D = dense(oracle.stokes_matrix(n, th))
    inter = np.flatnonzero(S.interior_nodes(n))
    idx = (4 * inter[:, None] + np.arange(4)).ravel()
    Dii = D[np.ix_(idx, idx)]
    assert np.array_equal(Dii, Dii.T)
    assert not np.array_equal(D, D.T)


def test_assembly_velocity_rows_are_viscous_laplacian():
    """Velocity rows: the u_c entries sum to zero (diffusion), and each off-diagonal is
    minus the edge viscosity (mean of the 4 cells on the edge) over h^2."""
    n = 5
    th = S.theta_field(n, 1.0, 3)
    A = oracle.stokes_matrix(n, th)
    D = dense(A)
    h2 = (n - 1) ** 2
    g = 1 + n * (1 + n * 1)           # node (1,1,1)
    r = 4 * g + 0
    ucols = [4 * m for m in range(n ** 3)]
    assert abs(D[r, ucols].sum()) < 1e-12 * abs(D[r, r])
    # edge (1,1,1) -> (2,1,1): cells (1, j, k) for j, k in {0, 1}
    cells = [1 + (n - 1) * (j + (n - 1) * k) for k in (0, 1) for j in (0, 1)]
    mu = 0.25 * th[cells].sum()
    assert D[r, 4 * (g + 1)] == pytest.approx(-mu * h2, rel=1e-15)
    # pressure coupling +-1/(2h) and stabilization h^2 lap_h p
    assert D[r, 4 * (g + 1) + 3] == 0.5 * (n - 1)
    assert D[r, 4 * (g - 1) + 3] == -0.5 * (n - 1)
    rp = 4 * g + 3
    assert D[rp, rp] == -6.0 and D[rp, 4 * (g + n) + 3] == 1.0
    assert D[rp, 4 * (g + 1)] == -0.5 * (n - 1) and D[rp, 4 * (g - 1)] == 0.5 * (n - 1)


def test_assembly_closed_form_residual():
    """A x* - b at interior rows equals 2((2 - 2cos h)/h^2 - 1) sin x cos y on u rows, its
    negative-cosine counterpart on v rows, and 0 on w and p rows (central differences of
    the manufactured u* and the linear p*); 0 on boundary rows."""
    n = 16
    A = oracle.stokes_matrix(n)
    xs, b = S.mms_solution(n), S.mms_rhs(n)
    res = (A @ xs - b).reshape(-1, 4)
    h = 1.0 / (n - 1)
    X = S.node_coords(n)
    k = 2.0 * ((2.0 - 2.0 * np.cos(h)) / h ** 2 - 1.0)
    inter = S.interior_nodes(n)
    expect_u = k * np.sin(X[:, 0]) * np.cos(X[:, 1])
    expect_v = -k * np.cos(X[:, 0]) * np.sin(X[:, 1])
    scale = (n - 1) ** 2
    assert np.allclose(res[inter, 0], expect_u[inter], atol=1e-12 * scale)
    assert np.allclose(res[inter, 1], expect_v[inter], atol=1e-12 * scale)
    assert np.allclose(res[inter, 2], 0.0, atol=1e-12 * scale)
    assert np.allclose(res[inter, 3], 0.0, atol=1e-12 * n)
    assert np.all(res[~inter] == 0.0)


def _solve_tight(A, b):
    s = oracle.Solver(A, 4)
    x, info = s.solve(b, 1e-12)
    assert info["converged"]
    return x


@pytest.mark.slow
def test_discretization_second_order():
    """Nodal error of the FD solution against the continuous manufactured solution falls
    by about 4 per halving of h."""
    errs = []
    for n in (9, 17, 33):
        A = oracle.stokes_matrix(n)
        x = _solve_tight(A, S.mms_rhs(n))
        e = (x - S.mms_solution(n)).reshape(-1, 4)
        errs.append(np.abs(e[:, :3]).max())
    # observed order over h = 1/8 .. 1/32 (pre-asymptotic ratios are 5.0 and 5.6)
    order = np.log(errs[0] / errs[2]) / np.log(4.0)
    assert 1.8 < order < 3.0 and errs[0] > errs[1] > errs[2], errs


def paper_cube_triple(X):
    """Analytic rotating flow of the unit-cube benchmark (Section 5.1, eq. UnitCubeProb).
    The printed f equals -lap(u~) + grad(p) for u~ = u/pi, i.e. the printed velocity without
    its leading factor pi (reading of a misprint; with mu = 1 the printed u and f differ by
    that factor)."""
    x, y, z = X[:, 0] * np.pi, X[:, 1] * np.pi, X[:, 2] * np.pi
    s, c = np.sin, np.cos
    u = np.stack([s(x) * c(y) - s(x) * c(z), s(y) * c(z) - s(y) * c(x),
                  s(z) * c(x) - s(z) * c(y)], axis=1)
    p = s(x) * s(y) * s(z) - 8.0 / np.pi ** 3
    pi = np.pi
    f = pi * np.stack([
        2 * pi * s(x) * c(y) - 2 * pi * s(x) * c(z) + s(y) * s(z) * c(x),
        -2 * pi * s(y) * c(x) + 2 * pi * s(y) * c(z) + s(x) * s(z) * c(y),
        2 * pi * s(z) * c(x) - 2 * pi * s(z) * c(y) + s(x) * s(y) * c(z)], axis=1)
    return u, p, f


def test_paper_triple_closed_form():
    """div u = 0, f = -lap(u) + grad p, and mean(p) = 0, checked with high-order central
    differences at random points (independent of the FD operator under test)."""
    rng = np.random.default_rng(0)
    P = rng.uniform(0.1, 0.9, size=(50, 3))
    d = 1e-3
    E = np.eye(3) * d

    def U(Q):
        return paper_cube_triple(Q)[0]

    def Pp(Q):
        return paper_cube_triple(Q)[1]

    lap = sum((U(P + E[a]) - 2 * U(P) + U(P - E[a])) / d ** 2 for a in range(3))
    gradp = np.stack([(Pp(P + E[a]) - Pp(P - E[a])) / (2 * d) for a in range(3)], axis=1)
    div = sum((U(P + E[a])[:, a] - U(P - E[a])[:, a]) / (2 * d) for a in range(3))
    f = paper_cube_triple(P)[2]
    assert np.allclose(f, -lap + gradp, atol=1e-4)
    assert np.abs(div).max() < 1e-6
    g = (np.arange(200) + 0.5) / 200
    mean_sss = np.sin(np.pi * g).mean() ** 3
    assert abs(mean_sss - 8 / np.pi ** 3) < 1e-4


@pytest.mark.slow
def test_paper_triple_second_order():
    """The paper's analytic solution, imposed through boundary rows and f, is reproduced by
    the FD operator to O(h^2)."""
    errs = []
    for n in (9, 17, 33):
        A = oracle.stokes_matrix(n)
        X = S.node_coords(n)
        u, p, f = paper_cube_triple(X)
        inter = S.interior_nodes(n)
        xs = np.concatenate([u, p[:, None]], axis=1)
        b = np.zeros((n ** 3, 4))
        b[inter, :3] = f[inter]
        b[~inter] = xs[~inter]
        x = _solve_tight(A, b.ravel()).reshape(-1, 4)
        errs.append(np.abs(x[:, :3] - u).max())
    # the pi-frequency field is under-resolved at n = 9; the 17 -> 33 ratio is near 4
    assert errs[0] > errs[1] > errs[2] and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_block_view_matches_paper_worked_example():
    """The node (block) view the oracle gathers from scalar CSR reproduces the block CSR
    arrays printed for the paper's 6x6 example (Section 4, block-valued backend)."""
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "bsr_worked_example.json")) as f:
        ex = json.load(f)
    c = ex["csr"]
    A = sp.csr_matrix((c["val"], c["col"], c["ptr"]), shape=(6, 6))
    ptr, cols, vals = [0], [], []
    for i in range(3):
        bc, bv = oracle.gather_block_row(A, 2, i)
        cols += bc.tolist()
        vals += bv.tolist()
        ptr.append(len(cols))
    assert ptr == ex["bsr"]["ptr"] and cols == ex["bsr"]["col"]
    assert vals == ex["bsr"]["val"]
    # BSR and scalar CSR products agree bitwise (ascending order, exact zeros add +0)
    x = np.random.default_rng(0).normal(size=6)
    y = np.zeros(6)
    for i in range(3):
        for t in range(ptr[i], ptr[i + 1]):
            for r in range(2):
                for q in range(2):
                    y[2 * i + r] += vals[t][r][q] * x[2 * cols[t] + q]
    assert np.array_equal(y, oracle.spmv(A, x))


# ---------------------------------------------------------------- hierarchy

def chain(m):
    """1D chain: identity rows at both ends, [-1, 2, -1] inside (columns to the ends kept)."""
    rows, cols, vals = [0, m - 1], [0, m - 1], [1.0, 1.0]
    for i in range(1, m - 1):
        rows += [i, i, i]
        cols += [i - 1, i, i + 1]
        vals += [-1.0, 2.0, -1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


def test_aggregation_1d_hand_derived():
    s = oracle.Solver(chain(11), 1, coarse_enough=1, max_levels=2)
    L0 = s.level(0)
    assert list(L0["agg"]) == [-1, 0, 0, 1, 1, 1, 2, 2, 2, 2, -1]
    assert L0["n_agg"] == 3


def test_prolongator_1d_hand_derived():
    """1D Laplacian: Gershgorin bound 2, omega = 2/3; P entries by hand."""
    s = oracle.Solver(chain(11), 1, coarse_enough=1, max_levels=2)
    L0 = s.level(0)
    assert L0["omega"] == pytest.approx(2.0 / 3.0, rel=1e-15)
    P = dense(L0["P"])
    expect = np.zeros((11, 3))
    expect[1] = [2 / 3, 0, 0]
    expect[2] = [2 / 3, 1 / 3, 0]
    expect[3] = [1 / 3, 2 / 3, 0]
    expect[4] = [0, 1, 0]
    expect[5] = [0, 2 / 3, 1 / 3]
    expect[6] = [0, 1 / 3, 2 / 3]
    expect[7] = [0, 0, 1]
    expect[8] = [0, 0, 1]
    expect[9] = [0, 0, 2 / 3]
    assert np.allclose(P, expect, atol=1e-15)
    # rows of A_F summing to zero keep P 1 = P_tent 1 = 1
    assert np.allclose(P[3:9].sum(axis=1), 1.0)


def scaled_chain(m, diag, off=-1.0, diag_odd=None):
    """chain(m) with interior diagonal `diag` (or `diag_odd` on odd nodes) and off-diagonal
    `off`; identity rows at both ends."""
    rows, cols, vals = [0, m - 1], [0, m - 1], [1.0, 1.0]
    for i in range(1, m - 1):
        d = diag_odd if (diag_odd is not None and i % 2) else diag
        rows += [i, i, i]
        cols += [i - 1, i, i + 1]
        vals += [off, d, off]
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


@pytest.mark.parametrize("diag,strong", [(10.0, True), (12.4, True), (12.6, False)])
def test_strength_threshold_is_eps_squared(diag, strong):
    """Strength (b = 1): a_ij^2 > eps^2 |a_ii| |a_jj| with eps = 0.08.  For the chain with
    interior rows [-1, d, -1] the interior couplings are strong iff 1 > 0.0064 d^2, i.e.
    d < 12.5: d = 10 and 12.4 aggregate like the plain chain.  With d = 12.6 the interior
    couplings are weak; only nodes 1 and 9 keep a strong coupling, to the identity rows at
    the ends (1 > 0.0064 * 12.6 * 1), whose nodes are isolated, so nodes 1 and 9 become
    singleton aggregates and every other node is isolated.  Reading the threshold as eps
    instead of eps^2 (1 > 0.08 d^2 for the interior couplings, d < 3.54) would leave no
    interior coupling strong in all three cases."""
    s = oracle.Solver(scaled_chain(11, diag), 1, coarse_enough=1, max_levels=2)
    assert s.nlevels() == 2
    if strong:
        assert list(s.level(0)["agg"]) == [-1, 0, 0, 1, 1, 1, 2, 2, 2, 2, -1]
    else:
        assert list(s.level(0)["agg"]) == [-1, 0, -1, -1, -1, -1, -1, -1, -1, 1, -1]


@pytest.mark.parametrize("c,strong", [(0.85, True), (0.75, False)])
def test_strength_uses_geometric_mean_of_both_diagonals(c, strong):
    """Interior diagonals alternate 1 (even nodes) and 100 (odd nodes), couplings -c.  The
    test c^2 > eps^2 sqrt(N_ii) sqrt(N_jj) = 0.0064 * 1 * 100 gives c > 0.8 for every
    coupling: 0.85 strong, 0.75 weak.  Using only the row's own diagonal would make even
    rows strong (c > 0.08) and odd rows weak (c > 8) for both values; the minimum or the
    maximum of the two diagonals would give the same answer for both values.  The end
    couplings (odd node 1 or 9 against the identity row, diagonals 100 and 1) follow the
    same rule, so with c = 0.75 every node is isolated."""
    A = scaled_chain(11, 1.0, off=-c, diag_odd=100.0)
    s = oracle.Solver(A, 1, coarse_enough=1, max_levels=2)
    if strong:
        assert s.nlevels() == 2
        assert list(s.level(0)["agg"]) == [-1, 0, 0, 1, 1, 1, 2, 2, 2, 2, -1]
    else:
        assert s.nlevels() == 1


def anisotropic_lines(mx=5, my=12, delta=1.0 / 32):
    """my x-lines of mx nodes, periodic in y.  Nodes i = 0 and mx - 1 of every line are
    identity rows (columns kept); interior nodes have 2 + 2 delta on the diagonal, -1 to
    their x-neighbours and -delta to their y-neighbours.  Node (i, j) is i + mx j."""
    rows, cols, vals = [], [], []
    g = lambda i, j: i + mx * (j % my)  # noqa: E731
    for j in range(my):
        for i in range(mx):
            r = g(i, j)
            if i == 0 or i == mx - 1:
                rows.append(r); cols.append(r); vals.append(1.0)  # noqa: E702
                continue
            for c, v in ((g(i - 1, j), -1.0), (g(i + 1, j), -1.0), (g(i, j - 1), -delta),
                         (g(i, j + 1), -delta), (r, 2.0 + 2.0 * delta)):
                rows.append(r); cols.append(c); vals.append(v)  # noqa: E702
    return sp.csr_matrix((vals, (rows, cols)), shape=(mx * my, mx * my))


def test_weak_lumping_and_eps_halving_hand_derived():
    """Anisotropic lines (delta = 1/32; every value below is exact in binary or derived
    by hand).

    Level 0 (eps = 0.08): x-couplings are strong (1 > 0.0064 * 2.0625^2), y-couplings weak
    (delta^2 = 0.00098 < 0.0272).  Each line's three interior nodes form one aggregate
    (phase 1 seeds {1, 2}, node 3 joins it in phase 2): 12 aggregates.  The weak
    y-couplings are lumped into the diagonal of the filtered matrix, so A_F has rows
    [-1, 2, -1] (2.0625 - 1/32 - 1/32 = 2): Gershgorin bound 2, omega = (4/3)/2 = 2/3, and
    the prolongator of each line is (2/3, 1, 2/3) with no entry in any other line
    (dropping instead of lumping gives omega = 0.6875 and P = 0.677...; keeping the weak
    couplings gives entries in the neighbouring lines).

    Level 1 = R A P: per line p^T A_x p = 10/9 and sum p_i^2 = 17/9, so a ring of 12 nodes
    with diagonal 10/9 + 34 delta/9 and couplings -17 delta/9 (relative strength 0.048).
    With eps halved to 0.04 the ring couplings are strong and the ring aggregates as
    {11, 0, 1}, {2, 3, 4}, {5, 6, 7}, {8, 9, 10}; with eps kept at 0.08 (or the eps
    threshold instead of eps^2) they are weak, every level-1 node is isolated and the
    hierarchy stops at two levels.  Level-1 omega: the Gershgorin bound of the ring is
    (10 + 68 delta) / (10 + 34 delta)."""
    delta = 1.0 / 32
    A = anisotropic_lines(delta=delta)
    s = oracle.Solver(A, 1, coarse_enough=5)
    assert s.nlevels() == 3
    L0 = s.level(0)
    agg = L0["agg"].reshape(12, 5)
    assert np.array_equal(agg[:, 0], -np.ones(12)) and np.array_equal(agg[:, 4], -np.ones(12))
    for j in range(12):
        assert list(agg[j, 1:4]) == [j, j, j]
    assert L0["n_agg"] == 12
    assert L0["omega"] == 2.0 / 3.0
    P = dense(L0["P"])
    expect = np.zeros((60, 12))
    for j in range(12):
        expect[5 * j + 1:5 * j + 4, j] = [2.0 / 3.0, 1.0, 2.0 / 3.0]
    assert np.abs(P - expect).max() <= 1e-15
    assert L0["P"].nnz == 36
    L1 = s.level(1)
    A1 = dense(L1["A"])
    ring = np.zeros((12, 12))
    for j in range(12):
        ring[j, j] = 10.0 / 9.0 + 34.0 * delta / 9.0
        ring[j, (j + 1) % 12] = ring[j, (j - 1) % 12] = -17.0 * delta / 9.0
    assert np.abs(A1 - ring).max() <= 1e-14
    assert list(L1["agg"]) == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 0]
    assert L1["omega"] == pytest.approx((4.0 / 3.0) * (10 + 34 * delta) / (10 + 68 * delta),
                                        rel=1e-14)


def test_two_phases_aggregate_every_connected_node():
    """The third aggregation phase (leftover nodes seeding aggregates) is unreachable: a
    node that phase 1 skips has a non-isolated strong neighbour already aggregated in
    phase 1, which phase 2 joins.  The oracle reports an error if a node were left; random
    nonsymmetric matrices with random strength patterns never trigger it, and every
    non-isolated node ends in an aggregate."""
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(6, 40))
        A = sp.random(n, n, density=float(rng.uniform(0.05, 0.4)), random_state=int(trial),
                      data_rvs=lambda k: rng.uniform(-1, 1, k))
        A = sp.csr_matrix(A + sp.diags(rng.uniform(1, 4, n)))
        s = oracle.Solver(A, 1, coarse_enough=1, max_levels=2)
        if s.nlevels() < 2:
            continue
        L0 = s.level(0)
        iso = np.array([all(abs(A[i, j]) ** 2 <= 0.0064 * abs(A[i, i]) * abs(A[j, j])
                            for j in A[i].indices if j != i) for i in range(n)])
        assert np.array_equal(L0["agg"] < 0, iso)


def test_damped_jacobi_smoother_closed_form():
    """Damped block Jacobi: M_i = omega_J A_ii^-1 on every level (omega_J = 2/3 and 0.5),
    against numpy's inverse of each diagonal block."""
    n = 7
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 13))
    for om in (2.0 / 3.0, 0.5):
        s = oracle.Solver(A, 4, smoother=oracle.JACOBI, jacobi_omega=om, coarse_enough=30)
        assert s.nlevels() >= 3
        for l in range(s.nlevels() - 1):
            L = s.level(l)
            Ad = dense(L["A"])
            for i in range(Ad.shape[0] // 4):
                Dii = Ad[4 * i:4 * i + 4, 4 * i:4 * i + 4]
                ref = om * np.linalg.inv(Dii)
                assert np.abs(L["M"][i] - ref).max() <= 1e-12 * np.abs(ref).max(), (om, l, i)


def test_plain_aggregation_1d_hand_derived():
    """Plain aggregation: P is the tentative prolongator (one unit entry per aggregated
    node, omega 0), and for the 1D Laplacian each aggregate sums to the coarse stencil
    (-1, 2, -1): an aggregate of m nodes has 2m - 2(m - 1) = 2 on the diagonal."""
    s = oracle.Solver(chain(11), 1, coarse_enough=1, max_levels=2, coarsening=oracle.PLAIN)
    L0 = s.level(0)
    assert list(L0["agg"]) == [-1, 0, 0, 1, 1, 1, 2, 2, 2, 2, -1]
    assert L0["omega"] == 0.0
    P = dense(L0["P"])
    expect = np.zeros((11, 3))
    for i, a in enumerate(L0["agg"]):
        if a >= 0:
            expect[i, a] = 1.0
    assert np.array_equal(P, expect)
    Ac = dense(s.level(1)["A"])
    assert np.array_equal(Ac, np.array([[2.0, -1, 0], [-1, 2, -1], [0, -1, 2]]))


def test_plain_aggregation_3d_invariants():
    """Block plain aggregation: every stored block of P is the identity, each aggregated
    node has exactly one, R = P^T, and A_{l+1} = R A_l P against a dense triple product."""
    n = 8
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 7))
    s = oracle.Solver(A, 4, coarse_enough=40, coarsening=oracle.PLAIN)
    assert s.nlevels() >= 3
    for l in range(s.nlevels() - 1):
        L, Lc = s.level(l), s.level(l + 1)
        P, R, Al = dense(L["P"]), dense(L["R"]), dense(L["A"])
        agg = L["agg"]
        expect = np.zeros_like(P)
        for i, a in enumerate(agg):
            if a >= 0:
                expect[4 * i:4 * i + 4, 4 * a:4 * a + 4] = np.eye(4)
        assert np.array_equal(P, expect) and np.array_equal(R, P.T)
        Ac = R @ Al @ P
        assert np.abs(dense(Lc["A"]) - Ac).max() <= 1e-13 * np.abs(Al).max() * 10


@pytest.fixture(scope="module")
def small_hierarchy():
    n = 8
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 7))
    s = oracle.Solver(A, 4, coarse_enough=40)
    return n, A, s


def test_aggregates_partition_and_connected(small_hierarchy):
    n, A, s = small_hierarchy
    assert s.nlevels() >= 3
    for l in range(s.nlevels() - 1):
        L = s.level(l)
        agg = L["agg"]
        nagg = L["n_agg"]
        used = agg[agg >= 0]
        assert set(used.tolist()) == set(range(nagg))
        # an aggregate is connected through nonzero blocks of A
        Ab = dense(L["A"])
        nn = Ab.shape[0] // 4
        G = np.zeros((nn, nn), bool)
        for i in range(nn):
            for j in range(nn):
                G[i, j] = np.any(Ab[4 * i:4 * i + 4, 4 * j:4 * j + 4] != 0)
        for a in range(nagg):
            mem = np.flatnonzero(agg == a)
            seen = {mem[0]}
            stack = [mem[0]]
            while stack:
                v = stack.pop()
                for w in mem:
                    if w not in seen and (G[v, w] or G[w, v]):
                        seen.add(w)
                        stack.append(w)
            assert len(seen) == len(mem)


def test_tentative_prolongator_invariants(small_hierarchy):
    """P_tent^T P_tent = diag(|agg|) I_b and P_tent 1 = 1 on non-isolated rows, with
    P_tent rebuilt from the aggregates (unnormalized identity blocks)."""
    n, A, s = small_hierarchy
    L = s.level(0)
    agg = L["agg"]
    nn = agg.size
    rows = [4 * i + c for i in range(nn) if agg[i] >= 0 for c in range(4)]
    cols = [4 * agg[i] + c for i in range(nn) if agg[i] >= 0 for c in range(4)]
    Pt = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(4 * nn, 4 * L["n_agg"]))
    sizes = np.bincount(agg[agg >= 0], minlength=L["n_agg"])
    assert np.array_equal(dense(Pt.T @ Pt), np.kron(np.diag(sizes), np.eye(4)))
    one = Pt @ np.ones(Pt.shape[1])
    assert np.array_equal(one.reshape(-1, 4)[agg >= 0], np.ones(((agg >= 0).sum(), 4)))
    # the smoothed prolongator keeps P_tent's block pattern plus strong neighbours' aggregates
    P = dense(L["P"])
    for i in range(nn):
        if agg[i] < 0:
            assert not np.any(P[4 * i:4 * i + 4])
        else:
            assert np.any(P[4 * i:4 * i + 4, 4 * agg[i]:4 * agg[i] + 4])


def test_galerkin_identity(small_hierarchy):
    """A_{l+1} = R_l A_l P_l against a dense triple product; R_l = P_l^T exactly."""
    n, A, s = small_hierarchy
    for l in range(s.nlevels() - 1):
        L, Lc = s.level(l), s.level(l + 1)
        P, R, Al = dense(L["P"]), dense(L["R"]), dense(L["A"])
        assert np.array_equal(R, P.T)
        Ac = R @ Al @ P
        scale = np.abs(R).max() * np.abs(Al).max() * np.abs(P).max()
        assert np.abs(dense(Lc["A"]) - Ac).max() <= 1e-13 * scale


def test_spai0_closed_forms():
    """Block SPAI0 M minimizes ||I - M A||_F over block-diagonal M: random perturbations
    never do better, and the residual of each row-block least-squares problem is
    orthogonal to that block row (normal equations)."""
    rng = np.random.default_rng(1)
    nb, b = 5, 3
    blocks = [rng.normal(size=(b, b)) + 4 * np.eye(b) for _ in range(nb)]
    A = sp.random(nb * b, nb * b, density=0.3, random_state=2) + sp.csr_matrix(sp.block_diag(blocks))
    A = sp.csr_matrix(A)
    s = oracle.Solver(A, b, coarse_enough=1, max_levels=2)
    if s.nlevels() < 2:
        pytest.skip("random matrix did not coarsen")
    M = s.level(0)["M"]
    Ad_ = dense(A)
    Mfull = sp.block_diag(list(M)).toarray()
    base = np.linalg.norm(np.eye(nb * b) - Mfull @ Ad_)
    for t in range(20):
        Pm = Mfull + 1e-3 * sp.block_diag([rng.normal(size=(b, b)) for _ in range(nb)]).toarray()
        assert np.linalg.norm(np.eye(nb * b) - Pm @ Ad_) >= base
    # the normal equations of the row-block least squares at the optimum
    for i in range(nb):
        Ai = Ad_[b * i:b * i + b]
        Ei = np.zeros_like(Ai)
        Ei[:, b * i:b * i + b] = np.eye(b)
        assert np.allclose((Ei - M[i] @ Ai) @ Ai.T, 0, atol=1e-12)


def test_spai0_scalar_reduces():
    A = chain(11) + sp.diags(np.linspace(0.1, 0.5, 11))
    A = sp.csr_matrix(A)
    s = oracle.Solver(A, 1, coarse_enough=1, max_levels=2)
    M = s.level(0)["M"][:, 0, 0]
    D = dense(A)
    assert np.allclose(M, np.diag(D) / (D ** 2).sum(axis=1), rtol=1e-15)


def vcycle_dense(s, l, nlev):
    """Dense V(1,1) operator from its definition: B = M + (I - M A) M
    + (I - M A) P B_c R (I - A M), with B_c the exact inverse at the coarsest level."""
    L = s.level(l)
    A = dense(L["A"])
    if l == nlev - 1:
        return np.linalg.inv(A)
    M = sp.block_diag(list(L["M"])).toarray()
    P, R = dense(L["P"]), dense(L["R"])
    Bc = vcycle_dense(s, l + 1, nlev)
    I = np.eye(A.shape[0])
    return M + (I - M @ A) @ M + (I - M @ A) @ P @ Bc @ R @ (I - A @ M)


def test_vcycle_brute_force(small_hierarchy):
    n, A, s = small_hierarchy
    B = vcycle_dense(s, 0, s.nlevels())
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.normal(size=A.shape[0])
        z = s.precond(r)
        assert np.allclose(z, B @ r, rtol=1e-10, atol=1e-12 * np.abs(B @ r).max())


def test_vcycle_with_ilu0_smoother_brute_force():
    """V(1,1) with block ILU(0) smoothing: the dense operator of the definition with the
    smoother S_l = the standalone ILU(0) preconditioner of A_l (pinned above), applied
    column by column."""
    n = 5
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 7))
    s = oracle.Solver(A, 4, coarse_enough=40, smoother=oracle.ILU0, ilu_sweeps=2)
    nlev = s.nlevels()
    assert nlev >= 2

    def smoother(l):
        Al = s.level(l)["A"]
        si = oracle.Solver(Al, 4, kind=oracle.KIND_ILU, ilu_level=0, ilu_sweeps=2)
        m = Al.shape[0]
        return np.column_stack([si.precond(np.eye(m)[:, j]) for j in range(m)])

    def dense_cycle(l):
        L = s.level(l)
        Al = dense(L["A"])
        if l == nlev - 1:
            return np.linalg.inv(Al)
        Sm = smoother(l)
        P, R = dense(L["P"]), dense(L["R"])
        I = np.eye(Al.shape[0])
        return Sm + (I - Sm @ Al) @ Sm + (I - Sm @ Al) @ P @ dense_cycle(l + 1) @ R @ (I - Al @ Sm)

    B = dense_cycle(0)
    r = np.random.default_rng(12).normal(size=A.shape[0])
    z = s.precond(r)
    assert np.allclose(z, B @ r, rtol=1e-10, atol=1e-12 * np.abs(B @ r).max())
    with pytest.raises(RuntimeError):
        s.solve(r, 1e-8, transposed=True)


def test_transposed_vcycle_is_adjoint(small_hierarchy):
    """<y, B x> = <B^T y, x> for the transposed-cycle preconditioner."""
    n, A, s = small_hierarchy
    rng = np.random.default_rng(4)
    x, y = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    lhs = y @ s.precond(x)
    rhs = s.precond(y, transposed=True) @ x
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)


def test_single_level_is_exact():
    """coarse_enough >= unknowns: the preconditioner is the exact inverse and BiCGStab
    converges in one iteration."""
    n = 4
    A = oracle.stokes_matrix(n)
    s = oracle.Solver(A, 4, coarse_enough=10 ** 6)
    assert s.nlevels() == 1
    b = S.mms_rhs(n)
    x, info = s.solve(b, 1e-12)
    assert info["iters"] == 1 and info["converged"]
    xd = np.linalg.solve(dense(A), b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


# ---------------------------------------------------------------- Krylov

@pytest.mark.parametrize("n", [4, 5, 6])
@pytest.mark.parametrize("krylov", [oracle.BICGSTAB, oracle.FGMRES, oracle.IDRS])
def test_solver_against_dense_lu(n, krylov):
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, n))
    xs = S.mms_solution(n)
    b = A @ xs
    s = oracle.Solver(A, 4, krylov=krylov, coarse_enough=100)
    x, info = s.solve(b, 1e-12)
    xd = np.linalg.solve(dense(A), b)
    assert info["converged"] and info["rel_resid"] <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert np.linalg.norm(xd - xs) <= 1e-9 * np.linalg.norm(xs)


def test_fgmres_terminates_in_n_steps():
    rng = np.random.default_rng(5)
    m = 12
    A = sp.csr_matrix(rng.normal(size=(m, m)) + 6 * np.eye(m))
    s = oracle.Solver(A, 1, kind=oracle.KIND_IDENTITY, krylov=oracle.FGMRES, fgmres_m=m)
    b = rng.normal(size=m)
    x, info = s.solve(b, 1e-13)
    assert info["iters"] <= m and info["converged"]
    assert np.allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-11)


def test_idr_shadow_space_is_splitmix64_orthonormalized():
    """Column 0 of the shadow space is the normalized SplitMix64 sequence from state 0
    (published first outputs below) mapped to [-1, 1); columns are orthonormal."""
    first = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    raw = np.array([(v >> 11) * 2.0 ** -53 * 2.0 - 1.0 for v in first])
    n, s = 50, 5
    P = oracle.idr_shadow(n, s)
    assert np.allclose(P[:4, 0] / P[0, 0], raw / raw[0], rtol=1e-13)
    assert np.abs(P.T @ P - np.eye(s)).max() <= 1e-14


@pytest.mark.parametrize("m,s", [(40, 4), (60, 2), (30, 1), (48, 6)])
def test_idrs_terminates_within_m_plus_m_over_s(m, s):
    """IDR(s) finds the solution of an m x m system in at most m + m/s products with A
    (exact arithmetic); nonsymmetric test matrices with spread spectrum."""
    rng = np.random.default_rng(3 + m + s)
    A = np.diag(np.linspace(1, 20, m)) + 0.5 * rng.normal(size=(m, m)) / np.sqrt(m)
    b = rng.normal(size=m)
    so = oracle.Solver(sp.csr_matrix(A), 1, kind=oracle.KIND_IDENTITY, krylov=oracle.IDRS,
                       idr_s=s, max_restarts=0)
    x, info = so.solve(b, 1e-10)
    assert info["converged"] and info["iters"] <= m + m // s
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8)


# ---------------------------------------------------------------- block ILU(k)

def split_lu(Fd, b):
    nb = Fd.shape[0] // b
    blk = np.kron(np.arange(nb), np.ones(b, int))
    lower = blk[:, None] > blk[None, :]
    L = np.where(lower, Fd, 0.0) + np.eye(Fd.shape[0])
    U = np.where(~lower, Fd, 0.0)
    return L, U


def test_ilu0_of_tridiagonal_is_exact_lu():
    """No fill is dropped for a tridiagonal matrix: L U = A, and with as many sweeps as
    rows the Jacobi-iterated triangular solves are exact."""
    m = 11
    A = sp.csr_matrix(chain(m) + sp.diags(np.linspace(0.1, 0.6, m - 1), 1))
    s = oracle.Solver(A, 1, kind=oracle.KIND_ILU, ilu_level=0, ilu_sweeps=m)
    L, U = split_lu(dense(s.ilu_factor()), 1)
    assert np.allclose(L @ U, dense(A), atol=1e-14)
    r = np.random.default_rng(8).normal(size=m)
    assert np.allclose(s.precond(r), np.linalg.solve(dense(A), r), rtol=1e-12)


@pytest.mark.parametrize("level", [0, 1])
def test_ilu_reproduces_a_on_its_pattern(level):
    """The defining property of ILU: (L U)_ij = A_ij on the stored block pattern, which
    contains A's pattern (plus level-1 fill for ILU(1)); block rows of 4x4."""
    n = 5
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 3))
    s = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_level=level, ilu_sweeps=2)
    F = s.ilu_factor()
    L, U = split_lu(dense(F), 4)
    Ad = dense(A)
    blk = np.kron(np.arange(n ** 3), np.ones(4, int))
    # block pattern of the factor
    Fc, Ac = F.tocoo(), A.tocoo()          # stored entries, explicit zeros included
    Fb = sp.csr_matrix((np.ones(Fc.nnz), (blk[Fc.row], blk[Fc.col])))
    Ab = sp.csr_matrix((np.ones(Ac.nnz), (blk[Ac.row], blk[Ac.col])))
    Fb.data[:] = 1.0
    Ab.data[:] = 1.0
    assert (Ab.multiply(Fb) != Ab).nnz == 0           # A's pattern is inside the factor's
    mask = np.kron(dense(Fb) != 0, np.ones((4, 4), bool))
    LU = L @ U
    assert np.abs((LU - Ad)[mask]).max() <= 1e-12 * np.abs(Ad).max()
    if level == 1:
        assert Fb.nnz > Ab.nnz                        # fill was kept
        F0 = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_level=0).ilu_factor()
        L0, U0 = split_lu(dense(F0), 4)
        # the level-1 factor is the better approximation of A
        assert np.linalg.norm(LU - Ad) < np.linalg.norm(L0 @ U0 - Ad)


def test_ilu_sweeps_limit_and_zero_sweeps():
    """Enough sweeps reach the exact solve with the factors; zero sweeps leave block
    Jacobi with the pivot blocks, z = D^-1 r."""
    n = 4
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 4))
    r = np.random.default_rng(9).normal(size=A.shape[0])
    many = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_level=1, ilu_sweeps=n ** 3)
    L, U = split_lu(dense(many.ilu_factor()), 4)
    assert np.allclose(many.precond(r), np.linalg.solve(U, np.linalg.solve(L, r)), rtol=1e-10)
    zero = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_level=1, ilu_sweeps=0)
    Dm = np.zeros_like(U)
    for i in range(n ** 3):
        Dm[4 * i:4 * i + 4, 4 * i:4 * i + 4] = U[4 * i:4 * i + 4, 4 * i:4 * i + 4]
    assert np.allclose(zero.precond(r), np.linalg.solve(Dm, r), rtol=1e-12)


def test_ilut_hand_derived():
    """ILUT(p = 1, tau = 0.05) of the 4 x 4 matrix [[4,1,0,1],[1,4,1,0],[0,1,4,1],[1,0,1,4]]
    by hand (every row norm is sqrt(18), so the drop tolerance is 0.05 sqrt(18) = 0.2121):
      row 0: U = (4, 1, 0, 1);
      row 1: l10 = 1/4 (kept), fill u13 = -1/4 passes the tolerance but the cap of
             p * 1 upper block keeps only u12 = 1; u11 = 4 - 1/4 = 3.75;
      row 2: l21 = 1/3.75, u22 = 4 - 1/3.75, u23 = 1;
      row 3: l30 = 1/4; the fill at (3,1), -1/4, becomes -1/4 / 3.75 = -0.0667 and is
             dropped (below 0.2121, and not eliminated further); l32 = 1 / u22;
             u33 = 4 - 1/4 - l32."""
    A = sp.csr_matrix(np.array([[4.0, 1, 0, 1], [1, 4, 1, 0], [0, 1, 4, 1], [1, 0, 1, 4]]))
    s = oracle.Solver(A, 1, kind=oracle.KIND_ILU, ilu_kind=1, ilut_p=1.0, ilut_tau=0.05)
    F = dense(s.ilu_factor())
    u22 = 4.0 - 1.0 / 3.75
    l32 = 1.0 / u22
    expect = np.array([[4.0, 1.0, 0.0, 1.0],
                       [0.25, 3.75, 1.0, 0.0],
                       [0.0, 1.0 / 3.75, u22, 1.0],
                       [0.25, 0.0, l32, 4.0 - 0.25 - l32]])
    assert np.abs(F - expect).max() <= 1e-15
    assert s.ilu_factor().nnz == 12          # neither (3,1) nor (1,3) is stored
    assert np.allclose(s.ilu_dinv()[:, 0, 0], 1.0 / np.diag(expect), rtol=1e-15)


def test_ilut_limits():
    """tau = 0 with an unlimited fill cap keeps every block: ILUT is then the exact block
    LU without pivoting, L U = A (the smallest pivot of this diagonally dominated system
    keeps it stable); a tolerance larger than any row norm drops every off-diagonal block,
    leaving the diagonal blocks of A and their inverses (block Jacobi)."""
    n = 4
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 6))
    b = 4
    full = oracle.Solver(A, b, kind=oracle.KIND_ILU, ilu_kind=1, ilut_p=1e6, ilut_tau=0.0)
    L, U = split_lu(dense(full.ilu_factor()), b)
    Ad = dense(A)
    assert np.abs(L @ U - Ad).max() <= 1e-11 * np.abs(Ad).max()
    diag = oracle.Solver(A, b, kind=oracle.KIND_ILU, ilu_kind=1, ilut_p=2.0, ilut_tau=1e9)
    Fd = dense(diag.ilu_factor())
    nb = n ** 3
    for i in range(nb):
        blk = Fd[b * i:b * i + b]
        Dii = Ad[b * i:b * i + b, b * i:b * i + b]
        assert np.array_equal(blk[:, b * i:b * i + b], Dii)
        assert np.count_nonzero(blk) == np.count_nonzero(Dii)
        assert np.allclose(diag.ilu_dinv()[i], np.linalg.inv(Dii), rtol=1e-12)


def test_ilut_cap_keeps_largest_blocks():
    """With tau = 0 the cap alone decides: every row of L and of U keeps at most
    floor(p * n) blocks (n: A's blocks of that row and triangle) and always its diagonal
    block.  Checked on a random block matrix with random fill for three caps."""
    rng = np.random.default_rng(3)
    nb, b = 12, 3
    D = sp.random(nb * b, nb * b, density=0.25, random_state=4, data_rvs=lambda k: rng.normal(size=k))
    A = sp.csr_matrix(D + sp.eye(nb * b) * 8.0)
    for p in (0.5, 1.0, 1.5):
        s = oracle.Solver(A, b, kind=oracle.KIND_ILU, ilu_kind=1, ilut_p=p, ilut_tau=0.0)
        Fd = dense(s.ilu_factor())
        Ad = dense(A)
        for i in range(nb):
            a_blocks = [j for j in range(nb) if np.any(Ad[b * i:b * i + b, b * j:b * j + b])]
            nL = sum(j < i for j in a_blocks)
            nU = sum(j > i for j in a_blocks)
            f_blocks = [j for j in range(nb) if np.any(Fd[b * i:b * i + b, b * j:b * j + b])]
            assert sum(j < i for j in f_blocks) <= int(np.floor(p * nL))
            assert sum(j > i for j in f_blocks) <= int(np.floor(p * nU))
            assert i in f_blocks


def test_idrs_with_ilu1_reaches_dense_solution():
    """The paper's monolithic configuration (IDR(5) with ILU(1)) on a small system."""
    n = 6
    A = oracle.stokes_matrix(n, S.theta_field(n, 0.5, 5))
    b = A @ S.mms_solution(n)
    s = oracle.Solver(A, 4, kind=oracle.KIND_ILU, ilu_level=1, ilu_sweeps=3,
                      krylov=oracle.IDRS, idr_s=5)
    x, info = s.solve(b, 1e-11)
    xd = np.linalg.solve(dense(A), b)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_bicgstab_edge_cases():
    n = 5
    A = oracle.stokes_matrix(n)
    s = oracle.Solver(A, 4, maxiter=1, max_restarts=0, coarse_enough=40)
    x, info = s.solve(np.zeros(A.shape[0]))
    assert info["converged"] and info["iters"] == 0 and not np.any(x)
    x, info = s.solve(S.mms_rhs(n), 1e-14)
    assert not info["converged"] and info["iters"] == 1


# ---------------------------------------------------------------- Schur

def test_schur_complement_closed_form():
    """Constant viscosity: the interior stencil of S = C - B_lo diag(A_uu)^-1 B_up is
    -6.25 at the node, 1 at the six neighbours and +1/24 at distance two."""
    n = 9
    A = oracle.stokes_matrix(n)
    s = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES)
    Sh = dense(s.level(0, which=1)["A"])
    i = j = k = 4
    g = i + n * (j + n * k)
    row = Sh[g]
    assert row[g] == pytest.approx(-6.25, rel=1e-14)
    for d in (1, n, n * n):
        assert row[g + d] == pytest.approx(1.0, rel=1e-14)
        assert row[g - d] == pytest.approx(1.0, rel=1e-14)
        assert row[g + 2 * d] == pytest.approx(1 / 24, rel=1e-12)
        assert row[g - 2 * d] == pytest.approx(1 / 24, rel=1e-12)
    assert np.count_nonzero(row) == 13


def test_schur_apply_is_block_factorization():
    """With single-level (exact) inner solves, the Schur preconditioner equals the dense
    block factorization: z_p = S^-1 (r_p - B_lo A_uu^-1 r_u), z_u = A_uu^-1 (r_u - B_up z_p)."""
    n = 5
    A = oracle.stokes_matrix(n, S.theta_field(n, 1.0, 9))
    s = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, krylov=oracle.FGMRES, coarse_enough=10 ** 6)
    D = dense(A)
    nn = n ** 3
    u = np.array([4 * g + c for g in range(nn) for c in range(3)])
    p = 4 * np.arange(nn) + 3
    Auu, Bup, Blo, Cc = D[np.ix_(u, u)], D[np.ix_(u, p)], D[np.ix_(p, u)], D[np.ix_(p, p)]
    Sh = Cc - Blo @ np.diag(1 / np.diag(Auu)) @ Bup
    assert np.allclose(dense(s.level(0, which=1)["A"]), Sh, rtol=1e-14, atol=1e-14)
    r = np.random.default_rng(6).normal(size=4 * nn)
    zp = np.linalg.solve(Sh, r[p] - Blo @ np.linalg.solve(Auu, r[u]))
    zu = np.linalg.solve(Auu, r[u] - Bup @ zp)
    z = s.precond(r)
    assert np.allclose(z[u], zu, rtol=1e-9, atol=1e-12)
    assert np.allclose(z[p], zp, rtol=1e-9, atol=1e-12)


def test_schur_diagonal_approximation_and_spai0_pressure():
    """eq. SchurApprox: S_diag = C - diag(B_lo diag(A_uu)^-1 B_up) keeps C off the diagonal
    and has the diagonal of the full approximation (itself pinned above).  The SPAI(0)
    pressure step m .* r_p (lower factorization, r_u = 0) minimizes ||I - diag(m) S_diag||_F."""
    n = 5
    A = oracle.stokes_matrix(n, S.theta_field(n, 1.0, 9))
    D = dense(A)
    nn = n ** 3
    p = 4 * np.arange(nn) + 3
    Cc = D[np.ix_(p, p)]
    full = dense(oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, coarse_enough=10 ** 6)
                 .level(0, which=1)["A"])
    sd = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, coarse_enough=10 ** 6, schur_approx=1)
    Sd = dense(sd.level(0, which=1)["A"])
    off = ~np.eye(nn, dtype=bool)
    assert np.array_equal(Sd[off], Cc[off])
    assert np.allclose(np.diag(Sd), np.diag(full), rtol=1e-15, atol=0)
    sp0 = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, coarse_enough=10 ** 6, schur_approx=1,
                        schur_spai0=1, schur_lower=1)
    r = np.zeros(4 * nn)
    r[p] = 1.0
    z = sp0.precond(r)
    m = z[p]
    assert not np.any(np.delete(z, p))
    base = np.linalg.norm(np.eye(nn) - np.diag(m) @ Sd)
    rng = np.random.default_rng(4)
    for _ in range(20):
        assert np.linalg.norm(np.eye(nn) - np.diag(m + 1e-4 * rng.normal(size=nn)) @ Sd) >= base
    # normal equations of each row's least-squares problem
    assert np.allclose(((np.eye(nn) - np.diag(m) @ Sd) * Sd).sum(axis=1), 0, atol=1e-12)


def test_schur_lower_is_block_lower_factorization():
    """Lower factorization with exact inner solves: z_u = A_uu^-1 r_u,
    z_p = S^-1 (r_p - B_lo z_u); no second velocity solve."""
    n = 5
    A = oracle.stokes_matrix(n, S.theta_field(n, 1.0, 9))
    s = oracle.Solver(A, 4, kind=oracle.KIND_SCHUR, coarse_enough=10 ** 6, schur_lower=1)
    D = dense(A)
    nn = n ** 3
    u = np.array([4 * g + c for g in range(nn) for c in range(3)])
    p = 4 * np.arange(nn) + 3
    Auu, Bup, Blo, Cc = D[np.ix_(u, u)], D[np.ix_(u, p)], D[np.ix_(p, u)], D[np.ix_(p, p)]
    Sh = Cc - Blo @ np.diag(1 / np.diag(Auu)) @ Bup
    r = np.random.default_rng(6).normal(size=4 * nn)
    zu = np.linalg.solve(Auu, r[u])
    zp = np.linalg.solve(Sh, r[p] - Blo @ zu)
    z = s.precond(r)
    assert np.allclose(z[u], zu, rtol=1e-9, atol=1e-12)
    assert np.allclose(z[p], zp, rtol=1e-9, atol=1e-12)


def test_schur_scalar_and_block_velocity_amg_coincide():
    """The finite-difference velocity block has no coupling between u, v and w, so its 3x3
    blocks are diagonal: block strength, aggregation, prolongation and SPAI(0) reduce to the
    scalar ones, and the velocity AMG on scalar values (the paper's V2 format) is the same
    preconditioner as on 3x3 blocks (V3) - two independent code paths agree."""
    n = 9
    A = oracle.stokes_matrix(n, S.theta_field(n, 1.0, 6))
    kw = dict(kind=oracle.KIND_SCHUR, coarse_enough=150)
    sb = oracle.Solver(A, 4, **kw)
    ss = oracle.Solver(A, 4, schur_scalar_u=1, **kw)
    assert sb.level(0, 0)["block"] == 3 and ss.level(0, 0)["block"] == 1
    assert sb.nlevels(0) == ss.nlevels(0) >= 2
    r = np.random.default_rng(10).normal(size=A.shape[0])
    zb, zs = sb.precond(r), ss.precond(r)
    assert np.allclose(zb, zs, rtol=1e-12, atol=1e-14 * np.abs(zb).max())


def test_schur_exact_complement_one_iteration():
    """If the pressure operator were the exact Schur complement C - B_lo A_uu^-1 B_up, the
    factorization would be A^-1 (eqs. SchurP/SchurU); the dense check of that identity pins
    the order of the three steps used by the oracle."""
    n = 4
    A = dense(oracle.stokes_matrix(n, S.theta_field(n, 1.0, 9)))
    nn = n ** 3
    u = np.array([4 * g + c for g in range(nn) for c in range(3)])
    p = 4 * np.arange(nn) + 3
    Auu, Bup, Blo, Cc = A[np.ix_(u, u)], A[np.ix_(u, p)], A[np.ix_(p, u)], A[np.ix_(p, p)]
    Sx = Cc - Blo @ np.linalg.solve(Auu, Bup)
    r = np.random.default_rng(7).normal(size=4 * nn)
    zp = np.linalg.solve(Sx, r[p] - Blo @ np.linalg.solve(Auu, r[u]))
    zu = np.linalg.solve(Auu, r[u] - Bup @ zp)
    z = np.empty(4 * nn)
    z[u], z[p] = zu, zp
    assert np.allclose(z, np.linalg.solve(A, r), rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- gradient

def test_gradient_is_exact_linear_derivative():
    """A is linear in theta, so dL/dtheta_e = -lambda^T (A(theta + e_e) - A(theta)) x
    exactly; the edge formula must agree for every cell."""
    n = 5
    th = S.theta_field(n, 0.5, 12)
    A = oracle.stokes_matrix(n, th)
    rng = np.random.default_rng(8)
    x, lam = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    g = oracle.theta_gradient(n, lam, x)
    for e in range(0, (n - 1) ** 3, 3):
        t2 = th.copy()
        t2[e] += 1.0
        dA = oracle.stokes_matrix(n, t2) - A
        assert g[e] == pytest.approx(-(lam @ (dA @ x)), rel=1e-9, abs=1e-9)


def test_gradient_matches_central_fd():
    n = 6
    th = S.theta_field(n, 0.5, 13)
    thr = S.theta_field(n, 0.5, 14)
    b = S.mms_rhs(n)

    def solve(t):
        s = oracle.Solver(oracle.stokes_matrix(n, t), 4, coarse_enough=100)
        x, info = s.solve(b, 1e-13)
        assert info["converged"]
        return x, s

    xt, _ = solve(thr)
    x, s = solve(th)
    lam, info = s.solve(x - xt, 1e-13, transposed=True)
    assert info["converged"]
    g = oracle.theta_gradient(n, lam, x)
    loss = lambda t: 0.5 * np.sum((solve(t)[0] - xt) ** 2)
    for e in S.fd_cells(n, 5, 15):
        d = np.zeros_like(th)
        d[e] = 1e-6
        fd = (loss(th + d) - loss(th - d)) / 2e-6
        assert fd == pytest.approx(g[e], rel=1e-5, abs=1e-9)
