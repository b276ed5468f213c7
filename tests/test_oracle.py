"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself.  Each pin uses an independent
route to the same number: a closed form on a hand grid, a dense inverse, the
Sherman-Morrison line-outage formula, the bridge / effective-reactance
identity, Kirchhoff's current law, the defining property of ILU(0).  The
last tests plant mistakes in the oracle (on the CPU) and check that a pin
catches each one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import gridgen
import oracle
from oracle import system as osys

RNG = np.random.default_rng(1234)


def _dense_inv(A):
    return np.linalg.inv(A.toarray())


def _net_outflow(g, f):
    out = np.zeros(g.n)
    np.add.at(out, g.br_from, f)
    np.add.at(out, g.br_to, -f)
    return out


def _lu_nopivot(A):
    """Exact LU without pivoting by dense Gaussian elimination (textbook)."""
    a = A.toarray().astype(float)
    n = a.shape[0]
    for k in range(n):
        a[k + 1:, k] /= a[k, k]
        a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k], a[k, k + 1:])
    L = sp.csr_matrix(np.tril(a, -1))
    U = sp.csr_matrix(np.triu(a))
    return L, U


# ---------------------------------------------------------------- hand grids


def test_two_bus_closed_form():
    # one branch: B' = [1/x], theta_1 = P_1 x
    g = gridgen.hand_grid("two_bus")
    th, A = oracle.base_case(g)
    assert A.shape == (1, 1) and A[0, 0] == pytest.approx(1 / 0.2)
    assert th[1] == pytest.approx(1.5 * 0.2, abs=1e-15)
    # its only branch out: bus 1 islanded, nothing left to dispatch to
    s = oracle.scenario(g, 0, A)
    assert s["island"].tolist() == [False, True]
    assert np.all(s["theta"] == 0) and s["status"] == oracle.STATUS_ISLANDED_NO_GEN


def test_ring3_closed_form():
    # equal reactances a: B' = (1/a)[[2,-1],[-1,2]], inverse (a/3)[[2,1],[1,2]]
    g = gridgen.hand_grid("ring3")
    a = 0.1
    th, A = oracle.base_case(g)
    np.testing.assert_allclose(A.toarray(), np.array([[2, -1], [-1, 2]]) / a, rtol=1e-15)
    P1, P2 = 0.3, 0.4
    np.testing.assert_allclose(th[1:], (a / 3) * np.array([2 * P1 + P2, P1 + 2 * P2]), rtol=1e-14)
    # branch (1,2) out: two radial branches, theta_k = a P_k
    s = oracle.scenario(g, 2, A)
    np.testing.assert_allclose(s["theta"][1:], [a * P1, a * P2], rtol=1e-14)
    # branch (0,1) out: path 0-2-1, theta_2 = a (P1+P2), theta_1 = theta_2 + a P1
    s = oracle.scenario(g, 0, A)
    np.testing.assert_allclose(s["theta"][1:], [a * (P1 + P2) + a * P1, a * (P1 + P2)], rtol=1e-14)


def test_path5_closed_form_and_redispatch():
    # radial grid: every flow is minus the injection sum beyond it
    g = gridgen.hand_grid("path5")
    P = g.P
    th, A = oracle.base_case(g)
    f = oracle.flows(g, th)
    np.testing.assert_allclose(f, [-(P[1:].sum()), -(P[2:].sum()), -(P[3:].sum()), -P[4]], atol=1e-14)
    assert th[1] == pytest.approx(0.02, abs=1e-15)
    assert th[4] == pytest.approx(-0.185, abs=1e-14)
    # branch (2,3) out: island {3,4} exported 0.6-0.5 = 0.1; the only main
    # generator (bus 1, P=0.5) takes it over: P'_1 = 0.5 (1 + 0.1/0.5) = 0.6
    s = oracle.scenario(g, 2, A)
    assert s["island"].tolist() == [False, False, False, True, True]
    np.testing.assert_allclose(s["Pp"], [-0.2, 0.6, -0.4, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(s["theta"], [0.0, 0.02, 0.02 - 0.4 * 0.2, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(s["flows"], [-0.2, 0.4, 0.0, 0.0], atol=1e-14)
    assert s["status"] == oracle.STATUS_CONVERGED_ISLANDED


def test_slack_leaf_outage_islands_everything():
    g = gridgen.hand_grid("slack_leaf")
    s = oracle.scenario(g, 0)
    assert s["island"][1:].all() and not s["island"][0]
    assert np.all(s["theta"] == 0) and np.all(s["flows"] == 0)
    assert s["status"] == oracle.STATUS_ISLANDED_NO_GEN


def test_parallel_branch_is_not_a_bridge():
    g = gridgen.hand_grid("parallel")
    assert not oracle.is_bridge(g, 0) and not oracle.is_bridge(g, 1)
    th, A = oracle.base_case(g)
    s = oracle.scenario(g, 0, A)
    assert not s["island"].any()
    # the remaining parallel branch and the ring still carry the injections
    np.testing.assert_allclose(_net_outflow(g, s["flows"])[1:], g.P[1:], atol=1e-13)
    assert s["flows"][0] == 0.0 and s["flows"][1] != 0.0


@pytest.mark.parametrize("name", gridgen.HAND_GRIDS)
def test_small_grids_dense_lu_pcg_agree(name):
    g = gridgen.hand_grid(name)
    th, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    for c in range(-1, g.m):
        d = oracle.scenario(g, c, A)
        main = np.flatnonzero(~d["island"][1:])
        if len(main):
            Ad = d["Ac"].toarray()[np.ix_(main, main)]
            dense = np.linalg.inv(Ad) @ d["Pp"][1:][main]
            np.testing.assert_allclose(d["theta"][1:][main], dense, rtol=1e-12, atol=1e-14)
        p = oracle.scenario_pcg(g, c, A, L, U, th, tol=1e-13)
        np.testing.assert_allclose(p["theta"], d["theta"], rtol=1e-11, atol=1e-13)
        assert p["status"] == d["status"]


def test_generated_10bus_dense_lu_pcg_agree():
    g = gridgen.make_grid(gridgen.GridSpec("t10", 10, 14, 7))
    th, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    for c in range(g.m):
        d = oracle.scenario(g, c, A)
        main = np.flatnonzero(~d["island"][1:])
        dense = np.linalg.inv(d["Ac"].toarray()[np.ix_(main, main)]) @ d["Pp"][1:][main]
        np.testing.assert_allclose(d["theta"][1:][main], dense, rtol=1e-12, atol=1e-14)
        p = oracle.scenario_pcg(g, c, A, L, U, th, tol=1e-13)
        np.testing.assert_allclose(p["theta"], d["theta"], rtol=1e-10, atol=1e-13)


# ------------------------------------------------------- structural pins


def test_outage_changes_four_entries(grids):
    """Section IV.B / Fig. 7: an outage changes A_ii, A_jj, A_ij, A_ji only
    (one entry when an endpoint is the slack)."""
    g = grids["grid200"]
    _, A = oracle.base_case(g)
    for c in range(g.m):
        D = (oracle.outage_matrix(g, A, c) - A).tocoo()
        D.eliminate_zeros()
        bc = 1 / g.x[c]
        if g.br_from[c] == 0:
            assert D.nnz == 1
            assert D.data[0] == pytest.approx(-bc, rel=1e-15)
        else:
            assert D.nnz == 4
            np.testing.assert_allclose(np.sort(np.abs(D.data)), bc, rtol=1e-12)


def test_bridge_iff_unit_effective_susceptance(grids):
    """R_eff(c) = u^T A^-1 u <= x_c with equality iff c is a bridge, so
    1 - b_c R_eff is 0 exactly for bridges and in (0, 1) otherwise."""
    g = grids["grid200"]
    _, A = oracle.base_case(g)
    Ainv = _dense_inv(A)
    for c in range(g.m):
        u = np.zeros(g.n)
        u[g.br_from[c]] += 1
        u[g.br_to[c]] -= 1
        u = u[1:]
        den = 1 - (u @ Ainv @ u) / g.x[c]
        if oracle.is_bridge(g, c):
            assert abs(den) < 1e-9
            assert oracle.island_of(g, c).any()
        else:
            assert 1e-9 < den < 1
            assert not oracle.island_of(g, c).any()


def test_line_outage_formula(grids):
    """Non-islanding angles equal the Sherman-Morrison update of the base
    angles (the classic DC line-outage distribution formula)."""
    g = grids["grid200"]
    thb, A = oracle.base_case(g)
    Ainv = _dense_inv(A)
    checked = 0
    for c in range(g.m):
        if oracle.is_bridge(g, c):
            continue
        u = np.zeros(g.n)
        u[g.br_from[c]] += 1
        u[g.br_to[c]] -= 1
        u = u[1:]
        b = 1 / g.x[c]
        w = Ainv @ u
        expect = thb[1:] + b * (u @ thb[1:]) / (1 - b * (u @ w)) * w
        got = oracle.scenario(g, c, A)["theta"][1:]
        np.testing.assert_allclose(got, expect, rtol=1e-9, atol=1e-11)
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("key", ["grid200", "grid2k"])
def test_kirchhoff_balance(grids, key):
    """Flows leaving each main bus sum to its (re-dispatched) injection; the
    slack balances the rest; islanded buses carry nothing."""
    g = grids[key]
    _, A = oracle.base_case(g)
    for c in RNG.choice(g.m, 12, replace=False):
        s = oracle.scenario(g, int(c), A)
        out = _net_outflow(g, s["flows"])
        Pp = s["Pp"].copy()
        Pp[0] = -Pp[1:].sum()
        scale = np.abs(g.P).max()
        np.testing.assert_allclose(out, Pp, atol=1e-10 * scale * g.n ** 0.5)
        assert np.all(out[s["island"]] == 0)


def test_redispatch_invariants(grids):
    """Slack output unchanged, islanded injections zero, only main
    generators change, all by the same factor."""
    g = grids["grid200"]
    P = g.P
    n_isl = 0
    for c in range(g.m):
        isl = oracle.island_of(g, c)
        if not isl.any():
            continue
        n_isl += 1
        Pp, nogen = oracle.redispatch(P, isl)
        assert np.all(Pp[isl] == 0)
        assert Pp[1:].sum() == pytest.approx(P[1:].sum(), abs=1e-12)
        gen = ~isl & (P > 0)
        gen[0] = False
        assert nogen == (not gen.any())
        changed = Pp != P
        assert np.all(~changed[~isl & ~gen])
        if gen.any():
            ratio = Pp[gen] / P[gen]
            np.testing.assert_allclose(ratio, ratio[0], rtol=1e-14)
    assert n_isl > 30


def test_base_reproduced_without_outage(grids):
    g = grids["grid2k"]
    thb, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    s = oracle.scenario(g, -1, A)
    np.testing.assert_array_equal(s["theta"], thb)
    p = oracle.scenario_pcg(g, -1, A, L, U, thb)
    assert p["iters"] == 0
    np.testing.assert_array_equal(p["theta"], thb)


# -------------------------------------------------------- solver pins


def test_refined_solve_accuracy(grids):
    g = grids["grid2k"]
    thb, A = oracle.base_case(g)
    b = g.P[1:]
    r = np.asarray(b, np.longdouble) - A.astype(np.longdouble) @ np.asarray(thb[1:], np.longdouble)
    # a correctly rounded solution x = fl(x*) has |b - A x| <= u |A| |x|
    # componentwise (u = 2^-53); the refined solve must be within 2x of that
    floor = 2.0 ** -53 * (abs(A) @ np.abs(thb[1:]))
    assert np.all(np.abs(np.asarray(r, float)) <= 2 * floor + 1e-300)
    # against a dense solve in extended precision on the small grid
    g2 = grids["grid200"]
    th2, A2 = oracle.base_case(g2)
    dense = np.linalg.solve(A2.toarray(), g2.P[1:])
    np.testing.assert_allclose(th2[1:], dense, rtol=1e-11, atol=1e-12)


def test_ilu0_defining_property(grids):
    """(L+I) U equals A on the pattern of A; the symmetric case gives
    U = diag(U) L^T."""
    g = grids["grid2k"]
    _, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    n = A.shape[0]
    LU = ((L + sp.eye(n)) @ U).tocsr()
    Ac = A.tocoo()
    got = np.asarray(LU[Ac.row, Ac.col]).ravel()
    np.testing.assert_allclose(got, Ac.data, rtol=1e-12, atol=1e-9)
    D = sp.diags(U.diagonal())
    np.testing.assert_allclose((D @ L.T).toarray()[np.triu_indices(50, 1)],
                               U.toarray()[np.triu_indices(50, 1)], rtol=1e-13, atol=1e-12)
    assert np.all(U.diagonal() > 0)


def test_inner_product_from_the_forward_solve(grids):
    """Reading of Section III.A's r'z for factors U = D L^T: with r zero on
    an outage's islanded rows and z = P_M (L U)^-1 r, r'z equals y' D^-1 y
    for y = L^-1 r (the masking drops out because r_I = 0).  Checked with
    the oracle's ILU(0) of B' on an islanding outage of the 2k grid, for
    seeded r; and the identity fails for a planted nonsymmetric U (the
    strict upper part scaled), which is why the device checks the form."""
    import scipy.sparse.linalg as spla

    g = grids["grid2k"]
    _, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    n = A.shape[0]
    Lu = (L + sp.eye(n)).tocsr()
    c = next(k for k in range(g.m) if oracle.is_bridge(g, k) and oracle.island_of(g, k).sum() > 3)
    main = ~oracle.island_of(g, c)[1:]
    rng = np.random.default_rng(43)
    d = U.diagonal()
    for Uc, same in ((U, True), (sp.triu(U, 1) * (1 + 1e-6) + sp.diags(d), False)):
        for _ in range(3):
            r = rng.normal(size=n) * main
            y = spla.spsolve_triangular(Lu, r, lower=True)
            z = spla.spsolve_triangular(Uc.tocsr(), y, lower=False) * main
            rz, yy = float(r @ z), float(y @ (y / d))
            assert (abs(rz - yy) <= 1e-11 * abs(rz)) == same, (rz, yy)


def test_ilu0_exact_on_tree():
    """With no fill possible (a tree eliminated leaves first), ILU(0) is the
    exact LU."""
    rng = np.random.default_rng(5)
    n = 40
    parent = [rng.integers(0, k) for k in range(1, n)]
    f = np.array(parent, dtype=np.int32)
    t = np.arange(1, n, dtype=np.int32)
    x = rng.uniform(0.01, 0.3, n - 1)
    # number buses by decreasing depth so that leaves come first
    depth = np.zeros(n, int)
    for k in range(1, n):
        depth[k] = depth[parent[k - 1]] + 1
    order = np.r_[0, 1 + np.argsort(-depth[1:], kind="stable")]
    relabel = np.empty(n, int)
    relabel[order] = np.arange(n)
    ff, tt = relabel[f], relabel[t]
    g = gridgen.Grid("tree", n, np.minimum(ff, tt).astype(np.int32), np.maximum(ff, tt).astype(np.int32), x,
                     np.zeros(n))
    _, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    np.testing.assert_allclose(((L + sp.eye(n - 1)) @ U).toarray(), A.toarray(), rtol=1e-12, atol=1e-10)


def test_pcg_identity_preconditioner_is_cg():
    """With M = I on an SPD system CG finishes in at most n steps (up to
    rounding) and returns the solution of numpy.linalg.solve."""
    rng = np.random.default_rng(3)
    n = 24
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = sp.csr_matrix(Q @ np.diag(np.linspace(1, 20, n)) @ Q.T)
    b = rng.normal(size=n)
    L = sp.csr_matrix((n, n))
    U = sp.eye(n, format="csr")
    x, its, st, _ = oracle.pcg_textbook(A, b, L, U, tol=1e-13)
    assert st == oracle.STATUS_CONVERGED and its <= n + 2
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-11)


def test_exact_factors_converge_in_one_step(grids):
    """With the exact LU of the base matrix as preconditioner, the base-state
    start makes the first search direction parallel to the correction (by
    Sherman-Morrison), so a non-islanding outage converges in one step."""
    g = grids["grid200"]
    thb, A = oracle.base_case(g)
    L, U = _lu_nopivot(A)
    n_checked = 0
    for c in range(0, g.m, 3):
        if oracle.is_bridge(g, c):
            continue
        p = oracle.scenario_pcg(g, c, A, L, U, thb, tol=1e-10)
        assert p["iters"] <= 2, (c, p["iters"])
        n_checked += 1
    assert n_checked > 40


def test_pcg_matches_direct(grids):
    g = grids["grid2k"]
    thb, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    for c in RNG.choice(g.m, 4, replace=False):
        d = oracle.scenario(g, int(c), A)
        p = oracle.scenario_pcg(g, int(c), A, L, U, thb, tol=1e-12)
        assert np.abs(p["theta"] - d["theta"]).max() < 1e-10
        assert p["status"] == d["status"]
        assert oracle.true_residual(g, A, int(c), p["theta"], d["Pp"], d["island"]) < 1e-10


# ------------------------------------------- iteration-count spread


def iteration_bar(k: int) -> int:
    """Iterations two valid PCG implementations may differ by at k
    iterations (the bar of the device parity tests): max(3, ceil(6 % k))."""
    return max(3, int(np.ceil(0.06 * k)))


def test_iteration_spread_between_summation_orders(grids):
    """The stop step of PCG moves with rounding: the recursive residual
    crosses tol ||b|| while it stagnates near the FP64 floor.  The oracle's
    own PCG with three valid inner products (NumPy's, the exactly rounded
    sum of the products, a reversed running sum) on 40 seeded outages of
    the 2,000-bus grid (rows in reverse Cuthill-McKee order, as the device
    runs them) at the benchmark's stop differs by several iterations
    (measured: up to 5 at 2k and 10 of about 300 at 10k), so +-1 cannot be
    asked of two correct implementations.  The device tests' bar covers
    every spread seen here."""
    import math

    def exact_dot(u, v):
        return math.fsum((np.asarray(u) * np.asarray(v)).tolist())

    def reversed_dot(u, v):
        acc = 0.0
        for t in (np.asarray(u) * np.asarray(v))[::-1].tolist():
            acc += t
        return acc

    g = gridgen.make_grid("grid2k", order="rcm")
    thb, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    spread = []
    for c in np.random.default_rng(41).choice(g.m, 40, replace=False):
        its = [oracle.scenario_pcg(g, int(c), A, L, U, thb, tol=5e-11, dot=d)["iters"]
               for d in (None, exact_dot, reversed_dot)]
        spread.append(max(its) - min(its))
        assert max(its) - min(its) <= iteration_bar(max(its)), (c, its)
    assert max(spread) >= 2


# ------------------------------------------------------- true residual


def test_true_residual_closed_form_ring3():
    """ring3 without branch (1,2): A_c = (1/a) I, so theta* + eps e_1 has
    residual A_c (eps e_1) = (eps / a) e_1 and a relative residual of
    (eps / a) / ||P_M||; theta* itself is at rounding level."""
    g = gridgen.hand_grid("ring3")
    _, A = oracle.base_case(g)
    d = oracle.scenario(g, 2, A)
    assert oracle.true_residual(g, A, 2, d["theta"], d["Pp"], d["island"]) < 1e-15
    a, eps = 0.1, 1e-6
    th = d["theta"].copy()
    th[1] += eps
    expect = (eps / a) / np.hypot(g.P[1], g.P[2])
    assert oracle.true_residual(g, A, 2, th, d["Pp"], d["island"]) == pytest.approx(expect, rel=1e-9)


def test_true_residual_closed_form_island():
    """path5 without the bridge (1,2): the main system is bus 1 alone (plus
    the slack), A_c[M,M] = [1/x_01] = [10], and the re-dispatch leaves
    P'_1 = 0.5 (1 + (-0.3) / 0.5) = 0.2.  theta_1* + eps with arbitrary
    values on the island has relative residual 10 eps / 0.2 = 50 eps: the
    island's rows and angles do not enter."""
    g = gridgen.hand_grid("path5")
    _, A = oracle.base_case(g)
    d = oracle.scenario(g, 1, A)
    assert d["Pp"][1] == pytest.approx(0.2, rel=1e-15)
    eps = 1e-7
    th = d["theta"].copy()
    th[1] += eps
    th[2:] = [3.0, -7.0, 11.0]
    assert oracle.true_residual(g, A, 1, th, d["Pp"], d["island"]) == pytest.approx(50 * eps, rel=1e-9)


def test_true_residual_pins_catch_mistakes(monkeypatch):
    """Planted mistakes: a residual that ignored the island (all rows kept)
    or dropped the outage's rank-1 term misses the closed forms above."""
    g = gridgen.hand_grid("path5")
    _, A = oracle.base_case(g)
    d = oracle.scenario(g, 1, A)
    th = d["theta"].copy()
    th[1] += 1e-7
    th[2:] = [3.0, -7.0, 11.0]
    no_mask = oracle.true_residual(g, A, 1, th, d["Pp"], np.zeros(g.n, bool))
    assert abs(no_mask - 50e-7) > 1e-3 * 50e-7
    g3 = gridgen.hand_grid("ring3")
    _, A3 = oracle.base_case(g3)
    d3 = oracle.scenario(g3, 2, A3)
    th3 = d3["theta"].copy()
    th3[1] += 1e-6
    expect = (1e-6 / 0.1) / np.hypot(g3.P[1], g3.P[2])
    monkeypatch.setattr(osys, "_u_reduced", lambda grid, c: np.zeros(grid.n - 1))
    dropped = oracle.true_residual(g3, A3, 2, th3, d3["Pp"], d3["island"])
    assert abs(dropped - expect) > 1e-3 * expect


# ------------------------------------------------- planted mistakes (CPU)


def test_pins_catch_dropped_rank1_term(grids, monkeypatch):
    """If the outage matrix forgot the diagonal half of the change, the
    line-outage pin would fail."""
    g = grids["grid200"]
    thb, A = oracle.base_case(g)
    c = next(c for c in range(g.m) if not oracle.is_bridge(g, c) and g.br_from[c] > 0)
    good = oracle.scenario(g, c, A)["theta"]

    orig = osys.outage_matrix

    def bad(grid, A_, c_):
        # keeps the off-diagonal coupling of the outaged branch
        M = orig(grid, A_, c_).tolil()
        i, j = grid.br_from[c_] - 1, grid.br_to[c_] - 1
        M[i, j] -= 1 / grid.x[c_]
        M[j, i] -= 1 / grid.x[c_]
        return M.tocsr()

    monkeypatch.setattr(osys, "outage_matrix", bad)
    wrong = osys.scenario(g, c, A)["theta"]
    assert np.abs(wrong - good).max() > 1e-6


def test_pins_catch_wrong_redispatch_sign(grids, monkeypatch):
    g = grids["grid200"]
    c = next(c for c in range(g.m) if oracle.island_of(g, c).sum() >= 2)
    orig = osys.redispatch

    def bad(P, island):
        Pp, nogen = orig(P, island)
        gen = ~island & (P > 0)
        gen[0] = False
        dP = P[island].sum()
        Pp[gen] = P[gen] * (1 - dP / P[gen].sum())
        return Pp, nogen

    monkeypatch.setattr(osys, "redispatch", bad)
    s = osys.scenario(g, c)
    out = _net_outflow(g, s["flows"])
    # Kirchhoff still holds for the (wrong) P', but the slack output moves:
    assert abs(out[0] - g.P[0]) > 1e-9


def test_pins_catch_transposed_factor(grids):
    g = grids["grid200"]
    _, A = oracle.base_case(g)
    L, U = oracle.ilu0(A)
    n = A.shape[0]
    LU = ((sp.eye(n) + U.T) @ L.T).tocsr()  # a plausible operand mix-up
    Ac = A.tocoo()
    got = np.asarray(LU[Ac.row, Ac.col]).ravel()
    assert np.abs(got - Ac.data).max() > 1e-3
