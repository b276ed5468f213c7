"""Pins of the oracle's overload loss and its dense-Jacobian gradients."""
import numpy as np
import pytest

import gridgen
from oracle import adjoint


def _fd(fun, v, j, h):
    vp, vm = v.copy(), v.copy()
    vp[j] += h
    vm[j] -= h
    return (fun(vp) - fun(vm)) / (2 * h)


def test_two_bus_closed_form():
    """One branch: theta_1 = P_1 x, f = -P_1 whatever x is, so
    L = softplus(k (|P_1| / F - 1)), dL/dP_1 = sigma(z) k sign(P_1) / F and
    dL/dx = 0."""
    g = gridgen.hand_grid("two_bus")
    F = np.array([2.0])
    k = 20.0
    L, dP, dx = adjoint.gradients_dense(g, -1, g.P, g.x, F, kappa=k)
    z = k * (abs(g.P[1]) / F[0] - 1.0)
    assert L == pytest.approx(np.logaddexp(0, z), rel=1e-14)
    assert dP[1] == pytest.approx(adjoint.sigmoid(z) * k * np.sign(g.P[1]) / F[0], rel=1e-13)
    assert dP[0] == 0.0 and abs(dx[0]) < 1e-15


@pytest.mark.parametrize("case", ["intact", "plain", "island"])
def test_gradients_match_central_differences(grids, case):
    """Central differences (h = 1e-6) of the refined direct loss on seeded
    entries of P and x, for the intact grid, a non-islanding outage and an
    islanding outage with main-system generators (re-dispatch chain rule)."""
    import oracle

    g = grids["grid200"]
    F = adjoint.flow_limits(g)
    if case == "intact":
        c = -1
    else:
        want = case == "island"
        c = next(e for e in range(g.m) if oracle.is_bridge(g, e) == want
                 and (not want or oracle.island_of(g, e).sum() >= 3))
    L, dP, dx = adjoint.gradients_dense(g, c, g.P, g.x, F)
    assert L == pytest.approx(adjoint.scenario_loss(g, c, g.P, g.x, F), rel=1e-12)
    rng = np.random.default_rng(5)
    isl = np.flatnonzero(oracle.island_of(g, c)) if c >= 0 else np.array([], int)
    jp = list(rng.choice(np.arange(1, g.n), 6, replace=False)) + list(isl[:2])
    for j in jp:
        fd = _fd(lambda v: adjoint.scenario_loss(g, c, v, g.x, F), g.P.copy(), j, 1e-6)
        assert abs(fd - dP[j]) <= 1e-6 * max(1.0, np.abs(dP).max()), (case, j, fd, dP[j])
    for e in list(rng.choice(g.m, 6, replace=False)) + ([c] if c >= 0 else []):
        fd = _fd(lambda v: adjoint.scenario_loss(g, c, g.P, v, F), g.x.copy(), e, 1e-6)
        assert abs(fd - dx[e]) <= 1e-6 * max(1.0, np.abs(dx).max()), (case, e, fd, dx[e])


def test_redispatch_jacobian_is_derivative():
    """The re-dispatch Jacobian against differences of the map itself."""
    import oracle

    g = gridgen.hand_grid("path5")
    island = oracle.island_of(g, 2)
    J = adjoint.redispatch_jacobian(g.P, island)
    for j in range(g.n):
        col = _fd(lambda v: oracle.redispatch(v, island)[0], g.P.copy(), j, 1e-7)
        np.testing.assert_allclose(J[:, j], col, rtol=0, atol=1e-8)


def test_pin_catches_dropped_direct_term(grids):
    """A planted mistake (the direct x-dependence of the flows left out) is
    caught by the difference check."""
    g = grids["grid200"]
    F = adjoint.flow_limits(g)
    L, dP, dx = adjoint.gradients_dense(g, 3, g.P, g.x, F)
    e = int(np.argmax(np.abs(dx)))
    fd = _fd(lambda v: adjoint.scenario_loss(g, 3, g.P, v, F), g.x.copy(), e, 1e-6)
    z = 20.0 * (np.abs(adjoint.flows(adjoint.with_reactances(g, g.x),
                                      adjoint.scenario(g, 3)["theta"], 3)) / F - 1.0)
    f = adjoint.scenario(g, 3)["flows"]
    direct = adjoint.sigmoid(z) * 20.0 * np.sign(f) / F * (-f / g.x)
    assert abs(fd - dx[e]) <= 1e-6 * np.abs(dx).max()
    assert abs(fd - (dx[e] - direct[e])) > 1e-3 * np.abs(dx).max()


def test_sparse_adjoint_equals_dense_jacobians(grids):
    """The adjoint form with sparse LU solves (used on the 10,000-bus grid,
    where a dense inverse is out of reach) against the dense-Jacobian chain
    rule, for the intact grid and every outage of the 200-bus grid
    (re-dispatch and islands included): relative 1e-9 of each gradient's
    largest entry."""
    g = grids["grid200"]
    F = adjoint.flow_limits(g)
    for c in range(-1, g.m):
        L1, p1, x1 = adjoint.gradients_dense(g, c, g.P, g.x, F)
        L2, p2, x2 = adjoint.gradients_sparse(g, c, g.P, g.x, F)
        assert L2 == pytest.approx(L1, rel=1e-10), c  # the dense inverse is the less accurate of the two
        assert np.abs(p1 - p2).max() <= 1e-9 * np.abs(p1).max(), c
        assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x1).max(), c


def test_sparse_adjoint_planted_mistake(grids, monkeypatch):
    """A sparse adjoint that forgot the re-dispatch chain rule (dL/dP =
    lambda on the island and generators unchanged) misses the dense
    gradients on an islanding outage with main-system generators."""
    import oracle

    g = grids["grid200"]
    F = adjoint.flow_limits(g)
    c = next(e for e in range(g.m) if oracle.island_of(g, e).sum() >= 2)
    _, p1, _ = adjoint.gradients_dense(g, c, g.P, g.x, F)
    monkeypatch.setattr(adjoint, "redispatch", lambda P, isl: (np.where(isl, 0.0, P), False))
    _, p2, _ = adjoint.gradients_sparse(g, c, g.P, g.x, F)
    assert np.abs(p1 - p2).max() > 1e-6 * np.abs(p1).max()
