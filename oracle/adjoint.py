"""Branch-overload screening loss of an outage scenario and its gradients
with respect to the bus injections and the branch reactances.

TEST INFRASTRUCTURE (see the package docstring).  The screening quantity of
Section IV is the branch flow after the outage; the differentiation workload
turns it into a smooth overload measure

    L = sum_e softplus(kappa (|f_e| / F_e - 1)),

with limits F_e = 1.2 |f_e^base| + 0.1 taken once from the intact base case
and held fixed.  The gradients here are formed with explicit dense Jacobians,
the chain rule written out matrix by matrix:

* the main-system angles depend on the re-dispatched injections through the
  dense inverse of A_c[M,M];
* the re-dispatch of Section IV.C has its own explicit Jacobian (it is
  piecewise smooth: the generator set is fixed away from P_k = 0);
* a reactance changes A_c by (dA_c/dx_e) = -(1/x_e^2) u_e u_e^T (e != c), so
  the angles move by -A_c[M,M]^{-1} (dA_c/dx_e)[M,M] theta_M, and the flow
  f_e = (theta_from - theta_to) / x_e also depends on x_e directly.

At f_e = 0 (the outaged branch, branches inside the island) the derivative
of |f_e| is taken as 0.  Pinned in the tests by central finite differences of
the loss and by a closed form on a two-bus grid.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .system import base_case, flows, island_of, outage_matrix, redispatch, reduced, scenario, susceptance_full


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def with_reactances(grid, x):
    """The same grid with its branch reactances replaced."""
    return dataclasses.replace(grid, x=np.asarray(x, dtype=np.float64))


def flow_limits(grid, P=None) -> np.ndarray:
    """F_e = 1.2 |f_e| + 0.1 from the intact base case (constants)."""
    th, _ = base_case(grid, rhs=P)
    return 1.2 * np.abs(flows(grid, th)) + 0.1


def scenario_loss(grid, c: int, P, x, F, kappa: float = 20.0, extended: bool = False) -> float:
    """The loss of outage c from the direct (refined) scenario solve.

    With ``extended`` the main-system angles, the flows and the loss are kept
    in ``longdouble`` (the refined solve's own precision) instead of being
    rounded to FP64: on large grids, where angles reach thousands of
    radians, the FP64 loss carries rounding of order 1e-13 relative, which
    central differences of small steps would amplify."""
    g = with_reactances(grid, x)
    P = np.asarray(P, dtype=np.float64)
    if not extended:
        d = scenario(g, int(c), rhs=P)
        z = kappa * (np.abs(d["flows"]) / F - 1.0)
        return float(np.sum(softplus(z)))
    from .system import refined_solve

    island = island_of(g, int(c))
    Pp, _ = redispatch(P, island)
    idx = np.flatnonzero(~island[1:])
    Amm = outage_matrix(g, reduced(susceptance_full(g)), int(c))[idx][:, idx].tocsr()
    th = np.zeros(g.n, dtype=np.longdouble)
    th[idx + 1] = refined_solve(Amm, Pp[idx + 1], steps=6, extended=True)
    ld = np.longdouble
    f = (th[g.br_from] - th[g.br_to]) / np.asarray(g.x, dtype=ld)
    if c >= 0:
        f[int(c)] = 0
    inside = island[g.br_from] & island[g.br_to]
    f[inside] = 0
    z = ld(kappa) * (np.abs(f) / np.asarray(F, dtype=ld) - 1)
    return float(np.sum(np.logaddexp(ld(0), z)))


def redispatch_jacobian(P, island) -> np.ndarray:
    """Dense Jacobian dP'/dP of the proportional re-dispatch (Section IV.C)."""
    P = np.asarray(P, dtype=np.float64)
    n = len(P)
    J = np.eye(n)
    if not island.any():
        return J
    J[island, island] = 0.0  # P'_I = 0
    gen = ~island & (P > 0)
    gen[0] = False
    if not gen.any():
        return J
    dP = P[island].sum()
    S = P[gen].sum()
    g = np.flatnonzero(gen)
    isl = np.flatnonzero(island)
    for k in g:  # P'_k = P_k (1 + dP / S)
        J[k, g] = -P[k] * dP / S**2
        J[k, k] = 1.0 + dP / S - P[k] * dP / S**2
        J[k, isl] = P[k] / S
    return J


def gradients_dense(grid, c: int, P, x, F, kappa: float = 20.0):
    """(L, dL/dP[n], dL/dx[m]) for outage c by dense Jacobians."""
    g = with_reactances(grid, x)
    P = np.asarray(P, dtype=np.float64)
    n, m = g.n, len(g.x)
    A = reduced(susceptance_full(g))
    island = island_of(g, int(c))
    Pp, _ = redispatch(P, island)
    idx = np.flatnonzero(~island[1:])  # main-system reduced rows
    bus = idx + 1
    Ac = outage_matrix(g, A, int(c)).toarray()
    Ainv = np.linalg.inv(Ac[np.ix_(idx, idx)])
    theta = np.zeros(n)
    theta[bus] = Ainv @ Pp[bus]
    f = flows(g, theta, int(c), island)
    z = kappa * (np.abs(f) / F - 1.0)
    L = float(np.sum(softplus(z)))
    dLdf = sigmoid(z) * kappa * np.sign(f) / F

    # flows as a linear map of the angles (rows of c and of island-internal
    # branches are zero)
    live = np.ones(m, bool)
    if c >= 0:
        live[c] = False
    live &= ~(island[g.br_from] & island[g.br_to])
    D = np.zeros((m, n))
    e = np.flatnonzero(live)
    D[e, g.br_from[e]] = 1.0 / g.x[e]
    D[e, g.br_to[e]] = -1.0 / g.x[e]
    dLdth = D.T @ dLdf

    # injections: theta_M = Ainv P'_M, P' = redispatch(P)
    Jth_P = np.zeros((n, n))
    Jth_P[np.ix_(bus, bus)] = Ainv
    dLdP = redispatch_jacobian(P, island).T @ (Jth_P.T @ dLdth)

    # reactances: direct dependence of f_e on x_e, and theta through A_c
    dLdx = dLdf * (-f / g.x)
    Jth_x = np.zeros((n, m))
    for k in range(m):
        if k == c:
            continue
        u = np.zeros(n)
        u[g.br_from[k]] += 1.0
        u[g.br_to[k]] -= 1.0
        uM = u[bus]
        if not uM.any():
            continue
        # d theta_M / d x_k = -Ainv (dA/dx_k)[M,M] theta_M, dA/dx_k = -(1/x_k^2) u u^T
        Jth_x[bus, k] = Ainv @ uM * (uM @ theta[bus]) / g.x[k] ** 2
    dLdx = dLdx + Jth_x.T @ dLdth
    return L, dLdP, dLdx


def gradients_sparse(grid, c: int, P, x, F, kappa: float = 20.0):
    """(L, dL/dP[n], dL/dx[m]) for outage c by the adjoint method with
    sparse LU solves (for grids where a dense inverse is out of reach).

    theta_M solves A_c[M,M] theta_M = P'_M and, A_c being symmetric, one more
    solve with the same matrix gives lambda_M = A_c[M,M]^{-1} (dL/dtheta)_M.
    Then, term by term as in ``gradients_dense``:
      dL/dP = (dP'/dP)^T lambda, written out for the proportional
        re-dispatch (Section IV.C): lambda_k on main buses outside the
        generator set G; lambda_k (1 + dP/S) - dP T / S^2 on G; T / S on the
        island; T = sum_G P_k lambda_k, S = sum_G P_k, dP = sum_I P_k;
      dL/dx_k = dL/df_k (-f_k / x_k) + (u_k'theta)(u_k'lambda) / x_k^2,
        the second term from d theta_M / d x_k = A^{-1} u (u'theta) / x_k^2.
    Both solves are sparse LU with extended-precision refinement."""
    from .system import refined_solve

    g = with_reactances(grid, x)
    P = np.asarray(P, dtype=np.float64)
    n, m = g.n, len(g.x)
    A = reduced(susceptance_full(g))
    island = island_of(g, int(c))
    Pp, _ = redispatch(P, island)
    idx = np.flatnonzero(~island[1:])
    bus = idx + 1
    Amm = outage_matrix(g, A, int(c))[idx][:, idx].tocsr()
    theta = np.zeros(n)
    theta[bus] = refined_solve(Amm, Pp[bus])
    f = flows(g, theta, int(c), island)
    z = kappa * (np.abs(f) / F - 1.0)
    L = float(np.sum(softplus(z)))
    dLdf = sigmoid(z) * kappa * np.sign(f) / F
    live = np.ones(m, bool)
    if c >= 0:
        live[c] = False
    live &= ~(island[g.br_from] & island[g.br_to])
    s = np.where(live, dLdf / g.x, 0.0)
    dLdth = np.zeros(n)
    np.add.at(dLdth, g.br_from, s)
    np.add.at(dLdth, g.br_to, -s)
    lam = np.zeros(n)
    lam[bus] = refined_solve(Amm, dLdth[bus])
    # injections through the re-dispatch
    dLdP = lam.copy()
    dLdP[0] = 0.0
    dLdP[island] = 0.0
    gen = ~island & (P > 0)
    gen[0] = False
    if island.any() and gen.any():
        dPi = P[island].sum()
        S = P[gen].sum()
        T = float(np.sum(P[gen] * lam[gen]))
        dLdP[gen] = lam[gen] * (1.0 + dPi / S) - dPi * T / S ** 2
        dLdP[island] = T / S
    # reactances: direct dependence of f_k on x_k, and the angles through A_c
    ut = theta[g.br_from] - theta[g.br_to]
    ul = lam[g.br_from] - lam[g.br_to]
    dLdx = dLdf * (-f / g.x) + ut * ul / g.x ** 2
    if c >= 0:
        dLdx[c] = dLdf[c] * (-f[c] / g.x[c])  # the outaged branch is out of A_c
    return L, dLdP, dLdx
