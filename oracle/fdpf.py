"""Fast-decoupled AC power flow of every outage, a fixed number of outer
iterations (Section II, eqs. (1)-(5)).

TEST INFRASTRUCTURE (see the package docstring).  The network is lossless
and tap-free: a branch has series reactance x only, a bus may have a shunt
susceptance b_sh (reactor sign, as in the B'' of ``system``).  With V the
bus voltage magnitudes and theta the angles, the injections the network
takes are

    P_i = sum_{j~i} V_i V_j sin(theta_i - theta_j) / x_ij,
    Q_i = V_i^2 (sum_{j~i} 1 / x_ij + b_sh,i) - sum_{j~i} V_i V_j cos(theta_i - theta_j) / x_ij.

The slack (bus 0) holds theta = 0 and V = 1; every other bus is a load bus
with specified P and Q.  One outer iteration is a P-theta half-iteration,
B' dtheta = dP / V, theta += dtheta, then a Q-V half-iteration with the
updated angles, B'' dV = dQ / V, V += dV (eqs. (4)-(5)), each solved
directly here.  An outage removes its branch from the network and from both
matrices; buses cut off from the slack are left out of every equation and
reported as theta = 0, V = 1; the islanded active power is re-dispatched as
in the DC screening (Section IV.C).  The base state is this iteration from
a flat start on the intact network; each outage starts from the base state.
"""
from __future__ import annotations

import numpy as np

from .system import island_of, outage_matrix, redispatch, reduced, refined_solve, susceptance_full


def injections(grid, theta, V, shunt, c: int = -1):
    """(P, Q) the network takes at (theta, V), with branch c out."""
    n = grid.n
    live = np.ones(len(grid.x), bool)
    if c >= 0:
        live[c] = False
    f, t = grid.br_from[live], grid.br_to[live]
    b = 1.0 / grid.x[live]
    d = theta[f] - theta[t]
    P = np.zeros(n)
    Q = np.zeros(n)
    vv = V[f] * V[t] * b
    np.add.at(P, f, vv * np.sin(d))
    np.add.at(P, t, -vv * np.sin(d))
    np.add.at(Q, f, -vv * np.cos(d))
    np.add.at(Q, t, -vv * np.cos(d))
    diag = np.zeros(n)
    np.add.at(diag, f, b)
    np.add.at(diag, t, b)
    Q += V * V * (diag + np.asarray(shunt, dtype=np.float64))
    return P, Q


def fdpf(grid, P, Q, shunt, theta0, V0, c: int = -1, iters: int = 3, redispatch_islands: bool = True,
         solve=None):
    """``iters`` outer fast-decoupled iterations of outage c from (theta0, V0).

    ``solve(A, b)`` solves each half's linear system (default: sparse LU
    with extended-precision refinement; any correct FP64 solve is valid).
    Returns (theta, V, island)."""
    solve = refined_solve if solve is None else solve
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    island = island_of(grid, c) if c >= 0 else np.zeros(grid.n, bool)
    Pp = redispatch(P, island)[0] if redispatch_islands else np.where(island, 0.0, P)
    Bp = outage_matrix(grid, reduced(susceptance_full(grid)), c)
    Bpp = outage_matrix(grid, reduced(susceptance_full(grid, shunt)), c)
    idx = np.flatnonzero(~island[1:])
    bus = idx + 1
    Bp = Bp[idx][:, idx].tocsr()
    Bpp = Bpp[idx][:, idx].tocsr()
    theta = np.array(theta0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    theta[0], V[0] = 0.0, 1.0
    for _ in range(iters):
        Pc, _ = injections(grid, theta, V, shunt, c)
        theta[bus] += solve(Bp, (Pp[bus] - Pc[bus]) / V[bus])
        _, Qc = injections(grid, theta, V, shunt, c)
        V[bus] += solve(Bpp, (Q[bus] - Qc[bus]) / V[bus])
    theta[island] = 0.0
    V[island] = 1.0
    return theta, V, island


def base_state(grid, P, Q, shunt, iters: int = 3, solve=None):
    """The intact network's state after ``iters`` iterations from flat start."""
    th, V, _ = fdpf(grid, P, Q, shunt, np.zeros(grid.n), np.ones(grid.n), -1, iters, solve=solve)
    return th, V
