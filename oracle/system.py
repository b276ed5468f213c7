"""Susceptance systems, islanding, re-dispatch and the direct scenario solve.

TEST INFRASTRUCTURE (see the package docstring): plain FP64 NumPy/SciPy, no
blocking, no fusion.  Bus 0 is the slack; the reduced system drops its row and
column, so reduced row ``k`` is bus ``k + 1``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla
from scipy.sparse.csgraph import connected_components

# Per-scenario outcome codes (shared meaning with the device library's
# documented status values; each side defines its own constants).
STATUS_CONVERGED = 0
STATUS_MAX_ITER = 1
STATUS_BREAKDOWN = 2
STATUS_NONFINITE = 3
STATUS_CONVERGED_ISLANDED = 4
STATUS_ISLANDED_NO_GEN = 5


def susceptance_full(grid, shunt=None) -> sp.csr_matrix:
    """Full n x n susceptance matrix of the lossless, tap-free network.

    B = sum_e (1/x_e) u_e u_e^T, u_e = e_from - e_to, i.e. the weighted
    Laplacian that is the fast-decoupled B' of eq. (4); with ``shunt`` the bus
    shunt susceptances are added to the diagonal, which gives the B'' of
    eq. (5) (reactor sign, so that B'' stays positive definite).
    Parallel branches simply add up.

    Every entry is the exact sum of its terms (the rounded 1/x_e of each
    branch, and the shunt) rounded once to FP64 (``math.fsum``), so the
    matrix does not depend on the order in which branches are visited.
    """
    n = grid.n
    b = 1.0 / np.asarray(grid.x, dtype=np.float64)
    terms = {}
    for e in range(grid.m):
        i, j, v = int(grid.br_from[e]), int(grid.br_to[e]), float(b[e])
        terms.setdefault((i, i), []).append(v)
        terms.setdefault((j, j), []).append(v)
        terms.setdefault((i, j), []).append(-v)
        terms.setdefault((j, i), []).append(-v)
    if shunt is not None:
        for k, v in enumerate(np.asarray(shunt, dtype=np.float64)):
            terms.setdefault((k, k), []).append(float(v))
    keys = sorted(terms)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int64)
    vals = np.array([math.fsum(terms[k]) for k in keys], dtype=np.float64)
    B = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    B.sort_indices()
    return B


def reduced(B: sp.csr_matrix) -> sp.csr_matrix:
    """Drop the slack (bus 0) row and column."""
    R = B[1:, 1:].tocsr()
    R.sort_indices()
    return R


def _u_reduced(grid, c: int) -> np.ndarray:
    """Incidence vector of branch c with the slack entry dropped (length n-1)."""
    u = np.zeros(grid.n)
    u[grid.br_from[c]] += 1.0
    u[grid.br_to[c]] -= 1.0
    return u[1:]


def outage_matrix(grid, A: sp.csr_matrix, c: int) -> sp.csr_matrix:
    """Reduced matrix with branch c taken out: A_c = A - b_c u u^T.

    Only the two diagonal entries and the two off-diagonal entries of the
    branch's endpoints change (Section IV.B, Fig. 7); one entry when an
    endpoint is the slack.  Built here as an explicit sparse matrix.
    """
    if c < 0:
        return A.copy()
    u = _u_reduced(grid, c)
    nz = np.flatnonzero(u)
    bc = 1.0 / grid.x[c]
    D = sp.coo_matrix((bc * np.outer(u[nz], u[nz]).ravel(), (np.repeat(nz, len(nz)), np.tile(nz, len(nz)))),
                      shape=A.shape).tocsr()
    Ac = (A - D).tocsr()
    Ac.sort_indices()
    return Ac


def island_of(grid, c: int) -> np.ndarray:
    """Buses cut off from the slack when branch c is out (bool[n]).

    Brute force: connected components of the graph without c; the island is
    every bus outside the slack's component (Section IV.C).  ``c = -1`` is the
    intact network.
    """
    n = grid.n
    keep = np.ones(grid.m, bool)
    if c >= 0:
        keep[c] = False
    f = grid.br_from[keep].astype(np.int64)
    t = grid.br_to[keep].astype(np.int64)
    G = sp.coo_matrix((np.ones(len(f)), (f, t)), shape=(n, n))
    _, lab = connected_components(G, directed=False)
    return lab != lab[0]


def is_bridge(grid, c: int) -> bool:
    """True when removing branch c disconnects the network (brute force)."""
    if c < 0:
        return False
    n = grid.n
    keep = np.arange(grid.m) != c
    f = grid.br_from[keep].astype(np.int64)
    t = grid.br_to[keep].astype(np.int64)
    G = sp.coo_matrix((np.ones(len(f)), (f, t)), shape=(n, n))
    return connected_components(G, directed=False)[0] > 1


def redispatch(P: np.ndarray, island: np.ndarray):
    """Proportional re-dispatch of islanded power (Section IV.C).

    The power the islanded buses exported (or imported), dP = sum_{k in I} P_k,
    is taken over by the generators left in the main system: every non-slack
    main bus with positive injection is scaled by the same factor
    (1 + dP / S), S their total injection.  Islanded buses get 0.  Other main
    buses keep their injection, so the slack's output is unchanged.  With no
    such generator the injections stay as they are and the slack absorbs.

    Returns (P', no_generator).
    """
    P = np.asarray(P, dtype=np.float64)
    Pp = P.copy()
    if not island.any():
        return Pp, False
    dP = P[island].sum()
    gen = ~island & (P > 0)
    gen[0] = False
    Pp[island] = 0.0
    if not gen.any():
        return Pp, True
    S = P[gen].sum()
    Pp[gen] = P[gen] * (1.0 + dP / S)
    return Pp, False


def _residual_ld(A: sp.csr_matrix, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b - A x with every product and sum in extended precision."""
    Ald = A.astype(np.longdouble)
    return np.asarray(b, dtype=np.longdouble) - Ald @ np.asarray(x, dtype=np.longdouble)


def refined_solve(A: sp.csr_matrix, b: np.ndarray, steps: int = 4, extended: bool = False) -> np.ndarray:
    """Sparse LU solve followed by iterative refinement.

    The residual of each refinement step is formed in extended precision
    (x86 80-bit ``longdouble``), the correction solved with the same FP64 LU
    factors; the result is the FP64 solution to within a few ulps (with
    ``extended``, the refined solution itself is returned in ``longdouble``,
    several digits beyond FP64).
    """
    if A.shape[0] == 0:
        return np.zeros(0, dtype=np.longdouble if extended else np.float64)
    lu = sla.splu(A.tocsc(), permc_spec="COLAMD")
    xl = np.asarray(lu.solve(np.asarray(b, dtype=np.float64)), dtype=np.longdouble)
    for _ in range(steps):
        r = np.asarray(b, dtype=np.longdouble) - A.astype(np.longdouble) @ xl
        d = lu.solve(np.asarray(r, dtype=np.float64))
        xl = xl + np.asarray(d, dtype=np.longdouble)
    return xl if extended else np.asarray(xl, dtype=np.float64)


def base_case(grid, rhs=None, shunt=None):
    """Base-case solution of the reduced system (Section IV.B: the base case
    is solved once and kept).  Returns (theta_b[n] with slack 0, A)."""
    A = reduced(susceptance_full(grid, shunt))
    b = np.asarray(grid.P if rhs is None else rhs, dtype=np.float64)[1:]
    th = np.zeros(grid.n)
    th[1:] = refined_solve(A, b)
    return th, A


def flows(grid, theta: np.ndarray, c: int = -1, island=None) -> np.ndarray:
    """Branch flows f_e = (theta_from - theta_to) / x_e.

    The outaged branch carries nothing, and neither do branches inside the
    island (their angles are pinned to zero there).
    """
    f = (theta[grid.br_from] - theta[grid.br_to]) / grid.x
    if c >= 0:
        f[c] = 0.0
    if island is not None and island.any():
        inside = island[grid.br_from] & island[grid.br_to]
        f[inside] = 0.0
    return f


def scenario(grid, c: int, A: sp.csr_matrix | None = None, rhs=None, redispatch_islands: bool = True,
             shunt=None):
    """Direct solve of outage scenario c (Section IV; LU rebuilt per scenario).

    The outage matrix A_c restricted to the main system M (the slack's
    component, without the slack) is solved against the re-dispatched
    injections.  Islanded angles are pinned to 0 (the islanded block is
    singular, so this choice makes the result unique).

    Returns a dict with theta[n], flows[m], island[n] (bool), Pp[n] (the
    re-dispatched injections), status, and Ac.
    """
    if A is None:
        A = reduced(susceptance_full(grid, shunt))
    P = np.asarray(grid.P if rhs is None else rhs, dtype=np.float64)
    island = island_of(grid, c)
    if redispatch_islands:
        Pp, nogen = redispatch(P, island)
    else:
        Pp, nogen = P.copy(), False
        Pp[island] = 0.0
    if not island.any():
        status = STATUS_CONVERGED
    else:
        status = STATUS_ISLANDED_NO_GEN if nogen else STATUS_CONVERGED_ISLANDED
    Ac = outage_matrix(grid, A, c)
    main = ~island[1:]
    idx = np.flatnonzero(main)
    th = np.zeros(grid.n)
    if len(idx):
        Amm = Ac[idx][:, idx].tocsr()
        th[1:][idx] = refined_solve(Amm, Pp[1:][idx])
    out = dict(theta=th, island=island, Pp=Pp, status=status, Ac=Ac)
    out["flows"] = flows(grid, th, c, island)
    return out


def true_residual(grid, A: sp.csr_matrix, c: int, theta: np.ndarray, Pp: np.ndarray, island: np.ndarray) -> float:
    """Relative residual ||P'_M - A_c[M,M] theta_M|| / ||P'_M|| over the
    main-system rows, in extended precision.

    A_c = A - b_c u u^T is applied with the outage's change taken exactly
    (Section IV.B: four entries change by +-b_c, b_c = 1/x_c as it enters A):
    A_c[M,M] theta_M = (A theta~)_M - b_c (u'theta~) u_M with theta~ the
    angles zeroed outside M, all in ``longdouble``.
    """
    main = ~np.asarray(island, bool)[1:]
    idx = np.flatnonzero(main)
    if len(idx) == 0:
        return 0.0
    th = np.where(main, np.asarray(theta, np.float64)[1:], 0.0).astype(np.longdouble)
    r = np.asarray(Pp, np.float64)[1:].astype(np.longdouble) - A.astype(np.longdouble) @ th
    if c >= 0:
        u = _u_reduced(grid, c).astype(np.longdouble)
        bc = np.longdouble(1.0 / grid.x[c])
        r = r + bc * (u @ th) * u
    b = np.asarray(Pp, np.longdouble)[1:][idx]
    nb = float(np.sqrt(np.sum(b ** 2)))
    nr = float(np.sqrt(np.sum(r[idx] ** 2)))
    return nr / nb if nb > 0 else nr
