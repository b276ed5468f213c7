"""Textbook preconditioned conjugate gradient, run per outage scenario.

TEST INFRASTRUCTURE (see the package docstring).

The iteration is the PCG of Section III.A: step length alpha = r'z / p'Ap,
update of the approximate solution and the residual, stop test on the
residual, preconditioned residual z = M^-1 r, improvement
beta = z_new'r_new / z_old'r_old, new search direction p = z + beta p.
Two readings are taken where the printed listing is garbled: the
preconditioner is applied to the *current* residual r_k (the listing's
duplicated step number indexes r_{k-1}), and "sufficiently small" means
||r_k||_2 <= tol * ||b||_2 with b the scenario right-hand side.

Section III.B (last paragraph) starts each outage from the base-case state.
That start is taken in correction form: the unknown is the change
delta = theta - theta_base, which starts at 0 with residual
r0 = b - A_c theta_base, formed in extended precision.  Every iterate equals
the one started at x0 = theta_base; only the rounding is better.

M = L U are the ILU(0) factors of the unmodified base-case matrix
(Section IV.B, eqs. 6-7).  Islanded rows are held at zero, so the operator and
the preconditioner both act on the main system only: M^-1 is applied as
P_M U^-1 L^-1 P_M.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

from .system import (
    STATUS_BREAKDOWN,
    STATUS_CONVERGED,
    STATUS_CONVERGED_ISLANDED,
    STATUS_ISLANDED_NO_GEN,
    STATUS_MAX_ITER,
    STATUS_NONFINITE,
    island_of,
    outage_matrix,
    redispatch,
)


def _apply_prec(Lf, U, r, mask):
    """z = P_M U^-1 L^-1 P_M r; ``Lf`` is the unit lower factor with its
    diagonal stored."""
    if r.shape[0] == 0:
        return r.copy()
    rm = np.where(mask, r, 0.0)
    y = spsolve_triangular(Lf, rm, lower=True, unit_diagonal=True)
    z = spsolve_triangular(U, y, lower=False)
    return np.where(mask, z, 0.0)


def pcg_textbook(A, b, L, U, x0=None, r0=None, mask=None, tol=1e-12, max_iter=10000, bnorm=None, dot=None):
    """PCG on A x = b with preconditioner M = (L+I) U.

    Either ``x0`` (then r0 = b - A x0) or ``r0`` directly may be given.  Rows
    where ``mask`` is False are held at zero.  Returns (x, iters, status,
    history of ||r_k||).  ``iters`` counts the step-length updates taken
    (0 when the starting residual already passes).  ``dot(u, v)`` forms the
    inner products and norms (default: NumPy's ``u @ v``); any correctly
    computed inner product is a valid choice, and the choice only moves
    rounding.
    """
    if dot is None:
        dot = lambda u, v: float(u @ v)  # noqa: E731
    n = A.shape[0]
    Lf = (L + sp.eye(n, format="csr")).tocsr()
    U = U.tocsr()
    mask = np.ones(n, bool) if mask is None else np.asarray(mask, bool)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if r0 is None:
        r = np.asarray(b, dtype=np.float64) - A @ x
    else:
        r = np.array(r0, dtype=np.float64)
    r = np.where(mask, r, 0.0)
    bnorm = float(np.linalg.norm(np.where(mask, b, 0.0))) if bnorm is None else bnorm
    hist = [float(np.sqrt(dot(r, r)))]
    if hist[0] <= tol * bnorm:
        return x, 0, STATUS_CONVERGED, hist
    z = _apply_prec(Lf, U, r, mask)
    p = z.copy()
    rho = dot(r, z)
    for k in range(1, max_iter + 1):
        q = A @ p
        q = np.where(mask, q, 0.0)
        sigma = dot(p, q)
        if not np.isfinite(sigma) or not np.isfinite(rho):
            return x, k - 1, STATUS_NONFINITE, hist
        if sigma <= 0.0:
            return x, k - 1, STATUS_BREAKDOWN, hist
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        hist.append(float(np.sqrt(dot(r, r))))
        if not np.isfinite(hist[-1]):
            return x, k, STATUS_NONFINITE, hist
        if hist[-1] <= tol * bnorm:
            return x, k, STATUS_CONVERGED, hist
        z = _apply_prec(Lf, U, r, mask)
        rho_new = dot(r, z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, max_iter, STATUS_MAX_ITER, hist


def pcg_correction(Ac, b_red, theta_b_red, L, U, mask, tol=1e-12, max_iter=10000, dot=None):
    """Correction-form PCG of one scenario on the reduced system.

    Solves A_c delta = r0 with r0 = b - A_c theta_b (extended precision) on
    the main rows, delta0 = 0, and returns (theta = theta_b + delta on main
    rows and 0 elsewhere, iters, status, history).  The stop test is relative
    to ||b|| over the main rows.
    """
    mask = np.asarray(mask, bool)
    thb = np.where(mask, theta_b_red, 0.0)
    r0 = (np.asarray(b_red, np.longdouble)
          - Ac.astype(np.longdouble) @ np.asarray(thb, np.longdouble))
    r0 = np.where(mask, np.asarray(r0, np.float64), 0.0)
    bnorm = float(np.linalg.norm(np.where(mask, b_red, 0.0)))
    d, its, st, hist = pcg_textbook(Ac, b_red, L, U, r0=r0, mask=mask, tol=tol, max_iter=max_iter, bnorm=bnorm,
                                    dot=dot)
    th = np.where(mask, thb + d, 0.0)
    return th, its, st, hist


def scenario_pcg(grid, c, A, L, U, theta_b, tol=1e-12, max_iter=10000, rhs=None, redispatch_islands=True,
                 dot=None):
    """One outage scenario solved by the paper's method: island detection,
    re-dispatch, then PCG from the base state with the base ILU factors.

    Returns a dict with theta[n] (slack and islanded buses 0), island[n],
    Pp[n], iters, status and the residual history.
    """
    P = np.asarray(grid.P if rhs is None else rhs, dtype=np.float64)
    island = island_of(grid, c)
    if redispatch_islands:
        Pp, nogen = redispatch(P, island)
    else:
        Pp, nogen = P.copy(), False
        Pp[island] = 0.0
    Ac = outage_matrix(grid, A, c)
    mask = ~island[1:]
    th_red, its, st, hist = pcg_correction(Ac, Pp[1:], theta_b[1:], L, U, mask, tol, max_iter, dot=dot)
    if st == STATUS_CONVERGED and island.any():
        st = STATUS_ISLANDED_NO_GEN if nogen else STATUS_CONVERGED_ISLANDED
    th = np.zeros(grid.n)
    th[1:] = th_red
    return dict(theta=th, island=island, Pp=Pp, iters=its, status=st, hist=hist, Ac=Ac)
