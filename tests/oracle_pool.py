"""Every-outage comparison of device results with the oracle, on CPU workers.

The oracle's direct solve (sparse LU + extended-precision refinement per
scenario) takes 10-25 ms per outage on the 10,000-bus grid, so the device's
angles, flows, island flags, statuses and true residuals of all outages are
checked in a pool of single-threaded worker processes.  The device results
are written to a temporary directory and memory-mapped by the workers.  The
workers are started with ``spawn`` (a fresh interpreter each), so nothing of
the parent's GPU state is inherited; they import only NumPy, SciPy and the
oracle.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import shutil
import tempfile

import numpy as np

_W: dict = {}


def _init(grid, A, rhs, shunt, redispatch, paths):
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except Exception:
        pass
    _W.update(grid=grid, A=A, rhs=rhs, shunt=shunt, redispatch=redispatch)
    for k, p in paths.items():
        _W[k] = np.load(p, mmap_mode="r")


def _chunk(rows):
    import oracle

    g, A = _W["grid"], _W["A"]
    out = []
    for s, c in rows:
        d = oracle.scenario(g, int(c), A, rhs=_W["rhs"], redispatch_islands=_W["redispatch"], shunt=_W["shunt"])
        x = np.asarray(_W["x"][s])
        ang = float(np.abs(x - d["theta"]).max())
        flow = float((np.abs(np.asarray(_W["flows"][s]) - d["flows"]) * g.x).max()) if "flows" in _W else 0.0
        isl = bool(np.array_equal(np.asarray(_W["island"][s]).astype(bool), d["island"])) if "island" in _W else True
        st = int(d["status"])
        res = oracle.true_residual(g, A, int(c), x, d["Pp"], d["island"])
        out.append((s, ang, flow, isl, st, res))
    return out


def compare_all(grid, A, outages, res, rhs=None, shunt=None, redispatch=True, workers=None):
    """Check every scenario of a device solve against the oracle.

    ``res`` holds NumPy arrays x [n_out, n_bus] and optionally flows, island.
    Returns a dict of per-scenario arrays: angle (max |dtheta|), flow
    (max |df| x_e), island_ok, status (the oracle's), resid (the oracle's
    true residual of the device angles)."""
    outages = np.asarray(outages)
    n = len(outages)
    tmp = tempfile.mkdtemp(prefix="gpcg_oracle_")
    try:
        paths = {}
        for k in ("x", "flows", "island"):
            if res.get(k) is not None:
                paths[k] = os.path.join(tmp, k + ".npy")
                np.save(paths[k], np.ascontiguousarray(res[k]))
        nw = workers or min(16, len(os.sched_getaffinity(0)))
        rows = [(s, int(outages[s])) for s in range(n)]
        step = max(1, min(64, n // (4 * nw) + 1))
        chunks = [rows[i:i + step] for i in range(0, n, step)]
        ctx = mp.get_context("spawn")
        with ctx.Pool(nw, initializer=_init, initargs=(grid, A, rhs, shunt, redispatch, paths)) as pool:
            parts = pool.map(_chunk, chunks)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    out = dict(angle=np.zeros(n), flow=np.zeros(n), island_ok=np.zeros(n, bool), status=np.zeros(n, np.int64),
               resid=np.zeros(n))
    for part in parts:
        for s, ang, flow, isl, st, r in part:
            out["angle"][s], out["flow"][s], out["island_ok"][s] = ang, flow, isl
            out["status"][s], out["resid"][s] = st, r
    return out


def _init_fdpf(grid, P, Q, bsh, th0, V0, paths):
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except Exception:
        pass
    _W.update(grid=grid, P=P, Q=Q, bsh=bsh, th0=th0, V0=V0)
    for k, p in paths.items():
        _W[k] = np.load(p, mmap_mode="r")


def _chunk_fdpf(rows):
    from oracle import fdpf

    out = []
    for s, c in rows:
        th, V, _ = fdpf.fdpf(_W["grid"], _W["P"], _W["Q"], _W["bsh"], _W["th0"], _W["V0"], int(c))
        out.append((s, float(np.abs(np.asarray(_W["theta"][s]) - th).max()),
                    float(np.abs(np.asarray(_W["V"][s]) - V).max())))
    return out


def compare_fdpf(grid, P, Q, bsh, th0, V0, outages, theta, V, workers=None):
    """Three fast-decoupled iterations of each outage by the oracle against
    the device's (theta, V) rows; returns per-scenario max |dtheta|, |dV|."""
    outages = np.asarray(outages)
    n = len(outages)
    tmp = tempfile.mkdtemp(prefix="gpcg_fdpf_")
    try:
        paths = {"theta": os.path.join(tmp, "theta.npy"), "V": os.path.join(tmp, "V.npy")}
        np.save(paths["theta"], np.ascontiguousarray(theta))
        np.save(paths["V"], np.ascontiguousarray(V))
        nw = workers or min(16, len(os.sched_getaffinity(0)))
        rows = [(s, int(outages[s])) for s in range(n)]
        step = max(1, min(16, n // (4 * nw) + 1))
        chunks = [rows[i:i + step] for i in range(0, n, step)]
        ctx = mp.get_context("spawn")
        with ctx.Pool(nw, initializer=_init_fdpf, initargs=(grid, P, Q, bsh, th0, V0, paths)) as pool:
            parts = pool.map(_chunk_fdpf, chunks)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    dth, dV = np.zeros(n), np.zeros(n)
    for part in parts:
        for s, a, b in part:
            dth[s], dV[s] = a, b
    return dth, dV
