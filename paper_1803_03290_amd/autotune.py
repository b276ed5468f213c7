"""Tile-shape autotuner for multi-grid batches, with a cache.

A tile shape is the scenario block S (scenarios per wavefront: rows per step
against scenarios per wave) and the look-ahead window of the triangular
schedules (rows a step may pick its ready rows from: a wider window fills
more of the R slots of a step, a narrower one keeps the LDS ring small).
The best shape depends on the grids' sizes, dependency depths and scenario
counts.  ``BlockTuner.best`` times a batch solve for each candidate (a block,
or a (block, lookahead) pair) through ``gpcg_batch_tune`` and remembers the
winner per set of grids (keyed by a digest of their branch tables, matrix
kind, scenario counts and tolerance), in memory and, when a path is given,
in a JSON file.  The kernels' prefetch depths are not searched: they are
fixed by the register budget of one wavefront per SIMD.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .binding import batch_tune


def grid_key(ctx) -> str:
    """Digest of what a context's schedules depend on."""
    h = hashlib.sha256()
    for a in (ctx.br_from, ctx.br_to, ctx.x):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(f"{ctx.n_bus}:{ctx.kind}".encode())
    return h.hexdigest()[:20]


class BlockTuner:
    def __init__(self, path: str | None = None):
        self.path = path
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def key(self, contexts, outages, tol) -> str:
        parts = [grid_key(c) + f"/{int(o.shape[0])}" for c, o in zip(contexts, outages)]
        return hashlib.sha256(("|".join(parts) + f"|{tol:g}").encode()).hexdigest()[:24]

    def best(self, contexts, outages, rhs, candidates=(4, 8, 16), tol=1e-12, max_iter=20000, reps=1):
        """The fastest of ``candidates`` for this batch (cached): a block when
        the candidates are blocks, a (block, lookahead) pair when they are
        pairs."""
        k = self.key(contexts, outages, tol) + "|" + ",".join(str(c) for c in candidates)
        if k in self.table:
            b = self.table[k]["best"]
            return int(b) if np.isscalar(candidates[0]) else tuple(int(v) for v in b)
        ms = batch_tune(contexts, outages, rhs, candidates, tol, max_iter, reps)
        best = min(ms, key=ms.get)
        self.table[k] = {"best": best if np.isscalar(best) else list(best),
                         "ms": {str(b): v for b, v in ms.items()}}
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.table, f, indent=1)
        return best
