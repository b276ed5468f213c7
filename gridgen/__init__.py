"""Seeded synthetic transmission grids: the inputs shared by the oracle and the GPU path.

This module only draws grids.  It holds none of the contingency method's
arithmetic (no susceptance assembly, no factorisation, no solve, no bridge
pass of the method): it returns a branch table, reactances and injections,
which both the oracle and the device library then turn into their own systems.

The paper evaluates on a non-public provincial grid (1,425 buses, 1,691
branches, about 41 % islanding outages; Section V, Table I).  These grids stand
in for it with the same sparsity (mean degree 2.4-2.8), the same share of
bridge branches and the same kind of injections.

Recipe (every draw comes from one ``numpy.random.default_rng(seed)`` in this
order):

1. bus coordinates: ``rng.random((n, 2))`` on the unit square;
2. branches: the Euclidean minimum spanning tree of the Delaunay edges, plus the
   shortest non-tree pairs from the 8-nearest-neighbour lists, sorted by
   (length, i, j), until ``m`` branches exist (no parallel branches);
3. slack: the highest-degree bus of the largest 2-edge-connected component
   (ties go to the bus nearest the centre), relabelled to index 0; the other
   buses are numbered 1..n-1 in reverse Cuthill-McKee order of the graph
   with the slack removed, the frame in which steps 4-7 draw;
4. branches sorted by (min endpoint, max endpoint) in that frame; ``from``
   is the smaller;
5. reactances ``x ~ U(x_lo, 0.3)``; optionally a seeded 5 % of branches become
   transformers with ``x ~ U(0.05, 0.2)``;
6. active injections ``P ~ N(0, 0.5)`` (standard deviation), slack entry set so
   that the injections sum to zero;
7. optionally reactive injections ``Q ~ N(0, 0.2)`` and shunts
   ``b_sh ~ U(0, 0.05)``;
8. the buses are then relabelled in generation order (slack 0, the others
   in the order of their points; ``order="generated"``, the default), a
   numbering unrelated to the graph, with the branch ids and orientations
   kept; ``order="rcm"`` keeps the frame of step 3.  Both describe the same
   physical grid.  A banded row order is a solver's concern: ``rcm_perm``
   gives SciPy's reverse Cuthill-McKee row order of a grid for a consumer
   that wants one, and ``renumber`` relabels a grid by it.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree
from scipy.spatial import Delaunay, cKDTree

__all__ = ["Grid", "GridSpec", "SPECS", "make_grid", "hand_grid", "HAND_GRIDS", "rcm_perm", "renumber"]


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """Parameters of one synthetic grid."""

    name: str
    n: int
    m: int
    seed: int
    x_lo: float = 0.005
    x_hi: float = 0.3
    transformer_share: float = 0.0
    reactive: bool = False
    order: str = "generated"


# The five workloads: a 200-bus grid, a 2,000-bus grid, a 10,000-bus grid
# (with transformers, reactive injections and shunts), and the eight grids of
# the uneven batch.
SPECS = {
    "grid200": GridSpec("grid200", 200, 280, 1, x_lo=0.01),
    "grid2k": GridSpec("grid2k", 2000, 2800, 2),
    "grid10k": GridSpec("grid10k", 10000, 13500, 3, transformer_share=0.05, reactive=True),
}
for _k, (_n, _seed) in enumerate(zip((500, 1000, 2000, 3000, 5000, 8000, 12000, 20000), range(41, 49))):
    SPECS[f"uneven{_n}"] = GridSpec(f"uneven{_n}", _n, int(round(1.4 * _n)), _seed)


@dataclasses.dataclass
class Grid:
    """A bus-branch grid.  Bus 0 is the slack.  Arrays are plain NumPy."""

    name: str
    n: int
    br_from: np.ndarray  # int32[m], smaller endpoint
    br_to: np.ndarray  # int32[m]
    x: np.ndarray  # float64[m], branch reactance (p.u.)
    P: np.ndarray  # float64[n], active injections; sums to zero
    Q: Optional[np.ndarray] = None  # float64[n], reactive injections
    bsh: Optional[np.ndarray] = None  # float64[n], bus shunt susceptance
    pts: Optional[np.ndarray] = None  # float64[n, 2], coordinates
    seed: Optional[int] = None

    @property
    def m(self) -> int:
        return int(self.br_from.shape[0])

    def digest(self) -> str:
        """SHA-256 over the arrays that define the grid."""
        h = hashlib.sha256()
        for a in (self.br_from, self.br_to, self.x, self.P, self.Q, self.bsh):
            if a is not None:
                h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _two_edge_components(n: int, edges: np.ndarray) -> np.ndarray:
    """Label each bus with its 2-edge-connected component.

    The bridges (branches whose removal disconnects their endpoints) are
    found by one depth-first search with low-link values (Tarjan 1974; a
    branch is identified by its index, so a doubled branch is never a
    bridge); the components are the connected pieces left when they are
    removed.
    """
    m = edges.shape[0]
    adj = [[] for _ in range(n)]
    for k, (a, b) in enumerate(edges.tolist()):
        adj[a].append((b, k))
        adj[b].append((a, k))
    pre = [-1] * n
    low = [0] * n
    bridge = np.zeros(m, bool)
    counter = 0
    for root in range(n):
        if pre[root] >= 0:
            continue
        pre[root] = low[root] = counter
        counter += 1
        stack = [(root, -1, 0)]  # (bus, branch into it, next neighbour position)
        while stack:
            v, via, k = stack[-1]
            if k < len(adj[v]):
                stack[-1] = (v, via, k + 1)
                w, e = adj[v][k]
                if e == via:
                    continue
                if pre[w] < 0:
                    pre[w] = low[w] = counter
                    counter += 1
                    stack.append((w, e, 0))
                else:
                    low[v] = min(low[v], pre[w])
            else:
                stack.pop()
                if stack:
                    u = stack[-1][0]
                    low[u] = min(low[u], low[v])
                    if low[v] > pre[u]:
                        bridge[via] = True
    kept = edges[~bridge]
    H = sp.coo_matrix((np.ones(len(kept)), (kept[:, 0], kept[:, 1])), shape=(n, n))
    _, lab = connected_components(H, directed=False)
    return lab


def make_grid(spec: GridSpec | str, order: Optional[str] = None) -> Grid:
    """Draw the grid described by ``spec`` (a GridSpec or a key of SPECS),
    optionally with another bus numbering ("generated" or "rcm")."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    if order is not None:
        spec = dataclasses.replace(spec, order=order)
    n, m = spec.n, spec.m
    if m < n - 1:
        raise ValueError("a connected grid needs m >= n - 1")
    rng = np.random.default_rng(spec.seed)
    pts = rng.random((n, 2))

    # Delaunay edges, then their Euclidean minimum spanning tree
    tri = Delaunay(pts)
    s = tri.simplices
    de = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    de = np.unique(np.sort(de, axis=1), axis=0)
    w = np.linalg.norm(pts[de[:, 0]] - pts[de[:, 1]], axis=1)
    T = minimum_spanning_tree(sp.coo_matrix((w, (de[:, 0], de[:, 1])), shape=(n, n)).tocsr()).tocoo()
    tree = {(min(a, b), max(a, b)) for a, b in zip(T.row.tolist(), T.col.tolist())}
    if len(tree) != n - 1:
        raise RuntimeError("spanning tree is not connected")

    # extra branches: shortest non-tree nearest-neighbour pairs
    kd = cKDTree(pts)
    d, nb = kd.query(pts, k=9)
    cand = {}
    for i in range(n):
        for kk in range(1, 9):
            j = int(nb[i, kk])
            key = (min(i, j), max(i, j))
            if key not in tree:
                cand[key] = float(d[i, kk])
    extra = sorted(cand.items(), key=lambda t: (t[1], t[0][0], t[0][1]))
    need = m - (n - 1)
    if len(extra) < need:
        raise RuntimeError("not enough candidate branches")
    edges = np.array(sorted(tree) + [k for k, _ in extra[:need]], dtype=np.int64)

    # slack: highest-degree bus of the largest 2-edge-connected component
    lab = _two_edge_components(n, edges)
    big = np.argmax(np.bincount(lab))
    deg = np.bincount(edges.ravel(), minlength=n)
    cands = np.flatnonzero(lab == big)
    dc = np.linalg.norm(pts[cands] - 0.5, axis=1)
    order = np.lexsort((dc, -deg[cands]))
    slack = int(cands[order[0]])

    # relabel: slack -> 0, the others in RCM order; the draws below are made
    # in this frame, so both numberings describe the same physical grid
    new = np.empty(n, np.int64)
    rest = np.array([i for i in range(n) if i != slack], dtype=np.int64)
    rest_rcm = rest[_rcm_order(n, edges, slack, rest)]
    new[slack] = 0
    new[rest_rcm] = np.arange(1, n)
    e = new[edges]
    e = np.sort(e, axis=1)
    e = e[np.lexsort((e[:, 1], e[:, 0]))]
    pts_new = np.empty_like(pts)
    pts_new[new] = pts

    x = rng.uniform(spec.x_lo, spec.x_hi, m)
    if spec.transformer_share > 0:
        k = int(round(spec.transformer_share * m))
        tr = rng.choice(m, k, replace=False)
        x[tr] = rng.uniform(0.05, 0.2, k)
    P = rng.normal(0.0, 0.5, n)
    P[0] = -P[1:].sum()
    Q = bsh = None
    if spec.reactive:
        Q = rng.normal(0.0, 0.2, n)
        bsh = rng.uniform(0.0, 0.05, n)
    if spec.order == "generated":
        # the same grid, buses relabelled in generation order (slack 0);
        # branches keep their ids and orientation
        gen = np.empty(n, np.int64)
        gen[slack] = 0
        gen[rest] = np.arange(1, n)
        r2g = np.empty(n, np.int64)
        r2g[new] = gen
        e = r2g[e]

        def bus(a):
            if a is None:
                return None
            out = np.empty_like(a)
            out[r2g] = a
            return out

        P, Q, bsh, pts_new = bus(P), bus(Q), bus(bsh), bus(pts_new)
    elif spec.order != "rcm":
        raise ValueError(f"unknown order {spec.order!r}")
    return Grid(spec.name, n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), x, P, Q, bsh, pts_new, spec.seed)


def _hand(name, n, pairs, x, P, bsh=None):
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    return Grid(name, n, pairs[:, 0].copy(), pairs[:, 1].copy(), np.asarray(x, float), np.asarray(P, float),
                bsh=None if bsh is None else np.asarray(bsh, float))


def hand_grid(name: str) -> Grid:
    """Small grids whose solutions can be written down by hand.

    * ``two_bus``: one branch; the non-slack angle is ``P1 * x``.
    * ``ring3``: a triangle with equal reactances ``a``.
    * ``path5``: a path; every branch is a bridge.
    * ``two_rings``: two triangles joined by one bridge (buses 2-3).
    * ``slack_leaf``: the slack hangs on a single branch off a ring.
    * ``parallel``: a ring with one doubled branch (two branches 0-1).
    """
    if name == "two_bus":
        return _hand(name, 2, [(0, 1)], [0.2], [-1.5, 1.5])
    if name == "ring3":
        return _hand(name, 3, [(0, 1), (0, 2), (1, 2)], [0.1, 0.1, 0.1], [-0.7, 0.3, 0.4])
    if name == "path5":
        return _hand(name, 5, [(0, 1), (1, 2), (2, 3), (3, 4)], [0.1, 0.2, 0.05, 0.3],
                     [-0.2, 0.5, -0.4, 0.6, -0.5])
    if name == "two_rings":
        return _hand(name, 6, [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (3, 5), (4, 5)],
                     [0.1, 0.2, 0.15, 0.05, 0.1, 0.2, 0.25], [-0.9, 0.4, -0.3, 0.5, 0.2, 0.1])
    if name == "slack_leaf":
        return _hand(name, 5, [(0, 1), (1, 2), (1, 3), (2, 4), (3, 4)], [0.1, 0.2, 0.1, 0.3, 0.15],
                     [-0.5, 0.3, -0.2, 0.6, -0.2])
    if name == "parallel":
        return _hand(name, 4, [(0, 1), (0, 1), (1, 2), (2, 3), (0, 3)], [0.2, 0.3, 0.1, 0.25, 0.15],
                     [-0.6, 0.5, -0.3, 0.4])
    raise KeyError(name)


HAND_GRIDS = ("two_bus", "ring3", "path5", "two_rings", "slack_leaf", "parallel")


def _rcm_order(n: int, edges: np.ndarray, slack: int, rest: np.ndarray) -> np.ndarray:
    """Positions into ``rest`` in reverse Cuthill-McKee order of the graph
    induced on ``rest`` (the buses other than the slack)."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    pos = np.full(n, -1, np.int64)
    pos[rest] = np.arange(len(rest))
    keep = (edges[:, 0] != slack) & (edges[:, 1] != slack)
    f, t = pos[edges[keep, 0]], pos[edges[keep, 1]]
    k = len(rest)
    G = sp.coo_matrix((np.ones(len(f)), (f, t)), shape=(k, k)).tocsr()
    G = (G + G.T).tocsr()
    return np.asarray(reverse_cuthill_mckee(G, symmetric_mode=True), dtype=np.int64)


def rcm_perm(grid: Grid) -> np.ndarray:
    """Reverse Cuthill-McKee order of the non-slack buses (SciPy's), as the
    bus of each reduced row: perm[k] is the bus held in row k."""
    n = grid.n
    edges = np.stack([grid.br_from, grid.br_to], axis=1).astype(np.int64)
    rest = np.arange(1, n, dtype=np.int64)
    return rest[_rcm_order(n, edges, 0, rest)].astype(np.int32)


def renumber(grid: Grid, perm: np.ndarray) -> Grid:
    """The same grid with bus perm[k] relabelled k + 1 (the slack stays 0);
    branches keep their order and orientation, so outage ids and flows are
    unchanged."""
    n = grid.n
    new = np.zeros(n, np.int64)
    new[np.asarray(perm, np.int64)] = np.arange(1, n)
    old = np.zeros(n, np.int64)
    old[new] = np.arange(n)

    def bus(a):
        return None if a is None else np.asarray(a)[old]

    return Grid(grid.name + ":renumbered", n, new[grid.br_from].astype(np.int32), new[grid.br_to].astype(np.int32),
                grid.x.copy(), bus(grid.P), bus(grid.Q), bus(grid.bsh),
                None if grid.pts is None else grid.pts[old], grid.seed)
