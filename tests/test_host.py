"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host passes (assembly, ILU(0), integer topology) agree with the
oracle and with brute force.  No GPU call is made here."""
import os
import re

import numpy as np
import pytest

import gridgen
import oracle
import paper_1803_03290_amd as gp
from paper_1803_03290_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "gpcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gpcg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gp.lib()
    names = _declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
        assert n in binding.SIGNATURES, n


@pytest.mark.parametrize("key", ["grid200", "grid2k", "grid10k"])
def test_assembly_matches_oracle(grids, key):
    """Both sides round every entry once from its exact sum, so the reduced
    B' (and B'' with the 10k grid's shunts) agree bit for bit."""
    g = grids[key]
    A = gp.assemble(g.n, g.br_from, g.br_to, g.x).to_scipy()
    Ao = oracle.reduced(oracle.susceptance_full(g))
    np.testing.assert_array_equal(A.indptr, Ao.indptr)
    np.testing.assert_array_equal(A.indices, Ao.indices)
    np.testing.assert_array_equal(A.data, Ao.data)
    if g.bsh is not None:
        A = gp.assemble(g.n, g.br_from, g.br_to, g.x, g.bsh).to_scipy()
        Ao = oracle.reduced(oracle.susceptance_full(g, g.bsh))
        np.testing.assert_array_equal(A.indices, Ao.indices)
        np.testing.assert_array_equal(A.data, Ao.data)


def test_assembly_with_shunts(grids):
    g = grids["grid200"]
    bsh = np.linspace(0.0, 0.05, g.n)
    A = gp.assemble(g.n, g.br_from, g.br_to, g.x, bsh).to_scipy()
    Ao = oracle.reduced(oracle.susceptance_full(g, bsh))
    np.testing.assert_array_equal(A.toarray(), Ao.toarray())


def test_assembly_parallel_branches():
    g = gridgen.hand_grid("parallel")
    A = gp.assemble(g.n, g.br_from, g.br_to, g.x).to_scipy()
    Ao = oracle.reduced(oracle.susceptance_full(g))
    np.testing.assert_array_equal(A.toarray(), Ao.toarray())


def test_assembly_entries_are_correctly_rounded_sums():
    """A star where the order of the additions decides the last bit: bus 1
    meets branches of susceptance 1, 2^-53 and 2^-53 (and a parallel pair
    to bus 2).  Left to right in FP64 the diagonal is 1 (each 2^-53 is a
    tie that rounds back to 1); the exact sum 1 + 2^-52 is representable.
    Both assemblies must give the exact value, checked with rationals,
    under every order of the branch table."""
    from fractions import Fraction
    import itertools

    pairs = [(0, 1), (1, 2), (1, 3), (1, 2), (0, 3)]
    x = [1.0, 2.0 ** 53, 2.0 ** 53, 3.0, 7.0]
    exact_11 = sum(Fraction(1) / Fraction(v) for v in x[:4])
    exact_12 = -(Fraction(1) / Fraction(x[1]) + Fraction(1) / Fraction(x[3]))
    for perm in itertools.permutations(range(len(pairs))):
        pr = np.array([pairs[k] for k in perm], np.int32)
        xx = np.array([x[k] for k in perm])
        g = gridgen.Grid("star", 4, pr[:, 0].copy(), pr[:, 1].copy(), xx, np.zeros(4))
        A = gp.assemble(4, g.br_from, g.br_to, g.x).to_scipy().toarray()
        Ao = oracle.reduced(oracle.susceptance_full(g)).toarray()
        assert A[0, 0] == float(exact_11) and Ao[0, 0] == float(exact_11), perm
        assert A[0, 1] == float(exact_12) and Ao[0, 1] == float(exact_12), perm
    # the naive left-to-right sum of the first three terms loses the last bit
    assert (1.0 + 2.0 ** -53) + 2.0 ** -53 == 1.0
    assert float(Fraction(1) + 2 * Fraction(1, 2 ** 53)) == 1.0 + 2.0 ** -52


@pytest.mark.parametrize("key", ["grid200", "grid2k", "grid10k"])
def test_rcm_row_order(grids, key):
    """gpcg_rcm: a permutation of the non-slack buses, deterministic, whose
    rows are banded (the generated numbering is not); gpcg_assemble with it
    equals P A P^T of the bus-order assembly bit for bit."""
    g = grids[key]
    perm = gp.rcm(g.n, g.br_from, g.br_to)
    assert sorted(perm.tolist()) == list(range(1, g.n))
    np.testing.assert_array_equal(perm, gp.rcm(g.n, g.br_from, g.br_to))
    Ap = gp.assemble(g.n, g.br_from, g.br_to, g.x, perm=perm).to_scipy()
    coo = Ap.tocoo()
    assert np.abs(coo.row - coo.col).max() <= 80
    A = gp.assemble(g.n, g.br_from, g.br_to, g.x).to_scipy()
    rows = perm - 1
    np.testing.assert_array_equal(Ap.toarray() if g.n <= 2000 else Ap[:50].toarray(),
                                  A[rows][:, rows].toarray() if g.n <= 2000 else A[rows[:50]][:, rows].toarray())


def test_rcm_on_a_disconnected_reduced_graph():
    """Without the slack the reduced graph may fall apart (slack_leaf: the
    slack's only branch; two_rings: pieces joined through the slack);
    every piece is ordered."""
    for name in gridgen.HAND_GRIDS:
        g = gridgen.hand_grid(name)
        perm = gp.rcm(g.n, g.br_from, g.br_to)
        assert sorted(perm.tolist()) == list(range(1, g.n)), name


@pytest.mark.parametrize("key", ["grid200", "grid2k"])
def test_ilu0_matches_oracle(grids, key):
    g = grids[key]
    Ah = gp.assemble(g.n, g.br_from, g.br_to, g.x)
    L, U = gp.ilu0(Ah)
    Lo, Uo = oracle.ilu0(Ah.to_scipy())
    np.testing.assert_array_equal(L.rowptr, Lo.indptr)
    np.testing.assert_array_equal(U.col, Uo.indices)
    np.testing.assert_allclose(L.val, Lo.data, rtol=1e-13, atol=0)
    np.testing.assert_allclose(U.val, Uo.data, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("name", gridgen.HAND_GRIDS)
def test_topology_hand_grids(name):
    g = gridgen.hand_grid(name)
    T = gp.topology(g.n, g.br_from, g.br_to)
    for c in range(g.m):
        isl = oracle.island_of(g, c)
        assert T["is_bridge"][c] == oracle.is_bridge(g, c)
        got = (T["pre"] >= T["island_lo"][c]) & (T["pre"] < T["island_hi"][c])
        np.testing.assert_array_equal(got, isl)


@pytest.mark.parametrize("key", ["grid200", "grid2k"])
def test_topology_bit_exact_against_brute_force(grids, key):
    g = grids[key]
    T = gp.topology(g.n, g.br_from, g.br_to)
    assert T["pre"][0] == 0 and T["subtree"][0] == g.n
    assert sorted(T["pre"].tolist()) == list(range(g.n))
    step = 1 if g.n <= 200 else 7
    for c in range(0, g.m, step):
        isl = oracle.island_of(g, c)
        assert bool(T["is_bridge"][c]) == bool(isl.any())
        got = (T["pre"] >= T["island_lo"][c]) & (T["pre"] < T["island_hi"][c])
        np.testing.assert_array_equal(got, isl)


def test_errors_are_reported():
    with pytest.raises(gp.GpcgError) as e:
        gp.assemble(3, [0, 1], [1, 5], [0.1, 0.1])
    assert e.value.code == -1 and "range" in str(e.value)
    with pytest.raises(gp.GpcgError) as e:
        gp.topology(4, [0, 2], [1, 3])
    assert e.value.code == -1 and "connected" in str(e.value)
    A = binding.Csr([0, 1, 2], [1, 0], [1.0, 1.0])  # no diagonal
    with pytest.raises(gp.GpcgError) as e:
        gp.ilu0(A)
    assert e.value.code == -4
    with pytest.raises(gp.GpcgError) as e:
        gp.assemble(3, [0, 1], [1, 2], [0.1, -0.1])
    assert e.value.code == -1


def test_jacobi_factors_are_the_diagonal(grids):
    """The Jacobi preconditioner's factor pair: L without entries, U = diag(A),
    in the library's factor format."""
    import scipy.sparse as sp

    g = grids["grid200"]
    A = binding.assemble(g.n, g.br_from, g.br_to, g.x)
    L, U = binding.jacobi_factors(A)
    assert L.nnz == 0 and len(L.rowptr) == A.n + 1
    np.testing.assert_array_equal(U.rowptr, np.arange(A.n + 1))
    np.testing.assert_array_equal(U.col, np.arange(A.n))
    np.testing.assert_array_equal(U.val, sp.csr_matrix(A.to_scipy()).diagonal())


def test_block_tuner_caches_and_persists(tmp_path, monkeypatch):
    """The autotuner keeps the fastest candidate per set of grids, answers
    repeated questions from its table and reloads it from its JSON file."""
    from paper_1803_03290_amd import autotune

    class FakeCtx:
        def __init__(self, n):
            self.n_bus, self.kind = n, 0
            self.br_from = np.arange(n - 1, dtype=np.int32)
            self.br_to = np.arange(1, n, dtype=np.int32)
            self.x = np.full(n - 1, 0.1)

    class FakeOut:
        shape = (7,)

    calls = []

    def fake_tune(ctxs, outs, rhs, cands, tol, max_iter, reps):
        calls.append(tuple(cands))
        return {c: {4: 3.0, 8: 1.5, 16: 2.0}[c] for c in cands}

    monkeypatch.setattr(autotune, "batch_tune", fake_tune)
    path = str(tmp_path / "tune.json")
    t = autotune.BlockTuner(path)
    ctxs = [FakeCtx(5), FakeCtx(9)]
    outs = [FakeOut(), FakeOut()]
    assert t.best(ctxs, outs, None, (4, 8, 16)) == 8
    assert t.best(ctxs, outs, None, (4, 8, 16)) == 8 and len(calls) == 1
    t2 = autotune.BlockTuner(path)
    assert t2.best(ctxs, outs, None, (4, 8, 16)) == 8 and len(calls) == 1
    assert t2.best(ctxs, outs, None, (4, 8, 16), tol=1e-10) == 8 and len(calls) == 2  # another key


def test_tuner_caches_tile_shapes(tmp_path, monkeypatch):
    """(block, lookahead) candidates: the tuner returns the fastest pair,
    and a cached pair comes back as a tuple after a JSON round trip."""
    from paper_1803_03290_amd import autotune

    class FakeCtx:
        n_bus, kind = 6, 1
        br_from = np.arange(5, dtype=np.int32)
        br_to = np.arange(1, 6, dtype=np.int32)
        x = np.full(5, 0.2)

    class FakeOut:
        shape = (3,)

    calls = []
    table = {(4, 16): 2.0, (8, 16): 1.0, (8, 64): 0.5, 8: 0.1}

    def fake_tune(ctxs, outs, rhs, cands, tol, max_iter, reps):
        calls.append(tuple(cands))
        return {c: table[c] for c in cands}

    monkeypatch.setattr(autotune, "batch_tune", fake_tune)
    path = str(tmp_path / "tune.json")
    cands = ((4, 16), (8, 16), (8, 64))
    assert autotune.BlockTuner(path).best([FakeCtx()], [FakeOut()], None, cands) == (8, 64)
    assert autotune.BlockTuner(path).best([FakeCtx()], [FakeOut()], None, cands) == (8, 64) and len(calls) == 1
    # another candidate list is another key
    assert autotune.BlockTuner(path).best([FakeCtx()], [FakeOut()], None, (8,)) == 8 and len(calls) == 2
