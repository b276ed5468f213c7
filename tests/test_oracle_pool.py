"""CPU check of the every-outage comparison helper used by the GPU tests:
fed the oracle's own solutions with one planted angle error and one flipped
island flag, it reports exactly those two scenarios."""
import numpy as np

import oracle
from oracle_pool import compare_all


def test_compare_all_reports_planted_differences(grids):
    g = grids["grid200"]
    _, A = oracle.base_case(g)
    outs = np.arange(g.m)
    sols = [oracle.scenario(g, int(c), A) for c in outs]
    res = dict(x=np.array([d["theta"] for d in sols]), flows=np.array([d["flows"] for d in sols]),
               island=np.array([d["island"] for d in sols]).astype(np.uint8))
    res["x"][17, 5] += 3e-8
    k = next(i for i, d in enumerate(sols) if d["island"].any())
    res["island"][k, 0] ^= 1
    out = compare_all(g, A, outs, res, workers=2)
    assert np.flatnonzero(out["angle"] > 1e-8).tolist() == [17]
    assert np.flatnonzero(~out["island_ok"]).tolist() == [k]
    assert np.array_equal(out["status"], [d["status"] for d in sols])
    assert out["resid"].max() < 1e-10 or np.argmax(out["resid"]) == 17


def test_compare_fdpf_reports_a_planted_difference(grids):
    """The power-flow comparison helper: the oracle's own three iterations
    of 12 outages with one planted angle error; only that one is reported."""
    from oracle import fdpf
    from oracle_pool import compare_fdpf

    g = grids["grid200"]
    rng = np.random.default_rng(4)
    P, Q, bsh = 0.01 * g.P, 0.01 * rng.normal(0, 0.2, g.n), 0.01 * rng.uniform(0, 0.05, g.n)
    thb, Vb = fdpf.base_state(g, P, Q, bsh)
    outs = np.arange(12)
    runs = [fdpf.fdpf(g, P, Q, bsh, thb, Vb, int(c)) for c in outs]
    T = np.array([r[0] for r in runs])
    V = np.array([r[1] for r in runs])
    T[3, 5] += 1e-7
    dth, dV = compare_fdpf(g, P, Q, bsh, thb, Vb, outs, T, V, workers=2)
    assert np.flatnonzero(dth > 1e-8).tolist() == [3] and dV.max() == 0.0
