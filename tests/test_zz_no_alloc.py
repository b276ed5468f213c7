"""The allocation-free solve (gpcg_solve_contingencies_noalloc) against the
ordinary batched solve, through the C ABI: identical results on two calls in
a row (all 2,800 outages of the 2,000-bus grid, with fewer wavefronts than
the ordinary solve runs, then 300 outages; a call on another grid's context
in between, all sharing the one fixed scratch), no device memory taken by
the call, and a clear refusal when the workspace would not fit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("x", "flows", "iters", "status", "island", "resid")


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_03290_amd as gp

    gp.lib()
    return gp


def _solve(gp, ctx, outs, rhs, noalloc, check_free=False):
    """One solve into preallocated outputs; with check_free, the device's
    free memory is read right before and after the call (the outputs and
    the outage list are the caller's and exist before)."""
    o = torch.tensor(outs.astype(np.int32), device="cuda")
    out = ctx.alloc_outputs(len(outs))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.solve(o, rhs, tol=1e-12, noalloc=noalloc, out=out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    if check_free:
        assert free0 - free1 < (2 << 20), (free0, free1)
    return {k: out[k].cpu().numpy() for k in KEYS}


def test_noalloc_matches_batched_solve(gp, grids):
    g = grids["grid2k"]
    small = grids["grid200"]
    ctx = gp.Context(g.n, g.br_from, g.br_to, g.x, g.P, block=4)
    ctx_small = gp.Context(small.n, small.br_from, small.br_to, small.x, small.P, block=16)
    rhs = torch.tensor(g.P, device="cuda")
    rhs_small = torch.tensor(small.P, device="cuda")
    rng = np.random.default_rng(3)
    first = np.arange(g.m)  # fewer wavefronts fit the fixed scratch than the ordinary solve runs
    second = np.concatenate([[-1, g.m + 5], np.sort(rng.choice(g.m, 298, replace=False))])
    for outs in (first, second):
        na = _solve(gp, ctx, outs, rhs, True, check_free=True)
        ref = _solve(gp, ctx, outs, rhs, False)
        for k in KEYS:
            np.testing.assert_array_equal(na[k], ref[k], err_msg=k)
        assert na["resid"][na["status"] != gp.BAD_OUTAGE].max() <= 1e-10
        # another context on the same GPU uses the same scratch in between
        so = np.arange(small.m)
        a = _solve(gp, ctx_small, so, rhs_small, True, check_free=True)
        b = _solve(gp, ctx_small, so, rhs_small, False)
        for k in KEYS:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_refuses_oversized_workspace(gp):
    """Three million scenarios of the two-bus grid need about 84 MB of
    per-scenario buffers (re-dispatch factors and the ordering), more than
    the 64 MiB of fixed scratch: refused on the host, outputs untouched."""
    import gridgen

    g = gridgen.hand_grid("two_bus")
    ctx = gp.Context(g.n, g.br_from, g.br_to, g.x, g.P, block=64)
    n = 3_000_000
    outs = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    out = ctx.alloc_outputs(n)
    out["x"].fill_(7.0)
    with pytest.raises(gp.GpcgError) as e:
        ctx.solve(outs, torch.tensor(g.P, device="cuda"), noalloc=True, out=out)
    assert e.value.code == -6 and "fixed scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out["x"] == 7.0).all())
