#!/usr/bin/env python3
"""Benchmark: N-1 scenario solves per second, batched vs plain PCG, on one MI355X.

One step is one pass of the whole hot path over one batch: every single-branch
outage of the grid (10,000-bus synthetic grid by default: 13,500 scenarios)
solved by the device library's batched PCG - base residual, init, PCG to the
tolerance, angles, flows, island flags and true residuals - with inputs
already resident in HBM.  Printed as one JSON line (rank 0).

Besides the contract fields the line carries:
  * "plain": the same scenarios (a seeded sample of 500) through the plain
    per-scenario PCG of the same library, and the batched/plain ratio;
  * "roofline": the PCG tile kernel's algorithmic HBM bytes per launch over
    its average launch time (HIP events on the context's stream), against
    the 8 TB/s HBM3E peak.  The bytes are the method's own work: 120 bytes
    per row per scenario per iteration of that scenario (15 vector passes),
    the matrix and factor entries once per wavefront per iteration it runs,
    and init and output passes; sweeps of columns that have already stopped
    are not counted (their share is reported as "idle_column_overhead").
    "traffic" comes from the committed rocprofv3 counter summary when it was
    taken on the current kernel source, workload and block;
  * "cpu_baseline": the FP64 oracle's direct solve (sparse LU + extended
    precision refinement per scenario, the paper's rebuild-per-scenario
    reference) on a bounded sample, on the host cores;
  * "verify": worst true residual, status counts, iteration statistics.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N-1 scenario solves/sec to 1e-10 residual, batched vs plain PCG; HBM GB/s %"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "pcg_wave_grid10k_counters.txt")
KERNEL_SRC = [os.path.join(ROOT, "paper_1803_03290_amd", "csrc", f)
              for f in ("gpcg_tile.hip", "gpcg_internal.h", "gpcg_device.h")]

# The method's algorithmic bytes per PCG iteration of one scenario: 15 vector
# passes of 8 bytes per row (product: read p, write q; update: read delta, p,
# r, q, write delta, r; forward solve: read r, write y; backward solve: read
# y, write z; direction: read z, p, write p), i.e. 120 bytes per row; the
# matrix A and the factors L, U are read once per iteration for all the
# columns of a tile (12 bytes per entry, 4 per row pointer); init and output
# move about six passes per scenario plus its flows.
VEC_BYTES_PER_ROW_ITER = 120.0


def own_work_bytes(info: dict, scen_iters, wave_iters: int, m: int) -> float:
    """Algorithmic bytes of one solve: every scenario's own iterations for
    the vectors, every wavefront iteration for the shared matrix entries
    (read once per iteration for the wave's S columns)."""
    nr = info["n_r"]
    vec = VEC_BYTES_PER_ROW_ITER * nr * float(sum(int(k) for k in scen_iters))
    mat_iter = 12.0 * (info["nnz_a"] + info["nnz_l"] + info["nnz_u"]) + 12.0 * (nr + 1)
    mat = mat_iter * float(wave_iters)
    io = (6.0 * 8.0 * nr + 8.0 * m) * len(scen_iters)
    return vec + mat + io


def kernel_digest() -> str:
    """First 16 hex digits of the SHA-256 of the PCG kernel's sources (the
    kernel file and the headers it is compiled with) with comments and
    whitespace removed (a comment edit keeps the counters of the same code
    valid)."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", re.sub(r"//[^\n]*", "", text), flags=re.S)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def auto_block(n_out: int) -> int:
    """Widest tile (scenarios per wavefront) that still gives about 600
    wavefronts, so every SIMD of the 1,024 holds a tile."""
    S = 64
    while S > 1 and (n_out + S - 1) // S < 600:
        S //= 2
    return S


def read_counters():
    """(fetch_kib, write_kib, fetch_factor, write_factor, digest, (workload,
    block, lookahead)) from the
    committed summary; each factor is what a plain copy of known size needs
    to turn that counter into bytes."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    try:
        return (float(vals["fetch_kib_per_dispatch"]), float(vals["write_kib_per_dispatch"]),
                float(vals["fetch_copy_factor"]), float(vals["write_copy_factor"]), vals["kernel_digest"],
                (vals["workload"], int(vals["block"]), int(vals.get("lookahead", "0"))))
    except KeyError:
        return None


# ----------------------------------------------------------- CPU baseline
_G = None


def _cpu_init(grid):
    global _G
    import oracle

    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except Exception:
        pass
    _G = (grid, oracle.reduced(oracle.susceptance_full(grid)))


def _cpu_one(c):
    import oracle

    grid, A = _G
    s = oracle.scenario(grid, int(c), A)
    return s["status"]


def cpu_baseline(grid, seconds: float = 20.0):
    """The oracle's per-scenario direct solve over a bounded seeded sample
    (about ``seconds`` of single-core work), one single-threaded worker per
    host core this process may use, at most 16 (the host share that goes
    with one GPU); run before the GPU is touched."""
    import multiprocessing as mp

    import numpy as np

    affinity = len(os.sched_getaffinity(0))
    cores = min(16, affinity)
    _cpu_init(grid)
    rng = np.random.default_rng(11)
    probe = rng.choice(grid.m, min(20, grid.m), replace=False)
    t0 = time.perf_counter()
    for c in probe:
        _cpu_one(c)
    per = (time.perf_counter() - t0) / len(probe)
    n = int(min(grid.m, max(cores, seconds / per)))
    sample = rng.choice(grid.m, n, replace=False)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_cpu_init, initargs=(grid,)) as pool:
        t0 = time.perf_counter()
        pool.map(_cpu_one, sample, chunksize=max(1, n // (8 * cores)))
        wall = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / wall, "unit": "scenarios/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded outages of {grid.name} (of {grid.m}), sparse LU + longdouble refinement per "
                      f"scenario, {cores} single-threaded workers; {wall:.2f} s wall; 1-core {1.0 / per:.1f} "
                      f"scenarios/s",
            "cpu_model": model, "affinity_cpus": affinity, "one_core_value": 1.0 / per}


# ------------------------------------------------------ stand-alone SpMM
def spmm_measure(gp, torch, grid, S: int = 64, reps: int = 20):
    """The outage-corrected product q = A_c p over every outage column of a
    grid in one launch (p ~ N(0, 1), seed 0, columns padded to a multiple
    of S), timed with HIP events; bytes are the product's algorithmic bytes
    12 nnz + 4 (n_r + 1) + 16 n_r s + 16 s for s columns."""
    import numpy as np

    ctx = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, grid.P, block=S)
    info = ctx.info()
    nr = info["n_r"]
    ncols = ((grid.m + S - 1) // S) * S
    dev = torch.device("cuda", 0)
    outs = torch.tensor(np.arange(ncols) % grid.m, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    p = torch.randn((ncols // S, nr, S), dtype=torch.float64, device=dev, generator=gen)
    q = torch.empty_like(p)
    pq = torch.empty(ncols, dtype=torch.float64, device=dev)
    for _ in range(3):
        ctx.spmm(outs, p, q, pq)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.spmm(outs, p, q, pq)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    nbytes = 12.0 * info["nnz_a"] + 4.0 * (nr + 1) + 16.0 * nr * ncols + 16.0 * ncols
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": f"{grid.name}: q = A_c p over {ncols} outage columns ({grid.m} outages)",
            "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "median_ms": ms, "algorithmic_bytes": nbytes, "block": S}


def adjoint_measure(gp, torch, grid, S: int = 16, reps: int = 2, tol: float = 1e-12):
    """The differentiation workload: the overload loss of every outage and
    its gradients in P (n) and x (m), one forward and one adjoint batched
    PCG per scenario, timed with HIP events on the context's stream.  Flow
    limits F = 1.2 |base flow| + 0.1 come from the library's own base-case
    solve (input preparation, outside the timed region)."""
    import numpy as np

    ctx = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, grid.P, block=S)
    dev = torch.device("cuda", 0)
    P = torch.tensor(grid.P, dtype=torch.float64, device=dev)
    base = ctx.solve(torch.tensor([-1], dtype=torch.int32, device=dev), P, tol=tol)
    F = 1.2 * base["flows"][0].abs() + 0.1
    outs = torch.arange(grid.m, dtype=torch.int32, device=dev)
    res = ctx.overload_gradients(outs, P, F, 20.0, tol=tol)
    torch.cuda.synchronize()
    stream = ctx.stream
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        res = ctx.overload_gradients(outs, P, F, 20.0, tol=tol)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    it = res["iters"].cpu().numpy()
    st = res["status"].cpu().numpy()
    return {"workload": f"{grid.name}: overload loss + dL/dP ({grid.n}) + dL/dx ({grid.m}) of all {grid.m} "
                        f"outages, forward + adjoint batched PCG (base ILU(0)), tol {tol:g}",
            "value": grid.m / (ms * 1e-3), "unit": "scenarios/s", "ms": ms, "block": S,
            "forward_iters_mean": float(it[:grid.m].mean()), "adjoint_iters_mean": float(it[grid.m:].mean()),
            "all_converged": bool(np.all(st <= 5))}


def fdpf_measure(gp, torch, grid, S: int = 16, scale: float = 1e-4, n_outer: int = 3, tol: float = 1e-12,
                 reps: int = 1):
    """The power-flow workload: n_outer fast-decoupled iterations (a B' and a
    B'' batched solve each) for every outage, from the base state, timed with
    HIP events on the shared stream.  Injections and shunts are scaled by
    ``scale``: at the full draws the AC iteration diverges on these grids,
    1e-4 is where it converges on the 10,000-bus grid.  The base state
    (n_outer iterations of the intact grid from a flat start) is computed
    by the same entry point outside the timed region."""
    import numpy as np

    rng = np.random.default_rng(4)
    Q = grid.Q if grid.Q is not None else rng.normal(0, 0.2, grid.n)
    bsh = grid.bsh if grid.bsh is not None else rng.uniform(0, 0.05, grid.n)
    P, Q, bsh = scale * grid.P, scale * Q, scale * bsh
    bp = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, P, block=S)
    bpp = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, Q, block=S, kind=gp.KIND_BPP, shunt=bsh)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.asarray(a, np.float64), device=dev)
    Pt, Qt = t(P), t(Q)
    base = bp.fdpf(bpp, torch.tensor([-1], dtype=torch.int32, device=dev), Pt, Qt, t(np.zeros(grid.n)),
                   t(np.ones(grid.n)), n_outer=n_outer, tol=tol)
    th0, V0 = base["theta"][0].contiguous(), base["V"][0].contiguous()
    outs = torch.arange(grid.m, dtype=torch.int32, device=dev)
    res = bp.fdpf(bpp, outs, Pt, Qt, th0, V0, n_outer=n_outer, tol=tol)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bp.stream)
        res = bp.fdpf(bpp, outs, Pt, Qt, th0, V0, n_outer=n_outer, tol=tol)
        e1.record(bp.stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    st = res["status"].cpu().numpy()
    return {"workload": f"{grid.name}: {n_outer} fast-decoupled iterations (B' + B'' batched PCG each) of all "
                        f"{grid.m} outages from the base state, injections and shunts x {scale:g}, tol {tol:g}",
            "value": grid.m / (ms * 1e-3), "unit": "scenarios/s", "ms": ms, "block": S,
            "pcg_iters_mean": float(res["iters"].float().mean().item()),
            "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}


def ablation_measure(gp, torch, grid, S: int, tol: float, max_iter: int, steps: int = 3):
    """The paper's own alternatives, same kernels: the Jacobi preconditioner
    of the GPCG listing and the zero start of the PCG listing, against the
    base-case ILU(0) and the base-state start (``base_ilu0``, the method
    itself on the same grid and block), and the plain per-scenario PCG over
    the grid's whole outage list beside it.  Run on the grid given
    (normally the 2,000-bus grid: Jacobi takes about 13 times the base-ILU
    iterations, too long a leg on the 10k grid)."""
    import numpy as np

    dev = torch.device("cuda", 0)
    outs = torch.arange(grid.m, dtype=torch.int32, device=dev)
    rhs = torch.tensor(grid.P, dtype=torch.float64, device=dev)
    res = {}
    for name, kw in (("base_ilu0", {}), ("jacobi", dict(precond="jacobi")), ("zero_start", dict(zero_start=True))):
        ctx = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, grid.P, block=S, **kw)
        out = ctx.solve(outs, rhs, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            ctx.solve(outs, rhs, tol=tol, max_iter=max_iter, out=out)
            e1.record(ctx.stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        it = out["iters"].cpu().numpy()
        res[name] = {"value": grid.m / (ms * 1e-3), "unit": "scenarios/s", "ms": ms,
                     "iters_mean": float(it.mean()), "iters_max": int(it.max()),
                     "max_true_rel_residual": float(out["resid"].max().item())}
        if name == "base_ilu0":
            # the plain per-scenario PCG over the whole outage list of this grid
            ctx.solve(outs[:16], rhs, tol=tol, max_iter=max_iter, plain=True)  # warm-up
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            pout = ctx.solve(outs, rhs, tol=tol, max_iter=max_iter, plain=True)
            e1.record(ctx.stream)
            torch.cuda.synchronize()
            p_ms = e0.elapsed_time(e1)
            res["plain_all_outages"] = {
                "value": grid.m / (p_ms * 1e-3), "unit": "scenarios/s", "ms": p_ms,
                "iters_mean": float(pout["iters"].float().mean().item()),
                "max_abs_diff_vs_batched_rad": float((pout["x"] - out["x"]).abs().max().item()),
                "batched_vs_plain": (grid.m / (ms * 1e-3)) / (grid.m / (p_ms * 1e-3))}
            del pout
    return res


UNEVEN = ("uneven500", "uneven1000", "uneven2000", "uneven3000", "uneven5000", "uneven8000", "uneven12000",
          "uneven20000")


BATCH_SHAPES = ((4, 0), (8, 0), (8, 64), (16, 0), (16, 64))
BATCH_DEFAULT_SHAPE = (8, 64)  # the autotuner's pick over BATCH_SHAPES on the uneven workload


def batch_measure(gp, torch, tol: float, max_iter: int, reps: int = 2, names=UNEVEN, shapes=BATCH_SHAPES):
    """The uneven workload: all outages of eight grids (500 to 20,000 buses)
    in one graph-captured launch; the tile shape (block, look-ahead window)
    is picked by the autotuner over ``shapes``, one timed solve each.  Timed
    with HIP events on the contexts' stream around ``reps`` graph replays."""
    import numpy as np

    import gridgen

    def progress(msg):
        print(f"[batch] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    grids, ctxs = [], []
    for n in names:
        t0 = time.perf_counter()
        g = gridgen.make_grid(n)
        t1 = time.perf_counter()
        ctxs.append(gp.Context(g.n, g.br_from, g.br_to, g.x, g.P, block=8))
        grids.append(g)
        progress(f"{n}: grid {t1 - t0:.1f} s, context {time.perf_counter() - t1:.1f} s")
    outs = [torch.arange(g.m, dtype=torch.int32, device=dev) for g in grids]
    rhs = [torch.tensor(g.P, dtype=torch.float64, device=dev) for g in grids]
    tune_ms = {}
    if len(shapes) > 1:
        for cand in shapes:  # the autotuner's search, one candidate per call so that progress shows
            tune_ms.update(gp.batch_tune(ctxs, outs, rhs, (cand,), tol, max_iter))
            progress(f"block {cand[0]}, look-ahead {cand[1] or 'default'}: {tune_ms[cand]:.1f} ms per solve")
        S, look = min(tune_ms, key=tune_ms.get)
    else:
        S, look = shapes[0]
    b = gp.Batch(ctxs, outs, rhs, block=S, tol=tol, max_iter=max_iter, flows=True, lookahead=look)
    b.run()
    torch.cuda.synchronize()
    progress("batch built and captured")
    stream = ctxs[0].stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = sum(g.m for g in grids)
    resid = max(float(d["resid"].max().item()) for d in b.out)
    st = np.concatenate([d["status"].cpu().numpy() for d in b.out])
    b.close()
    return {"workload": f"uneven batch: {len(grids)} grids of {grids[0].n} to {grids[-1].n} buses, all {n} outages "
                        f"in one graph-captured launch, tol {tol:g}",
            "value": n / (ms * 1e-3), "unit": "scenarios/s", "ms": ms, "block": S, "lookahead": look,
            "tuner_ms_per_solve": {f"{b}/{lk}": v for (b, lk), v in tune_ms.items()} or None,
            "max_true_rel_residual": resid,
            "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}


# ------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="grid10k", help="grid spec key (grid200, grid2k, grid10k, ...)")
    ap.add_argument("--block", type=int, default=16, help="scenarios per wavefront (0: auto)")
    ap.add_argument("--lookahead", type=int, default=64,
                    help="look-ahead window of the triangular schedules, rows (0: the library's 256)")
    ap.add_argument("--tol", type=float, default=1e-12,
                    help="stop on the recursive relative residual; on the 10k grid 1e-12 meets both the 1e-10 "
                         "true-residual bar and the 1e-8 rad angle bar on every outage")
    ap.add_argument("--tol-alt", type=float, default=5e-11, help="second stop reported beside the headline")
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--plain-sample", type=int, default=500, help="scenarios timed through the plain PCG")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--dump-iters", default="", help="save per-outage iterations, status and queue order (.npz)")
    ap.add_argument("--spmm-workload", default="grid10k", help="grid of the stand-alone product measurement")
    ap.add_argument("--no-spmm", action="store_true")
    ap.add_argument("--spmm-block", type=int, default=16)
    ap.add_argument("--spmm-only", action="store_true", help="only the stand-alone product measurement")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-workload", default="grid10k", help="grid of the overload-gradient measurement")
    ap.add_argument("--adjoint-block", type=int, default=16)
    ap.add_argument("--adjoint-only", action="store_true", help="only the overload-gradient measurement")
    ap.add_argument("--no-fdpf", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--ablation-workload", default="grid2k", help="grid of the ablations (Jacobi, x0 = 0)")
    ap.add_argument("--ablation-block", type=int, default=4)
    ap.add_argument("--batch", action="store_true",
                    help="run the uneven multi-grid batch with the autotuner's search over five tile shapes "
                         "(several minutes) instead of at the shape it picks on this workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven multi-grid batch")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the uneven multi-grid batch (at the tuned shape; add --batch for the search)")
    ap.add_argument("--fdpf-workload", default="grid10k", help="grid of the power-flow measurement")
    ap.add_argument("--fdpf-only", action="store_true", help="only the power-flow measurement")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the scenarios are independent, so more GPUs would each run the "
              "same kernel on a share of the outage list; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import gridgen

    grid = gridgen.make_grid(args.workload)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(grid, args.cpu_seconds)  # before any GPU call

    import torch

    if args.copy_probe:
        n = 1 << 27  # 1 GiB of float64
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.copy_(a)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 6,
                          "ms_per_copy": ms, "GBps": 2 * n * 8 / (ms * 1e-3) / 1e9}))
        return

    import paper_1803_03290_amd as gp

    gp.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    aux_grids = {}

    def aux_grid(name):
        if name not in aux_grids:
            aux_grids[name] = grid if name == grid.name else gridgen.make_grid(name)
        return aux_grids[name]

    if args.spmm_only:
        print(json.dumps(spmm_measure(gp, torch, aux_grid(args.spmm_workload), args.spmm_block)), flush=True)
        return
    if args.batch_only:
        # at the tuned shape; with --batch, the tuner's whole search first
        print(json.dumps(batch_measure(gp, torch, args.tol, args.max_iter, reps=2,
                                       shapes=BATCH_SHAPES if args.batch else (BATCH_DEFAULT_SHAPE,))),
              flush=True)
        return
    if args.fdpf_only:
        print(json.dumps(fdpf_measure(gp, torch, aux_grid(args.fdpf_workload))), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_measure(gp, torch, aux_grid(args.adjoint_workload), args.adjoint_block)),
              flush=True)
        return
    t0 = time.perf_counter()
    block = args.block or auto_block(grid.m)
    ctx = gp.Context(grid.n, grid.br_from, grid.br_to, grid.x, grid.P, block=block, lookahead=args.lookahead)
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    m = grid.m
    outages = torch.arange(m, dtype=torch.int32, device=dev)
    rhs = torch.tensor(grid.P, dtype=torch.float64, device=dev)
    out = ctx.alloc_outputs(m, flows=True, island=True, resid=True)

    def step():
        ctx.solve(outages, rhs, tol=args.tol, max_iter=args.max_iter, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps

    # PCG kernel time per launch, from the library's own events
    ctx.set_timing(True)
    kms = []
    for _ in range(max(3, min(args.steps, 10))):
        step()
        kms.append(ctx.pcg_ms())
    ctx.set_timing(False)
    torch.cuda.synchronize()
    pcg_ms = float(np.mean(kms))

    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    resid = out["resid"].cpu().numpy()
    S = info["block"]
    waves, wave_iters = ctx.sweeps()  # persistent wavefronts and their iterations, last solve
    if args.dump_iters:
        np.savez(args.dump_iters, iters=iters, status=status, order=ctx.order(m), perm=ctx.perm)
    algo_bytes = own_work_bytes(info, iters, wave_iters, m)
    achieved = algo_bytes / (pcg_ms * 1e-3) / 1e9
    idle_overhead = float(S * wave_iters) / max(1, int(iters.sum()))
    progress(f"headline: {m / (ms_step * 1e-3):.0f} scenarios/s, pcg kernel {pcg_ms:.1f} ms")

    alt = None
    if args.tol_alt and args.tol_alt != args.tol:
        aout = ctx.alloc_outputs(m, flows=True, island=True, resid=True)
        ctx.solve(outages, rhs, tol=args.tol_alt, max_iter=args.max_iter, out=aout)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.solve(outages, rhs, tol=args.tol_alt, max_iter=args.max_iter, out=aout)
        e1.record(stream)
        torch.cuda.synchronize()
        a_ms = e0.elapsed_time(e1)
        alt = {"tol": args.tol_alt, "value": m / (a_ms * 1e-3), "unit": "scenarios/s", "ms": a_ms,
               "max_true_rel_residual": float(aout["resid"].max().item()),
               "iters_mean": float(aout["iters"].float().mean().item()),
               "max_abs_diff_vs_headline_rad": float((aout["x"] - out["x"]).abs().max().item())}
        del aout
    traffic = None
    cnt = read_counters()
    if cnt and cnt[4] == kernel_digest() and cnt[5] == (args.workload, S, args.lookahead):
        traffic = cnt[0] * 1024.0 * cnt[2] + cnt[1] * 1024.0 * cnt[3]

    plain = None
    if not args.no_plain:
        rng = np.random.default_rng(5)
        samp = np.sort(rng.choice(m, min(args.plain_sample, m), replace=False)).astype(np.int32)
        so = torch.tensor(samp, device=dev)
        pout = ctx.alloc_outputs(len(samp), flows=True, island=True, resid=True)
        ctx.solve(so, rhs, tol=args.tol, max_iter=args.max_iter, plain=True, out=pout)  # warm-up
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.solve(so, rhs, tol=args.tol, max_iter=args.max_iter, plain=True, out=pout)
        e1.record(stream)
        torch.cuda.synchronize()
        p_ms = e0.elapsed_time(e1)
        same = float(np.abs(pout["x"].cpu().numpy() - out["x"][so.long()].cpu().numpy()).max())
        isl_share = float((status[samp] >= 4).mean())
        plain = {"value": len(samp) / (p_ms * 1e-3), "unit": "scenarios/s", "scenarios": int(len(samp)),
                 "ms": p_ms, "max_abs_diff_vs_batched_rad": same, "islanding_share": isl_share,
                 "islanding_share_all": float((status >= 4).mean()),
                 "iters_mean": float(pout["iters"].float().mean().item()),
                 "note": f"seeded sample of {len(samp)} of the {m} outages (seed 5), one scenario per launch, "
                         f"lanes spread over rows (S=1); the rate of the sample stands for the whole list"}
        progress(f"plain: {plain['value']:.1f} scenarios/s")

    spmm = None if args.no_spmm else spmm_measure(gp, torch, aux_grid(args.spmm_workload), args.spmm_block)
    adj = None if args.no_adjoint else adjoint_measure(gp, torch, aux_grid(args.adjoint_workload),
                                                       args.adjoint_block)
    pf = None if args.no_fdpf else fdpf_measure(gp, torch, aux_grid(args.fdpf_workload))
    progress("spmm, adjoint and power-flow legs done")
    abl = None if args.no_ablations else ablation_measure(gp, torch, aux_grid(args.ablation_workload),
                                                          args.ablation_block, 5e-11, args.max_iter)
    bat = None
    if not args.no_batch:
        # the whole uneven workload (72,100 outages); by default at the tile shape the autotuner picks on it
        bat = batch_measure(gp, torch, args.tol, args.max_iter, reps=1,
                            shapes=BATCH_SHAPES if args.batch else (BATCH_DEFAULT_SHAPE,))

    value = m / (ms_step * 1e-3)
    st_counts = {int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))}
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "scenarios/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{grid.name}: {grid.n}-bus synthetic grid, all {m} N-1 branch outages, batched PCG with "
                        f"base-case ILU(0), FP64, recursive residual stop {args.tol:g}, true residual <= 1e-10",
            "n_bus": grid.n, "n_branches": m, "scenarios": m, "block": S, "lookahead": args.lookahead or 256,
            "tol": args.tol, "grid_sha256": grid.digest()[:16],
        },
        "batched_vs_plain": (value / plain["value"]) if plain else None,
        "plain": plain,
        "alt_tol": alt,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"pcg_wave_kernel<{S}>", "algorithmic_bytes_per_launch": algo_bytes,
            "avg_launch_ms": pcg_ms, "kernel_digest": kernel_digest(), "idle_column_overhead": idle_overhead,
            "bytes": "120 B per row per scenario-iteration + 12 B per matrix/factor entry per wave-iteration + "
                     "init/output; stopped columns not counted",
        },
        "spmm": spmm,
        "adjoint": adj,
        "fdpf": pf,
        "ablations": abl,
        "batch": bat,
        "cpu_baseline": cpu,
        "verify": {
            "status_counts": st_counts,
            "max_true_rel_residual": float(resid.max()),
            "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
            "waves": waves, "wave_iters_sum": int(wave_iters), "scenario_iters_sum": int(iters.sum()),
            "bridges": info["n_bridges"], "setup_s": setup_s, "base_iters": info["base_iters"],
            "base_resid": info["base_resid"],
        },
        "schedule": {k: info[k] for k in ("rows_per_step", "ring_fwd", "ring_bwd", "steps_fwd", "steps_bwd",
                                          "bandwidth", "nnz_a", "nnz_l", "nnz_u")},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
