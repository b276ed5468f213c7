"""The benchmark's roofline accounting (CPU): the committed counter summary
belongs to the kernel source and launch the benchmark runs by default, and
the algorithmic bytes follow their stated formula."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    import bench

    return bench


def test_counter_summary_matches_the_default_launch():
    """A kernel change without new counters would report stale traffic:
    the summary's digest must be that of the current kernel sources, and its
    workload, block and look-ahead those of the default command line."""
    b = _bench()
    cnt = b.read_counters()
    assert cnt is not None
    fetch, write, ff, wf, digest, key = cnt
    assert digest == b.kernel_digest()
    # the defaults as main() declares them

    src = open(os.path.join(ROOT, "bench.py")).read()
    assert '"--workload", default="grid10k"' in src
    assert '"--block", type=int, default=16' in src
    assert '"--lookahead", type=int, default=64' in src
    assert key == ("grid10k", 16, 64)
    assert fetch > 0 and write > 0 and ff == 2.0 and wf == 1.0


def test_kernel_digest_ignores_comments(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("int f(int x) { return x + 1; }  // one\n/* two */\n")
    monkeypatch.setattr(b, "KERNEL_SRC", [str(src)])
    d0 = b.kernel_digest()
    src.write_text("int f(int x) {\n  return x + 1;  // changed comment\n}\n")
    assert b.kernel_digest() == d0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert b.kernel_digest() != d0


def test_own_work_bytes_formula():
    """120 B per row per scenario-iteration, 12 B per matrix/factor entry and
    per row (+1) per wavefront-iteration, and 6 vector passes + 8 B per
    branch per scenario for init and output."""
    b = _bench()
    info = {"n_r": 10, "nnz_a": 28, "nnz_l": 9, "nnz_u": 19}
    iters = [3, 5]
    got = b.own_work_bytes(info, iters, 7, m=12)
    want = 120 * 10 * 8 + (12 * (28 + 9 + 19) + 12 * 11) * 7 + (6 * 8 * 10 + 8 * 12) * 2
    assert got == want
