"""FP64 CPU oracle for N-1 contingency screening with base-case-ILU preconditioned CG.

TEST INFRASTRUCTURE.  This package is the plain, slow, obviously-correct
reference that the device library is checked against.  Only the tests, the
``smoke()`` entry point of ``__graft_entry__.py`` and the CPU-baseline leg of the
benchmark may import it.  The device library never calls it and shares no code
with it: the only common input is the seeded grid drawn by ``gridgen``.

What it computes, following the paper (arXiv 1803.03290):

* ``system``: the fast-decoupled susceptance matrices B' (eq. 4) and B''
  (eq. 5), the base case, the islanded buses of each single-branch outage by
  brute-force connectivity (Section IV.C), the proportional re-dispatch of the
  islanded power (Section IV.C), the direct solve of every outage scenario
  (sparse LU plus extended-precision iterative refinement; the rebuild-per-
  scenario "LUD" reference of Section V) and the branch flows.
* ``ilu``: the zero-fill incomplete LU factors of the base-case matrix, the
  preconditioner every scenario shares (Section IV.B, eqs. 6-7).
* ``pcg``: the textbook preconditioned conjugate gradient of Section III.A,
  run on each outage matrix in correction form from the base state
  (Section III.B, last paragraph) with the base-case ILU factors.

Every function is pinned in ``tests/test_oracle.py`` by something other than
itself (closed forms on hand grids, the Sherman-Morrison line-outage formula,
the bridge / effective-reactance identity, Kirchhoff balance, dense inverses,
the ILU(0) defining property); none is left "parity unpinned".
"""
from .system import (  # noqa: F401
    STATUS_CONVERGED,
    STATUS_MAX_ITER,
    STATUS_BREAKDOWN,
    STATUS_NONFINITE,
    STATUS_CONVERGED_ISLANDED,
    STATUS_ISLANDED_NO_GEN,
    susceptance_full,
    reduced,
    outage_matrix,
    island_of,
    is_bridge,
    redispatch,
    refined_solve,
    base_case,
    scenario,
    flows,
    true_residual,
)
from .ilu import ilu0  # noqa: F401
from .pcg import pcg_correction, pcg_textbook, scenario_pcg  # noqa: F401
