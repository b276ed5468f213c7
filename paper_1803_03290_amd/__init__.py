"""MI355X-native batched PCG for "N-1" contingency screening (arXiv 1803.03290).

A thin binding over the C ABI of ``libgpcg.so`` (declared in
``include/gpcg.h``).  Python only marshals arguments: the susceptance
assembly, ILU(0), topology pass and scheduling run in the library's host
C++, every solve step in its HIP kernels.  PyTorch provides device memory
and the stream.  There is no fallback: without the built library every call
raises.
"""
from .binding import (  # noqa: F401
    BAD_OUTAGE,
    BREAKDOWN,
    CONVERGED,
    CONVERGED_ISLANDED,
    ISLANDED_NO_GEN,
    KIND_BP,
    KIND_BPP,
    MAX_ITER,
    NONFINITE,
    Context,
    GpcgError,
    assemble,
    ilu0,
    lib,
    rcm,
    topology,
)
from .overload import OverloadLoss, overload_loss  # noqa: F401,E402
from .binding import Batch, batch_tune  # noqa: F401,E402
from .autotune import BlockTuner  # noqa: F401,E402
