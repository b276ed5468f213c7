"""Zero-fill incomplete LU of the base-case matrix (the shared preconditioner).

TEST INFRASTRUCTURE (see the package docstring).

Section IV.B makes the factors of the unmodified base-case matrix the
preconditioner of every outage scenario.  Here they are the ILU(0) factors:
no fill outside the pattern of A, no pivoting, the rows in the order given.
This is the IKJ form of Gaussian elimination restricted to the pattern
(Saad, "Iterative Methods for Sparse Linear Systems", 2nd ed., Alg. 10.4),
written with plain Python loops over the rows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def ilu0(A: sp.csr_matrix):
    """Return (L, U): L strictly lower (unit diagonal implied), U upper with
    the diagonal, both CSR with sorted indices, such that (L+I)U agrees with A
    on the pattern of A."""
    A = A.tocsr().copy()
    A.sort_indices()
    n = A.shape[0]
    ptr, ind = A.indptr, A.indices
    val = A.data.astype(np.float64).copy()
    # position of each (row, col) of the pattern
    pos = [dict(zip(ind[ptr[i]:ptr[i + 1]].tolist(), range(ptr[i], ptr[i + 1]))) for i in range(n)]
    diag = np.empty(n, dtype=np.int64)
    for i in range(n):
        if i not in pos[i]:
            raise ValueError(f"row {i} has no diagonal entry")
        diag[i] = pos[i][i]
    for i in range(1, n):
        for p in range(ptr[i], ptr[i + 1]):
            k = int(ind[p])
            if k >= i:
                break
            if val[diag[k]] == 0.0:
                raise ZeroDivisionError(f"zero pivot at row {k}")
            val[p] = val[p] / val[diag[k]]
            lik = val[p]
            # subtract lik * (row k of U) where the pattern of row i allows
            for q in range(diag[k] + 1, ptr[k + 1]):
                j = int(ind[q])
                pj = pos[i].get(j)
                if pj is not None:
                    val[pj] -= lik * val[q]
    F = sp.csr_matrix((val, ind.copy(), ptr.copy()), shape=A.shape)
    L = sp.tril(F, k=-1, format="csr")
    U = sp.triu(F, k=0, format="csr")
    L.sort_indices()
    U.sort_indices()
    return L, U
