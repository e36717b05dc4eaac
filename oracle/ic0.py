"""Oracle: incomplete Cholesky with no fill, IC(0), as a PCG preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper solves both corrector systems by PCG with an incomplete Cholesky
factorisation computed once before the time loop (Sec. 3.2.2 and 3.2.3,
citing Meijerink and van der Vorst).  Its triangular sweeps are sequential,
so the GPU library does not use it; this module exists only to put the GPU
preconditioners' iteration counts beside the paper's choice.

Definition (textbook IC(0)): L is lower triangular with the sparsity of the
lower triangle of A, and L L^T equals A on every position of A's pattern.
Row by row,
    L_ik = (A_ik - sum_{j<k} L_ij L_kj) / L_kk   for k < i in the pattern,
    L_ii = sqrt(A_ii - sum_{k<i} L_ik^2),
where the sums run over the pattern only.  For an M-matrix every pivot is
positive (Meijerink and van der Vorst, 1977).  Plain Python loops: small
systems only.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def ic0(A) -> sp.csr_matrix:
    """L of IC(0) for a symmetric matrix A with a symmetric pattern."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rows = []  # rows[i]: dict col -> L_ij for j <= i
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        cols, vals = A.indices[lo:hi], A.data[lo:hi]
        Li = {}
        for k, a in zip(cols, vals):
            if k >= i:
                continue
            Lk = rows[k]
            s = a
            for j, lij in Li.items():
                if j < k:
                    lkj = Lk.get(j)
                    if lkj is not None:
                        s -= lij * lkj
            Li[k] = s / Lk[k]
        diag = A[i, i] - sum(v * v for v in Li.values())
        if not diag > 0.0:
            raise ValueError(f"IC(0) breakdown at row {i}: pivot {diag}")
        Li[i] = math.sqrt(diag)
        rows.append(Li)
    r, c, v = [], [], []
    for i, Li in enumerate(rows):
        for j, x in Li.items():
            r.append(i)
            c.append(j)
            v.append(x)
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def ic0_apply(L, r) -> np.ndarray:
    """z = (L L^T)^{-1} r by a forward and a backward triangular solve."""
    y = spl.spsolve_triangular(L, np.asarray(r, np.float64), lower=True)
    return spl.spsolve_triangular(sp.csr_matrix(L.T), y, lower=False)
