"""Incomplete LU factorisation with zero fill, ILU(0) (oracle).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module.

The paper's two-domain preconditioners P^td_BJ(Uzawa, ILU(0)) and
P^td_BGS(Uzawa, ILU(0)) (Sec. 5 solver setup, Table 2) precondition the Darcy
block with an ILU(0) factorisation (Meijerink & van der Vorst, Math. Comp. 31,
1977).  Its definition: Gaussian elimination without pivoting in which every
entry outside the sparsity pattern of the matrix is dropped, so the unit lower
factor L and the upper factor U occupy exactly the pattern of A.  In the row
(IKJ) order used here, row i is finished by

    for each k < i in the pattern of row i, ascending:
        l_ik = a_ik / u_kk
        for each j > k in the pattern of row k, ascending:
            if (i, j) is in the pattern:  a_ij = a_ij - l_ik u_kj

and then holds l_ij (j < i) and u_ij (j >= i).  Consequence: (L U)_ij = a_ij
on the pattern, and L U = A when elimination creates no fill (a tridiagonal or
a dense matrix).  Applying the preconditioner solves L y = r by forward and
U z = y by backward substitution; each row's sum runs over its entries in
ascending column order and the diagonal of U divides last.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class ILU0:
    F: sp.csr_matrix           # strict lower part = L (unit diagonal implied), rest = U
    diag: np.ndarray           # position of the diagonal entry of each row in F.data

    @property
    def n(self) -> int:
        return self.F.shape[0]

    def L(self) -> sp.csr_matrix:
        return (sp.tril(self.F, -1) + sp.identity(self.n)).tocsr()

    def U(self) -> sp.csr_matrix:
        return sp.triu(self.F, 0).tocsr()

    def solve(self, r: np.ndarray) -> np.ndarray:
        """z = U^-1 L^-1 r by substitution, row by row."""
        F = self.F
        ptr, idx, val, d = F.indptr, F.indices, F.data, self.diag
        n = self.n
        z = np.zeros(n)
        for i in range(n):                       # L y = r (y kept in z)
            s = float(r[i])
            for e in range(ptr[i], d[i]):
                s = s - val[e] * z[idx[e]]
            z[i] = s
        for i in range(n - 1, -1, -1):           # U z = y
            s = z[i]
            for e in range(d[i] + 1, ptr[i + 1]):
                s = s - val[e] * z[idx[e]]
            z[i] = s / val[d[i]]
        return z


def ilu0(A) -> ILU0:
    """ILU(0) of a square sparse matrix whose diagonal is in the pattern and
    stays nonzero during the elimination (raises otherwise)."""
    F = sp.csr_matrix(A, dtype=np.float64, copy=True)
    F.sort_indices()
    F.sum_duplicates()
    n = F.shape[0]
    if F.shape != (n, n):
        raise ValueError("ILU(0) needs a square matrix")
    ptr, idx, val = F.indptr, F.indices, F.data
    diag = np.empty(n, dtype=np.int64)
    for i in range(n):
        hit = np.nonzero(idx[ptr[i]:ptr[i + 1]] == i)[0]
        if hit.size != 1:
            raise ValueError(f"row {i} has no diagonal entry")
        diag[i] = ptr[i] + hit[0]
    for i in range(n):
        pos = {int(idx[e]): e for e in range(ptr[i], ptr[i + 1])}
        for e in range(ptr[i], diag[i]):
            k = int(idx[e])
            ukk = val[diag[k]]
            if ukk == 0.0:
                raise ValueError(f"zero pivot in row {k}")
            lik = val[e] / ukk
            val[e] = lik
            for f in range(diag[k] + 1, ptr[k + 1]):
                g = pos.get(int(idx[f]))
                if g is not None:
                    val[g] = val[g] - lik * val[f]
        if val[diag[i]] == 0.0:
            raise ValueError(f"zero pivot in row {i}")
    return ILU0(F=F, diag=diag)
