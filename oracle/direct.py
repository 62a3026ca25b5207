"""Reference solution x* = A^-1 b by sparse LU (SciPy SuperLU).

The monolithic system of Sec. 2 has a unique solution; every iterative
method on the hot path converges to it.  The paper's own direct baseline is
UMFPACK (Sec. 5); SuperLU, a library sparse LU, serves the same purpose.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def solve(A, b) -> np.ndarray:
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    return lu.solve(np.asarray(b, dtype=np.float64))


def refined_solve(A, b, steps: int = 2) -> np.ndarray:
    """LU solve followed by a few steps of FP64 iterative refinement, used
    where the reference must be tighter than one LU solve guarantees."""
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    x = lu.solve(b)
    for _ in range(steps):
        x = x + lu.solve(b - A @ x)
    return x
