"""Backward-Euler time stepping of the coupled system (oracle).

Test infrastructure, like the rest of this package.

The free flow obeys the transient Stokes equations and the porous medium the
stationary Darcy equations (Sec. 2); the paper advances them with a
first-order backward Euler step and solves one monolithic linear system per
step.  With the system matrix assembled for a step dt (``assemble`` with
``Problem.dt > 0``: |CV|/dt on the diagonal of every interior velocity row),
step n -> n+1 solves

    A x^{n+1} = b^{n+1} + M x^n,    M = diag(|CV|/dt on those rows, 0 elsewhere),

where b^{n+1} holds the boundary data and sources at t_{n+1}.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from .assemble import Assembled
from .direct import solve as lu_solve


def step_rhs(a: Assembled, b_data: np.ndarray, x_prev: np.ndarray) -> np.ndarray:
    """b^{n+1} + M x^n: the data part plus the previous velocity times
    |CV|/dt, one product and one sum per row with a time derivative; the
    other rows are the data part unchanged."""
    if a.mass is None:
        raise ValueError("problem was assembled without a time step")
    has = a.mass != 0.0
    return np.where(has, b_data + a.mass * x_prev, b_data)


def backward_euler(a: Assembled, x0: np.ndarray, n_steps: int,
                   b_data: Optional[Callable[[int], np.ndarray]] = None,
                   solve: Callable = None) -> list:
    """Advance ``n_steps`` steps from x0.  ``b_data(n)`` gives the data part
    of step n's right-hand side (n = 1..n_steps; default: the assembled b,
    constant in time); ``solve(A, rhs)`` the linear solve (default: sparse
    LU).  Returns the iterates x^1..x^n."""
    solve = solve or (lambda A, r: lu_solve(A, r))
    x = np.asarray(x0, dtype=np.float64)
    out = []
    for n in range(1, n_steps + 1):
        bd = a.b if b_data is None else b_data(n)
        x = solve(a.A, step_rhs(a, bd, x))
        out.append(x)
    return out
