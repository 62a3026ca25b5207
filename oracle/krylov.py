"""Outer Krylov solvers (oracle).

FGMRES(m) (Saad, Iterative Methods for Sparse Linear Systems, flexible GMRES
with right preconditioning): Arnoldi with classical Gram-Schmidt applied
twice, Givens rotations on the Hessenberg matrix, update x += Z y at the end
of each cycle.  Convergence is decided on the true FP64 residual
||b - A x||_2 <= tol ||b||_2, recomputed at every restart; the rotated
right-hand side |g_{j+1}| only ends a cycle early.

Mixed precision (iterative refinement): the preconditioner and the Arnoldi
product A z_j run in float32; the basis, Hessenberg matrix, rotations, x and
the restart residual stay FP64.  A cycle ends once the implicit estimate has
dropped by ``cycle_drop`` relative to its start (float32 cannot certify more
per cycle) or reached the target.

BiCGSTAB (van der Vorst), right-preconditioned, with a true-residual check
on exit and restart from the current iterate if the recursive residual has
drifted.

PD-GMRES (the outer solver of the paper's Sec. 5 setup and of every iterative
row of its Table 2; Cuevas Nunez, Schaerer, Bhaya, J. Comput. Appl. Math.
337, 2018): restarted FGMRES whose restart length is set before each cycle
by a proportional-derivative controller on the true residual norms at the
restarts.  The paper fixes m_init = m_min = 3 and m_step = 5 and takes the
other parameters from that publication, which is not at hand here; the
controller's form and its gains are a reading (``PDControl``), so the
restart-length sequence is parity unpinned beyond what the tests state.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List

import numpy as np


@dataclasses.dataclass
class KrylovResult:
    x: np.ndarray
    converged: bool
    iters: int
    restarts: int
    rel_res: float
    history: List[float]


def fgmres(A, b, M: Callable, tol: float = 1e-8, m: int = 30,
           maxit: int = 2000, x0=None, A_inner=None,
           inner_dtype=np.float64, cycle_drop: float = 0.0) -> KrylovResult:
    return _restarted(A, b, M, tol, lambda res: m, maxit, x0, A_inner, inner_dtype,
                      cycle_drop)[0]


def _restarted(A, b, M, tol, length, maxit, x0, A_inner, inner_dtype, cycle_drop):
    """Restarted FGMRES; length(res) gives the next cycle's restart length from
    the true residual norms at the restarts so far (res[-1] the newest).
    Returns the result and the cycle lengths used."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return KrylovResult(np.zeros(n), True, 0, 0, 0.0, [0.0]), []
    A_in = A if A_inner is None else A_inner
    target = tol * nb
    it = 0
    restarts = 0
    hist = []
    res = []
    lengths = []
    while True:
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        hist.append(beta / nb)
        res.append(beta)
        if beta <= target:
            return KrylovResult(x, True, it, restarts, beta / nb, hist), lengths
        if it >= maxit or not math.isfinite(beta):
            return KrylovResult(x, False, it, restarts, beta / nb, hist), lengths
        m = int(length(res))
        lengths.append(m)
        cycle_target = max(target, cycle_drop * beta)
        V = np.zeros((m + 1, n))
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = M(V[j].astype(inner_dtype))
            Z.append(z)
            w = np.asarray(A_in @ z, dtype=np.float64)
            # classical Gram-Schmidt, twice
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            H[:j + 1, j] = h + h2
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if hn == 0.0 or abs(g[j + 1]) <= cycle_target or it >= maxit:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x += y[i] * np.asarray(Z[i], dtype=np.float64)
        restarts += 1


@dataclasses.dataclass
class PDControl:
    """Restart-length controller of PD-GMRES (reading).  Before cycle j + 1,
    with r_j the true residual norm at restart j (r_0 at the start):

        m_{j+1} = m_j + floor(alpha_p r_j / r_{j-1}
                               + alpha_d (r_j - r_{j-2}) / (2 r_{j-1}))

    (the derivative term from the third restart on), the first cycle taking
    m_init.  When m_{j+1} falls below m_min, m_init grows by m_step and
    m_{j+1} = m_init.  Lengths are capped at m_max (the basis capacity).
    With the negative proportional gain the length shrinks while the
    residual falls and jumps back to a growing m_init, the cycling of
    restart lengths this family of methods uses against stagnation."""
    m_init: int = 3
    m_min: int = 3
    m_step: int = 5
    alpha_p: float = -3.0
    alpha_d: float = 5.0
    m_max: int = 60


def pd_lengths(ctl: PDControl):
    """The controller as a function of the residual history: length(res)
    for _restarted, keeping m_j and the grown m_init between calls."""
    state = {"m": None, "m_init": ctl.m_init}

    def length(res):
        if state["m"] is None:
            m = state["m_init"]
        else:
            rj, rj1 = res[-1], res[-2]
            d = ctl.alpha_p * rj / rj1
            if len(res) >= 3:
                d += ctl.alpha_d * (rj - res[-3]) / (2.0 * rj1)
            m = state["m"] + math.floor(d)
            if m < ctl.m_min:
                state["m_init"] += ctl.m_step
                m = state["m_init"]
        m = max(1, min(m, ctl.m_max))
        state["m"] = m
        return m

    return length


def pd_fgmres(A, b, M: Callable, tol: float = 1e-8, ctl: PDControl | None = None,
              maxit: int = 2000, x0=None):
    """PD-GMRES with the flexible (right-preconditioned) cycles of fgmres.
    Returns the result and the restart lengths of its cycles."""
    ctl = ctl or PDControl()
    return _restarted(A, b, M, tol, pd_lengths(ctl), maxit, x0, None, np.float64, 0.0)


def bicgstab(A, b, M: Callable, tol: float = 1e-8, maxit: int = 2000,
             x0=None) -> KrylovResult:
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return KrylovResult(np.zeros(n), True, 0, 0, 0.0, [0.0])
    target = tol * nb
    it = 0
    restarts = 0
    hist = []
    while True:
        r = b - A @ x
        rn = float(np.linalg.norm(r))
        hist.append(rn / nb)
        if rn <= target:
            return KrylovResult(x, True, it, restarts, rn / nb, hist)
        if it >= maxit or not math.isfinite(rn):
            return KrylovResult(x, False, it, restarts, rn / nb, hist)
        rhat = r.copy()
        rho = alpha = omega = 1.0
        v = np.zeros(n)
        pvec = np.zeros(n)
        while it < maxit:
            rho_new = float(rhat @ r)
            if rho_new == 0.0:
                break
            beta = (rho_new / rho) * (alpha / omega)
            pvec = r + beta * (pvec - omega * v)
            y = M(pvec)
            v = A @ y
            alpha = rho_new / float(rhat @ v)
            s = r - alpha * v
            x = x + alpha * y
            it += 1
            if float(np.linalg.norm(s)) <= target:
                break
            zs = M(s)
            t = A @ zs
            tt = float(t @ t)
            if tt == 0.0:
                break
            omega = float(t @ s) / tt
            x = x + omega * zs
            r = s - omega * t
            rho = rho_new
            if float(np.linalg.norm(r)) <= target or omega == 0.0:
                break
        restarts += 1


def least_squares_iterate(A, b, Z: np.ndarray, x0: np.ndarray) -> np.ndarray:
    """argmin over x0 + span(Z) of ||b - A x||_2 (dense, small problems)."""
    AZ = A @ Z
    y, *_ = np.linalg.lstsq(AZ, b - A @ x0, rcond=None)
    return x0 + Z @ y
