"""Partitioned Dirichlet-Neumann coupling (oracle), Sec. 3 of the paper.

Serial implicit coupling: the free-flow solver S_ff maps the interface
normal velocity v^Gamma (Dirichlet data for the free flow) to the interface
normal stress sigma = p - 2 mu dv/dy (the free-flow side of the normal-stress
balance); the porous-medium solver S_pm takes sigma as the interface
pressure, closed over the half porous cell by Darcy's law, and returns the
interface normal velocity.  The coupling iterates the fixed-point problem
S_pm(S_ff(v)) = v with a post-processing step -- Aitken's dynamic
relaxation, or the paper's choice, the interface quasi-Newton method with an
inverse Jacobian from a least-squares fit of the input/output history
(IQN-ILS, Degroote, Bathe, Vierendeels 2009) -- and stops with the paper's
two relative convergence measures on the interface pressure and velocity.
At the fixed point every interface row of the monolithic system holds, so
the result equals the monolithic solution.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from sdinputs import Problem

from .assemble import Assembled


@dataclasses.dataclass
class DNResult:
    x: np.ndarray              # monolithic ordering
    iters: int
    converged: bool
    history: list


def subsolvers(p: Problem, a: Assembled):
    """The two subdomain solution operators of the coupling (sparse LU of each
    subdomain system, factorised here once) and the map back to the
    monolithic ordering: S_ff(v) -> (sigma, x_ff), S_pm(sigma) -> (vt, q),
    to_mono(x_ff, v, q)."""
    L = a.layout
    nx, nyp, npm, i0 = L.nx, L.ny_pm, L.nx_pm, L.i0
    A = a.A.tocsr()
    N = L.N
    cols = np.arange(i0, i0 + npm)                    # free-flow columns over the block
    gam = L.v(cols, 0)                                # interface v unknowns
    ff = np.arange(L.off_q)
    ff_int = np.setdiff1d(ff, gam)                    # free-flow unknowns/rows
    pm = np.arange(L.off_q, N)
    A_ff = A[ff_int][:, ff_int].tocsc()
    A_ffg = A[ff_int][:, gam].tocsr()
    lu_ff = spla.splu(A_ff)
    b_ff = a.b[ff_int]

    dy = p.H_ff / p.ny
    dyp = p.H_pm / nyp
    dx = p.Lx / nx
    K = np.asarray(p.K, dtype=np.float64).reshape(nyp, npm)
    Kt = K[nyp - 1, :]
    mu = p.mu
    top = L.q(np.arange(npm), nyp - 1) - L.off_q
    TB = dx * Kt / (mu * 0.5 * dyp)                   # half-cell Darcy transmissibility
    D = A[pm][:, pm].tocsr()
    D = (D + sp.csr_matrix((TB, (top, top)), shape=D.shape)).tocsc()
    lu_pm = spla.splu(D)
    b_pm = a.b[pm]
    pos = {int(g): k for k, g in enumerate(ff_int)}
    ip0 = np.array([pos[int(L.p(i, 0))] for i in cols])
    iv1 = np.array([pos[int(L.v(i, 1))] for i in cols])

    def S_ff(vg):
        x = lu_ff.solve(b_ff - A_ffg @ vg)
        sigma = x[ip0] - 2.0 * mu * (x[iv1] - vg) / dy
        return sigma, x

    def S_pm(sigma):
        rhs = b_pm.copy()
        rhs[top] += TB * sigma
        q = lu_pm.solve(rhs)
        vg = (Kt / mu) * (q[top] - sigma) / (0.5 * dyp)
        return vg, q

    def to_monolithic(x_ff, vg, q):
        x = np.zeros(N)
        x[ff_int] = x_ff
        x[gam] = vg
        x[pm] = q
        return x

    return S_ff, S_pm, to_monolithic


def solve_dn(p: Problem, a: Assembled, eps: float = 1e-10, maxit: int = 500,
             omega0: float = 0.5, accel: str = "aitken", subs=None) -> DNResult:
    """Dirichlet-Neumann fixed point with Aitken relaxation (accel="aitken")
    or IQN-ILS post-processing (accel="iqn-ils").  Iteration k maps the
    interface velocity v_k to sigma_k = S_ff(v_k) and vt_k = S_pm(sigma_k),
    r_k = vt_k - v_k, and stops once both relative measures of Sec. 3 hold:
    ||sigma_k - sigma_{k-1}|| < eps ||sigma_k|| and ||r_k|| < eps ||vt_k||."""
    S_ff, S_pm, to_mono = subs if subs is not None else subsolvers(p, a)
    nx = a.layout.n_gamma
    v = np.zeros(nx)
    sigma_old = None
    r_old = None
    omega = omega0
    hist = []
    x_ff = q = None
    R_hist, Vt_hist = [], []          # IQN-ILS: residuals and outputs so far
    for k in range(1, maxit + 1):
        sigma, x_ff = S_ff(v)
        vt, q = S_pm(sigma)
        r = vt - v
        dp = np.inf if sigma_old is None else np.linalg.norm(sigma - sigma_old)
        ok_p = dp < eps * np.linalg.norm(sigma)
        ok_v = np.linalg.norm(r) < eps * np.linalg.norm(vt)
        hist.append((float(dp), float(np.linalg.norm(r))))
        if ok_p and ok_v:
            return DNResult(to_mono(x_ff, v, q), k, True, hist)
        if accel == "aitken":
            if r_old is not None:
                dr = r - r_old
                den = float(dr @ dr)
                # Aitken's update; a step that left the residual unchanged gives
                # no secant information, so the initial relaxation is restored
                omega = -omega * float(r_old @ dr) / den if den > 0 else omega0
            v = v + omega * r
        elif accel == "iqn-ils":
            v = _iqn_ils_step(v, vt, r, R_hist, Vt_hist, omega0)
        else:
            raise ValueError(accel)
        r_old = r
        sigma_old = sigma
    return DNResult(to_mono(x_ff, v, q), maxit, False, hist)


def _iqn_ils_step(v, vt, r, R_hist, Vt_hist, omega0):
    """One IQN-ILS update.  With the history of residuals r_i and outputs
    vt_i, the columns dR_i = r_{i+1} - r_i and dVt_i = vt_{i+1} - vt_i are
    secant pairs of the inverse Jacobian; the coefficients c minimise
    ||dR c + r_k|| (the residual change that would cancel r_k, in the span of
    the observed changes) and the next input is vt_k + dVt c.  The first
    iteration, without history, relaxes with omega0."""
    R_hist.append(r.copy())
    Vt_hist.append(vt.copy())
    if len(R_hist) == 1:
        return v + omega0 * r
    dR = np.column_stack([R_hist[i + 1] - R_hist[i] for i in range(len(R_hist) - 1)])
    dV = np.column_stack([Vt_hist[i + 1] - Vt_hist[i] for i in range(len(Vt_hist) - 1)])
    c = np.linalg.lstsq(dR, -r, rcond=1e-12)[0]
    return vt + dV @ c


def solve_interface_gmres(p: Problem, a: Assembled, tol: float = 1e-14) -> np.ndarray:
    """The fixed-point residual R(v) = S_pm(S_ff(v)) - v is affine in v; its
    root is found here by dense Newton (one linear solve with the exactly
    assembled interface Jacobian), an alternative route to the same fixed
    point used as a cross-check of the Aitken iteration."""
    S_ff, S_pm, to_mono = subsolvers(p, a)
    nx = a.layout.n_gamma

    def R(v):
        return S_pm(S_ff(v)[0])[0] - v

    r0 = R(np.zeros(nx))
    J = np.empty((nx, nx))
    for k in range(nx):
        e = np.zeros(nx)
        e[k] = 1.0
        J[:, k] = R(e) - r0
    v = np.linalg.solve(J, -r0)
    sigma, x_ff = S_ff(v)
    vt, q = S_pm(sigma)
    return to_mono(x_ff, v, q)
