"""Pressure-velocity block preconditioners (oracle), Sec. 4 of the paper.

P_BJ(P_V, P_D')  = diag(P_V, X, P_D')
P_BGS(P_V, P_D') = [[P_V, 0, 0], [-X C P_V, X, 0], [-P_D' C1' P_V, 0, P_D']]

applied to a residual r = (r_v, r_p, r_pm):
  block-Jacobi:       y_v = P_V r_v,  y_p = X r_p,              y_pm = P_D' r_pm
  block-Gauss-Seidel: y_v = P_V r_v,  y_p = X (r_p - C y_v),    y_pm = P_D' (r_pm - C1' y_v)

P_V and P_D' are one AMG V-cycle each.  P_D' is built on the Darcy block as
the coupled system sees it, D~ = D' - C1' diag(V)^-1 B1': with no-flow outer
porous boundaries D' alone is singular (pure Neumann), while the coupled
matrix fixes the porous pressure through the interface; the correction adds
dx^2 / V_gg to the diagonal of each porous top cell (one interface face per
cell), evaluated as D[t,t] - (c1 * b1) / V[g,g].  X replaces the inverse of the zero
diagonal block: the paper's identity, or the inverse of a viscosity-scaled
pressure mass matrix, X = mu M_p^-1 with M_p = diag(dx dy) (the Schur
complement B^T V^-1 B is approximated by M_p / mu; with C = -B^T its sign is
positive).

Two-domain variants (Sec. 4, Table 2): with the free-flow block A' =
[[V, B], [C, 0]] preconditioned by one inexact Uzawa step (y_v = P_V r_v,
y_p = omega (r_p - C y_v), a Richardson step on the Schur complement
-C V^-1 B with omega = 1/lambda_max, lambda_max estimated by power
iteration on -C P_V B), P^td_BGS(P_A', P_D') coincides with the pv
block-Gauss-Seidel form with X = omega I, and P^td_BJ(P_A', P_D') =
diag(P_A', P_D') keeps the v -> p coupling inside A' but drops the porous
coupling C1' (y_pm = P_D' r_pm).

Darcy sub-solve P_D': one AMG V-cycle on D~ (default), or the ILU(0)
factorisation of D~ (forward and backward substitution, `oracle.ilu`), the
Darcy preconditioner of Table 2's P^td(Uzawa, ILU(0)) rows.

For the system of one backward-Euler step (mass |CV|/dt on the velocity
diagonal) M_p / mu only describes the Schur complement of the viscous part:
once sqrt(nu dt) is small against the domain, the mass term governs the
smooth pressure modes and FGMRES with X = mu M_p^-1 stalls.  The third choice
is the Cahouet-Chabard approximation (Cahouet & Chabard, "Some fast 3D finite
element solvers for the generalized Stokes problem", 1988), the sum of the
inverses of the viscous and the mass parts of the Schur complement:
X = mu M_p^-1 + L_p^-1 with L_p = B^T D^-1 B, D the velocity mass |CV|/dt on
the rows with a time derivative and V's own diagonal on the others (Gamma
and outflow faces, which have none); L_p^-1 is one AMG V-cycle.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import amg as amg_mod
from . import ilu as ilu_mod
from .assemble import Assembled

SCHUR_IDENTITY = "identity"
SCHUR_MASS = "mass"
SCHUR_CC = "cc"
SCHUR_UZAWA = "uzawa"
UZAWA_POWER_ITERS = 30
DARCY_AMG = "amg"
DARCY_ILU0 = "ilu0"


@dataclasses.dataclass
class BlockPreconditioner:
    variant: str               # "BJ" or "BGS"
    schur: str
    hV: amg_mod.Hierarchy
    hD: amg_mod.Hierarchy      # None when the Darcy block uses ILU(0)
    C: object                  # continuity rows x velocity columns
    C1: object                 # porous rows x velocity columns
    off: np.ndarray            # [0, off_v, off_p, off_q, N]
    xscale: float              # X = xscale * I (+ L_p^-1 with SCHUR_CC)
    dtype: type = np.float64
    hL: amg_mod.Hierarchy = None   # AMG hierarchy of L_p (SCHUR_CC only)
    ilu: ilu_mod.ILU0 = None       # ILU(0) of D~ (DARCY_ILU0 only)

    def __post_init__(self):
        dt = self.dtype
        self._C = self.C.astype(dt)
        self._C1 = self.C1.astype(dt)
        self._mV = amg_mod.level_mats(self.hV, dt)
        self._mD = None if self.hD is None else amg_mod.level_mats(self.hD, dt)
        self._mL = None if self.hL is None else amg_mod.level_mats(self.hL, dt)

    def middle(self, t: np.ndarray) -> np.ndarray:
        y = self.dtype(self.xscale) * t
        if self.hL is not None:
            y = y + amg_mod.vcycle(self.hL, t, self.dtype, mats=self._mL)
        return y

    def darcy(self, t: np.ndarray) -> np.ndarray:
        if self.ilu is not None:
            return self.ilu.solve(t).astype(self.dtype)
        return amg_mod.vcycle(self.hD, t, self.dtype, mats=self._mD)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        dt = self.dtype
        o = self.off
        r = r.astype(dt)
        rv, rp, rq = r[o[0]:o[2]], r[o[2]:o[3]], r[o[3]:o[4]]
        yv = amg_mod.vcycle(self.hV, rv, dt, mats=self._mV)
        if self.variant == "BJ":
            yp = self.middle(rp)
            yq = self.darcy(rq)
        elif self.variant == "TD_BJ":
            yp = self.middle(rp - self._C @ yv)
            yq = self.darcy(rq)
        elif self.variant in ("BGS", "TD_BGS"):
            yp = self.middle(rp - self._C @ yv)
            yq = self.darcy(rq - self._C1 @ yv)
        else:
            raise ValueError(self.variant)
        return np.concatenate([yv, yp, yq])


def velocity_components(a: Assembled) -> np.ndarray:
    """Component of every velocity unknown: 0 = u, 1 = v, 2 = w (3-D)."""
    o = a.layout.block_off
    comp = np.zeros(int(o[2]), dtype=np.int32)
    comp[o[1]:o[2]] = 1
    off_w = getattr(a.layout, "off_w", None)
    if off_w is not None:
        comp[off_w:o[2]] = 2
    return comp


def darcy_interface_block(blk) -> "sp.csr_matrix":
    """D~ = D' - C1' diag(V)^-1 B1' (diagonal correction on porous top cells)."""
    D = blk["D"].tocsr().copy()
    D.sort_indices()
    C1 = blk["C1"].tocsr()
    B1 = blk["B1"].tocsr()
    Vd = blk["V"].diagonal()
    for t in range(D.shape[0]):
        for kk in range(C1.indptr[t], C1.indptr[t + 1]):
            g = C1.indices[kk]
            c1 = C1.data[kk]
            for ll in range(B1.indptr[g], B1.indptr[g + 1]):
                tp = B1.indices[ll]
                b1 = B1.data[ll]
                pos = D.indptr[t] + np.searchsorted(D.indices[D.indptr[t]:D.indptr[t + 1]], tp)
                D.data[pos] = D.data[pos] - (c1 * b1) / Vd[g]
    return D


def pressure_operator(a: Assembled) -> "sp.csr_matrix":
    """L_p = B^T D^-1 B = -C D^-1 B on the free-flow pressure cells, with
    D = |CV|/dt on the velocity rows with a time derivative and diag(V) on the
    others.  Evaluated as ((-C) diag(1/D)) B."""
    if a.mass is None or not np.any(a.mass):
        raise ValueError("the Cahouet-Chabard middle block needs a backward-Euler system")
    blk = a.blocks()
    o = a.layout.block_off
    m = a.mass[o[0]:o[2]]
    Vd = blk["V"].diagonal()
    d = np.where(m != 0.0, m, Vd)
    C = blk["C"].tocsr()
    C.sort_indices()
    # (-C) diag(1/D), entry by entry, then the product with B: each entry of
    # L_p sums its terms in ascending velocity index
    X = sp.csr_matrix(((-C.data) * (1.0 / d)[C.indices], C.indices, C.indptr), shape=C.shape)
    L = (X @ blk["B"].tocsr()).tocsr()
    L.sort_indices()
    return L


def uzawa_relaxation(blk, hV, iters: int = UZAWA_POWER_ITERS) -> float:
    """omega = 1/lambda_max of the inexact Schur complement -C P_V B (P_V one
    V-cycle on V), lambda_max from `iters` power iterations started at the
    normalised ones vector: x <- y/||y|| with y = -C P_V B x, lambda = ||y||
    of the last step (Sec. 5: one Richardson iteration, its relaxation
    estimated by power iteration)."""
    B, C = blk["B"], blk["C"]
    n = B.shape[1]
    x = np.ones(n) / np.sqrt(n)
    lam = 1.0
    for _ in range(iters):
        y = -(C @ amg_mod.vcycle(hV, B @ x))
        lam = float(np.linalg.norm(y))
        x = y / lam
    return 1.0 / lam


def build(p, a: Assembled, variant: str = "BGS", schur: str = SCHUR_MASS,
          opts: amg_mod.AMGOptions | None = None, dtype=np.float64,
          darcy: str = DARCY_AMG) -> BlockPreconditioner:
    opts = opts or amg_mod.AMGOptions()
    blk = a.blocks()
    hV = amg_mod.setup(blk["V"], velocity_components(a), False, opts)
    Dt = darcy_interface_block(blk)
    hD, ilu = None, None
    if darcy == DARCY_ILU0:
        ilu = ilu_mod.ilu0(Dt)
    elif darcy == DARCY_AMG:
        hD = amg_mod.setup(Dt, np.zeros(Dt.shape[0], dtype=np.int32), False, opts)
    else:
        raise ValueError(darcy)
    vol = ((p.Lx / p.nx) * (p.H_ff / p.ny)) * p.dz     # dz = 1 in 2-D
    xscale = p.mu / vol if schur in (SCHUR_MASS, SCHUR_CC) else 1.0
    if variant in ("TD_BJ", "TD_BGS"):
        schur = SCHUR_UZAWA
        xscale = uzawa_relaxation(blk, hV)
    hL = None
    if schur == SCHUR_CC:
        Lp = pressure_operator(a)
        hL = amg_mod.setup(Lp, np.zeros(Lp.shape[0], dtype=np.int32), False, opts)
    return BlockPreconditioner(variant=variant, schur=schur, hV=hV, hD=hD,
                               C=blk["C"], C1=blk["C1"], off=a.layout.block_off,
                               xscale=xscale, dtype=dtype, hL=hL, ilu=ilu)


def exact_block_preconditioner(a: Assembled, variant: str, S_inv):
    """Block preconditioner with exact V^-1, D'^-1 (sparse LU) and a given
    middle-block operator S_inv; used to check the block algebra."""
    import scipy.sparse.linalg as spla
    blk = a.blocks()
    o = a.layout.block_off
    luV = spla.splu(blk["V"].tocsc())
    luD = spla.splu(blk["D"].tocsc())

    def apply(r):
        rv, rp, rq = r[o[0]:o[2]], r[o[2]:o[3]], r[o[3]:o[4]]
        yv = luV.solve(rv)
        if variant == "BJ":
            return np.concatenate([yv, S_inv(rp), luD.solve(rq)])
        return np.concatenate([yv, S_inv(rp - blk["C"] @ yv),
                               luD.solve(rq - blk["C1"] @ yv)])
    return apply
