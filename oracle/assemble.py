"""Assembly of the monolithic coupled Stokes-Darcy system (oracle).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package; the library never does.

Follows Sec. 2 of the paper: creeping Stokes flow in symmetric
gradient form (momentum flux (pI - tau) n with tau = mu (grad v + grad v^T),
rho = 1), Darcy's law with continuity in the porous medium, and at the
interface the normal-stress balance, the Beavers-Joseph-Saffman slip
condition and normal mass-flux continuity.  Space discretisation as the paper
states it: staggered (MAC) finite volumes in the free flow, two-point flux
approximation in the porous medium.  The unknown ordering is the paper's
pressure-velocity (pv) block form [v^ff (u then v), p^ff, p^pm].

The paper leaves the discrete interface and boundary closures to its
references; this oracle fixes them as follows (every row is "sum of outward
momentum / mass fluxes = source x |CV|"):

* interior u and v rows: 11-point MAC stencil of div(-tau + pI);
* top wall: tangential shear over a half cell, normal wall velocity known;
* BJS slip at Gamma (u rows of the first free-flow row): the slip velocity is
  eliminated from u_s = (sqrt(K)/alpha)(du/dy + dv/dx) with du/dy taken over
  the half cell; the south shear flux becomes
  gamma mu [(2 dx/dy) u + (v_i - v_{i-1})], gamma = beta / (beta + 2/dy),
  beta = alpha/sqrt(K_f), K_f the harmonic mean of the two porous cells below;
* outflow (traction) u faces: n.(pI - tau)n evaluated at the last cell
  centre equals the prescribed flux;
* Gamma rows (one per interface face v_{i,0}): normal-stress balance with the
  Darcy pressure reconstructed at Gamma over the half porous cell,
  dx [p_{i,0} - 2 mu (v_{i,1} - v_{i,0})/dy - q_top + (mu/K_top)(dy_pm/2) v_{i,0}] = 0;
* mass-flux continuity: the porous top cell's outward interface flux is
  dx * v_{i,0}, the same unknown as the free-flow normal velocity;
* Dirichlet velocity faces are eliminated and lifted into b;
* full Beavers-Joseph (``Problem.bj_full``): the slip condition keeps the
  porous tangential velocity u_pm = -(K_f/mu)(q_i - q_{i-1})/dx at the face,
  so the south shear flux becomes g mu [(2 dx/dy)(u - u_pm) + (v_i - v_{i-1})]:
  the u rows of the first free-flow row couple to the two porous top cells
  below with +-cg (K_f/mu)/dx (the paper's experiments use BJS);
* time (dt > 0): the transient momentum equation of Sec. 2 with the paper's
  first-order backward Euler step.  A momentum row integrates dv/dt over its
  control volume, which adds |CV|/dt to the diagonal of every interior u and
  v face row (rho = 1); b then holds the data part only, and one step's
  right-hand side adds (|CV|/dt) v^n on those rows (``oracle.transient``).
  The outflow u rows and the Gamma rows are boundary and interface
  conditions, not momentum balances of a control volume, and the Darcy
  equations carry no storage term, so none of these rows gets one.

Floating-point evaluation order of every coefficient is fixed (see the
named coefficients below); the assembled values are reproducible bit-for-bit
by any implementation that evaluates the same expressions in IEEE double
without contraction.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from sdinputs import (BC_NOFLOW, BC_PRESSURE, BC_TRACTION, BC_VELOCITY,
                      Problem)


@dataclasses.dataclass
class Layout:
    """Unknown index maps.  u faces i = i_first..i_last per free-flow row j
    (i_first = 0 with a traction left boundary, 1 otherwise; i_last = nx with
    a traction right boundary, nx - 1 otherwise; nu_x of them); v faces: the
    n_gamma interface faces first (free-flow columns i0..i0+nx_pm-1 of row
    j = 0, over the porous block), then rows j = 1..ny-1; p cells; porous
    cells q (nx_pm columns, row k = 0 at the bottom).  With the porous block
    as wide as the free flow this is the plain (row j, column i) order."""

    nx: int
    ny: int
    ny_pm: int
    nu_x: int
    nx_pm: int = 0
    i0: int = 0
    i_first: int = 1

    def __post_init__(self):
        if self.nx_pm == 0:
            self.nx_pm = self.nx

    @property
    def n_gamma(self):
        return self.nx_pm

    @property
    def off_u(self):
        return 0

    @property
    def off_v(self):
        return self.nu_x * self.ny

    @property
    def off_p(self):
        return self.off_v + self.n_gamma + self.nx * (self.ny - 1)

    @property
    def off_q(self):
        return self.off_p + self.nx * self.ny

    @property
    def N(self):
        return self.off_q + self.nx_pm * self.ny_pm

    @property
    def block_off(self):
        return np.array([0, self.off_v, self.off_p, self.off_q, self.N],
                        dtype=np.int64)

    def u(self, i, j):
        return self.off_u + j * self.nu_x + (i - self.i_first)

    def v(self, i, j):
        """v face (i, j); for j = 0 only the interface faces are unknowns."""
        return np.where(np.asarray(j) == 0, self.off_v + (np.asarray(i) - self.i0),
                        self.off_v + self.n_gamma + (np.asarray(j) - 1) * self.nx
                        + np.asarray(i))

    def p(self, i, j):
        return self.off_p + j * self.nx + i

    def q(self, i, k):
        """Porous cell of porous column i (0..nx_pm-1) and row k."""
        return self.off_q + k * self.nx_pm + i

    def over(self, i):
        """Free-flow column i lies over the porous block."""
        i = np.asarray(i)
        return (i >= self.i0) & (i < self.i0 + self.nx_pm)


def all_faces_dof(nx: int, ny: int, ny_pm: int) -> int:
    """Degrees of freedom when every face and cell is an unknown (Dirichlet
    faces kept), the count of Table 1: u (nx+1) ny + v nx (ny+1) + p + q."""
    return (nx + 1) * ny + nx * (ny + 1) + nx * ny + nx * ny_pm


def layout_of(p: Problem) -> Layout:
    if p.nx < 2 or p.ny < 2 or p.ny_pm < 1:
        raise ValueError("need nx >= 2, ny >= 2, ny_pm >= 1")
    if p.ff_top != BC_VELOCITY:
        raise ValueError("the top free-flow boundary must be velocity")
    for side in (p.ff_left, p.ff_right):
        if side not in (BC_VELOCITY, BC_TRACTION):
            raise ValueError("left/right free-flow boundaries: velocity or traction")
    nx_pm = p.nx_pm or p.nx
    if nx_pm < 1 or p.pm_i0 < 0 or p.pm_i0 + nx_pm > p.nx:
        raise ValueError("the porous block must lie under the free flow")
    i_first = 0 if p.ff_left == BC_TRACTION else 1
    i_last = p.nx if p.ff_right == BC_TRACTION else p.nx - 1
    return Layout(p.nx, p.ny, p.ny_pm, i_last - i_first + 1, nx_pm, p.pm_i0, i_first)


def _arr(a, n):
    return np.zeros(n) if a is None else np.asarray(a, dtype=np.float64).reshape(n)


@dataclasses.dataclass
class Assembled:
    A: sp.csr_matrix
    b: np.ndarray
    layout: Layout
    pm_singular: bool          # D' has the constant vector in its kernel
    mass: np.ndarray = None    # |CV|/dt on the rows with a time derivative

    @property
    def N(self):
        return self.layout.N

    def blocks(self):
        """pv blocks of eq. (pressure-velocity form): V, B, B1', C, C1', D'."""
        o = self.layout.block_off
        A = self.A
        s = lambda r0, r1, c0, c1: A[r0:r1, c0:c1].tocsr()
        return dict(V=s(o[0], o[2], o[0], o[2]), B=s(o[0], o[2], o[2], o[3]),
                    B1=s(o[0], o[2], o[3], o[4]), C=s(o[2], o[3], o[0], o[2]),
                    Z=s(o[2], o[3], o[2], o[3]), C1=s(o[3], o[4], o[0], o[2]),
                    Dz=s(o[3], o[4], o[2], o[3]), D=s(o[3], o[4], o[3], o[4]))


def assemble(p: Problem) -> Assembled:
    L = layout_of(p)
    nx, ny, nyp = p.nx, p.ny, p.ny_pm
    npm, i0 = L.nx_pm, L.i0
    mu, alpha = float(p.mu), float(p.alpha_bj)
    K = np.asarray(p.K, dtype=np.float64).reshape(nyp, npm)
    if not np.all(np.isfinite(K)) or np.any(K <= 0):
        raise ValueError("K must be finite and positive")
    dx = p.Lx / nx
    dy = p.H_ff / ny
    dyp = p.H_pm / nyp
    vol = dx * dy
    volp = dx * dyp
    dt = float(p.dt)
    if not (math.isfinite(dt) and dt >= 0.0):
        raise ValueError("dt must be finite and >= 0")
    mvol = vol / dt if dt > 0.0 else 0.0   # backward-Euler mass coefficient
    mass = np.zeros(L.N)
    # named coefficients (fixed evaluation order)
    cx = (2.0 * mu) * (dy / dx)          # u rows, normal stress E/W
    cy = mu * (dx / dy)                  # u rows, shear N/S
    cyt = mu * (dx / (0.5 * dy))         # u rows, shear at the top wall
    cyy = (2.0 * mu) * (dx / dy)         # v rows, normal stress N/S
    cxv = mu * (dy / dx)                 # v rows, shear E/W
    cxw = mu * (dy / (0.5 * dx))         # v rows, shear at a side wall
    right_tr = p.ff_right == BC_TRACTION
    left_tr = p.ff_left == BC_TRACTION

    uL = _arr(p.ff_left_n, ny)
    vL = _arr(p.ff_left_t, ny + 1)
    uR = _arr(p.ff_right_n, ny)
    vR = _arr(p.ff_right_t, ny + 1)
    uT = _arr(p.ff_top_t, nx + 1)
    vT = _arr(p.ff_top_n, nx)
    pL = _arr(p.pm_left_p, nyp)
    pR = _arr(p.pm_right_p, nyp)
    pB = _arr(p.pm_bottom_p, npm)
    fu = _arr(p.f_u, (ny, nx + 1))
    fv = _arr(p.f_v, (ny + 1, nx))
    fq = _arr(p.q_pm, (nyp, npm))

    rows, cols, vals = [], [], []
    b = np.zeros(L.N)

    def add(r, c, v, mask=None):
        r = np.asarray(r)
        c = np.broadcast_to(np.asarray(c), r.shape)
        v = np.broadcast_to(np.asarray(v, dtype=np.float64), r.shape)
        if mask is not None:
            r, c, v = r[mask], c[mask], v[mask]
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(v.ravel())

    # ---------------- u rows, interior faces i = 1..nx-1 ----------------
    j, i = np.meshgrid(np.arange(ny), np.arange(1, nx), indexing="ij")
    r = L.u(i, j)
    top = j == ny - 1
    bot = j == 0
    # faces of the first row whose two cells lie over the porous block obey
    # BJS; the others meet the bottom wall (no slip over half a cell)
    gam = bot & L.over(i - 1) & L.over(i)
    # BJS factor per face (harmonic mean of the two porous top cells below)
    Ka = K[nyp - 1, np.clip(i - 1 - i0, 0, npm - 1)]
    Kb = K[nyp - 1, np.clip(i - i0, 0, npm - 1)]
    Kf = (2.0 * Ka * Kb) / (Ka + Kb)
    beta = alpha / np.sqrt(Kf)
    g = beta / (beta + 2.0 / dy)
    cg = (g * mu) * ((2.0 * dx) / dy)
    gm = g * mu
    aN = np.where(top, cyt, cy)
    aS = np.where(gam, cg, np.where(bot, cyt, cy))
    diag = ((cx + cx) + aN) + aS
    if dt > 0.0:
        diag = diag + mvol
        mass[r.ravel()] = mvol
    add(r, r, diag)
    add(r, L.u(i - 1, j), -cx, (i - 1 >= 1) | left_tr)
    east_unknown = (i + 1 <= nx - 1) | right_tr
    add(r, L.u(np.minimum(i + 1, L.nu_x), j), -cx, east_unknown)
    add(r, L.u(i, np.minimum(j + 1, ny - 1)), -cy, ~top)
    add(r, L.u(i, np.maximum(j - 1, 0)), -cy, ~bot)
    # shear cross terms: -mu[(v_{i,j+1} - v_{i-1,j+1}) - (v_{i,j} - v_{i-1,j})]
    jn = np.minimum(j + 1, ny - 1)
    add(r, L.v(i, jn), -mu, ~top)
    add(r, L.v(i - 1, jn), mu, ~top)
    # the first row's bottom v faces are interface unknowns or wall (zero)
    add(r, L.v(i, j), np.where(gam, gm, mu), ~bot | L.over(i))
    add(r, L.v(i - 1, j), np.where(gam, -gm, -mu), ~bot | L.over(i - 1))
    add(r, L.p(i, j), dy)
    add(r, L.p(i - 1, j), -dy)
    if p.bj_full:
        cbj = cg * ((Kf / mu) / dx)
        add(r, L.q(np.clip(i - i0, 0, npm - 1), nyp - 1), cbj, gam)
        add(r, L.q(np.clip(i - 1 - i0, 0, npm - 1), nyp - 1), -cbj, gam)
    rhs = fu[j, i] * vol
    if not left_tr:
        rhs = np.where(i - 1 == 0, rhs + cx * uL[j], rhs)
    if not right_tr:
        rhs = np.where(i + 1 == nx, rhs + cx * uR[j], rhs)
    rhs = np.where(top, rhs + cyt * uT[i], rhs)
    rhs = np.where(top, rhs + mu * (vT[np.minimum(i, nx - 1)] - vT[i - 1]), rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- u rows, traction faces i = 0 (inflow side) -------------
    # n.(pI - tau)n at the first cell centre equals the datum (pressure-driven
    # inflow: the datum is the prescribed pressure)
    if left_tr:
        jj = np.arange(ny)
        r = L.u(0, jj)
        add(r, r, np.full(ny, cx))
        add(r, L.u(1, jj), -cx)
        add(r, L.p(0, jj), dy)
        b[r] = uL * dy

    # ---------------- u rows, outflow faces i = nx ----------------
    if right_tr:
        jj = np.arange(ny)
        r = L.u(nx, jj)
        add(r, r, np.full(ny, cx))
        add(r, L.u(nx - 1, jj), -cx)
        add(r, L.p(nx - 1, jj), -dy)
        b[r] = (-uR) * dy

    # ---------------- v rows, interior faces j = 1..ny-1 ----------------
    j, i = np.meshgrid(np.arange(1, ny), np.arange(nx), indexing="ij")
    r = L.v(i, j)
    west = i == 0
    east = i == nx - 1
    aE = np.where(east, 0.0 if right_tr else cxw, cxv)
    aW = np.where(west, 0.0 if left_tr else cxw, cxv)
    diag = ((cyy + cyy) + aE) + aW
    if dt > 0.0:
        diag = diag + mvol
        mass[r.ravel()] = mvol
    add(r, r, diag)
    add(r, L.v(i, np.minimum(j + 1, ny - 1)), -cyy, j + 1 <= ny - 1)
    add(r, L.v(i, j - 1), -cyy, (j - 1 >= 1) | L.over(i))   # wall faces are zero
    add(r, L.v(np.minimum(i + 1, nx - 1), j), -cxv, ~east)
    add(r, L.v(np.maximum(i - 1, 0), j), -cxv, ~west)
    # shear cross terms: -mu[(u_{i+1,j} - u_{i+1,j-1}) - (u_{i,j} - u_{i,j-1})]
    e_unk = (i + 1 <= nx - 1)            # east u face is an interior unknown
    ie = np.clip(i + 1, 1, L.nu_x)
    add(r, L.u(ie, j), -mu, e_unk)
    add(r, L.u(ie, j - 1), mu, e_unk)
    iw = np.maximum(i, 1)
    add(r, L.u(iw, j), mu, ~west)
    add(r, L.u(iw, j - 1), -mu, ~west)
    add(r, L.p(i, j), dx)
    add(r, L.p(i, j - 1), -dx)
    rhs = fv[j, i] * vol
    rhs = np.where(j + 1 == ny, rhs + cyy * vT[i], rhs)
    if left_tr:
        rhs = np.where(west, rhs - vL[j] * dy, rhs)
    else:
        rhs = np.where(west, rhs + cxw * vL[j], rhs)
        rhs = np.where(west, rhs - mu * (uL[j] - uL[j - 1]), rhs)
    if right_tr:
        rhs = np.where(east, rhs - vR[j] * dy, rhs)
    else:
        rhs = np.where(east, rhs + cxw * vR[j], rhs)
        rhs = np.where(east, rhs + mu * (uR[j] - uR[j - 1]), rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- Gamma rows (v_{i,0}) ----------------
    i = np.arange(i0, i0 + npm)
    r = L.v(i, 0)
    Kt = K[nyp - 1, i - i0]
    dg = ((mu / Kt) * (0.5 * dyp)) * dx
    add(r, r, cyy + dg)
    add(r, L.v(i, 1), -cyy)
    add(r, L.p(i, 0), dx)
    add(r, L.q(i - i0, nyp - 1), -dx)
    b[r] = 0.0

    # ---------------- free-flow continuity ----------------
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = L.p(i, j)
    e_unk = (i + 1 <= nx - 1) | right_tr
    add(r, L.u(np.minimum(i + 1, L.nu_x), j), dy, e_unk)
    add(r, L.u(np.maximum(i, L.i_first), j), -dy, (i >= 1) | left_tr)
    add(r, L.v(i, np.minimum(j + 1, ny - 1)), dx, j + 1 <= ny - 1)
    add(r, L.v(i, j), -dx, (j >= 1) | L.over(i))
    rhs = np.zeros_like(r, dtype=np.float64)
    if not left_tr:
        rhs = np.where(i == 0, rhs + dy * uL[j], rhs)
    if not right_tr:
        rhs = np.where(i + 1 == nx, rhs - dy * uR[j], rhs)
    rhs = np.where(j + 1 == ny, rhs - dx * vT[i], rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- porous medium (TPFA) ----------------
    k, i = np.meshgrid(np.arange(nyp), np.arange(npm), indexing="ij")
    r = L.q(i, k)
    Kc = K[k, i]

    def t_int(area, d, Kn):
        return ((area / mu) * ((2.0 * Kc * Kn) / (Kc + Kn))) / d

    def t_dir(area, d):
        return ((area / mu) * Kc) / (0.5 * d)

    zero = np.zeros_like(Kc)
    TE = np.where(i + 1 <= npm - 1, t_int(dyp, dx, K[k, np.minimum(i + 1, npm - 1)]),
                  t_dir(dyp, dx) if p.pm_right == BC_PRESSURE else zero)
    TW = np.where(i >= 1, t_int(dyp, dx, K[k, np.maximum(i - 1, 0)]),
                  t_dir(dyp, dx) if p.pm_left == BC_PRESSURE else zero)
    TN = np.where(k + 1 <= nyp - 1, t_int(dx, dyp, K[np.minimum(k + 1, nyp - 1), i]), zero)
    TS = np.where(k >= 1, t_int(dx, dyp, K[np.maximum(k - 1, 0), i]),
                  t_dir(dx, dyp) if p.pm_bottom == BC_PRESSURE else zero)
    add(r, r, ((TE + TW) + TN) + TS)
    add(r, L.q(np.minimum(i + 1, npm - 1), k), -TE, i + 1 <= npm - 1)
    add(r, L.q(np.maximum(i - 1, 0), k), -TW, i >= 1)
    add(r, L.q(i, np.minimum(k + 1, nyp - 1)), -TN, k + 1 <= nyp - 1)
    add(r, L.q(i, np.maximum(k - 1, 0)), -TS, k >= 1)
    add(r, L.v(i + i0, 0), dx, k == nyp - 1)
    rhs = fq[k, i] * volp
    if p.pm_right == BC_PRESSURE:
        rhs = np.where(i == npm - 1, rhs + TE * pR[k], rhs)
    if p.pm_left == BC_PRESSURE:
        rhs = np.where(i == 0, rhs + TW * pL[k], rhs)
    if p.pm_bottom == BC_PRESSURE:
        rhs = np.where(k == 0, rhs + TS * pB[i], rhs)
    b[r.ravel()] = rhs.ravel()

    R = np.concatenate(rows)
    C = np.concatenate(cols)
    Vv = np.concatenate(vals)
    # every (row, col) pair is produced once; no duplicate summation happens
    key = R.astype(np.int64) * L.N + C
    if np.unique(key).size != key.size:
        raise AssertionError("duplicate matrix entry")
    A = sp.csr_matrix((Vv, (R, C)), shape=(L.N, L.N))
    A.sort_indices()
    pm_singular = (p.pm_left == BC_NOFLOW and p.pm_right == BC_NOFLOW
                   and p.pm_bottom == BC_NOFLOW)
    return Assembled(A=A, b=b, layout=L, pm_singular=pm_singular, mass=mass)


def split_solution(x: np.ndarray, L: Layout):
    """Return (u [ny, nu_x], v [ny, nx], p [ny, nx], q [ny_pm, nx_pm]); the
    bottom wall faces of v (outside the porous block) are zero."""
    o = L.block_off
    v = np.zeros((L.ny, L.nx))
    v[0, L.i0:L.i0 + L.nx_pm] = x[o[1]:o[1] + L.n_gamma]
    v[1:] = x[o[1] + L.n_gamma:o[2]].reshape(L.ny - 1, L.nx)
    return (x[o[0]:o[1]].reshape(L.ny, L.nu_x), v,
            x[o[2]:o[3]].reshape(L.ny, L.nx), x[o[3]:o[4]].reshape(L.ny_pm, L.nx_pm))
