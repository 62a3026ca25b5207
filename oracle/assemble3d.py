"""Three-dimensional assembly of the coupled Stokes-Darcy system (oracle).

Test infrastructure, like the rest of this package.

The model and the closures are those of ``oracle.assemble`` (Sec. 2 of the
paper: creeping Stokes flow in symmetric-gradient form on a staggered grid,
two-point-flux Darcy, normal-stress balance, Beavers-Joseph-Saffman slip and
normal mass-flux continuity on Gamma, optional backward-Euler mass), on a box
grid: x streamwise (nx cells), y normal to Gamma (ny free-flow and ny_pm
porous cells), z spanwise (nz cells).  Every row is "sum of outward momentum
or mass fluxes = source x |CV|" with face areas Ax = dy dz, Ay = dx dz,
Az = dx dy; with dz = 1 and no z faces the coefficients are those of the 2-D
assembly.  Additional closures in 3-D:

* w (z velocity) faces k = 1..nz-1 are unknowns; the z walls are velocity
  walls (data for u, v and the normal w), eliminated like every Dirichlet face;
* both tangential velocities obey BJS on Gamma: the south shear flux of a u
  face is g mu [(2 Ay/dy) u + dz (v_i - v_{i-1})] and that of a w face
  g mu [(2 Ay/dy) w + dx (v_k - v_{k-1})], g = beta/(beta + 2/dy),
  beta = alpha/sqrt(K_f), K_f the harmonic mean of the two porous top cells
  beside the face (along x for u, along z for w);
* Gamma rows Ay [p - 2 mu (v_1 - v_0)/dy - q_top + (mu/K_top)(dy_pm/2) v_0] = 0;
* porous cells: six two-point fluxes, interface flux Ay v_{i,0,k};
* full Beavers-Joseph (``bj_full``): as in 2-D, for u along x and for w
  along z (porous tangential velocity -(K_f/mu) dq/dz at a w face).

Unknown order (pv blocks): u (j, k, i), v (j, k, i), w (j, k, i), p (j, k, i),
q (j, k, i), the last index fastest.  Velocity block = u, v, w.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from sdinputs import BC_NOFLOW, BC_PRESSURE, BC_TRACTION, BC_VELOCITY, Problem


@dataclasses.dataclass
class Layout3:
    nx: int
    ny: int
    ny_pm: int
    nz: int
    nu_x: int

    @property
    def off_v(self):
        return self.nu_x * self.ny * self.nz

    @property
    def off_w(self):
        return self.off_v + self.nx * self.ny * self.nz

    @property
    def off_p(self):
        return self.off_w + self.nx * self.ny * (self.nz - 1)

    @property
    def off_q(self):
        return self.off_p + self.nx * self.ny * self.nz

    @property
    def N(self):
        return self.off_q + self.nx * self.ny_pm * self.nz

    @property
    def block_off(self):
        return np.array([0, self.off_v, self.off_p, self.off_q, self.N], dtype=np.int64)

    def u(self, i, j, k):
        return (j * self.nz + k) * self.nu_x + (i - 1)

    def v(self, i, j, k):
        return self.off_v + (j * self.nz + k) * self.nx + i

    def w(self, i, j, k):
        return self.off_w + (j * (self.nz - 1) + (k - 1)) * self.nx + i

    def p(self, i, j, k):
        return self.off_p + (j * self.nz + k) * self.nx + i

    def q(self, i, j, k):
        return self.off_q + (j * self.nz + k) * self.nx + i


@dataclasses.dataclass
class Assembled3:
    A: sp.csr_matrix
    b: np.ndarray
    layout: Layout3
    pm_singular: bool
    mass: np.ndarray

    @property
    def N(self):
        return self.layout.N

    def blocks(self):
        o = self.layout.block_off
        A = self.A
        s = lambda r0, r1, c0, c1: A[r0:r1, c0:c1].tocsr()
        return dict(V=s(o[0], o[2], o[0], o[2]), B=s(o[0], o[2], o[2], o[3]),
                    B1=s(o[0], o[2], o[3], o[4]), C=s(o[2], o[3], o[0], o[2]),
                    Z=s(o[2], o[3], o[2], o[3]), C1=s(o[3], o[4], o[0], o[2]),
                    Dz=s(o[3], o[4], o[2], o[3]), D=s(o[3], o[4], o[3], o[4]))


def _arr(a, shape):
    return np.zeros(shape) if a is None else np.asarray(a, dtype=np.float64).reshape(shape)


def layout3_of(p: Problem) -> Layout3:
    if p.nx < 2 or p.ny < 2 or p.ny_pm < 1 or p.nz < 1:
        raise ValueError("need nx >= 2, ny >= 2, ny_pm >= 1, nz >= 1")
    if p.ff_left != BC_VELOCITY or p.ff_top != BC_VELOCITY:
        raise ValueError("left and top free-flow boundaries must be velocity")
    if p.ff_right not in (BC_VELOCITY, BC_TRACTION):
        raise ValueError("right free-flow boundary: velocity or traction")
    nu_x = p.nx if p.ff_right == BC_TRACTION else p.nx - 1
    return Layout3(p.nx, p.ny, p.ny_pm, p.nz, nu_x)


def assemble3d(p: Problem) -> Assembled3:
    L = layout3_of(p)
    nx, ny, nyp, nz = p.nx, p.ny, p.ny_pm, p.nz
    mu, alpha = float(p.mu), float(p.alpha_bj)
    K = np.asarray(p.K, dtype=np.float64).reshape(nyp, nz, nx)
    if not np.all(np.isfinite(K)) or np.any(K <= 0):
        raise ValueError("K must be finite and positive")
    dx, dy, dyp, dz = p.Lx / nx, p.H_ff / ny, p.H_pm / nyp, p.Lz / nz
    dt = float(p.dt)
    if not (math.isfinite(dt) and dt >= 0.0):
        raise ValueError("dt must be finite and >= 0")
    Ax, Ay, Az = dy * dz, dx * dz, dx * dy
    vol = (dx * dy) * dz
    volp = (dx * dyp) * dz
    mvol = vol / dt if dt > 0.0 else 0.0
    # named coefficients (fixed evaluation order)
    cx = (2.0 * mu) * (Ax / dx)          # x normal stress (u rows)
    cy = mu * (Ay / dy)                  # y shear (u, w rows)
    cyt = mu * (Ay / (0.5 * dy))         # y shear at the top wall
    cz = mu * (Az / dz)                  # z shear (u, v rows)
    czt = mu * (Az / (0.5 * dz))         # z shear at a z wall
    cyy = (2.0 * mu) * (Ay / dy)         # y normal stress (v rows)
    cxv = mu * (Ax / dx)                 # x shear (v, w rows)
    cxw = mu * (Ax / (0.5 * dx))         # x shear at a side wall
    czz = (2.0 * mu) * (Az / dz)         # z normal stress (w rows)
    mdx, mdy, mdz = mu * dx, mu * dy, mu * dz
    right_tr = p.ff_right == BC_TRACTION

    uL = _arr(p.ff_left_n, (ny, nz))
    vL = _arr(p.ff_left_t, (ny + 1, nz))
    wL = _arr(p.ff_left_tz, (ny, nz + 1))
    uR = _arr(p.ff_right_n, (ny, nz))
    vR = _arr(p.ff_right_t, (ny + 1, nz))
    wR = _arr(p.ff_right_tz, (ny, nz + 1))
    uT = _arr(p.ff_top_t, (nz, nx + 1))
    vT = _arr(p.ff_top_n, (nz, nx))
    wT = _arr(p.ff_top_tz, (nz + 1, nx))
    uB = _arr(p.ff_back_u, (ny, nx + 1))
    vB = _arr(p.ff_back_v, (ny + 1, nx))
    wB = _arr(p.ff_back_n, (ny, nx))
    uF = _arr(p.ff_front_u, (ny, nx + 1))
    vF = _arr(p.ff_front_v, (ny + 1, nx))
    wF = _arr(p.ff_front_n, (ny, nx))
    pL = _arr(p.pm_left_p, (nyp, nz))
    pR = _arr(p.pm_right_p, (nyp, nz))
    pBo = _arr(p.pm_bottom_p, (nz, nx))
    pBk = _arr(p.pm_back_p, (nyp, nx))
    pFr = _arr(p.pm_front_p, (nyp, nx))
    fu = _arr(p.f_u, (ny, nz, nx + 1))
    fv = _arr(p.f_v, (ny + 1, nz, nx))
    fw = _arr(p.f_w, (ny, nz + 1, nx))
    fq = _arr(p.q_pm, (nyp, nz, nx))

    rows, cols, vals = [], [], []
    b = np.zeros(L.N)
    mass = np.zeros(L.N)

    def add(r, c, v, mask=None):
        r = np.asarray(r)
        c = np.broadcast_to(np.asarray(c), r.shape)
        v = np.broadcast_to(np.asarray(v, dtype=np.float64), r.shape)
        if mask is not None:
            r, c, v = r[mask], c[mask], v[mask]
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(v.ravel())

    def grid(a, b_, c):
        return np.meshgrid(a, b_, c, indexing="ij")

    def harm(a, c):
        return (2.0 * a * c) / (a + c)

    # ---------------- u rows, interior faces i = 1..nx-1 ----------------
    j, k, i = grid(np.arange(ny), np.arange(nz), np.arange(1, nx))
    r = L.u(i, j, k)
    top, gam = j == ny - 1, j == 0
    front, back = k == nz - 1, k == 0
    beta = alpha / np.sqrt(harm(K[nyp - 1, k, i - 1], K[nyp - 1, k, i]))
    g = beta / (beta + 2.0 / dy)
    cg = (g * mu) * ((2.0 * Ay) / dy)
    gm = (g * mu) * dz
    diag = ((((cx + cx) + np.where(top, cyt, cy)) + np.where(gam, cg, cy))
            + np.where(front, czt, cz)) + np.where(back, czt, cz)
    if dt > 0.0:
        diag = diag + mvol
        mass[r.ravel()] = mvol
    add(r, r, diag)
    add(r, L.u(i - 1, j, k), -cx, i - 1 >= 1)
    add(r, L.u(np.minimum(i + 1, L.nu_x), j, k), -cx, (i + 1 <= nx - 1) | right_tr)
    add(r, L.u(i, np.minimum(j + 1, ny - 1), k), -cy, ~top)
    add(r, L.u(i, np.maximum(j - 1, 0), k), -cy, ~gam)
    add(r, L.u(i, j, np.minimum(k + 1, nz - 1)), -cz, ~front)
    add(r, L.u(i, j, np.maximum(k - 1, 0)), -cz, ~back)
    jn = np.minimum(j + 1, ny - 1)
    add(r, L.v(i, jn, k), -mdz, ~top)
    add(r, L.v(i - 1, jn, k), mdz, ~top)
    add(r, L.v(i, j, k), np.where(gam, gm, mdz))
    add(r, L.v(i - 1, j, k), np.where(gam, -gm, -mdz))
    kf = np.clip(k + 1, 1, max(nz - 1, 1))
    kb = np.clip(k, 1, max(nz - 1, 1))
    add(r, L.w(i, j, kf), -mdy, ~front)
    add(r, L.w(i - 1, j, kf), mdy, ~front)
    add(r, L.w(i, j, kb), mdy, ~back)
    add(r, L.w(i - 1, j, kb), -mdy, ~back)
    add(r, L.p(i, j, k), Ax)
    add(r, L.p(i - 1, j, k), -Ax)
    if p.bj_full:          # porous tangential velocity in the slip condition
        Kf = harm(K[nyp - 1, k, i - 1], K[nyp - 1, k, i])
        cbj = cg * ((Kf / mu) / dx)
        add(r, L.q(i, nyp - 1, k), cbj, gam)
        add(r, L.q(i - 1, nyp - 1, k), -cbj, gam)
    rhs = fu[j, k, i] * vol
    rhs = np.where(i - 1 == 0, rhs + cx * uL[j, k], rhs)
    if not right_tr:
        rhs = np.where(i + 1 == nx, rhs + cx * uR[j, k], rhs)
    rhs = np.where(top, rhs + cyt * uT[k, i], rhs)
    rhs = np.where(top, rhs + mdz * (vT[k, np.minimum(i, nx - 1)] - vT[k, i - 1]), rhs)
    rhs = np.where(back, rhs + czt * uB[j, i], rhs)
    rhs = np.where(back, rhs - mdy * (wB[j, np.minimum(i, nx - 1)] - wB[j, i - 1]), rhs)
    rhs = np.where(front, rhs + czt * uF[j, i], rhs)
    rhs = np.where(front, rhs + mdy * (wF[j, np.minimum(i, nx - 1)] - wF[j, i - 1]), rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- u rows, outflow faces i = nx ----------------
    if right_tr:
        j, k = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
        r = L.u(nx, j, k)
        add(r, r, np.full(r.shape, cx))
        add(r, L.u(nx - 1, j, k), -cx)
        add(r, L.p(nx - 1, j, k), -Ax)
        b[r.ravel()] = ((-uR) * Ax).ravel()

    # ---------------- v rows, interior faces j = 1..ny-1 ----------------
    j, k, i = grid(np.arange(1, ny), np.arange(nz), np.arange(nx))
    r = L.v(i, j, k)
    west, east = i == 0, i == nx - 1
    front, back = k == nz - 1, k == 0
    aE = np.where(east, 0.0 if right_tr else cxw, cxv)
    aW = np.where(west, cxw, cxv)
    diag = ((((cyy + cyy) + aE) + aW) + np.where(front, czt, cz)) + np.where(back, czt, cz)
    if dt > 0.0:
        diag = diag + mvol
        mass[r.ravel()] = mvol
    add(r, r, diag)
    add(r, L.v(i, np.minimum(j + 1, ny - 1), k), -cyy, j + 1 <= ny - 1)
    add(r, L.v(i, j - 1, k), -cyy)
    add(r, L.v(np.minimum(i + 1, nx - 1), j, k), -cxv, ~east)
    add(r, L.v(np.maximum(i - 1, 0), j, k), -cxv, ~west)
    add(r, L.v(i, j, np.minimum(k + 1, nz - 1)), -cz, ~front)
    add(r, L.v(i, j, np.maximum(k - 1, 0)), -cz, ~back)
    e_unk = i + 1 <= nx - 1
    ie = np.clip(i + 1, 1, L.nu_x)
    add(r, L.u(ie, j, k), -mdz, e_unk)
    add(r, L.u(ie, j - 1, k), mdz, e_unk)
    iw = np.maximum(i, 1)
    add(r, L.u(iw, j, k), mdz, ~west)
    add(r, L.u(iw, j - 1, k), -mdz, ~west)
    add(r, L.w(i, j, kf := np.clip(k + 1, 1, max(nz - 1, 1))), -mdx, ~front)
    add(r, L.w(i, j - 1, kf), mdx, ~front)
    kb = np.clip(k, 1, max(nz - 1, 1))
    add(r, L.w(i, j, kb), mdx, ~back)
    add(r, L.w(i, j - 1, kb), -mdx, ~back)
    add(r, L.p(i, j, k), Ay)
    add(r, L.p(i, j - 1, k), -Ay)
    rhs = fv[j, k, i] * vol
    rhs = np.where(j + 1 == ny, rhs + cyy * vT[k, i], rhs)
    rhs = np.where(west, rhs + cxw * vL[j, k], rhs)
    rhs = np.where(west, rhs - mdz * (uL[j, k] - uL[j - 1, k]), rhs)
    if right_tr:
        rhs = np.where(east, rhs - vR[j, k] * Ax, rhs)
    else:
        rhs = np.where(east, rhs + cxw * vR[j, k], rhs)
        rhs = np.where(east, rhs + mdz * (uR[j, k] - uR[j - 1, k]), rhs)
    rhs = np.where(back, rhs + czt * vB[j, i], rhs)
    rhs = np.where(back, rhs - mdx * (wB[j, i] - wB[j - 1, i]), rhs)
    rhs = np.where(front, rhs + czt * vF[j, i], rhs)
    rhs = np.where(front, rhs + mdx * (wF[j, i] - wF[j - 1, i]), rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- Gamma rows (v_{i,0,k}) ----------------
    k, i = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    r = L.v(i, 0, k)
    dg = ((mu / K[nyp - 1, k, i]) * (0.5 * dyp)) * Ay
    add(r, r, cyy + dg)
    add(r, L.v(i, 1, k), -cyy)
    add(r, L.p(i, 0, k), Ay)
    add(r, L.q(i, nyp - 1, k), -Ay)
    b[r.ravel()] = 0.0

    # ---------------- w rows, interior faces k = 1..nz-1 ----------------
    if nz > 1:
        j, k, i = grid(np.arange(ny), np.arange(1, nz), np.arange(nx))
        r = L.w(i, j, k)
        west, east = i == 0, i == nx - 1
        top, gam = j == ny - 1, j == 0
        beta = alpha / np.sqrt(harm(K[nyp - 1, k - 1, i], K[nyp - 1, k, i]))
        g = beta / (beta + 2.0 / dy)
        cgw = (g * mu) * ((2.0 * Ay) / dy)
        gmw = (g * mu) * dx
        aE = np.where(east, 0.0 if right_tr else cxw, cxv)
        aW = np.where(west, cxw, cxv)
        diag = ((((czz + czz) + aE) + aW) + np.where(top, cyt, cy)) + np.where(gam, cgw, cy)
        if dt > 0.0:
            diag = diag + mvol
            mass[r.ravel()] = mvol
        add(r, r, diag)
        add(r, L.w(i, j, np.minimum(k + 1, nz - 1)), -czz, k + 1 <= nz - 1)
        add(r, L.w(i, j, np.maximum(k - 1, 1)), -czz, k - 1 >= 1)
        add(r, L.w(np.minimum(i + 1, nx - 1), j, k), -cxv, ~east)
        add(r, L.w(np.maximum(i - 1, 0), j, k), -cxv, ~west)
        add(r, L.w(i, np.minimum(j + 1, ny - 1), k), -cy, ~top)
        add(r, L.w(i, np.maximum(j - 1, 0), k), -cy, ~gam)
        e_unk = i + 1 <= nx - 1
        ie = np.clip(i + 1, 1, L.nu_x)
        add(r, L.u(ie, j, k), -mdy, e_unk)
        add(r, L.u(ie, j, k - 1), mdy, e_unk)
        iw = np.maximum(i, 1)
        add(r, L.u(iw, j, k), mdy, ~west)
        add(r, L.u(iw, j, k - 1), -mdy, ~west)
        jn = np.minimum(j + 1, ny - 1)
        add(r, L.v(i, jn, k), -mdx, ~top)
        add(r, L.v(i, jn, k - 1), mdx, ~top)
        add(r, L.v(i, j, k), np.where(gam, gmw, mdx))
        add(r, L.v(i, j, k - 1), np.where(gam, -gmw, -mdx))
        add(r, L.p(i, j, k), Az)
        add(r, L.p(i, j, k - 1), -Az)
        if p.bj_full:
            Kf = harm(K[nyp - 1, k - 1, i], K[nyp - 1, k, i])
            cbj = cgw * ((Kf / mu) / dz)
            add(r, L.q(i, nyp - 1, k), cbj, gam)
            add(r, L.q(i, nyp - 1, k - 1), -cbj, gam)
        rhs = fw[j, k, i] * vol
        rhs = np.where(k - 1 == 0, rhs + czz * wB[j, i], rhs)
        rhs = np.where(k + 1 == nz, rhs + czz * wF[j, i], rhs)
        rhs = np.where(top, rhs + cyt * wT[k, i], rhs)
        rhs = np.where(top, rhs + mdx * (vT[np.minimum(k, nz - 1), i] - vT[k - 1, i]), rhs)
        rhs = np.where(west, rhs + cxw * wL[j, k], rhs)
        rhs = np.where(west, rhs - mdy * (uL[j, np.minimum(k, nz - 1)] - uL[j, k - 1]), rhs)
        if right_tr:
            rhs = np.where(east, rhs - wR[j, k] * Ax, rhs)
        else:
            rhs = np.where(east, rhs + cxw * wR[j, k], rhs)
            rhs = np.where(east, rhs + mdy * (uR[j, np.minimum(k, nz - 1)] - uR[j, k - 1]), rhs)
        b[r.ravel()] = rhs.ravel()

    # ---------------- free-flow continuity ----------------
    j, k, i = grid(np.arange(ny), np.arange(nz), np.arange(nx))
    r = L.p(i, j, k)
    add(r, L.u(np.minimum(i + 1, L.nu_x), j, k), Ax, (i + 1 <= nx - 1) | right_tr)
    add(r, L.u(np.maximum(i, 1), j, k), -Ax, i >= 1)
    add(r, L.v(i, np.minimum(j + 1, ny - 1), k), Ay, j + 1 <= ny - 1)
    add(r, L.v(i, j, k), -Ay)
    add(r, L.w(i, j, np.clip(k + 1, 1, max(nz - 1, 1))), Az, k + 1 <= nz - 1)
    add(r, L.w(i, j, np.clip(k, 1, max(nz - 1, 1))), -Az, k >= 1)
    rhs = np.zeros(r.shape)
    rhs = np.where(i == 0, rhs + Ax * uL[j, k], rhs)
    if not right_tr:
        rhs = np.where(i + 1 == nx, rhs - Ax * uR[j, k], rhs)
    rhs = np.where(j + 1 == ny, rhs - Ay * vT[k, i], rhs)
    rhs = np.where(k == 0, rhs + Az * wB[j, i], rhs)
    rhs = np.where(k + 1 == nz, rhs - Az * wF[j, i], rhs)
    b[r.ravel()] = rhs.ravel()

    # ---------------- porous medium (TPFA, six faces) ----------------
    j, k, i = grid(np.arange(nyp), np.arange(nz), np.arange(nx))
    r = L.q(i, j, k)
    Kc = K[j, k, i]
    zero = np.zeros_like(Kc)
    Apx, Apy, Apz = dyp * dz, dx * dz, dx * dyp

    def t_int(area, d, Kn):
        return ((area / mu) * ((2.0 * Kc * Kn) / (Kc + Kn))) / d

    def t_dir(area, d):
        return ((area / mu) * Kc) / (0.5 * d)

    TE = np.where(i + 1 <= nx - 1, t_int(Apx, dx, K[j, k, np.minimum(i + 1, nx - 1)]),
                  t_dir(Apx, dx) if p.pm_right == BC_PRESSURE else zero)
    TW = np.where(i >= 1, t_int(Apx, dx, K[j, k, np.maximum(i - 1, 0)]),
                  t_dir(Apx, dx) if p.pm_left == BC_PRESSURE else zero)
    TN = np.where(j + 1 <= nyp - 1, t_int(Apy, dyp, K[np.minimum(j + 1, nyp - 1), k, i]), zero)
    TS = np.where(j >= 1, t_int(Apy, dyp, K[np.maximum(j - 1, 0), k, i]),
                  t_dir(Apy, dyp) if p.pm_bottom == BC_PRESSURE else zero)
    TF = np.where(k + 1 <= nz - 1, t_int(Apz, dz, K[j, np.minimum(k + 1, nz - 1), i]),
                  t_dir(Apz, dz) if p.pm_front == BC_PRESSURE else zero)
    TB = np.where(k >= 1, t_int(Apz, dz, K[j, np.maximum(k - 1, 0), i]),
                  t_dir(Apz, dz) if p.pm_back == BC_PRESSURE else zero)
    add(r, r, ((((TE + TW) + TN) + TS) + TF) + TB)
    add(r, L.q(np.minimum(i + 1, nx - 1), j, k), -TE, i + 1 <= nx - 1)
    add(r, L.q(np.maximum(i - 1, 0), j, k), -TW, i >= 1)
    add(r, L.q(i, np.minimum(j + 1, nyp - 1), k), -TN, j + 1 <= nyp - 1)
    add(r, L.q(i, np.maximum(j - 1, 0), k), -TS, j >= 1)
    add(r, L.q(i, j, np.minimum(k + 1, nz - 1)), -TF, k + 1 <= nz - 1)
    add(r, L.q(i, j, np.maximum(k - 1, 0)), -TB, k >= 1)
    add(r, L.v(i, 0, k), Ay, j == nyp - 1)
    rhs = fq[j, k, i] * volp
    if p.pm_right == BC_PRESSURE:
        rhs = np.where(i == nx - 1, rhs + TE * pR[j, k], rhs)
    if p.pm_left == BC_PRESSURE:
        rhs = np.where(i == 0, rhs + TW * pL[j, k], rhs)
    if p.pm_bottom == BC_PRESSURE:
        rhs = np.where(j == 0, rhs + TS * pBo[k, i], rhs)
    if p.pm_front == BC_PRESSURE:
        rhs = np.where(k == nz - 1, rhs + TF * pFr[j, i], rhs)
    if p.pm_back == BC_PRESSURE:
        rhs = np.where(k == 0, rhs + TB * pBk[j, i], rhs)
    b[r.ravel()] = rhs.ravel()

    R = np.concatenate(rows)
    C = np.concatenate(cols)
    V = np.concatenate(vals)
    key = R.astype(np.int64) * L.N + C
    if np.unique(key).size != key.size:
        raise AssertionError("duplicate matrix entry")
    A = sp.csr_matrix((V, (R, C)), shape=(L.N, L.N))
    A.sort_indices()
    pm_singular = all(t == BC_NOFLOW for t in (p.pm_left, p.pm_right, p.pm_bottom,
                                                p.pm_back, p.pm_front))
    return Assembled3(A=A, b=b, layout=L, pm_singular=pm_singular, mass=mass)


def split_solution3(x: np.ndarray, L: Layout3):
    """(u [ny, nz, nu_x], v [ny, nz, nx], w [ny, nz-1, nx], p [ny, nz, nx],
    q [ny_pm, nz, nx])."""
    return (x[:L.off_v].reshape(L.ny, L.nz, L.nu_x),
            x[L.off_v:L.off_w].reshape(L.ny, L.nz, L.nx),
            x[L.off_w:L.off_p].reshape(L.ny, L.nz - 1, L.nx),
            x[L.off_p:L.off_q].reshape(L.ny, L.nz, L.nx),
            x[L.off_q:].reshape(L.ny_pm, L.nz, L.nx))
