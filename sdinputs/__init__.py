"""Seeded synthetic inputs for the coupled Stokes-Darcy solver.

This module is shared by the CPU oracle, the tests and the benchmark.  It
produces *inputs only* -- grids, permeability fields, boundary data, forcing
terms sampled from a manufactured solution and request traces -- and holds
none of the solver's arithmetic (no discretisation, no linear algebra).

Geometry (Sec. 2 of the paper, model problem): the porous medium occupies
[0, Lx] x [0, H_pm], the free flow [0, Lx] x [H_pm, H_pm + H_ff]; the
interface Gamma is the line y = H_pm.  Both subdomains have nx cell columns
(conforming at Gamma); the free flow has ny cell rows, the porous medium
ny_pm.  Staggered free-flow unknowns: u on vertical faces (x = i dx,
y = y_G + (j + 1/2) dy), v on horizontal faces (x = (i + 1/2) dx,
y = y_G + j dy), p at cell centres; porous-medium pressures q at cell centres.
Arrays are stored row-major with the row index counted from the bottom.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BC_VELOCITY = "velocity"
BC_TRACTION = "traction"
BC_PRESSURE = "pressure"
BC_NOFLOW = "noflow"


@dataclasses.dataclass
class Problem:
    """Everything that defines one coupled solve: a stationary problem, or
    (dt > 0) the linear system of one backward-Euler time step, whose
    right-hand side the data below give without the previous-step term.

    Boundary data conventions (all optional, ``None`` means zero):
      ff_left_n  [ny]     normal velocity u at the left faces (x = 0)
      ff_left_t  [ny+1]   tangential velocity v on the left wall at y_G + j dy
      ff_right_n [ny]     velocity u (velocity BC) or normal momentum flux
                          n.(pI - tau)n (traction BC) at x = Lx
      ff_right_t [ny+1]   velocity v (velocity BC) or tangential momentum
                          flux t.(pI - tau)n (traction BC) at x = Lx, y_G + j dy
      ff_top_t   [nx+1]   tangential velocity u on the top wall at x = i dx
      ff_top_n   [nx]     normal velocity v on the top wall
      pm_left_p/pm_right_p [ny_pm], pm_bottom_p [nx]  Dirichlet pressures
    Forcing: f_u [ny, nx+1] at u faces, f_v [ny+1, nx] at v faces,
    q_pm [ny_pm, nx] volumetric source at porous-medium cell centres.
    """

    nx: int
    ny: int
    ny_pm: int
    Lx: float = 1.0
    H_ff: float = 0.5
    H_pm: float = 0.5
    mu: float = 1.0
    alpha_bj: float = 1.0
    K: Optional[np.ndarray] = None          # [ny_pm, nx]
    ff_left: str = BC_VELOCITY
    ff_right: str = BC_TRACTION
    ff_top: str = BC_VELOCITY
    pm_left: str = BC_NOFLOW
    pm_right: str = BC_NOFLOW
    pm_bottom: str = BC_NOFLOW
    ff_left_n: Optional[np.ndarray] = None
    ff_left_t: Optional[np.ndarray] = None
    ff_right_n: Optional[np.ndarray] = None
    ff_right_t: Optional[np.ndarray] = None
    ff_top_t: Optional[np.ndarray] = None
    ff_top_n: Optional[np.ndarray] = None
    pm_left_p: Optional[np.ndarray] = None
    pm_right_p: Optional[np.ndarray] = None
    pm_bottom_p: Optional[np.ndarray] = None
    f_u: Optional[np.ndarray] = None
    f_v: Optional[np.ndarray] = None
    q_pm: Optional[np.ndarray] = None
    dt: float = 0.0                          # backward-Euler step, 0 = stationary
    bj_full: bool = False                    # slip with the porous tangential velocity
    # ---- porous block narrower than the free flow (2-D) ----
    nx_pm: int = 0                           # porous columns (0 = nx)
    pm_i0: int = 0                           # first free-flow column over the block
    # ---- third dimension (nz = 0: the 2-D problem above) ----
    nz: int = 0                              # spanwise cells (z), both subdomains
    Lz: float = 1.0
    pm_back: str = BC_NOFLOW                 # porous sides z = 0 / z = Lz
    pm_front: str = BC_NOFLOW
    ff_left_tz: Optional[np.ndarray] = None   # w on the left wall [ny, nz+1]
    ff_right_tz: Optional[np.ndarray] = None  # w or t_z.(pI - tau)n at x = Lx [ny, nz+1]
    ff_top_tz: Optional[np.ndarray] = None    # w on the top wall [nz+1, nx]
    ff_back_u: Optional[np.ndarray] = None    # wall z = 0: u [ny, nx+1], v [ny+1, nx],
    ff_back_v: Optional[np.ndarray] = None    #   normal w [ny, nx]
    ff_back_n: Optional[np.ndarray] = None
    ff_front_u: Optional[np.ndarray] = None   # wall z = Lz: same shapes
    ff_front_v: Optional[np.ndarray] = None
    ff_front_n: Optional[np.ndarray] = None
    pm_back_p: Optional[np.ndarray] = None    # [ny_pm, nx]
    pm_front_p: Optional[np.ndarray] = None
    f_w: Optional[np.ndarray] = None          # [ny, nz+1, nx]

    @property
    def dx(self) -> float:
        return self.Lx / self.nx

    @property
    def dy(self) -> float:
        return self.H_ff / self.ny

    @property
    def dy_pm(self) -> float:
        return self.H_pm / self.ny_pm

    @property
    def y_gamma(self) -> float:
        return self.H_pm

    @property
    def dz(self) -> float:
        return self.Lz / self.nz if self.nz > 0 else 1.0


# ----------------------------------------------------------------------------
# Face / cell coordinates
# ----------------------------------------------------------------------------

def u_face_xy(p: Problem):
    """Coordinates of all u faces, arrays of shape [ny, nx+1]."""
    x = np.arange(p.nx + 1) * p.dx
    y = p.y_gamma + (np.arange(p.ny) + 0.5) * p.dy
    return np.meshgrid(x, y)


def v_face_xy(p: Problem):
    """Coordinates of all v faces, arrays of shape [ny+1, nx]."""
    x = (np.arange(p.nx) + 0.5) * p.dx
    y = p.y_gamma + np.arange(p.ny + 1) * p.dy
    return np.meshgrid(x, y)


def ff_cell_xy(p: Problem):
    x = (np.arange(p.nx) + 0.5) * p.dx
    y = p.y_gamma + (np.arange(p.ny) + 0.5) * p.dy
    return np.meshgrid(x, y)


def pm_cell_xy(p: Problem):
    x = (np.arange(p.nx) + 0.5) * p.dx
    y = (np.arange(p.ny_pm) + 0.5) * p.dy_pm
    return np.meshgrid(x, y)


def u_face_xyz(p: Problem):
    """3-D: coordinates of all u faces, arrays of shape [ny, nz, nx+1]."""
    y = p.y_gamma + (np.arange(p.ny) + 0.5) * p.dy
    z = (np.arange(p.nz) + 0.5) * p.dz
    x = np.arange(p.nx + 1) * p.dx
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


def v_face_xyz(p: Problem):
    """3-D: all v faces, [ny+1, nz, nx]."""
    y = p.y_gamma + np.arange(p.ny + 1) * p.dy
    z = (np.arange(p.nz) + 0.5) * p.dz
    x = (np.arange(p.nx) + 0.5) * p.dx
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


def w_face_xyz(p: Problem):
    """3-D: all w faces, [ny, nz+1, nx]."""
    y = p.y_gamma + (np.arange(p.ny) + 0.5) * p.dy
    z = np.arange(p.nz + 1) * p.dz
    x = (np.arange(p.nx) + 0.5) * p.dx
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


def ff_cell_xyz(p: Problem):
    """3-D: free-flow cell centres, [ny, nz, nx]."""
    y = p.y_gamma + (np.arange(p.ny) + 0.5) * p.dy
    z = (np.arange(p.nz) + 0.5) * p.dz
    x = (np.arange(p.nx) + 0.5) * p.dx
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


def pm_cell_xyz(p: Problem):
    """3-D: porous cell centres, [ny_pm, nz, nx]."""
    y = (np.arange(p.ny_pm) + 0.5) * p.dy_pm
    z = (np.arange(p.nz) + 0.5) * p.dz
    x = (np.arange(p.nx) + 0.5) * p.dx
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


# ----------------------------------------------------------------------------
# Permeability fields
# ----------------------------------------------------------------------------

def lognormal_K(nx: int, ny_pm: int, K_geo: float, sigma: float,
                corr_cells: float, seed: int, nz: Optional[int] = None) -> np.ndarray:
    """ln K ~ N(ln K_geo, sigma^2) per cell with a Gaussian-smoothed
    correlation: iid N(0,1) (PCG64 from ``seed``), Gaussian filter with a
    standard deviation of ``corr_cells`` cells (reflecting borders, truncated
    at 4 sigma), re-standardised to zero mean and unit variance.  With ``nz``
    the field is 3-D, shape [ny_pm, nz, nx]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny_pm, nx) if nz is None else (ny_pm, nz, nx))
    if corr_cells > 0:
        z = gaussian_filter(z, sigma=corr_cells, mode="reflect", truncate=4.0)
    z = (z - z.mean()) / z.std()
    return np.exp(math.log(K_geo) + sigma * z)


# ----------------------------------------------------------------------------
# Manufactured solution (satisfies the three interface conditions exactly)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class MMS:
    """Stream function psi = -sin(pi x) h(s)/pi with s = y - y_G,
    u = d psi/dy, v = -d psi/dx; free-flow pressure cos(pi x)(Q0 + s);
    porous-medium pressure y cos(pi x).  h = h0 + h1 s + s^2 with
    h0 = -K/mu (normal mass flux continuity), h1 = (sqrt(K)/alpha)(2 + pi^2 h0)
    (Beavers-Joseph-Saffman slip) and Q0 = y_G + 2 mu h1 (normal stress
    balance).  Valid for constant K.  With bj_full the slip condition keeps
    the porous tangential velocity -(K/mu) dP/dx (full Beavers-Joseph), and
    h1 = (sqrt(K)/alpha)(2 + pi^2 h0) - (K/mu) pi^2 y_G."""

    K: float
    mu: float
    alpha: float
    y_gamma: float
    bj_full: bool = False

    @property
    def h0(self):
        return -self.K / self.mu

    @property
    def h1(self):
        h1 = math.sqrt(self.K) / self.alpha * (2.0 + math.pi ** 2 * self.h0)
        if self.bj_full:
            h1 -= self.K / self.mu * math.pi ** 2 * self.y_gamma
        return h1

    @property
    def Q0(self):
        return self.y_gamma + 2.0 * self.mu * self.h1

    def h(self, s):
        return self.h0 + self.h1 * s + s * s

    def dh(self, s):
        return self.h1 + 2.0 * s

    def u(self, x, y):
        s = y - self.y_gamma
        return -np.sin(np.pi * x) * self.dh(s) / np.pi

    def v(self, x, y):
        s = y - self.y_gamma
        return np.cos(np.pi * x) * self.h(s)

    def p(self, x, y):
        s = y - self.y_gamma
        return np.cos(np.pi * x) * (self.Q0 + s)

    def P(self, x, y):
        return y * np.cos(np.pi * x)

    def f_x(self, x, y):
        s = y - self.y_gamma
        return (-self.mu * np.pi * np.sin(np.pi * x) * self.dh(s)
                - np.pi * np.sin(np.pi * x) * (self.Q0 + s))

    def f_y(self, x, y):
        s = y - self.y_gamma
        return (-self.mu * np.cos(np.pi * x) * (2.0 - np.pi ** 2 * self.h(s))
                + np.cos(np.pi * x))

    def s_pm(self, x, y):
        return self.K / self.mu * np.pi ** 2 * y * np.cos(np.pi * x)

    def flux_n(self, x, y):
        """n.(pI - tau)n on a boundary with outward normal (1, 0)."""
        s = y - self.y_gamma
        return np.cos(np.pi * x) * (self.Q0 + s + 2.0 * self.mu * self.dh(s))

    def flux_t(self, x, y):
        """t.(pI - tau)n on a boundary with outward normal (1, 0)."""
        s = y - self.y_gamma
        return self.mu * np.sin(np.pi * x) * (2.0 / np.pi + np.pi * self.h(s))


def mms_problem(nx: int, ny: int, ny_pm: Optional[int] = None, K: float = 1e-2,
                mu: float = 1.0, alpha: float = 1.0, Lx: float = 1.0,
                H_ff: float = 0.5, H_pm: float = 0.5,
                bj_full: bool = False) -> tuple[Problem, MMS]:
    """Manufactured-solution problem: free-flow velocity given on the left and
    top, momentum flux (traction) on the right, Dirichlet pressure on the three
    outer porous-medium sides; bj_full: the full Beavers-Joseph variant."""
    ny_pm = ny if ny_pm is None else ny_pm
    p = Problem(nx=nx, ny=ny, ny_pm=ny_pm, Lx=Lx, H_ff=H_ff, H_pm=H_pm, mu=mu,
                alpha_bj=alpha, K=np.full((ny_pm, nx), K),
                ff_left=BC_VELOCITY, ff_right=BC_TRACTION, ff_top=BC_VELOCITY,
                pm_left=BC_PRESSURE, pm_right=BC_PRESSURE, pm_bottom=BC_PRESSURE,
                bj_full=bj_full)
    m = MMS(K=K, mu=mu, alpha=alpha, y_gamma=H_pm, bj_full=bj_full)
    yc = p.y_gamma + (np.arange(ny) + 0.5) * p.dy
    yv = p.y_gamma + np.arange(ny + 1) * p.dy
    xu = np.arange(nx + 1) * p.dx
    xv = (np.arange(nx) + 0.5) * p.dx
    ytop = p.y_gamma + H_ff
    ypm = (np.arange(ny_pm) + 0.5) * p.dy_pm
    p.ff_left_n = m.u(0.0, yc)
    p.ff_left_t = m.v(0.0, yv)
    p.ff_right_n = m.flux_n(Lx, yc)
    p.ff_right_t = m.flux_t(Lx, yv)
    p.ff_top_t = m.u(xu, ytop)
    p.ff_top_n = m.v(xv, ytop)
    p.pm_left_p = m.P(0.0, ypm)
    p.pm_right_p = m.P(Lx, ypm)
    p.pm_bottom_p = m.P(xv, 0.0)
    xu2, yu2 = u_face_xy(p)
    xv2, yv2 = v_face_xy(p)
    xq, yq = pm_cell_xy(p)
    p.f_u = m.f_x(xu2, yu2)
    p.f_v = m.f_y(xv2, yv2)
    p.q_pm = m.s_pm(xq, yq)
    return p, m


def mms_transient_problem(nx: int, ny: int, dt: float, t: float, g, dg,
                          **kw) -> tuple[Problem, MMS]:
    """Time-scaled manufactured solution (u, v, p, P)(x, y, t) =
    g(t) (u, v, p, P)(x, y) at time ``t``: the boundary data and the porous
    source of ``mms_problem`` times g(t); the free-flow forcing times g(t) plus
    dg(t) (u, v), the velocity's time derivative (the porous medium has no
    storage term).  ``dt`` is the step the matrix is assembled for."""
    p, m = mms_problem(nx, ny, **kw)
    gt, dgt = float(g(t)), float(dg(t))
    for name in ("ff_left_n", "ff_left_t", "ff_right_n", "ff_right_t",
                 "ff_top_t", "ff_top_n", "pm_left_p", "pm_right_p",
                 "pm_bottom_p", "q_pm"):
        setattr(p, name, gt * getattr(p, name))
    xu, yu = u_face_xy(p)
    xv, yv = v_face_xy(p)
    p.f_u = gt * p.f_u + dgt * m.u(xu, yu)
    p.f_v = gt * p.f_v + dgt * m.v(xv, yv)
    p.dt = float(dt)
    return p, m


# ----------------------------------------------------------------------------
# Channel flow over a heterogeneous porous bed
# ----------------------------------------------------------------------------

def channel_problem(nx: int, ny: int, ny_pm: Optional[int] = None, *,
                    mu: float = 1e-3, K_geo: float = 1e-4, sigma: float = 1.0,
                    corr_cells: float = 8.0, seed: int = 1, U: float = 1e-2,
                    alpha: float = 1.0, Lx: float = 1.0,
                    H_ff: float = 0.5, H_pm: float = 0.5) -> Problem:
    """Parabolic inflow of peak ``U`` on the free-flow left side, zero
    traction on the right, no-slip top, no-flow on every outer porous side;
    lognormal permeability."""
    ny_pm = ny if ny_pm is None else ny_pm
    K = lognormal_K(nx, ny_pm, K_geo, sigma, corr_cells, seed)
    p = Problem(nx=nx, ny=ny, ny_pm=ny_pm, Lx=Lx, H_ff=H_ff, H_pm=H_pm, mu=mu,
                alpha_bj=alpha, K=K, ff_left=BC_VELOCITY, ff_right=BC_TRACTION,
                ff_top=BC_VELOCITY, pm_left=BC_NOFLOW, pm_right=BC_NOFLOW,
                pm_bottom=BC_NOFLOW)
    yc = p.y_gamma + (np.arange(ny) + 0.5) * p.dy
    ytop = p.y_gamma + H_ff
    p.ff_left_n = 4.0 * U * (yc - p.y_gamma) * (ytop - yc) / (H_ff * H_ff)
    return p


# ----------------------------------------------------------------------------
# Three dimensions: x streamwise, y normal to Gamma, z spanwise
# ----------------------------------------------------------------------------

def mms3d_problem(nx: int, ny: int, nz: int, plane: str = "xy",
                  K: float = 1e-2, mu: float = 1.0, alpha: float = 1.0) -> tuple[Problem, MMS]:
    """3-D manufactured solution made of the 2-D one of ``MMS``.  plane "xy":
    (u, v, p, P) = MMS(x, y) and w = 0, constant in z; plane "zy": the same
    solution turned into the (z, y) plane, u = 0, v = MMS.v(z, y),
    w = MMS.u(z, y), p = MMS.p(z, y), P = MMS.P(z, y), constant in x.  Both
    meet the three interface conditions (BJS on u and on w).  Unit box
    [0,1] x [0,1] x [0,1] with Gamma at y = 1/2; free-flow velocity data on the
    left, top and both z walls, traction on the right, Dirichlet pressure on
    every outer porous side."""
    p = Problem(nx=nx, ny=ny, ny_pm=ny, nz=nz, Lx=1.0, H_ff=0.5, H_pm=0.5, Lz=1.0, mu=mu,
                alpha_bj=alpha, K=np.full((ny, nz, nx), K), ff_left=BC_VELOCITY,
                ff_right=BC_TRACTION, ff_top=BC_VELOCITY, pm_left=BC_PRESSURE,
                pm_right=BC_PRESSURE, pm_bottom=BC_PRESSURE, pm_back=BC_PRESSURE,
                pm_front=BC_PRESSURE)
    m = MMS(K=K, mu=mu, alpha=alpha, y_gamma=0.5)
    if plane == "xy":
        U = lambda x, y, z: m.u(x, y) + np.zeros(np.broadcast(x, y, z).shape)
        V = lambda x, y, z: m.v(x, y) + np.zeros(np.broadcast(x, y, z).shape)
        W = lambda x, y, z: np.zeros(np.broadcast(x, y, z).shape)
        Pf = lambda x, y, z: m.p(x, y) + np.zeros(np.broadcast(x, y, z).shape)
        Pm = lambda x, y, z: m.P(x, y) + np.zeros(np.broadcast(x, y, z).shape)
        Fx = lambda x, y, z: m.f_x(x, y)
        Fy = lambda x, y, z: m.f_y(x, y)
        Fz = lambda x, y, z: np.zeros(np.broadcast(x, y, z).shape)
        S = lambda x, y, z: m.s_pm(x, y)
        Tn = lambda y, z: m.flux_n(1.0, y) + np.zeros(np.broadcast(y, z).shape)
        Tt = lambda y, z: m.flux_t(1.0, y) + np.zeros(np.broadcast(y, z).shape)
        Tz = lambda y, z: np.zeros(np.broadcast(y, z).shape)
    elif plane == "zy":
        U = lambda x, y, z: np.zeros(np.broadcast(x, y, z).shape)
        V = lambda x, y, z: m.v(z, y) + np.zeros(np.broadcast(x, y, z).shape)
        W = lambda x, y, z: m.u(z, y) + np.zeros(np.broadcast(x, y, z).shape)
        Pf = lambda x, y, z: m.p(z, y) + np.zeros(np.broadcast(x, y, z).shape)
        Pm = lambda x, y, z: m.P(z, y) + np.zeros(np.broadcast(x, y, z).shape)
        Fx = lambda x, y, z: np.zeros(np.broadcast(x, y, z).shape)
        Fy = lambda x, y, z: m.f_y(z, y)
        Fz = lambda x, y, z: m.f_x(z, y)
        S = lambda x, y, z: m.s_pm(z, y)
        Tn = lambda y, z: m.p(z, y)           # n.(pI - tau)n with u = 0, d/dx = 0
        Tt = lambda y, z: np.zeros(np.broadcast(y, z).shape)
        Tz = lambda y, z: np.zeros(np.broadcast(y, z).shape)
    else:
        raise ValueError(plane)
    dx, dy, dz, yg = p.dx, p.dy, p.dz, 0.5
    yc = yg + (np.arange(ny) + 0.5) * dy
    yv = yg + np.arange(ny + 1) * dy
    zc = (np.arange(nz) + 0.5) * dz
    zw = np.arange(nz + 1) * dz
    xu = np.arange(nx + 1) * dx
    xc = (np.arange(nx) + 0.5) * dx
    ytop = yg + 0.5
    ypm = (np.arange(ny) + 0.5) * p.dy_pm
    g2 = lambda a, b: np.meshgrid(a, b, indexing="ij")
    Y, Z = g2(yc, zc)
    p.ff_left_n = U(0.0, Y, Z)
    Y, Z = g2(yv, zc)
    p.ff_left_t = V(0.0, Y, Z)
    p.ff_right_t = Tt(Y, Z)
    Y, Z = g2(yc, zw)
    p.ff_left_tz = W(0.0, Y, Z)
    p.ff_right_tz = Tz(Y, Z)
    Y, Z = g2(yc, zc)
    p.ff_right_n = Tn(Y, Z)
    Z, X = g2(zc, xu)
    p.ff_top_t = U(X, ytop, Z)
    Z, X = g2(zc, xc)
    p.ff_top_n = V(X, ytop, Z)
    Z, X = g2(zw, xc)
    p.ff_top_tz = W(X, ytop, Z)
    for zval, tag in ((0.0, "back"), (1.0, "front")):
        Y, X = g2(yc, xu)
        setattr(p, f"ff_{tag}_u", U(X, Y, zval))
        Y, X = g2(yv, xc)
        setattr(p, f"ff_{tag}_v", V(X, Y, zval))
        Y, X = g2(yc, xc)
        setattr(p, f"ff_{tag}_n", W(X, Y, zval))
        Y, X = g2(ypm, xc)
        setattr(p, f"pm_{tag}_p", Pm(X, Y, zval))
    Y, Z = g2(ypm, zc)
    p.pm_left_p = Pm(0.0, Y, Z)
    p.pm_right_p = Pm(1.0, Y, Z)
    Z, X = g2(zc, xc)
    p.pm_bottom_p = Pm(X, 0.0, Z)
    X, Y, Z = u_face_xyz(p)
    p.f_u = Fx(X, Y, Z)
    X, Y, Z = v_face_xyz(p)
    p.f_v = Fy(X, Y, Z)
    X, Y, Z = w_face_xyz(p)
    p.f_w = Fz(X, Y, Z)
    X, Y, Z = pm_cell_xyz(p)
    p.q_pm = S(X, Y, Z)
    ex = dict(u=U, v=V, w=W, p=Pf, P=Pm)
    return p, ex


def channel3d_problem(nx: int, ny: int, nz: int, ny_pm: Optional[int] = None, *,
                      mu: float = 1e-3, K_geo: float = 1e-4, sigma: float = 1.0,
                      corr_cells: float = 6.0, seed: int = 4, U: float = 1e-2,
                      alpha: float = 1.0, Lx: float = 1.0, H_ff: float = 0.5,
                      H_pm: float = 0.5, Lz: float = 1.0) -> Problem:
    """3-D channel over a porous bed: inflow u = 16 U s (H - s) z (Lz - z) /
    (H^2 Lz^2) on the left (s = y - y_G), zero traction on the right, no-slip
    top and z walls, no-flow on every outer porous side, lognormal K."""
    ny_pm = ny if ny_pm is None else ny_pm
    K = lognormal_K(nx, ny_pm, K_geo, sigma, corr_cells, seed, nz=nz)
    p = Problem(nx=nx, ny=ny, ny_pm=ny_pm, nz=nz, Lx=Lx, H_ff=H_ff, H_pm=H_pm, Lz=Lz,
                mu=mu, alpha_bj=alpha, K=K, ff_left=BC_VELOCITY, ff_right=BC_TRACTION,
                ff_top=BC_VELOCITY, pm_left=BC_NOFLOW, pm_right=BC_NOFLOW,
                pm_bottom=BC_NOFLOW, pm_back=BC_NOFLOW, pm_front=BC_NOFLOW)
    s = (np.arange(ny) + 0.5) * p.dy
    z = (np.arange(nz) + 0.5) * p.dz
    S, Z = np.meshgrid(s, z, indexing="ij")
    p.ff_left_n = 16.0 * U * S * (H_ff - S) * Z * (Lz - Z) / (H_ff * H_ff * Lz * Lz)
    return p


def paper_setup_problem(n: int, p_in: float = 0.0, *, K: float = 1e-6, mu: float = 1e-3,
                        alpha: float = 1.0, dt: float = 2e5) -> Problem:
    """The geometry of the paper's experiments (Sec. 5): a 3 x 1 free-flow
    channel [0,3] x [1,2] over a 1 x 1 porous block [1,2] x [0,1] under its
    middle third, n x n cells per unit square; pressure p_in on the left and 0
    on the right of the channel (traction data: the normal momentum flux equals
    the pressure, no tangential traction), no-slip top and bottom walls beside
    the block, p = 0 at the bottom of the block and no flow through its sides;
    constant K; one backward-Euler step of dt."""
    p = Problem(nx=3 * n, ny=n, ny_pm=n, Lx=3.0, H_ff=1.0, H_pm=1.0, mu=mu, alpha_bj=alpha,
                K=np.full((n, n), K), ff_left=BC_TRACTION, ff_right=BC_TRACTION,
                ff_top=BC_VELOCITY, pm_left=BC_NOFLOW, pm_right=BC_NOFLOW,
                pm_bottom=BC_PRESSURE, nx_pm=n, pm_i0=n, dt=dt)
    p.ff_left_n = np.full(n, float(p_in))
    return p


def paper_inflow_pressure(t: float, t_end: float = 50e5, dp_max: float = 1e-9) -> float:
    """Half-cosine pressure difference rising from 0 at t = 0 to dp_max at
    t_end: dp_max (1 - cos(pi t / t_end)) / 2."""
    return dp_max * 0.5 * (1.0 - math.cos(math.pi * t / t_end))


# Named workloads (cells per subdomain) ---------------------------------------

def config_problem(name: str) -> Problem:
    """C0: 32x16 manufactured solution; C1: 512x256 channel (seed 1);
    C2: 1024x512 channel (seed 2); T1: the C1 channel as the system of one
    backward-Euler step of 0.1 (its flow started from rest); C4: 3-D channel,
    96 x 48 x 96 cells per subdomain (x, y, z), one backward-Euler step of
    0.1."""
    if name == "T1":
        p = channel_problem(512, 256, seed=1)
        p.dt = 0.1
        return p
    if name == "C4":
        p = channel3d_problem(96, 48, 96, seed=4)
        p.dt = 0.1
        return p
    if name == "C0":
        return mms_problem(32, 16)[0]
    if name == "C1":
        return channel_problem(512, 256, seed=1)
    if name == "C2":
        return channel_problem(1024, 512, seed=2)
    raise KeyError(name)


# ----------------------------------------------------------------------------
# Serving trace
# ----------------------------------------------------------------------------

SERVING_GRIDS = ((64, 32), (128, 64), (256, 128), (512, 256))


def serving_trace(n_requests: int, rate_per_s: float, seed: int = 7,
                  grids=SERVING_GRIDS):
    """Poisson arrivals (exponential gaps at ``rate_per_s``), grid uniform over
    ``grids``, sigma ~ U[0.5, 2], inflow peak ~ U[1e-3, 1e-1], permeability
    seed 1000 + r.  Returns a list of dicts (arrival time and parameters)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests) if rate_per_s > 0 \
        else np.zeros(n_requests)
    t = np.cumsum(gaps) - (gaps[0] if n_requests else 0.0)
    gi = rng.integers(0, len(grids), n_requests)
    sig = rng.uniform(0.5, 2.0, n_requests)
    U = rng.uniform(1e-3, 1e-1, n_requests)
    out = []
    for r in range(n_requests):
        nx, ny = grids[int(gi[r])]
        out.append(dict(t_arrival=float(t[r]), nx=nx, ny=ny, sigma=float(sig[r]),
                        U=float(U[r]), seed=1000 + r))
    return out


def trace_problem(req: dict) -> Problem:
    return channel_problem(req["nx"], req["ny"], sigma=req["sigma"], U=req["U"],
                           seed=req["seed"])
