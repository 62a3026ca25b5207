"""Pins of the oracle's backward-Euler time stepping (Sec. 2: transient free
flow, stationary Darcy, first-order backward Euler in time) against what the
mathematics fixes: backward Euler integrates a solution that is linear in
time exactly, so only the spatial error of the stationary scheme remains;
its error is first order in dt; a stationary solution is a fixed point of
the step.  A planted wrong mass scale fails the first pin."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from sdinputs import (channel_problem, ff_cell_xy, mms_transient_problem,
                      pm_cell_xy, u_face_xy, v_face_xy)
from oracle.assemble import assemble
from oracle.direct import refined_solve, solve
from oracle.transient import backward_euler, step_rhs


def _exact(p, m, gt):
    """Manufactured solution at time t (scaled by g(t)) in the unknown order."""
    xu, yu = u_face_xy(p)
    xv, yv = v_face_xy(p)
    xc, yc = ff_cell_xy(p)
    xq, yq = pm_cell_xy(p)
    return gt * np.concatenate([m.u(xu, yu)[:, 1:].ravel(), m.v(xv, yv)[:-1, :].ravel(),
                                m.p(xc, yc).ravel(), m.P(xq, yq).ravel()])


def _march(n, dt, n_steps, g, dg, mass_scale=1.0):
    """Backward Euler from the exact state at t = 0; returns the block-wise
    max errors against the exact state at t = n_steps dt."""
    p0, m = mms_transient_problem(n, n // 2, dt, 0.0, g, dg)
    a = assemble(p0)
    if mass_scale != 1.0:        # planted mistake: a wrong |CV|/dt on both sides
        a.A = (a.A + sp.diags((mass_scale - 1.0) * a.mass)).tocsr()
        a.mass = mass_scale * a.mass
    data = lambda k: assemble(mms_transient_problem(n, n // 2, dt, k * dt, g, dg)[0]).b
    x = backward_euler(a, _exact(p0, m, g(0.0)), n_steps, b_data=data)[-1]
    xe = _exact(p0, m, g(n_steps * dt))
    o = a.layout.block_off
    return np.array([np.abs(x[o[i]:o[i + 1]] - xe[o[i]:o[i + 1]]).max() for i in range(4)])


LIN = (lambda t: 1.0 + 20.0 * t, lambda t: 20.0)


def test_linear_in_time_solution_leaves_the_spatial_error():
    # the velocity's time derivative (20 u) is as large as its viscous term,
    # so a wrong mass coefficient would leave an O(1) error at every h
    ns = [32, 64, 128]
    errs = np.array([_march(n, 0.01, 5, *LIN) for n in ns])
    assert np.all(np.diff(errs, axis=0) < 0)
    slope = -np.polyfit(np.log2(ns), np.log2(errs), 1)[0]
    assert np.all(slope >= 0.9), slope
    assert errs[-1, 0] < 2e-3 and errs[-1, 1] < 5e-3


def test_planted_wrong_mass_scale_is_caught():
    good = _march(32, 0.01, 5, *LIN)
    bad = _march(32, 0.01, 5, *LIN, mass_scale=2.0)
    assert np.all(bad[:2] > 5.0 * good[:2])


def test_first_order_in_time():
    g = (lambda t: math.exp(-10.0 * t), lambda t: -10.0 * math.exp(-10.0 * t))
    T, n = 0.2, 32
    xs = []
    for k in (8, 16, 32, 64):
        dt = T / k
        p0, m = mms_transient_problem(n, n // 2, dt, 0.0, *g)
        a = assemble(p0)
        data = lambda j, dt=dt: assemble(mms_transient_problem(n, n // 2, dt, j * dt, *g)[0]).b
        xs.append(backward_euler(a, _exact(p0, m, g[0](0.0)), k, b_data=data)[-1])
    d = [np.abs(xs[i] - xs[i + 1]).max() for i in range(3)]
    ratios = [d[i] / d[i + 1] for i in range(2)]
    assert all(1.8 <= r <= 2.4 for r in ratios), ratios


@pytest.mark.parametrize("dt", [1e-3, 0.1, 10.0])
def test_stationary_solution_is_a_fixed_point(dt):
    p = channel_problem(48, 24, seed=6)
    xs = refined_solve(assemble(p).A, assemble(p).b)
    p.dt = dt
    a = assemble(p)
    x1 = refined_solve(a.A, step_rhs(a, a.b, xs))
    assert np.linalg.norm(x1 - xs) <= 1e-11 * np.linalg.norm(xs)


def test_mass_rows_and_values():
    p = channel_problem(12, 6, 8, seed=2)
    A0 = assemble(p).A
    p.dt = 0.25
    a = assemble(p)
    L = a.layout
    vol = (p.Lx / p.nx) * (p.H_ff / p.ny)
    has = np.zeros(L.N, dtype=bool)
    for j in range(p.ny):
        for i in range(1, p.nx):           # interior u faces; the outflow face i = nx has none
            has[L.u(i, j)] = True
        if j >= 1:                         # v faces off Gamma
            has[L.v(np.arange(p.nx), j)] = True
    assert np.array_equal(a.mass != 0.0, has)
    assert np.all(a.mass[has] == vol / 0.25)
    d = (a.A - A0).tocsr()
    d.eliminate_zeros()
    assert np.array_equal(np.unique(d.indices), np.flatnonzero(has))
    assert np.allclose(d.diagonal()[has], vol / 0.25, rtol=1e-12, atol=0)
    # the step's right-hand side touches exactly those rows
    x = np.random.default_rng(0).standard_normal(L.N)
    r = step_rhs(a, a.b, x)
    assert np.array_equal(r[~has], a.b[~has])
    assert np.allclose(r[has] - a.b[has], (vol / 0.25) * x[has], rtol=1e-12)


def test_zero_dt_is_the_stationary_assembly():
    p = channel_problem(16, 8, seed=3)
    a0 = assemble(p)
    assert not np.any(a0.mass)
    with pytest.raises(ValueError):
        p.dt = -1.0
        assemble(p)


# ---- Cahouet-Chabard middle block for backward-Euler systems ----

from sdinputs import mms_problem  # noqa: E402
from oracle import krylov, precond  # noqa: E402


def test_pressure_operator_is_the_scaled_pressure_laplacian():
    """Away from Gamma and the outflow, L_p = B^T D^-1 B with D = dx dy / dt
    is dt times the 5-point pressure Laplacian with unit-ratio weights
    (dy/dx, dx/dy); at walls and inflow faces (eliminated velocities) it has
    Neumann rows (zero row sums)."""
    p = channel_problem(12, 8, 6, seed=2)
    p.dt = 0.3
    a = assemble(p)
    Lp = precond.pressure_operator(a).toarray()
    dx, dy = p.Lx / p.nx, p.H_ff / p.ny
    assert np.array_equal(Lp, Lp.T)
    cell = lambda i, j: j * p.nx + i
    for j in range(1, p.ny):                   # rows off Gamma
        for i in range(0, p.nx - 1):           # cells off the outflow
            c = cell(i, j)
            nb = {}
            if i > 0:
                nb[cell(i - 1, j)] = 0.3 * dy / dx
            nb[cell(i + 1, j)] = 0.3 * dy / dx
            nb[cell(i, j - 1)] = 0.3 * dx / dy
            if j + 1 < p.ny:
                nb[cell(i, j + 1)] = 0.3 * dx / dy
            row = Lp[c]
            for k, w in nb.items():
                assert row[k] == pytest.approx(-w, rel=1e-12)
            assert row[c] == pytest.approx(sum(nb.values()), rel=1e-12)
            assert np.count_nonzero(row) == len(nb) + 1
            assert abs(row.sum()) <= 1e-12 * row[c]
    assert np.all(np.linalg.eigvalsh(Lp) > 0)


@pytest.mark.parametrize("maker", ["channel", "mms"])
def test_cahouet_chabard_spectral_equivalence(maker):
    """The preconditioned Schur complement X S (S = B^T V^-1 B exact, X the
    Cahouet-Chabard block with an exact L_p solve) keeps its spectrum in a
    fixed interval as dt shrinks and h halves; mu M_p^-1 alone lets the
    smallest eigenvalue go to zero with dt."""
    for n in (16, 32):
        for dt in (1e-4, 1e-2):
            p = channel_problem(n, n // 2, seed=2) if maker == "channel" else mms_problem(n, n // 2)[0]
            p.dt = dt
            a = assemble(p)
            blk = a.blocks()
            V, B = blk["V"].toarray(), blk["B"].toarray()
            S = B.T @ np.linalg.solve(V, B)
            vol = (p.Lx / p.nx) * (p.H_ff / p.ny)
            X = (p.mu / vol) * np.eye(S.shape[0]) + np.linalg.inv(
                precond.pressure_operator(a).toarray())
            ev = np.linalg.eigvals(X @ S)
            assert np.abs(ev.imag).max() <= 1e-8 * np.abs(ev).max()
            assert 0.25 <= ev.real.min() and ev.real.max() <= 6.0, (n, dt, ev.real.min(),
                                                                     ev.real.max())
            ev0 = np.linalg.eigvals((p.mu / vol) * S).real
            if dt == 1e-4:
                assert ev0.min() < 0.01


def test_cahouet_chabard_fgmres_iterations_do_not_grow_with_h():
    its = []
    for n in (96, 192):
        p = channel_problem(n, n // 2, seed=3)
        p.dt = 0.1
        a = assemble(p)
        M = precond.build(p, a, "BGS", schur=precond.SCHUR_CC)
        r = krylov.fgmres(a.A, a.b, M, tol=1e-8, m=30, maxit=300)
        assert r.converged
        its.append(r.iters)
    assert its[1] <= its[0] + 8 and its[1] <= 70, its


def test_cahouet_chabard_rejects_stationary_systems():
    p = channel_problem(16, 8, seed=3)
    with pytest.raises(ValueError):
        precond.build(p, assemble(p), "BGS", schur=precond.SCHUR_CC)
