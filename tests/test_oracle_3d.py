"""Pins of the oracle's 3-D assembly (Sec. 2 model on a box grid): block
identities of the pv form, second-order consistency of every interior
stencil on manufactured solutions, the mirror symmetry between the x and z
directions, convergence of the discrete solution, discrete mass
conservation, and the backward-Euler mass rows."""
import numpy as np
import pytest
import scipy.sparse as sp

from sdinputs import (channel3d_problem, ff_cell_xyz, mms3d_problem, pm_cell_xyz,
                      u_face_xyz, v_face_xyz, w_face_xyz)
from oracle import krylov, precond
from oracle.assemble3d import assemble3d, split_solution3
from oracle.direct import refined_solve, solve


def _exact(p, ex):
    X, Y, Z = u_face_xyz(p)
    ue = ex["u"](X, Y, Z)[:, :, 1:]
    X, Y, Z = v_face_xyz(p)
    ve = ex["v"](X, Y, Z)[:-1]
    X, Y, Z = w_face_xyz(p)
    we = ex["w"](X, Y, Z)[:, 1:-1]
    X, Y, Z = ff_cell_xyz(p)
    pe = ex["p"](X, Y, Z)
    X, Y, Z = pm_cell_xyz(p)
    Pe = ex["P"](X, Y, Z)
    return np.concatenate([ue.ravel(), ve.ravel(), we.ravel(), pe.ravel(), Pe.ravel()])


def _interior_rows(a, p):
    """Rows whose stencils touch no boundary and not Gamma, per block
    (u, v, w, p, q)."""
    L = a.layout
    def box(n0, n1, n2, lo=2):
        j, k, i = np.meshgrid(np.arange(lo, n0 - lo), np.arange(lo, n1 - lo),
                              np.arange(lo, n2 - lo), indexing="ij")
        return j.ravel(), k.ravel(), i.ravel()
    j, k, i = box(p.ny, p.nz, p.nx)
    jq, kq, iq = box(p.ny_pm, p.nz, p.nx)
    return [L.u(i, j, k), L.v(i, j, k), L.w(i, j, k), L.p(i, j, k), L.q(iq, jq, kq)]


def _interior_truncation(n, plane):
    p, ex = mms3d_problem(n, n // 2, n, plane)
    a = assemble3d(p)
    r = a.A @ _exact(p, ex) - a.b
    vol = p.dx * p.dy * p.dz
    return np.array([np.abs(r[rows]).max() / vol for rows in _interior_rows(a, p)])


@pytest.mark.parametrize("plane", ["xy", "zy"])
def test_interior_stencils_second_order_consistent(plane):
    """The exact solution sampled at the unknowns leaves a residual per unit
    volume that falls 4x per halving of h on interior rows of every block
    (momentum u, v, w with their cross terms, continuity, porous TPFA)."""
    e1, e2 = _interior_truncation(24, plane), _interior_truncation(48, plane)
    active = e1 > 0
    assert np.all(e2[active] * 3.0 <= e1[active]), (e1, e2)
    # the velocity component the solution does not have stays exactly zero
    assert np.count_nonzero(~active) == 1


def test_x_and_z_directions_mirror_each_other():
    """The same solution in the (x, y) and in the (z, y) plane gives the same
    interior residuals with u and w exchanged."""
    exy, ezy = _interior_truncation(16, "xy"), _interior_truncation(16, "zy")
    assert exy[2] == 0.0 and ezy[0] == 0.0
    np.testing.assert_allclose(ezy[2], exy[0], rtol=1e-10)
    np.testing.assert_allclose(ezy[[1, 3, 4]], exy[[1, 3, 4]], rtol=1e-10)


@pytest.mark.parametrize("plane", ["xy", "zy"])
def test_manufactured_solution_errors_decrease(plane):
    errs = []
    for n in (8, 16):
        p, ex = mms3d_problem(n, n // 2, n, plane)
        a = assemble3d(p)
        x = solve(a.A, a.b)
        xe = _exact(p, ex)
        L = a.layout
        cuts = [0, L.off_v, L.off_w, L.off_p, L.off_q, L.N]
        errs.append([np.abs(x[cuts[t]:cuts[t + 1]] - xe[cuts[t]:cuts[t + 1]]).max()
                     for t in range(5)])
    errs = np.array(errs)
    assert np.all(errs[1] < errs[0]), errs
    assert np.all(errs[1, :3] < 6e-3) and np.all(errs[1, 3:] < 0.1), errs


@pytest.mark.parametrize("maker", [lambda: mms3d_problem(8, 4, 6, "zy")[0],
                                   lambda: channel3d_problem(10, 6, 8, 5, seed=2)])
def test_block_identities(maker):
    p = maker()
    a = assemble3d(p)
    blk = a.blocks()
    assert blk["Z"].nnz == 0 and blk["Dz"].nnz == 0
    for x, y in (("C", "B"), ("C1", "B1")):
        d = (blk[x] + blk[y].T).tocsr()
        d.eliminate_zeros()
        assert d.nnz == 0
    assert abs(blk["D"] - blk["D"].T).max() == 0.0
    if a.pm_singular:
        assert np.abs(blk["D"] @ np.ones(blk["D"].shape[0])).max() <= 1e-14 * abs(blk["D"]).max()
    cnt = np.diff(a.A.indptr)
    L = a.layout
    # interior stencils: a velocity row has 7 entries of its own component,
    # 4 of each other component and 2 pressures; continuity 6; TPFA 7
    i, j, k = p.nx // 2, p.ny // 2, p.nz // 2
    assert cnt[L.u(i, j, k)] == 7 + 4 + 4 + 2
    assert cnt[L.v(i, j, k)] == 17 and cnt[L.w(i, j, k)] == 17
    assert cnt[L.p(i, j, k)] == 6
    assert cnt[L.q(i, p.ny_pm // 2, k)] == 7


def test_mass_conservation_channel3d():
    p = channel3d_problem(12, 6, 8, seed=3)
    a = assemble3d(p)
    x = refined_solve(a.A, a.b)
    u, v, w, pp, q = split_solution3(x, a.layout)
    dx, dy, dz = p.dx, p.dy, p.dz
    uf = np.concatenate([p.ff_left_n[:, :, None], u], axis=2)             # [ny, nz, nx+1]
    vf = np.concatenate([v, np.zeros((1, p.nz, p.nx))], axis=0)          # top wall v = 0
    wf = np.concatenate([np.zeros((p.ny, 1, p.nx)), w, np.zeros((p.ny, 1, p.nx))], axis=1)
    div = ((uf[:, :, 1:] - uf[:, :, :-1]) * (dy * dz) + (vf[1:] - vf[:-1]) * (dx * dz)
           + (wf[:, 1:] - wf[:, :-1]) * (dx * dy))
    inflow = float(np.sum(p.ff_left_n) * dy * dz)
    assert np.abs(div).max() <= 1e-12 * inflow
    outflow = float(np.sum(u[:, :, -1]) * dy * dz)
    assert abs(inflow - outflow) <= 1e-10 * inflow
    assert abs(float(np.sum(v[0]) * dx * dz)) <= 1e-10 * inflow


def test_backward_euler_mass_rows_3d():
    p = channel3d_problem(6, 4, 5, 3, seed=1)
    A0 = assemble3d(p).A
    p.dt = 0.5
    a = assemble3d(p)
    L = a.layout
    has = np.zeros(L.N, dtype=bool)
    j, k, i = np.meshgrid(np.arange(p.ny), np.arange(p.nz), np.arange(1, p.nx), indexing="ij")
    has[L.u(i, j, k).ravel()] = True                     # outflow faces i = nx excluded
    j, k, i = np.meshgrid(np.arange(1, p.ny), np.arange(p.nz), np.arange(p.nx), indexing="ij")
    has[L.v(i, j, k).ravel()] = True
    has[L.off_w:L.off_p] = True
    assert np.array_equal(a.mass != 0.0, has)
    vol = p.dx * p.dy * p.dz
    d = (a.A - A0).tocsr()
    d.eliminate_zeros()
    assert np.array_equal(np.unique(d.indices), np.flatnonzero(has))
    assert np.allclose(d.diagonal()[has], vol / 0.5, rtol=1e-12, atol=0)


def test_block_preconditioned_fgmres_3d():
    p = channel3d_problem(16, 8, 12, seed=5)
    a = assemble3d(p)
    M = precond.build(p, a, "BGS")
    r = krylov.fgmres(a.A, a.b, M, tol=1e-10, m=60)
    assert r.converged and r.iters < 100
    xs = refined_solve(a.A, a.b)
    assert np.linalg.norm(r.x - xs) <= 1e-6 * np.linalg.norm(xs)
