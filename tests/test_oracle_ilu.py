"""Pins of the oracle's ILU(0) (Table 2's Darcy preconditioner of the
P^td(Uzawa, ILU(0)) rows) against what the definition and linear algebra fix:
exact LU where elimination creates no fill (tridiagonal: direct solve; dense:
the LU of a library routine), (L U)_ij = a_ij on the pattern with the dropped
fill showing up only outside it, the substitution against a library
triangular solver, and FGMRES with the ILU(0) block preconditioners reaching
the direct solution."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import krylov, precond
from oracle.assemble import assemble
from oracle.direct import refined_solve
from oracle.ilu import ilu0
from sdinputs import channel_problem, mms_problem


def _tridiag(n, seed):
    rng = np.random.default_rng(seed)
    lo, up = -rng.uniform(0.5, 1.0, n - 1), -rng.uniform(0.5, 1.0, n - 1)
    d = 2.5 + rng.uniform(0.0, 1.0, n)
    return sp.diags([lo, d, up], [-1, 0, 1], format="csr")


def _grid5(nx, ny, seed):
    """5-point operator with random positive couplings (diagonally dominant,
    nonsymmetric): elimination fills in, so ILU(0) differs from LU."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    rows, cols, vals = [], [], []
    for j in range(ny):
        for i in range(nx):
            r = i + nx * j
            s = 0.0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    c = rng.uniform(0.2, 1.0)
                    rows.append(r)
                    cols.append(ii + nx * jj)
                    vals.append(-c)
                    s += c
            rows.append(r)
            cols.append(r)
            vals.append(s + rng.uniform(0.1, 0.5))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def test_tridiagonal_is_exact_lu():
    A = _tridiag(40, 1)
    f = ilu0(A)
    assert np.abs((f.L() @ f.U() - A).toarray()).max() <= 1e-14
    r = np.random.default_rng(2).standard_normal(40)
    x = spla.spsolve(A.tocsc(), r)
    assert np.linalg.norm(f.solve(r) - x) <= 1e-13 * np.linalg.norm(x)


def test_dense_pattern_equals_library_lu():
    rng = np.random.default_rng(3)
    n = 7
    M = rng.uniform(-1.0, 1.0, (n, n))
    M += np.diag(np.abs(M).sum(axis=0) + 1.0)       # column dominance: no row exchanges
    P, Lr, Ur = sla.lu(M)
    assert np.array_equal(P, np.eye(n))
    f = ilu0(sp.csr_matrix(M))
    assert np.allclose(f.L().toarray(), Lr, rtol=0, atol=1e-13)
    assert np.allclose(f.U().toarray(), Ur, rtol=0, atol=1e-13)


def test_grid_factors_match_a_on_its_pattern_and_drop_fill():
    A = _grid5(7, 5, 4)
    f = ilu0(A)
    assert np.array_equal(f.F.indptr, A.indptr) and np.array_equal(f.F.indices, A.indices)
    LU = (f.L() @ f.U()).toarray()
    Ad = A.toarray()
    on = Ad != 0.0
    assert np.abs(LU[on] - Ad[on]).max() <= 1e-13 * np.abs(Ad).max()
    # the fill that elimination would create is dropped: L U differs from A
    # outside the pattern, and the full LU (no dropping) differs from ILU(0)
    assert np.abs(LU[~on]).max() > 1e-3
    _, Lr, _ = sla.lu(Ad)
    assert np.abs(Lr[np.tril(~on, -1)]).max() > 1e-3


def test_substitution_matches_library_triangular_solves():
    p, _ = mms_problem(16, 8)
    a = assemble(p)
    Dt = precond.darcy_interface_block(a.blocks())
    f = ilu0(Dt)
    r = np.random.default_rng(5).standard_normal(Dt.shape[0])
    y = spla.spsolve_triangular(f.L(), r, lower=True, unit_diagonal=True)
    z = spla.spsolve_triangular(f.U(), y, lower=False)
    assert np.linalg.norm(f.solve(r) - z) <= 1e-13 * np.linalg.norm(z)


def test_singular_pivot_is_rejected():
    A = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(ValueError):
        ilu0(A)
    with pytest.raises(ValueError):
        ilu0(sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 1.0]])))


@pytest.mark.parametrize("variant", ["TD_BJ", "TD_BGS"])
def test_fgmres_with_ilu_darcy_block_reaches_direct_solution(variant):
    p = channel_problem(32, 16, seed=3)
    a = assemble(p)
    xs = refined_solve(a.A, a.b)
    M = precond.build(p, a, variant, darcy=precond.DARCY_ILU0)
    assert M.hD is None and M.ilu is not None
    res = krylov.fgmres(a.A, a.b, M, tol=1e-10, m=60, maxit=2000)
    assert res.converged
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)
    # ILU(0) is a weaker Darcy preconditioner than the AMG V-cycle
    amg = krylov.fgmres(a.A, a.b, precond.build(p, a, variant), tol=1e-10, m=60)
    assert res.iters > amg.iters
