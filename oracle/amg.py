"""Aggregation algebraic multigrid (oracle).

The paper preconditions the velocity block V and the Darcy block with one
V-cycle of an aggregation AMG (Sec. 5, solver setup: DUNE-ISTL non-smooth
aggregation, one smoothing step before and after, direct coarse solve).  The
oracle fixes every step so that the hierarchy is reproducible bit-for-bit:

1. strength: j is a strong neighbour of i iff j != i, both unknowns belong to
   the same physical component, and a_ij^2 >= theta^2 |a_ii a_jj| (evaluated
   as (a*a) >= (theta*theta) * |a_ii * a_jj|); the graph is symmetrised;
2. roots: a maximal independent set by synchronous Luby rounds with hashed
   priorities (fmix32(i xor seed(level)), i) -- on the strength graph
   ("mis1") or on its square ("mis2", roots at distance >= 3);
3. aggregates: roots are numbered in index order; every other node with a
   root among its strong neighbours joins the root with the largest |a_ij|
   (ties: smallest index); for "mis2" the nodes left over then join, in one
   synchronous sweep, the aggregate of the strong neighbour with the largest
   |a_ij| among the nodes aggregated so far (ties: smallest index);
4. prolongation: tentative P_t[i, agg(i)] = 1.  "plain" (non-smooth, the
   paper's choice) uses P = P_t; "smoothed" uses the smoothed-aggregation
   prolongator of Vanek, Mandel and Brezina (Computing 56, 1996),
   P = (I - w_p D_F^-1 A_F) P_t, with the filtered matrix A_F = strong
   entries of A plus a diagonal into which the weak entries are lumped,
   a_F,ii = a_ii + sum of the row's weak a_ij (ascending j), so that A_F and
   A have the same row sums; w_p = 4 / (3 rho_G), rho_G = max_i sum_j
   |a_F,ij| / |a_F,ii| the Gershgorin bound of D_F^-1 A_F; entry
   P[i, J] = [J == agg(i)] - (w_p / a_F,ii) * (sum over the row's A_F
   entries with agg(j) = J, in ascending j).  A row whose lumped diagonal
   vanishes (|a_F,ii| <= 1e-8 |a_ii|: every connection weak and zero row
   sum) keeps its tentative row and is left out of rho_G;
5. restriction R = P^T; Galerkin A_c = R (A P), each product summed in the
   row-by-row (Gustavson) order: (A P)[i, J] accumulates a_ik p_kJ over
   ascending k, then over P's row k in ascending J; A_c[I, J] accumulates
   r_Ii (AP)_iJ over ascending i;
6. levels stop at n <= coarse_max, a coarsening ratio below min_ratio or
   max_levels; the coarsest level is solved with an explicit FP64 inverse,
   regularised by tr(A_c)/n_c^2 * 1 1^T when the block is known to be
   singular with the constant vector in its kernel.

V-cycle: x = 0; nu_pre damped-Jacobi sweeps x <- x + (omega / a_ii)(b - A x);
r = b - A x; b_c = R r; recurse; x <- x + P x_c; nu_post sweeps.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .hashing import priority_key

UNDECIDED, ROOT, NONROOT = 0, 1, 2


@dataclasses.dataclass
class AMGOptions:
    theta: float = 0.08
    omega: float = 2.0 / 3.0
    nu_pre: int = 2
    nu_post: int = 2
    coarse_max: int = 2048
    max_levels: int = 20
    min_ratio: float = 1.2
    smoothed: bool = True        # smoothed (True) or plain (False) aggregation
    mis: int = 2                 # 1 or 2: distance of the root independent set


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    comp: np.ndarray
    agg: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None


@dataclasses.dataclass
class Hierarchy:
    levels: List[Level]
    Ainv: np.ndarray
    opts: AMGOptions

    @property
    def n_levels(self):
        return len(self.levels)


def _rows_of(A: sp.csr_matrix) -> np.ndarray:
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def strong_mask(A: sp.csr_matrix, comp: np.ndarray, theta: float) -> np.ndarray:
    """Boolean mask over A's stored entries: strong off-diagonal couplings."""
    rows = _rows_of(A)
    cols = A.indices
    a = A.data
    d = A.diagonal()
    th2 = theta * theta
    return ((rows != cols) & (comp[rows] == comp[cols])
            & ((a * a) >= th2 * np.abs(d[rows] * d[cols])))


def strength_graph(A: sp.csr_matrix, comp: np.ndarray, theta: float) -> sp.csr_matrix:
    n = A.shape[0]
    m = strong_mask(A, comp, theta)
    rows = _rows_of(A)
    S = sp.csr_matrix((np.ones(int(m.sum()), dtype=np.int8),
                       (rows[m], A.indices[m])), shape=(n, n))
    S = ((S + S.T) > 0).astype(np.int8).tocsr()
    S.sort_indices()
    return S


def square_graph(S: sp.csr_matrix) -> sp.csr_matrix:
    """Distance-<=2 neighbours (no self loops)."""
    S2 = ((S.astype(np.int32) @ S.astype(np.int32) + S) > 0).tocsr().astype(np.int8)
    S2.setdiag(0)
    S2.eliminate_zeros()
    S2.sort_indices()
    return S2


def mis(G: sp.csr_matrix, level: int) -> np.ndarray:
    """Synchronous Luby rounds on graph G; returns the state per node."""
    n = G.shape[0]
    key = priority_key(n, level)
    rows = _rows_of(G)
    cols = G.indices
    state = np.full(n, UNDECIDED, dtype=np.int8)
    while True:
        und = state == UNDECIDED
        if not und.any():
            break
        beaten = und[rows] & und[cols] & (key[cols] > key[rows])
        lost = np.zeros(n, dtype=bool)
        lost[rows[beaten]] = True
        new_root = und & ~lost
        state[new_root] = ROOT
        hit = new_root[cols] & (state[rows] == UNDECIDED)
        state[rows[hit]] = NONROOT
    return state


def _join(A_abs_vals, S, agg, src_ok):
    """One synchronous sweep: every unaggregated node with a strong neighbour
    j satisfying src_ok[j] joins agg[j] of the neighbour with the largest
    |a_ij| (ties: smallest j).  Returns the new agg array."""
    rows = _rows_of(S)
    cols = S.indices
    sel = (agg[rows] < 0) & src_ok[cols]
    r, c = rows[sel], cols[sel]
    w = A_abs_vals(r, c)
    order = np.lexsort((c, -w, r))
    r, c = r[order], c[order]
    first = np.ones(r.size, dtype=bool)
    first[1:] = r[1:] != r[:-1]
    out = agg.copy()
    out[r[first]] = agg[c[first]]
    return out


def aggregate(A: sp.csr_matrix, S: sp.csr_matrix, level: int, mis_dist: int):
    """Returns (agg, roots)."""
    n = A.shape[0]
    G = S if mis_dist == 1 else square_graph(S)
    state = mis(G, level)
    roots = np.flatnonzero(state == ROOT)
    agg = np.full(n, -1, dtype=np.int64)
    agg[roots] = np.arange(roots.size)
    Aabs = abs(A.tocsr())

    def wfun(r, c):
        if r.size == 0:          # no candidate left (sparse indexing would give 1 x 0)
            return np.zeros(0)
        return np.asarray(Aabs[r, c]).ravel()

    is_root = state == ROOT
    agg = _join(wfun, S, agg, is_root)
    if mis_dist == 2:
        agg = _join(wfun, S, agg, agg >= 0)
    if np.any(agg < 0):
        raise AssertionError("node left without an aggregate")
    return agg, roots


def tentative(agg: np.ndarray, n_c: int) -> sp.csr_matrix:
    n = agg.size
    return sp.csr_matrix((np.ones(n), agg, np.arange(n + 1)), shape=(n, n_c))


def smoothed_prolongator(A: sp.csr_matrix, comp: np.ndarray, theta: float,
                         agg: np.ndarray, n_c: int) -> sp.csr_matrix:
    A = A.tocsr()
    n = A.shape[0]
    rows = _rows_of(A)
    isdiag = rows == A.indices
    strong = strong_mask(A, comp, theta)
    weak = ~strong & ~isdiag
    aii = A.diagonal()
    # lumped diagonal: a_ii plus the row's weak entries in stored (ascending) order
    dF = aii.copy()
    np.add.at(dF, rows[weak], A.data[weak])
    valid = np.abs(dF) > 1e-8 * np.abs(aii)
    keep = strong | isdiag
    vals = A.data.copy()
    vals[isdiag] = dF[rows[isdiag]]
    # Gershgorin bound of D_F^-1 A_F over the smoothed rows, stored order
    absum = np.zeros(n)
    np.add.at(absum, rows[keep], np.abs(vals[keep]))
    rho = float(np.max(absum[valid] / np.abs(dF[valid]))) if valid.any() else 0.0
    wp = 4.0 / (3.0 * rho) if rho > 0.0 else 0.0
    sel = keep & valid[rows]
    r, c, a = rows[sel], A.indices[sel], vals[sel]
    J = agg[c]
    # per (i, J): sum of a_F,ij over ascending j (entries are in CSR order)
    key = r * n_c + J
    ukey, inv = np.unique(key, return_inverse=True)
    s = np.zeros(ukey.size)
    np.add.at(s, inv, a)
    ri = ukey // n_c
    cj = ukey % n_c
    base = (cj == agg[ri]).astype(np.float64)
    val = base - (wp / dF[ri]) * s
    # rows left unsmoothed keep P_t
    fixed = np.flatnonzero(~valid)
    ri = np.concatenate([ri, fixed])
    cj = np.concatenate([cj, agg[fixed]])
    val = np.concatenate([val, np.ones(fixed.size)])
    order = np.lexsort((cj, ri))
    ri, cj, val = ri[order], cj[order], val[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, ri + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.csr_matrix((val, cj, indptr), shape=(n, n_c))


def spgemm(X: sp.csr_matrix, Y: sp.csr_matrix) -> sp.csr_matrix:
    """Sparse product in Gustavson order: (XY)[i, J] accumulates x_ik y_kJ
    over X's row i in ascending k, then Y's row k in ascending J.  The
    result's pattern is the structural product (zeros kept), columns sorted."""
    X = X.tocsr()
    Y = Y.tocsr()
    X.sort_indices()
    Y.sort_indices()
    n, m = X.shape[0], Y.shape[1]
    xr = _rows_of(X)
    cnt = np.diff(Y.indptr)[X.indices]                 # products per X entry
    pr = np.repeat(xr, cnt)
    xv = np.repeat(X.data, cnt)
    start = np.repeat(Y.indptr[X.indices], cnt)
    within = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    yidx = start + within
    pc = Y.indices[yidx]
    prod = xv * Y.data[yidx]
    key = pr.astype(np.int64) * m + pc
    ukey, inv = np.unique(key, return_inverse=True)
    vals = np.zeros(ukey.size)
    np.add.at(vals, inv, prod)                         # sequential, product order
    ri = ukey // m
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, ri + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.csr_matrix((vals, ukey % m, indptr), shape=(n, m))


def coarse_inverse(Ac: sp.csr_matrix, singular: bool) -> np.ndarray:
    D = Ac.toarray()
    n = D.shape[0]
    if singular:
        D = D + (np.trace(D) / (n * n)) * np.ones((n, n))
    return np.linalg.inv(D)


def setup(A: sp.csr_matrix, comp: np.ndarray, singular: bool = False,
          opts: Optional[AMGOptions] = None) -> Hierarchy:
    opts = opts or AMGOptions()
    A = A.tocsr()
    A.sort_indices()
    comp = np.asarray(comp)
    levels = [Level(A=A, comp=comp)]
    # strength threshold of the current level: halved (for this level and
    # all coarser ones) whenever aggregation would shrink a level by less
    # than a factor of 2 -- the level-dependent threshold of smoothed
    # aggregation (Vanek, Mandel, Brezina 1996), applied where coarsening
    # stalls (the wide Galerkin stencils of 3-D hierarchies); at most 6
    # halvings; below min_ratio the hierarchy ends
    theta = opts.theta
    while (levels[-1].A.shape[0] > opts.coarse_max
           and len(levels) < opts.max_levels):
        L = levels[-1]
        lev = len(levels) - 1
        S = strength_graph(L.A, L.comp, theta)
        agg, roots = aggregate(L.A, S, lev, opts.mis)
        n_c = roots.size
        if L.A.shape[0] < 2.0 * n_c and theta > opts.theta / 64.0:
            theta = theta / 2.0
            continue
        if L.A.shape[0] < opts.min_ratio * n_c:
            break
        if opts.smoothed:
            P = smoothed_prolongator(L.A, L.comp, theta, agg, n_c)
        else:
            P = tentative(agg, n_c)
        R = P.T.tocsr()
        R.sort_indices()
        Ac = spgemm(R, spgemm(L.A, P))
        L.agg, L.P, L.R = agg, P, R
        levels.append(Level(A=Ac, comp=L.comp[roots]))
    return Hierarchy(levels=levels, Ainv=coarse_inverse(levels[-1].A, singular),
                     opts=opts)


def level_mats(h: Hierarchy, dtype):
    o = h.opts
    return [(L.A.astype(dtype), (o.omega / L.A.diagonal()).astype(dtype),
             None if L.P is None else L.P.astype(dtype),
             None if L.R is None else L.R.astype(dtype)) for L in h.levels]


def vcycle(h: Hierarchy, b: np.ndarray, dtype=np.float64, level: int = 0,
           mats=None) -> np.ndarray:
    """One V-cycle on A_0 x = b from x = 0.  ``dtype`` float32 runs smoothing,
    residuals and transfers in single precision; the coarsest solve is FP64."""
    o = h.opts
    if mats is None:
        mats = level_mats(h, dtype)
    if level == len(h.levels) - 1:
        return (h.Ainv @ b.astype(np.float64)).astype(dtype)
    A, wd, P, R = mats[level]
    b = b.astype(dtype)
    x = np.zeros_like(b)
    for _ in range(o.nu_pre):
        x = x + wd * (b - A @ x)
    r = b - A @ x
    xc = vcycle(h, R @ r, dtype, level + 1, mats)
    x = x + P @ xc
    for _ in range(o.nu_post):
        x = x + wd * (b - A @ x)
    return x


def vcycle_operator(h: Hierarchy) -> np.ndarray:
    """Dense matrix of the V-cycle (small hierarchies only)."""
    n = h.levels[0].A.shape[0]
    M = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = vcycle(h, e)
    return M
