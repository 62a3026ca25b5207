"""The device matrix layout (sliced ELLPACK with stencil slices), checked on
the host through sd_sell_build: every slice, read the way the kernels read
it (column indices, or the slice's stencil offsets), gives the CSR row sums
bit for bit, and the stored arrays are consistent with each other."""
import numpy as np
import pytest
import scipy.sparse as sp

from sdinputs import channel_problem, mms_problem
from oracle.assemble import assemble

sd = pytest.importorskip("paper_2108_13229_amd.sd")

IRREGULAR = -2 ** 31


def _rows_of_entries(L, n):
    """(row, k, position) of every stored entry of a SELL-64 layout."""
    sptr, W = L["sptr"], L["width"]
    ns = (n + 63) // 64
    width = np.full(ns, W) if W else np.diff(sptr[: ns + 1]) // 64
    base = sptr[:ns] if not W else np.arange(ns) * 64 * W
    out = []
    for s in range(ns):
        for k in range(width[s]):
            r = s * 64 + np.arange(64)
            out.append((r, np.full(64, k), base[s] + 64 * k + np.arange(64)))
    return width, base, out


def _sequential_csr(A, x):
    """Row sums of A x, entries added one by one in column order from +0."""
    A = A.tocsr()
    n = A.shape[0]
    lens = np.diff(A.indptr)
    acc = np.zeros(n)
    for k in range(lens.max(initial=0)):
        m = lens > k
        e = A.indptr[:-1][m] + k
        acc[m] = acc[m] + A.data[e] * x[A.indices[e]]
    return acc


def _sequential_sell(L, n, x, stencil):
    """Row sums the way the SELL-64 kernels form them: entries k = 0, 1, ...
    of each row from +0, the column from col or (stencil slices) row + o_k."""
    width, base, _ = _rows_of_entries(L, n)
    ns = len(width)
    acc = np.zeros(ns * 64)
    rows = np.arange(ns * 64)
    for k in range(width.max(initial=0)):
        sl = np.nonzero(width > k)[0]
        r = (sl[:, None] * 64 + np.arange(64)).ravel()
        e = (base[sl][:, None] + 64 * k + np.arange(64)).ravel()
        c = L["col"][e]
        if stencil and L["stencil"]:
            d = L["doff"][(base[sl] // 64)]
            st = np.repeat((d != IRREGULAR) | (L["stencil"] == 2), 64)
            o = np.repeat(L["doff"][base[sl] // 64 + k], 64)
            c = np.where(st, np.clip(r + o, 0, len(x) - 1), c)
        ok = r < n        # phantom rows of the last slice are never stored
        acc[r[ok]] = acc[r[ok]] + L["val"][e[ok]] * x[c[ok]]
    return acc[:n]


def _check(A, allow_csr=False, min_stencil=None):
    A = A.tocsr()
    A.sort_indices()
    n, m = A.shape
    L = sd.sell_layout(A.indptr, A.indices, A.data, m, allow_csr=allow_csr, stencil=True)
    L0 = sd.sell_layout(A.indptr, A.indices, A.data, m, allow_csr=allow_csr, stencil=False)
    assert L0["doff"] is None and L0["idx"] == A.nnz and L0["stencil"] == 0
    assert (L["doff"] is None) == (L["stencil"] == 0)
    x = np.random.default_rng(5).standard_normal(m)
    ref = _sequential_csr(A, x)
    if L["lpr"] != 1:
        assert L["doff"] is None
        return L
    for lay in (L, L0):
        assert np.array_equal(_sequential_sell(lay, n, x, stencil=False), ref)
    assert np.array_equal(_sequential_sell(L, n, x, stencil=True), ref)
    if L["doff"] is None:
        return L
    width, base, _ = _rows_of_entries(L, n)
    ns = len(width)
    assert len(L["doff"]) == len(L["col"]) // 64 + 1 and L["doff"][-1] == IRREGULAR
    flags = L["doff"][base // 64]
    stencil_slices = ((flags != IRREGULAR) | (L["stencil"] == 2)) & (width > 0)
    assert (L["stencil"] == 2) == stencil_slices[width > 0].all()
    idx = len(L["doff"])
    w0 = np.diff(L0["sptr"][: ns + 1]) // 64 if not L0["width"] else np.full(ns, L0["width"])
    for s in range(ns):
        w = width[s]
        if not stencil_slices[s]:
            lo, hi = A.indptr[s * 64], A.indptr[min(n, s * 64 + 64)]
            idx += hi - lo
            assert w == w0[s]
            continue
        assert w0[s] <= w <= w0[s] + 8 and (L["width"] == 0 or w == w0[s])
        o = L["doff"][base[s] // 64: base[s] // 64 + w]
        assert np.all(np.diff(o) >= 0)               # ascending, tail repeats the last
        r = s * 64 + np.arange(64)
        for k in range(w):
            e = base[s] + 64 * k + np.arange(64)
            c = r + o[k]
            out = (c < 0) | (c >= m)
            assert np.array_equal(L["col"][e], np.clip(c, 0, m - 1))   # col stays complete
            assert np.all(L["val"][e][out] == 0)     # the kernels' clamp meets zeros only
            if k > 0 and o[k] == o[k - 1]:
                assert np.all(L["val"][e] == 0)
    assert L["idx"] == idx
    if min_stencil is not None:
        assert stencil_slices[width > 0].mean() >= min_stencil
    return L


def _laplace(nx, ny):
    I = sp.identity(nx)
    J = sp.identity(ny)
    Tx = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(nx, nx))
    Ty = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(ny, ny))
    return (sp.kron(J, Tx) + sp.kron(Ty, I)).tocsr()


def test_coupled_matrix_is_almost_all_stencil_slices():
    """The assembled Stokes-Darcy matrix: away from grid-line ends every
    64-row slice is one stencil; the few slices at block or grid ends that
    are not stay exact through their indices."""
    a = assemble(channel_problem(256, 128, 64, seed=3))
    L = _check(a.A, min_stencil=0.98)
    assert L["stencil"] == 2 and L["idx"] < 0.05 * a.A.nnz


def test_manufactured_solution_matrix():
    a = assemble(mms_problem(48, 24)[0])
    _check(a.A, min_stencil=0.9)


def test_laplacian_with_ragged_tail_and_uniform_width():
    """A 5-point Laplacian of 75,000 rows (a ragged last slice) in the
    hierarchy form: one lane per row, one width for all slices."""
    L = _check(_laplace(300, 250), allow_csr=True, min_stencil=0.99)
    assert L["lpr"] == 1 and L["width"] == 5 and L["stencil"] == 2


def test_small_and_degenerate_matrices():
    # fewer rows than a slice
    _check(_laplace(5, 7))
    # empty rows between stencil rows, and an empty matrix
    A = _laplace(40, 20).tolil()
    A[100, :] = 0
    A[101, :] = 0
    _check(sp.csr_matrix(A))
    _check(sp.csr_matrix((0, 0)))
    _check(sp.csr_matrix((70, 70)))
    # empty slices (whole 64-row groups without entries) inside and at the end
    Lp = _laplace(40, 20)
    Z = sp.csr_matrix((192, 192))
    L = _check(sp.block_diag([Lp, Z, Lp, Z]).tocsr(), min_stencil=0.5)
    assert L["doff"] is not None and L["doff"][-1] == IRREGULAR
    # rectangular: a coupling block wider than it is tall
    B = sp.random(200, 900, density=0.01, random_state=1, format="csr")
    _check(B)
    _check(sp.hstack([_laplace(16, 8), sp.identity(128)]).tocsr())


def _alternating(n, offs_even, offs_odd, m=None):
    """Rows alternating between two offset patterns (diagonal-dominant)."""
    m = m or n
    rows, cols = [], []
    for r in range(n):
        for o in (offs_even if r % 2 == 0 else offs_odd):
            if 0 <= r + o < m:
                rows.append(r)
                cols.append(r + o)
    v = np.random.default_rng(n).standard_normal(len(rows))
    return sp.csr_matrix((v, (rows, cols)), shape=(n, m))


def test_slices_widen_to_their_offset_union():
    """Rows of two patterns {-3, 0, 1} / {-1, 0, 4}: the union has 5 offsets
    against rows of 3, so each slice is widened by two zero positions (per-slice
    widths); with more than 8 extra offsets a slice keeps its indices."""
    A = _alternating(1000, (-3, 0, 1), (-1, 0, 4))
    L = _check(A, min_stencil=1.0)
    assert L["stencil"] == 2 and np.all(np.diff(L["sptr"]) == 5 * 64)
    B = _alternating(1000, tuple(range(0, 20, 2)), tuple(range(1, 21, 2)))    # 20 > 10 + 8
    L = _check(B)
    assert L["stencil"] == 0


def test_uniform_width_does_not_widen():
    """One width for all slices (the hierarchy form): a slice whose union
    exceeds it is read through its indices (stencil mode 1)."""
    A = _laplace(300, 250).tolil()
    A[640, 900] = 0.5                  # one extra far offset in slice 10 only
    L = _check(sp.csr_matrix(A), allow_csr=True, min_stencil=0.99)
    assert L["width"] == 6 and L["stencil"] == 2     # 6 wide: the union still fits
    A[641, 900] = 0.5                  # a second one: 7 offsets in a 6-wide layout
    L = _check(sp.csr_matrix(A), allow_csr=True, min_stencil=0.99)
    assert L["width"] == 6 and L["stencil"] == 1
    assert L["doff"][L["width"] * 10] == IRREGULAR


def test_irregular_matrix_keeps_indices():
    """Random columns: no slice is a stencil, the layout reads all indices."""
    A = sp.random(5000, 5000, density=2e-3, random_state=7, format="csr") + sp.identity(5000)
    L = _check(A)
    assert L["doff"] is None and L["idx"] == A.nnz


def test_repeated_columns_make_a_slice_irregular():
    """A row that names one column twice cannot be expanded onto offsets;
    its slice is read through its indices and stays exact."""
    A = _laplace(64, 8).tocsr()
    rp, ci, va = A.indptr.copy(), A.indices.copy(), A.data.copy()
    r = 70                                 # second slice
    ci = np.insert(ci, rp[r + 1], ci[rp[r + 1] - 1])
    va = np.insert(va, rp[r + 1], 0.25)
    rp[r + 1:] += 1
    L = sd.sell_layout(rp, ci, va, 512, stencil=True)
    assert L["stencil"] == 1 and L["doff"][L["sptr"][1] // 64] == IRREGULAR
    M = sp.csr_matrix((va, ci, rp), shape=(512, 512))
    x = np.random.default_rng(2).standard_normal(512)
    ref = _sequential_csr(M, x)
    assert np.array_equal(_sequential_sell(L, 512, x, stencil=True), ref)


def test_layout_input_validation():
    rp = np.array([0, 1, 2], dtype=np.int64)
    with pytest.raises(sd.SDError):
        sd.sell_layout(rp, np.array([0, 5]), np.ones(2), 3)          # column out of range
    with pytest.raises(sd.SDError):
        sd.sell_layout(np.array([1, 1, 2]), np.array([0, 1]), np.ones(2), 3)
    with pytest.raises(sd.SDError):
        sd.sell_layout(np.array([0, 2, 1]), np.array([0, 1]), np.ones(2), 3)
