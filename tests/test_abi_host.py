"""C-ABI checks that need no GPU: exported symbols, argument validation, and
bit-exact parity of the host assembly and AMG setup with the oracle."""
import os
import re

import numpy as np
import pytest

from sdinputs import channel_problem, mms_problem
from oracle import amg, precond
from oracle.assemble import assemble

sd = pytest.importorskip("paper_2108_13229_amd.sd")
HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sd.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sd.SIGNATURES)


def _cases():
    p_vel = channel_problem(20, 10, 8, seed=9)
    p_vel.ff_right = "velocity"
    p_vel.ff_right_n = np.linspace(0.0, 1e-3, 10)
    p_vel.ff_right_t = np.linspace(-1e-4, 1e-4, 11)
    p_mixbc = channel_problem(30, 12, 14, seed=11)
    p_mixbc.pm_left = "pressure"
    p_mixbc.pm_left_p = np.linspace(1.0, 2.0, 14)
    p_tr = channel_problem(40, 20, 12, seed=4)
    p_tr.dt = 0.1                                    # one backward-Euler step
    p_vel_tr = channel_problem(20, 10, 8, seed=9)
    p_vel_tr.ff_right = "velocity"
    p_vel_tr.ff_right_n = np.linspace(0.0, 1e-3, 10)
    p_vel_tr.dt = 3e-4
    p_bj = channel_problem(30, 14, 9, seed=6)
    p_bj.bj_full = True
    from sdinputs import paper_setup_problem
    p_paper = paper_setup_problem(6, p_in=1e-9)                   # narrow block, transient
    p_lt = mms_problem(20, 10)[0]
    p_lt.ff_left = "traction"
    p_lt.ff_left_n = np.linspace(1.0, 2.0, 10)
    p_lt.ff_left_t = np.linspace(-0.1, 0.1, 11)
    p_narrow = channel_problem(24, 8, 6, seed=7)
    p_narrow.nx_pm, p_narrow.pm_i0 = 10, 5
    p_narrow.K = p_narrow.K[:, :10].copy()
    p_narrow.pm_left, p_narrow.pm_left_p = "pressure", np.linspace(0.0, 1.0, 6)
    p_narrow.bj_full = True
    return [mms_problem(32, 16)[0], mms_problem(24, 12, 9, K=3e-3, mu=0.5, alpha=0.7)[0],
            channel_problem(64, 32, seed=1), channel_problem(45, 22, 17, seed=5), p_vel, p_mixbc,
            p_tr, p_vel_tr, mms_problem(20, 10, bj_full=True)[0], p_bj, p_paper, p_lt, p_narrow]


@pytest.mark.parametrize("p", _cases())
def test_host_assembly_bit_exact(p):
    P = sd.Problem(p, device=False)
    rp, col, val, b = P.csr()
    a = assemble(p)
    assert np.array_equal(rp, a.A.indptr)
    assert np.array_equal(col, a.A.indices)
    assert np.array_equal(val, a.A.data)        # bit-for-bit
    assert np.array_equal(b, a.b)
    assert np.array_equal(P.block_off, a.layout.block_off)


@pytest.mark.parametrize("amg_kind,mis", [("smoothed", 2), ("plain", 1), ("smoothed", 1),
                                          ("plain", 2)])
@pytest.mark.parametrize("pi", [0, 2, 3, 6, 10, 12])
def test_host_amg_bit_exact(amg_kind, mis, pi):
    p = _cases()[pi]
    P = sd.Problem(p, device=False)
    S = sd.Solver(P, device=False, amg=amg_kind, mis=mis, coarse_max=64)
    a = assemble(p)
    opts = amg.AMGOptions(smoothed=amg_kind == "smoothed", mis=mis, coarse_max=64)
    M = precond.build(p, a, "BGS", opts=opts)
    for blk, h in [(0, M.hV), (1, M.hD)]:
        nl = S.n_levels(blk)
        assert nl == h.n_levels
        for lev in range(nl):
            L = h.levels[lev]
            shape, rp, col, val = S.level_csr(blk, lev, 0)
            assert np.array_equal(rp, L.A.indptr) and np.array_equal(col, L.A.indices)
            assert np.array_equal(val, L.A.data)
            if lev + 1 < nl:
                assert np.array_equal(S.level_agg(blk, lev), L.agg)
                for which, M_ in [(1, L.P), (2, L.R)]:
                    _, rp, col, val = S.level_csr(blk, lev, which)
                    assert np.array_equal(rp, M_.indptr) and np.array_equal(col, M_.indices)
                    assert np.array_equal(val, M_.data)
        inv = S.coarse_inverse(blk)
        assert np.allclose(inv, h.Ainv, rtol=0, atol=1e-12 * np.abs(h.Ainv).max())


def test_invalid_inputs_are_rejected():
    p = channel_problem(16, 8, seed=1)
    p.K = p.K.copy()
    p.K[3, 4] = np.nan
    with pytest.raises(sd.SDError) as e:
        sd.Problem(p, device=False)
    assert e.value.code == sd.SD_E_INVALID
    p = channel_problem(16, 8, seed=1)
    p.K = -p.K
    with pytest.raises(sd.SDError):
        sd.Problem(p, device=False)
    p = channel_problem(1, 8, seed=1, corr_cells=0)
    with pytest.raises(sd.SDError):
        sd.Problem(p, device=False)
    p = channel_problem(16, 8, seed=1)
    p.ff_top = "traction"
    with pytest.raises(sd.SDError):
        sd.Problem(p, device=False)
    for dt in (-0.1, float("nan"), float("inf")):
        p = channel_problem(16, 8, seed=1)
        p.dt = dt
        with pytest.raises(sd.SDError) as e:
            sd.Problem(p, device=False)
        assert e.value.code == sd.SD_E_INVALID
    p = channel_problem(16, 8, seed=1)
    P = sd.Problem(p, device=False)
    with pytest.raises(sd.SDError):
        sd.Solver(P, device=False, restart=64)
    with pytest.raises(sd.SDError):
        sd.Solver(P, device=False, tol=0.0)
    with pytest.raises(sd.SDError):
        sd.Solver(P, device=True)        # host-only problem cannot get device data
    for bad in (dict(precision=3), dict(precision=-1), dict(nu_pre=-1), dict(coarse_max=0),
                dict(mis=3), dict(omega=0.0), dict(precond=4), dict(precond=-1)):
        with pytest.raises(sd.SDError):
            sd.Solver(P, device=False, **bad)
    assert sd.lib().sd_status_string(-4) == b"SD_E_NOCONV"


def test_smallest_grid():
    p = channel_problem(2, 2, 1, seed=1, corr_cells=0)
    P = sd.Problem(p, device=False)
    rp, col, val, b = P.csr()
    a = assemble(p)
    assert np.array_equal(val, a.A.data) and P.N == a.N == 2 * 2 + 2 * 2 + 4 + 2


@pytest.mark.parametrize("amg_kind,mis", [("smoothed", 2), ("plain", 1)])
@pytest.mark.parametrize("pi", [6, 7])
def test_host_pressure_operator_hierarchy_bit_exact(amg_kind, mis, pi):
    """Cahouet-Chabard middle block: L_p and its AMG hierarchy (block 2)."""
    p = _cases()[pi]
    P = sd.Problem(p, device=False)
    S = sd.Solver(P, device=False, amg=amg_kind, mis=mis, coarse_max=64, schur="cc")
    a = assemble(p)
    opts = amg.AMGOptions(smoothed=amg_kind == "smoothed", mis=mis, coarse_max=64)
    M = precond.build(p, a, "BGS", schur=precond.SCHUR_CC, opts=opts)
    h = M.hL
    assert S.n_levels(2) == h.n_levels >= 2
    for lev in range(h.n_levels):
        L = h.levels[lev]
        _, rp, col, val = S.level_csr(2, lev, 0)
        assert np.array_equal(rp, L.A.indptr) and np.array_equal(col, L.A.indices)
        assert np.array_equal(val, L.A.data)
        if lev + 1 < h.n_levels:
            assert np.array_equal(S.level_agg(2, lev), L.agg)
    inv = S.coarse_inverse(2)
    assert np.allclose(inv, h.Ainv, rtol=0, atol=1e-12 * np.abs(h.Ainv).max())


def test_pressure_operator_needs_a_time_step():
    P = sd.Problem(channel_problem(16, 8, seed=1), device=False)
    with pytest.raises(sd.SDError) as e:
        sd.Solver(P, device=False, schur="cc")
    assert e.value.code == sd.SD_E_INVALID
    S = sd.Solver(P, device=False)
    assert S.n_levels(2) == 0


def _cases3d():
    from sdinputs import channel3d_problem, mms3d_problem
    c_vel = channel3d_problem(9, 6, 7, 4, seed=3)
    c_vel.ff_right = "velocity"
    c_vel.ff_right_n = np.full((6, 7), 1e-3)
    c_vel.ff_right_tz = np.linspace(-1e-4, 1e-4, 6 * 8).reshape(6, 8)
    c_vel.dt = 0.05
    c_p = channel3d_problem(10, 6, 8, 5, seed=2)
    c_p.pm_back, c_p.pm_front = "pressure", "pressure"
    c_p.pm_back_p = np.linspace(0.0, 1.0, 5 * 10).reshape(5, 10)
    c_p.dt = 0.2
    c_bj = channel3d_problem(9, 5, 7, 4, seed=5)
    c_bj.bj_full = True
    return [mms3d_problem(8, 4, 6, "xy")[0], mms3d_problem(9, 5, 7, "zy")[0],
            channel3d_problem(12, 6, 8, seed=1), c_vel, c_p,
            mms3d_problem(6, 4, 1, "xy")[0], c_bj]


@pytest.mark.parametrize("ci", range(7))
def test_host_assembly_3d_bit_exact(ci):
    from oracle.assemble3d import assemble3d
    p = _cases3d()[ci]
    P = sd.Problem(p, device=False)
    rp, col, val, b = P.csr()
    a = assemble3d(p)
    assert np.array_equal(rp, a.A.indptr)
    assert np.array_equal(col, a.A.indices)
    assert np.array_equal(val, a.A.data)        # bit-for-bit
    assert np.array_equal(b, a.b)
    assert np.array_equal(P.block_off, a.layout.block_off)


@pytest.mark.parametrize("ci", [2, 3])
@pytest.mark.parametrize("schur", ["mass", "cc"])
def test_host_amg_3d_bit_exact(ci, schur):
    from oracle.assemble3d import assemble3d
    p = _cases3d()[ci]
    if schur == "cc" and not p.dt:
        p.dt = 0.1
    P = sd.Problem(p, device=False)
    S = sd.Solver(P, device=False, coarse_max=64, schur=schur)
    a = assemble3d(p)
    M = precond.build(p, a, "BGS", schur=schur, opts=amg.AMGOptions(coarse_max=64))
    hs = [(0, M.hV), (1, M.hD)] + ([(2, M.hL)] if schur == "cc" else [])
    for blk, h in hs:
        assert S.n_levels(blk) == h.n_levels
        for lev in range(h.n_levels):
            L = h.levels[lev]
            _, rp, col, val = S.level_csr(blk, lev, 0)
            assert np.array_equal(rp, L.A.indptr) and np.array_equal(col, L.A.indices)
            assert np.array_equal(val, L.A.data)
            if lev + 1 < h.n_levels:
                assert np.array_equal(S.level_agg(blk, lev), L.agg)



@pytest.mark.parametrize("variant", ["TD_BJ", "TD_BGS"])
def test_two_domain_setup_on_host(variant):
    p = channel_problem(24, 12, seed=2)
    P = sd.Problem(p, device=False)
    S = sd.Solver(P, device=False, precond=variant, coarse_max=64)
    assert S.n_levels(0) >= 2 and S.n_levels(1) >= 2
    assert S.middle_scale() == 1.0      # omega needs the device V-cycle


def _ilu_cases():
    from sdinputs import paper_setup_problem
    return [("channel", lambda: channel_problem(24, 12, seed=2)),
            ("ragged", lambda: channel_problem(45, 22, 17, seed=5)),
            ("paper_geometry", lambda: paper_setup_problem(16, p_in=1e-9, dt=2e5)),
            ("channel3d", lambda: __import__("sdinputs").channel3d_problem(8, 5, 6, seed=1))]


@pytest.mark.parametrize("ci", range(4))
def test_host_ilu0_bit_exact_and_level_schedule_valid(ci):
    """The host ILU(0) factors of D~ equal the oracle's bit for bit, and each
    substitution level references only rows of earlier levels."""
    from oracle import precond
    from oracle.assemble3d import assemble3d
    from oracle.ilu import ilu0
    name, make = _ilu_cases()[ci]
    p = make()
    a = assemble3d(p) if name == "channel3d" else assemble(p)
    ref = ilu0(precond.darcy_interface_block(a.blocks()))
    F, d = ref.F, ref.diag
    P = sd.Problem(p, device=False)
    S = sd.Solver(P, device=False, precond="TD_BGS", darcy="ilu0")
    assert S.n_levels(1) == 0
    n = F.shape[0]
    for lower in (True, False):
        f = S.ilu(lower)
        lev, ordr = f["lev"], f["ord"]
        assert lev[0] == 0 and lev[-1] == n and np.all(np.diff(lev) > 0)
        assert np.array_equal(np.sort(ordr), np.arange(n))
        level = np.empty(n, dtype=np.int64)
        for lv in range(len(lev) - 1):
            level[ordr[lev[lv]:lev[lv + 1]]] = lv
        for q in range(n):
            i = ordr[q]
            e0, e1 = (F.indptr[i], d[i]) if lower else (d[i] + 1, F.indptr[i + 1])
            cols, vals = F.indices[e0:e1], F.data[e0:e1]
            k = len(cols)
            assert np.array_equal(f["col"][:k, q], cols) and np.all(f["col"][k:, q] == -1)
            assert np.array_equal(f["val"][:k, q], vals) and np.all(f["val"][k:, q] == 0.0)
            assert np.all(level[cols] < level[i])
            if not lower:
                assert f["diag"][q] == F.data[d[i]]


def test_ilu0_option_validation():
    p = channel_problem(16, 8, seed=1)
    P = sd.Problem(p, device=False)
    for bad in (dict(darcy=2), dict(darcy=-1)):
        with pytest.raises(sd.SDError) as e:
            sd.Solver(P, device=False, **bad)
        assert e.value.code == sd.SD_E_INVALID
    S = sd.Solver(P, device=False)
    with pytest.raises(sd.SDError):
        S.ilu(True)                    # AMG Darcy block: no factors


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without the built HIP library the binding raises; there is no CPU
    fallback."""
    monkeypatch.setattr(sd, "_lib", None)
    monkeypatch.setattr(sd, "LIB_PATH", str(tmp_path / "libsd.so"))
    with pytest.raises(RuntimeError, match="not built"):
        sd.lib()
    with pytest.raises(RuntimeError):
        sd.Problem(channel_problem(8, 4, seed=1), device=False)


def test_arnoldi_row_blocking_stays_within_lds_and_partials():
    """The Gram-Schmidt projection keeps a block's rows of w and u_j in LDS
    (16 B per row): for every admissible size the blocks cover the rows, the
    LDS stays within 64 KiB and the grid within the 4096 partial-sum slots;
    sizes beyond the limit are rejected (so sd_setup refuses them before the
    host set-up)."""
    limit = 4096 * 4096
    for n in (1, 63, 1024, 1025, 524_288, 1_048_577, 2_097_152, 2_207_232, 4_194_305,
              8_388_608, 8_388_609, limit - 1, limit):
        rp, nb, lds = sd.arnoldi_layout(n)
        assert rp % 1024 == 0 and rp <= 4096
        assert nb * rp >= n and (nb - 1) * rp < n
        assert nb <= 4096
        assert lds == 16 * rp and lds <= 64 * 1024
    assert sd.arnoldi_layout(2_097_152)[:2] == (2048, 1024)   # the 1024x512 workload
    for bad in (0, -5, limit + 1):
        with pytest.raises(sd.SDError):
            sd.arnoldi_layout(bad)


def test_setup_refuses_more_unknowns_than_the_row_blocking_covers():
    """A channel of 4096 x 1025 cells per subdomain (16,789,504 unknowns,
    just above 4096 x 4096): assembly accepts it, the solver set-up refuses
    it with SD_E_INVALID before any AMG work."""
    p = channel_problem(4096, 1025, seed=1)
    P = sd.Problem(p, device=False)
    assert P.N > 4096 * 4096
    with pytest.raises(sd.SDError) as e:
        sd.Solver(P, device=False)
    assert e.value.code == sd.SD_E_INVALID
    P.close()
