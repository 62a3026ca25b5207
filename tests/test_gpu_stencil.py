"""Stencil slices on the GPU: a solver whose SELL-64 matrices read stencil
offsets (stencil_slices = 1, the default) computes exactly what the same
solver reading column indices computes (stencil_slices = 0): the same
preconditioner application, V-cycle, iterate, iteration count and residual,
bit for bit.  256x128 cells per subdomain, so the finest velocity level
(65,920 rows) is stored one lane per row as well as the coupled matrix."""
import numpy as np
import pytest

from sdinputs import channel_problem
from oracle.assemble import assemble

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2108_13229_amd.sd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    sd.lib()


@pytest.fixture(scope="module")
def problem():
    p = channel_problem(256, 128, 64, seed=3)
    return p, assemble(p)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed32"])
def test_stencil_slices_change_nothing(problem, precision):
    p, a = problem
    print("case stencil", precision, flush=True)
    P = sd.Problem(p, device=True)
    out = []
    for stencil in (1, 0):
        S = sd.Solver(P, precond="BGS", schur="mass", tol=1e-8, restart=60,
                      precision=precision, stencil_slices=stencil)
        r = _dev(np.random.default_rng(4).standard_normal(a.N))
        z = S.apply_preconditioner(r)
        nv = S.block_size(0)
        xv = S.apply_vcycle(0, _dev(np.random.default_rng(6).standard_normal(nv)))
        x, st, rc = S.solve()
        torch.cuda.synchronize()
        assert rc == sd.SD_OK
        out.append((z.cpu(), xv.cpu(), x.cpu(), st["iters"], st["rel_res"]))
        S.close()
    P.close()
    (z1, v1, x1, i1, r1), (z0, v0, x0, i0, r0) = out
    assert torch.equal(z1, z0)
    assert torch.equal(v1, v0)
    assert i1 == i0 and r1 == r0
    assert torch.equal(x1, x0)
    res = np.linalg.norm(a.b - a.A @ x1.numpy()) / np.linalg.norm(a.b)
    assert res <= 1e-8


def test_stencil_option_is_validated(problem):
    p, _ = problem
    P = sd.Problem(p, device=False)
    with pytest.raises(sd.SDError):
        sd.Solver(P, device=False, stencil_slices=2)
    P.close()


def test_stencil_flag_path_3d():
    """A 3-D channel (40x20x40 cells per subdomain): its finest velocity level
    (95,200 rows, one lane per row, width 15) has slices whose offset union
    does not fit the width, so the kernels read the per-slice flag and take
    those slices through their indices (stencil mode 1).  V-cycle,
    preconditioner and solve match the index form bit for bit."""
    from sdinputs import channel3d_problem
    p = channel3d_problem(40, 20, 40, seed=3)
    Ph = sd.Problem(p, device=False)
    Sh = sd.Solver(Ph, device=False)
    shape, rp, col, val = Sh.level_csr(0, 0, 0)
    L = sd.sell_layout(rp, col, val, shape[1], allow_csr=True)
    assert L["lpr"] == 1 and L["stencil"] == 1
    Sh.close()
    Ph.close()
    print("case stencil flag path 3-D", flush=True)
    P = sd.Problem(p, device=True)
    out = []
    for stencil in (1, 0):
        S = sd.Solver(P, precond="BGS", schur="mass", tol=1e-8, restart=60, precision="mixed",
                      stencil_slices=stencil)
        nv = S.block_size(0)
        xv = S.apply_vcycle(0, _dev(np.random.default_rng(8).standard_normal(nv)))
        z = S.apply_preconditioner(_dev(np.random.default_rng(9).standard_normal(P.N)))
        x, st, rc = S.solve()
        torch.cuda.synchronize()
        assert rc == sd.SD_OK
        out.append((xv.cpu(), z.cpu(), x.cpu(), st["iters"]))
        S.close()
    P.close()
    (v1, z1, x1, i1), (v0, z0, x0, i0) = out
    assert torch.equal(v1, v0) and torch.equal(z1, z0)
    assert i1 == i0 and torch.equal(x1, x0)
