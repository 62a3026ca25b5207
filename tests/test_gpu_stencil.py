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
