"""The allocation-free residual entry point (sd_residual_noalloc) against
sd_residual through the C ABI: the same kernels with the norms' block
partials in the library's static device scratch instead of the solver's
workspace, so r and the four norms agree bit for bit; two calls in a row on
different solvers, the second on a smaller system, and no device allocation
during the call."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_noalloc_residual_matches_allocating_entry_point():
    cases = [channel_problem(160, 80, seed=31), channel_problem(24, 12, 9, seed=32)]
    assert cases[1].nx * cases[1].ny < cases[0].nx * cases[0].ny
    for k, p in enumerate(cases):
        print("case noalloc residual", k, p.nx, p.ny, flush=True)
        a = assemble(p)
        P = sd.Problem(p)
        S = sd.Solver(P, tol=1e-8, restart=30)
        rng = np.random.default_rng(40 + k)
        x = _dev(rng.standard_normal(a.N))
        b = _dev(rng.standard_normal(a.N))
        r1, n1 = S.residual(x=x, b=b)
        r2 = torch.full((a.N,), np.nan, dtype=torch.float64, device="cuda")
        n2 = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        s0 = dict(sd.ALLOC_STATS)
        m0 = torch.cuda.memory_allocated()
        S.residual(x=x, b=b, r=r2, norms=n2, noalloc=True)
        torch.cuda.synchronize()
        assert sd.ALLOC_STATS["allocs"] == s0["allocs"]
        assert torch.cuda.memory_allocated() == m0
        assert torch.equal(r1, r2) and torch.equal(n1, n2)
        # against the oracle's matrix
        ref = b.cpu().numpy() - a.A @ x.cpu().numpy()
        assert np.allclose(r2.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert abs(n2[0].item() - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
        # defaults: x = 0 and the assembled b
        r3, n3 = S.residual(noalloc=True)
        r4, n4 = S.residual()
        assert torch.equal(r3, r4) and torch.equal(n3, n4)
        assert np.array_equal(r3.cpu().numpy(), a.b)
        S.close()
        P.close()
