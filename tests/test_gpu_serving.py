"""Request loop: admission, overlap, alone-vs-mix equality, failure paths."""
import time

import numpy as np
import pytest

from sdinputs import channel_problem, serving_trace, trace_problem
from oracle.assemble import assemble

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sd = pytest.importorskip("paper_2108_13229_amd.sd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    sd.lib()


def _mix():
    return [channel_problem(64, 32, seed=11, U=3e-2),
            channel_problem(48, 24, 20, seed=12, sigma=1.5),
            channel_problem(96, 48, seed=13, U=1e-3),
            channel_problem(64, 32, seed=14, sigma=0.5)]


def _run(server, probs, **opts):
    tickets = [server.submit(p, **opts) for p in probs]
    out = [server.wait(t, timeout=120) for t in tickets]
    for t in tickets:
        server.release(t)
    return out


def test_server_results_match_direct_solve_and_residual():
    probs = _mix()
    S = sd.Server(max_slots=4)
    res = _run(S, probs, tol=1e-8, restart=40)
    S.close()
    for p, r in zip(probs, res):
        print("request", r["N"], r["stats"]["iters"], flush=True)
        assert r["state"] == "done" and r["status"] == sd.SD_OK
        a = assemble(p)
        assert np.linalg.norm(a.b - a.A @ r["x"]) <= 1e-8 * np.linalg.norm(a.b)
        # same library, same kernels: bit-identical to a direct sd_solve
        P = sd.Problem(p)
        Sv = sd.Solver(P, tol=1e-8, restart=40)
        x, st, rc = Sv.solve()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), r["x"]) and st["iters"] == r["stats"]["iters"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_alone_vs_mix_bit_identical(precision):
    probs = _mix()
    alone = []
    S1 = sd.Server(max_slots=1)
    for p in probs:
        alone += _run(S1, [p], tol=1e-8, precision=precision)
    S1.close()
    S8 = sd.Server(max_slots=8)
    mix = _run(S8, probs, tol=1e-8, precision=precision)
    S8.close()
    for a_, m_ in zip(alone, mix):
        assert a_["status"] == m_["status"] == sd.SD_OK
        assert np.array_equal(a_["x"], m_["x"])
        assert a_["stats"]["iters"] == m_["stats"]["iters"]


def _peak_concurrency(res):
    ev = sorted([(m["t_admit"], 1) for m in res] + [(m["t_done"], -1) for m in res])
    live = peak = 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    return peak


def test_mix_overlaps_on_device():
    # equal-size requests are prepared in parallel and iterate concurrently
    probs = [channel_problem(128, 64, seed=40 + k) for k in range(8)]
    S = sd.Server(max_slots=8)
    res = _run(S, probs, tol=1e-8)
    S.close()
    assert all(r["status"] == sd.SD_OK for r in res)
    assert _peak_concurrency(res) >= 2


def test_admission_respects_slots_and_fifo():
    probs = [channel_problem(64, 32, seed=20 + k) for k in range(5)]
    S = sd.Server(max_slots=2)
    res = _run(S, probs, tol=1e-8)
    S.close()
    assert all(r["status"] == sd.SD_OK for r in res)
    # at most two requests in flight at any time
    ev = sorted([(r["t_admit"], 1) for r in res] + [(r["t_done"], -1) for r in res])
    live = 0
    for _, d in ev:
        live += d
        assert live <= 2


def test_budget_cancel_and_errors():
    S = sd.Server(max_slots=2, hbm_budget=1 << 20)   # 1 MiB: nothing fits
    with pytest.raises(sd.SDError) as e:
        S.submit(channel_problem(64, 32, seed=1))
    assert e.value.code == sd.SD_E_NOMEM
    S.close()
    S = sd.Server(max_slots=1)
    p = channel_problem(128, 64, seed=2)
    t1 = S.submit(p, tol=1e-8)
    t2 = S.submit(p, tol=1e-8)
    S.cancel(t2)
    r1 = S.wait(t1, timeout=120)
    r2 = S.wait(t2, timeout=120)
    assert r1["status"] == sd.SD_OK
    assert r2["state"] == "failed"
    with pytest.raises(sd.SDError) as e:
        S.poll(987654)
    assert e.value.code == sd.SD_E_NOTFOUND
    bad = channel_problem(32, 16, seed=3)
    bad.K = bad.K.copy()
    bad.K[0, 0] = -1.0
    t3 = S.submit(bad)
    r3 = S.wait(t3, timeout=60)
    assert r3["state"] == "failed" and r3["status"] == sd.SD_E_INVALID
    t4 = S.submit(channel_problem(32, 16, seed=4), maxit=2)
    r4 = S.wait(t4, timeout=60)
    assert r4["status"] == sd.SD_E_NOCONV and r4["stats"]["iters"] == 2
    S.close()


def test_serving_trace_small():
    trace = serving_trace(12, rate_per_s=0.0, seed=7, grids=((64, 32), (128, 64)))
    S = sd.Server(max_slots=8)
    res = _run(S, [trace_problem(t) for t in trace], tol=1e-8, precision="mixed")
    S.close()
    for t, r in zip(trace, res):
        assert r["status"] == sd.SD_OK, (t, r["status"])


def test_device_memory_comes_from_torch_allocator():
    """The binding registers torch's caching allocator as the library's
    sd_allocator: a solver's matrices, hierarchies and Krylov state, and every
    request of the loop, are torch blocks, all returned when the handles
    close."""
    torch.cuda.synchronize()
    s0 = dict(sd.ALLOC_STATS)
    m0 = torch.cuda.memory_allocated()
    p = channel_problem(96, 48, seed=13)
    P = sd.Problem(p)
    S = sd.Solver(P, tol=1e-8, restart=40)
    s1 = dict(sd.ALLOC_STATS)
    got = s1["bytes_allocated"] - s0["bytes_allocated"]
    assert s1["allocs"] > s0["allocs"] and got > 0
    assert torch.cuda.memory_allocated() - m0 >= got
    x, st, rc = S.solve()
    assert rc == sd.SD_OK
    del x
    S.close()
    P.close()
    torch.cuda.synchronize()
    assert sd.ALLOC_STATS["bytes_live"] == s0["bytes_live"]
    # the request loop's requests
    sv = sd.Server(max_slots=2)
    res = _run(sv, _mix()[:2], tol=1e-8, restart=40)
    assert all(r["status"] == sd.SD_OK for r in res)
    s2 = dict(sd.ALLOC_STATS)
    assert s2["allocs"] > s1["allocs"] + 1
    sv.close()
    assert sd.ALLOC_STATS["bytes_live"] == s0["bytes_live"]


def test_shared_launches_serve_every_member_bit_identically():
    """Requests with the same kernel sequence (one grid and permeability
    field, different inflow) form one group: each graph replay runs an
    Arnoldi column for several of them in one batched launch per kernel, and
    each result equals its direct sd_solve bit for bit."""
    probs = [channel_problem(128, 64, seed=50, U=u) for u in (1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.3)]
    S = sd.Server(max_slots=6)
    res = _run(S, probs, tol=1e-8, restart=40)
    st = S.batch_stats()
    S.close()
    print("batch stats", st, flush=True)
    assert st["groups"] >= 1 and st["replays"] > 0
    assert st["max_members"] >= 2
    assert st["member_columns"] > st["replays"]
    for p, r in zip(probs, res):
        assert r["status"] == sd.SD_OK
        P = sd.Problem(p)
        Sv = sd.Solver(P, tol=1e-8, restart=40)
        x, s1, rc = Sv.solve()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), r["x"]) and s1["iters"] == r["stats"]["iters"]
        Sv.close()
        P.close()


@pytest.mark.parametrize("krylov", ["fgmres", "pdgmres"])
def test_shared_launches_across_restarts(krylov):
    """Short cycles (restart 8, and PD-GMRES's controlled lengths): members
    leave the group at every cycle end, restart on their own stream and
    join again; results still equal the direct solves bit for bit."""
    probs = [channel_problem(64, 32, seed=60, U=u) for u in (1e-3, 1e-2, 0.1)]
    S = sd.Server(max_slots=4)
    res = _run(S, probs, tol=1e-8, restart=8, krylov=krylov)
    S.close()
    for p, r in zip(probs, res):
        assert r["status"] == sd.SD_OK and r["stats"]["restarts"] >= 2
        P = sd.Problem(p)
        Sv = sd.Solver(P, tol=1e-8, restart=8, krylov=krylov)
        x, s1, rc = Sv.solve()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), r["x"]) and s1["iters"] == r["stats"]["iters"]
        Sv.close()
        P.close()


def test_cancel_while_in_shared_launches():
    """A request cancelled while its columns run in a group's shared launches
    leaves the group (its workgroup counts cleared, its stream ordered after
    the group's last replay) before its memory is freed; the other members
    still equal their direct solves bit for bit."""
    probs = [channel_problem(256, 128, seed=70, U=u) for u in (1e-3, 1e-2, 0.1, 0.3)]
    S = sd.Server(max_slots=4)
    tickets = [S.submit(p, tol=1e-10, restart=60) for p in probs]
    victim = tickets[1]
    t_end = time.time() + 60
    while S.poll(victim)["state"] == "pending" and time.time() < t_end:
        time.sleep(0.0005)
    time.sleep(0.002)
    S.cancel(victim)
    res = [S.wait(t, timeout=120) for t in tickets]
    st = S.batch_stats()
    for t in tickets:
        S.release(t)
    S.close()
    print("victim", res[1]["state"], res[1]["status"], "batch stats", st, flush=True)
    assert res[1]["state"] in ("failed", "done")
    if res[1]["state"] == "failed":
        assert res[1]["status"] == sd.SD_E_INVALID
    assert st["max_members"] >= 2
    for k, (p, r) in enumerate(zip(probs, res)):
        if k == 1:
            continue
        assert r["status"] == sd.SD_OK
        P = sd.Problem(p)
        Sv = sd.Solver(P, tol=1e-10, restart=60)
        x, s1, rc = Sv.solve()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), r["x"]) and s1["iters"] == r["stats"]["iters"]
        Sv.close()
        P.close()
