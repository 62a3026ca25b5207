"""Host set-up under concurrency: assembly, AMG set-up and the device layout
built from several threads at once, each with its own cap on the threads its
set-up steps use (sd_set_host_threads), give the hierarchies of a sequential
set-up bit for bit.  This is how the request loop prepares requests: eight
preparation threads, each with a share of the host."""
import threading

import numpy as np
import pytest

from sdinputs import channel_problem, serving_trace, trace_problem

sd = pytest.importorskip("paper_2108_13229_amd.sd")


def _hierarchy(p, cap=None):
    if cap is not None:
        sd.set_host_threads(cap)
    try:
        P = sd.Problem(p, device=False)
        S = sd.Solver(P, device=False, coarse_max=256)
        out = []
        for blk in (0, 1):
            for lev in range(S.n_levels(blk)):
                shape, rp, col, val = S.level_csr(blk, lev, 0)
                out.append((shape, rp.copy(), col.copy(), val.copy()))
                if lev + 1 < S.n_levels(blk):
                    out.append(S.level_agg(blk, lev).copy())
            out.append(S.coarse_inverse(blk).copy())
        rp, col, val, b = P.csr()
        L = sd.sell_layout(rp, col, val, P.N)
        out.append((L["stencil"], L["doff"].copy(), L["val"].copy()))
        S.close()
        P.close()
        return out
    finally:
        if cap is not None:
            sd.set_host_threads(0)


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        if isinstance(x, tuple):
            for u, v in zip(x, y):
                assert np.array_equal(np.asarray(u), np.asarray(v))
        else:
            assert np.array_equal(x, y)


def test_concurrent_setups_match_sequential():
    probs = [trace_problem(t) for t in serving_trace(6, rate_per_s=0.0, seed=7)]
    probs.append(channel_problem(192, 96, 48, seed=3))     # levels above 8192 rows
    ref = [_hierarchy(p) for p in probs]
    caps = [1, 2, 3, 16, 0, 2, 1]
    got = [None] * len(probs)
    errs = []

    def work(i):
        try:
            got[i] = _hierarchy(probs[i], caps[i])
        except Exception as e:         # reported below
            errs.append(repr(e))

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(probs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs
    for r, g in zip(ref, got):
        _same(r, g)


def test_host_thread_cap_validated():
    with pytest.raises(sd.SDError):
        sd.set_host_threads(-1)
    sd.set_host_threads(4)
    sd.set_host_threads(0)
