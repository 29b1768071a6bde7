"""The library's serving loop (continuous batching of a request trace into
rounds) against the oracle.

With every request arriving at time 0, each tick admits exactly the next
max_tick requests, so the ticks are a fixed sequence of rounds: the oracle runs
the same rounds (the tick's deletes, inserts and searches in request order,
reclaim every few ticks) and the exported states must agree bit for bit.
"""

import numpy as np
import pytest

from common import assert_same_state, index_params, make_gpu, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph", [False, True])
def test_serve_ticks_match_oracle_rounds(graph):
    import torch
    wl = small_workload(seed=51, n_base=1500, rounds=6, churn=0.05)
    p = index_params(wl, n_entry=48)
    o, g = make_oracle(p), make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        x = st.base(b)
        o.insert(x)
        g.insert(torch.from_numpy(x).cuda())
    rng = np.random.default_rng(7)
    n, T, every = 700, 90, 3
    kind = rng.choice(3, size=n, p=[0.6, 0.2, 0.2]).astype(np.uint32)
    n_ins = int((kind == 1).sum())
    qpool = st.queries(64)
    rows = np.concatenate([qpool, st.inserts(n_ins)])
    live = np.nonzero(~o.export()["deleted"])[0]
    dels = rng.choice(live, size=int((kind == 2).sum()), replace=False).astype(np.uint32)
    arg = np.zeros(n, np.uint32)
    arg[kind == 0] = rng.integers(0, 64, size=int((kind == 0).sum()))
    arg[kind == 1] = 64 + np.arange(n_ins)
    arg[kind == 2] = dels
    t = np.zeros(n)
    print(f"[serve] graph={graph} n={n} tick={T}", flush=True)
    lat, stats = g.serve(t, kind, arg, torch.from_numpy(rows).cuda(), k=10, L=48, max_tick=T, reclaim_every=every,
                         graph=graph)
    for tick, s in enumerate(range(0, n, T)):
        kk, aa = kind[s:s + T], arg[s:s + T]
        o.round(del_ids=aa[kk == 2], x=rows[aa[kk == 1]], q=rows[aa[kk == 0]], k=10, L=48,
                reclaim=(tick + 1) % every == 0)
    assert (lat >= 0).all()
    assert stats["ticks"] == (n + T - 1) // T
    assert stats["inserts"] == n_ins and stats["deletes"] == dels.size
    assert stats["searches"] == int((kind == 0).sum())
    assert stats["failed_ticks"] == 0 and stats["rejected_inserts"] == 0
    assert stats["reclaims"] == stats["ticks"] // every
    assert_same_state(o, g, "after serving")
    g.close()


def test_serve_budget_rejects_inserts():
    import torch
    wl = small_workload(seed=52, n_base=800, rounds=2, churn=0.05)
    p = index_params(wl, n_entry=16)
    g = make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        g.insert(torch.from_numpy(st.base(b)).cuda())
    n = 40
    kind = np.ones(n, np.uint32)
    rows = torch.from_numpy(st.inserts(n)).cuda()
    used = g.stats()["device_bytes"]
    # a budget already exceeded by the index's fixed buffers admits no insert
    lat, stats = g.serve(np.arange(n) * 1e-3, kind, np.arange(n, dtype=np.uint32), rows, max_tick=16,
                         hbm_budget_bytes=used // 2)
    assert stats["rejected_inserts"] == n and stats["inserts"] == 0
    assert (lat == -1).all()
    g.close()
