"""The library's serving loop against the oracle and against the same queries
run alone.

Each tick's searches run on a snapshot of the state the previous tick left,
concurrently with the tick's own deletes and inserts (one round) on a second
stream. So a search in the mix must return exactly what the same query returns
alone on that state:

- saturated mode (arrival times ignored, max_tick requests per tick) makes the
  ticks a fixed function of the trace, so the oracle replays them itself
  (searches of the tick, then the tick's deletes and inserts as one round,
  reclaim every few ticks) and every result and the final state must agree
  bit for bit;
- real-time mode forms ticks from what has arrived on the wall clock; a second
  GPU index replays the served ticks one call at a time (each tick's searches
  alone, then its round) and every result and the final state must agree bit
  for bit.
"""

import numpy as np
import pytest

from common import assert_same_state, index_params, make_gpu, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _trace(o_or_live, st, rng, n, p_kind, n_pool=64):
    kind = rng.choice(3, size=n, p=p_kind).astype(np.uint32)
    n_ins = int((kind == 1).sum())
    qpool = st.queries(n_pool)
    rows = np.concatenate([qpool, st.inserts(n_ins)])
    dels = rng.choice(o_or_live, size=int((kind == 2).sum()), replace=False).astype(np.uint32)
    arg = np.zeros(n, np.uint32)
    arg[kind == 0] = rng.integers(0, n_pool, size=int((kind == 0).sum()))
    arg[kind == 1] = n_pool + np.arange(n_ins)
    arg[kind == 2] = dels
    return kind, arg, rows


@pytest.mark.parametrize("graph", [False, True])
def test_serve_matches_oracle_replay(graph):
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
    n, T, every, k, L = 700, 90, 3, 10, 48
    live = np.nonzero(~o.export()["deleted"])[0]
    kind, arg, rows = _trace(live, st, rng, n, [0.6, 0.2, 0.2])
    print(f"[serve] saturated graph={graph} n={n} tick={T}", flush=True)
    lat, ticks, stats, (ri, rd) = g.serve(np.zeros(n), kind, arg, torch.from_numpy(rows).cuda(), k=k, L=L,
                                          max_tick=T, reclaim_every=every, graph=graph, results=True)
    ri, rd = ri.cpu().numpy().astype(np.uint32), rd.cpu().numpy()
    assert stats["deferred"] == 0 and stats["failed_ticks"] == 0 and stats["rejected_inserts"] == 0
    assert np.array_equal(ticks, np.arange(n) // T)  # the next max_tick requests per tick
    for tick, s in enumerate(range(0, n, T)):
        kk, aa = kind[s:s + T], arg[s:s + T]
        qi = np.nonzero(kk == 0)[0] + s
        if qi.size:
            io, do = o.search(rows[arg[qi]], k, L)
            assert np.array_equal(io, ri[qi]), f"tick {tick}: result ids differ"
            assert np.array_equal(do, rd[qi]), f"tick {tick}: result distances differ"
        dl, xs = aa[kk == 2], rows[aa[kk == 1]]
        if dl.size or xs.shape[0] or (tick + 1) % every == 0:
            o.round(del_ids=dl if dl.size else None, x=xs if xs.shape[0] else None, reclaim=(tick + 1) % every == 0)
    assert (lat >= 0).all()
    assert stats["ticks"] == (n + T - 1) // T
    assert stats["inserts"] == int((kind == 1).sum()) and stats["deletes"] == int((kind == 2).sum())
    assert stats["searches"] == int((kind == 0).sum())
    assert stats["reclaims"] == stats["ticks"] // every
    assert_same_state(o, g, "after serving")
    g.close()


def test_serve_realtime_results_equal_queries_alone():
    import torch
    wl = small_workload(seed=53, n_base=4000, rounds=4, churn=0.05, batch=1000)
    p = index_params(wl, n_entry=64)
    g, h = make_gpu(p), make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        x = torch.from_numpy(st.base(b)).cuda()
        g.insert(x)
        h.insert(x)
    rng = np.random.default_rng(11)
    n, T, every, k, L = 3000, 128, 4, 10, 64
    kind, arg, rows = _trace(np.arange(4000), st, rng, n, [0.8, 0.1, 0.1])
    t = np.cumsum(rng.exponential(1.0 / 20000.0, size=n))  # Poisson arrivals at 20k/s: 0.15 s
    rows_d = torch.from_numpy(rows).cuda()
    print(f"[serve] realtime n={n} tick<={T}", flush=True)
    lat, ticks, stats, (ri, rd) = g.serve(t, kind, arg, rows_d, k=k, L=L, max_tick=T, reclaim_every=every,
                                          graph=False, realtime=True, results=True)
    ri, rd = ri.cpu().numpy(), rd.cpu().numpy()
    assert stats["failed_ticks"] == 0 and stats["rejected_inserts"] == 0
    assert (ticks != 0xFFFFFFFF).all() and (lat >= 0).all()
    assert stats["searches"] + stats["inserts"] + stats["deletes"] == n
    nt = int(ticks.max()) + 1
    assert nt == stats["ticks"]
    print(f"[serve] {nt} ticks, mean {n / nt:.1f} requests, p50 {np.median(lat):.3f} ms", flush=True)
    for tick in range(nt):
        mem = np.nonzero(ticks == tick)[0]  # arrival order
        kk, aa = kind[mem], arg[mem]
        qi = mem[kk == 0]
        if qi.size:
            i2, d2 = h.search(rows_d[torch.from_numpy(arg[qi].astype(np.int64)).cuda()], k, L)
            assert np.array_equal(i2.cpu().numpy(), ri[qi]), f"tick {tick}: ids differ from the query alone"
            assert np.array_equal(d2.cpu().numpy(), rd[qi]), f"tick {tick}: distances differ from the query alone"
        dl = aa[kk == 2]
        xi = aa[kk == 1]
        rec = (tick + 1) % every == 0
        if dl.size or xi.size or rec:
            out = h.round(del_ids=torch.from_numpy(dl.astype(np.int32)).cuda() if dl.size else None,
                          x=rows_d[torch.from_numpy(xi.astype(np.int64)).cuda()] if xi.size else None,
                          reclaim=rec)
            assert not out["status"].cpu().numpy().any()
    eg, eh = g.export(), h.export()
    for f in ("nbr", "rho", "deg", "deleted", "has_slab"):
        assert np.array_equal(eg[f], eh[f]), f"final state differs in {f}"
    g.close()
    h.close()


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
    lat, ticks, stats = g.serve(np.arange(n) * 1e-3, kind, np.arange(n, dtype=np.uint32), rows, max_tick=16,
                                hbm_budget_bytes=used // 2)
    assert stats["rejected_inserts"] == n and stats["inserts"] == 0
    assert (lat == -1).all() and (ticks == 0xFFFFFFFF).all()
    g.close()


def test_serve_defers_updates_the_pool_cannot_cover():
    import torch
    wl = small_workload(seed=54, n_base=600, rounds=2, churn=0.05, batch=50)
    p = index_params(wl, n_entry=16)
    # after the build the free pool covers one tick of 50 inserts (50 * (R + 2)
    # slabs) but not two, so the tick behind a running one gets few inserts
    p["slab_capacity"] = 600 + 50 * (wl.R + 2) + 100
    p["max_batch"] = 100
    p["id_capacity"] = 800
    g = make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        g.insert(torch.from_numpy(st.base(b)).cuda())
    n = 200
    kind = np.where(np.arange(n) % 2 == 0, 1, 0).astype(np.uint32)
    rows = torch.from_numpy(np.concatenate([st.queries(8), st.inserts(n // 2)])).cuda()
    arg = np.where(kind == 1, 8 + np.cumsum(kind) - 1, np.arange(n) % 8).astype(np.uint32)
    lat, ticks, stats = g.serve(np.zeros(n), kind, arg, rows, max_tick=100)
    # every request is served eventually; inserts wait for slabs while searches go ahead
    assert stats["inserts"] == n // 2 and stats["searches"] == n // 2 and stats["failed_ticks"] == 0
    assert stats["deferred"] > 0
    assert (ticks != 0xFFFFFFFF).all()
    ins_ticks, srch_ticks = ticks[kind == 1], ticks[kind == 0]
    assert srch_ticks.max() <= ins_ticks.max()
    assert g.stats()["error_bits"] == 0
    g.close()
