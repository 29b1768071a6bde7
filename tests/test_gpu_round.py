"""The round call on the GPU (deletes, inserts and queries in one epoch) against
the oracle's round, bit-exact on the uint8 path: directly, and replayed from a
captured HIP graph with counts that change from round to round.

After every round the whole exported state is compared (lists, distances,
degrees, flags, pool counts, publication counters, entry set), together with
the delete statuses, the new ids and the query results.
"""

import numpy as np
import pytest

from common import assert_same_state, index_params, make_gpu, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _build(wl, p, W=1, **gpu_kw):
    torch = _torch()
    o = make_oracle(p)
    g = make_gpu(p, **gpu_kw)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        x = st.base(b)
        o.insert(x)
        g.insert(torch.from_numpy(x).cuda())
    assert_same_state(o, g, "build")
    return o, g, st


def _check_round(o, g_out, sd, ids_o, qi_o, qd_o, where):
    torch = _torch()
    torch.cuda.synchronize()
    st = g_out["status"].cpu().numpy()
    assert st[0] == 0 and st[1] == 0, f"{where}: round status {st}"
    assert np.array_equal(sd, g_out["del_status"].cpu().numpy()), f"{where}: delete statuses"
    assert np.array_equal(ids_o, g_out["ids"].cpu().numpy().astype(np.uint32)), f"{where}: new ids"
    assert np.array_equal(qi_o, g_out["q_ids"].cpu().numpy().astype(np.uint32)), f"{where}: query ids"
    assert np.array_equal(qd_o, g_out["q_dists"].cpu().numpy()), f"{where}: query distances"


@pytest.mark.parametrize("reclaim", [False, True])
def test_round_parity_direct(reclaim):
    torch = _torch()
    wl = small_workload(seed=41, n_base=1500, rounds=3, churn=0.05)
    p = index_params(wl, n_entry=48)
    o, g, st = _build(wl, p)
    print(f"[round] direct reclaim={reclaim}", flush=True)
    for r in range(3):
        live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
        dl = st.deletes(live, 40 + 17 * r)
        dl = np.concatenate([dl, dl[:2], [10**7]]).astype(np.uint32)  # duplicates, unknown id
        x = st.inserts(55 + 23 * r)
        q = st.queries(37 + r)
        sd, ids, qi, qd = o.round(del_ids=dl, x=x, q=q, k=10, L=40, reclaim=reclaim)
        out = g.round(torch.from_numpy(dl.astype(np.int32)).cuda(), torch.from_numpy(x).cuda(),
                      torch.from_numpy(q).cuda(), k=10, L=40, reclaim=reclaim)
        _check_round(o, out, sd, ids, qi, qd, f"round {r}")
        assert_same_state(o, g, f"round {r}")
    g.close()


@pytest.mark.parametrize("buckets", [False, True])
def test_round_parity_graph_replay_uneven_counts(buckets):
    # one captured graph (or one per size bucket) serves rounds of different
    # sizes; eager calls run between the replays and every replay is checked
    torch = _torch()
    from paper_2607_02543_amd import etale
    wl = small_workload(seed=42, n_base=1500, rounds=6, churn=0.05)
    p = index_params(wl, n_entry=48)
    o, g, st = _build(wl, p)
    runner = etale.RoundRunner(g, max_del=90, max_ins=90, max_q=64, k=10, L=48, reclaim=True, graph=True,
                               buckets=buckets)
    sizes = [(80, 33, 64), (0, 90, 5), (61, 0, 1), (17, 71, 0), (90, 90, 64), (3, 1, 2), (80, 33, 60)]
    for r, (nd, ni, nq) in enumerate(sizes):
        print(f"[round] graph replay {r} sizes {nd, ni, nq}", flush=True)
        live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
        dl = st.deletes(live, nd)
        x = st.inserts(ni) if ni else None
        q = st.queries(nq) if nq else None
        sd, ids, qi, qd = o.round(del_ids=dl, x=x, q=q, k=10, L=48, reclaim=True)
        out = runner(torch.from_numpy(dl.astype(np.int32)).cuda() if nd else None,
                     torch.from_numpy(x).cuda() if ni else None, torch.from_numpy(q).cuda() if nq else None)
        _check_round(o, out, sd, ids, qi, qd, f"replay {r}")
        assert_same_state(o, g, f"replay {r}")
        # eager work on the same stream between replays
        ids_e, _ = g.search(torch.from_numpy(st.queries(8)).cuda(), 5, 32)
        torch.cuda.synchronize()
    g.close()


def test_round_gate_rejects_without_changing_state():
    torch = _torch()
    from paper_2607_02543_amd import etale
    wl = small_workload(seed=43, n_base=800, rounds=1, batch=100)
    p = index_params(wl, n_entry=32)
    p["id_capacity"] = 1100
    p["slab_capacity"] = 800 + 100 * (wl.R + 2) + 1000
    p["max_batch"] = 120
    o, g, st = _build(wl, p)
    before = g.export()
    live = np.nonzero(~before["deleted"])[0].astype(np.uint32)
    # pool: 100 inserts and 40 deletes need 100 (R + 2) + 40 R slabs
    dl = st.deletes(live, 40)
    x = st.inserts(100)
    for graph in (False, True):
        print(f"[round] gate graph={graph}", flush=True)
        runner = etale.RoundRunner(g, max_del=40, max_ins=100, max_q=4, graph=graph)
        out = runner(torch.from_numpy(dl.astype(np.int32)).cuda(), torch.from_numpy(x).cuda(),
                     torch.from_numpy(st.queries(4)).cuda())
        torch.cuda.synchronize()
        assert out["status"].cpu().numpy()[0] == etale.EPOOL
        after = g.export()
        for f in ("nbr", "deg", "deleted", "has_slab", "rho"):
            assert np.array_equal(before[f], after[f]), f
        # counts above the launch shapes are refused on the device
        out = runner(counts=(41, 0, 0))
        torch.cuda.synchronize()
        assert out["status"].cpu().numpy()[0] == etale.EINVAL
    assert_same_state(o, g, "after refused rounds")
    # the index still works: a round that fits
    sd, ids, qi, qd = o.round(del_ids=dl[:10], x=x[:20], q=None)
    out = g.round(torch.from_numpy(dl[:10].astype(np.int32)).cuda(), torch.from_numpy(x[:20]).cuda())
    torch.cuda.synchronize()
    assert out["status"].cpu().numpy()[0] == 0
    assert_same_state(o, g, "after a fitting round")
    g.close()


def test_round_bootstrap_and_empty_rounds():
    torch = _torch()
    from paper_2607_02543_amd import etale
    wl = small_workload(seed=44, n_base=600, rounds=1)
    p = index_params(wl, n_entry=16)
    o, g = make_oracle(p), make_gpu(p)
    st = dg.Stream(wl)
    runner = etale.RoundRunner(g, max_del=50, max_ins=400, max_q=16, k=5, L=24, graph=True)
    x = st.base(400)
    q = st.queries(16)
    print("[round] bootstrap through a graph", flush=True)
    sd, ids, qi, qd = o.round(x=x, q=q, k=5, L=24)
    out = runner(None, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    _check_round(o, out, sd, ids, qi, qd, "bootstrap")
    assert_same_state(o, g, "bootstrap")
    # an empty round, then a round with queries only
    sd, ids, qi, qd = o.round(k=5, L=24)
    out = runner()
    _check_round(o, out, sd, ids, qi, qd, "empty")
    sd, ids, qi, qd = o.round(q=q, k=5, L=24)
    out = runner(None, None, torch.from_numpy(q).cuda())
    _check_round(o, out, sd, ids, qi, qd, "queries only")
    # delete everything, then bootstrap again in one round
    live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
    for i in range(0, live.size, 50):
        dl = live[i:i + 50]
        o.round(del_ids=dl)
        out = runner(torch.from_numpy(dl.astype(np.int32)).cuda())
        torch.cuda.synchronize()
        assert out["status"].cpu().numpy()[0] == 0
    assert_same_state(o, g, "all deleted")
    x2 = st.inserts(100)
    sd, ids, qi, qd = o.round(x=x2, q=q, k=5, L=24)
    out = runner(None, torch.from_numpy(x2).cuda(), torch.from_numpy(q).cuda())
    _check_round(o, out, sd, ids, qi, qd, "second bootstrap")
    assert_same_state(o, g, "second bootstrap")
    g.close()
