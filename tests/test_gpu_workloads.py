"""The measured workloads on the GPU.

tiny uint8 (10,000 x 128-d, 32 clusters, batches of 1,000, five 1% churn rounds,
1,000 queries per round, seed 0): bit-exact against the oracle after every call.

scale uint8 (1,000,000 x 128-d, 1,024 clusters, the configuration bench.py times):
the oracle cannot build it, so sampled outputs are checked one by one (stored
distances against numpy, returned distances against numpy, the brute-force kernel
against numpy) and properties that hold at any size are checked in full (degree
bound, no self loops or duplicates, sorted lists, deletion flags, no edge into a
tombstone after reclaim, resident slabs = live nodes, deleted ids never returned).
"""

import numpy as np
import pytest

from common import assert_same_state, index_params, make_gpu, make_oracle, recall_at
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_tiny_workload_bit_exact():
    torch = _torch()
    wl = dg.tiny_u8()
    p = index_params(wl, n_entry=128)
    o, g = make_oracle(p), make_gpu(p)
    st = dg.Stream(wl)
    dev = torch.device("cuda")
    for bi, b in enumerate(wl.build_batches()):
        x = st.base(b)
        o.insert(x)
        g.insert(torch.from_numpy(x).to(dev))
        assert_same_state(o, g, f"build batch {bi}")
    q = st.queries(wl.n_queries)
    qd = torch.from_numpy(q).to(dev)
    for r in range(wl.churn_rounds):
        live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
        dl = st.deletes(live, wl.churn_count())
        assert np.array_equal(o.delete(dl), g.delete(torch.from_numpy(dl.astype(np.int32)).to(dev)).cpu().numpy())
        x = st.inserts(wl.churn_count())
        o.insert(x)
        g.insert(torch.from_numpy(x).to(dev))
        o.reclaim()
        g.reclaim()
        assert_same_state(o, g, f"round {r}")
        io, do, eo, no = o.search(q, 10, 64, counts=True)
        ig, dgp, cg = g.search(qd, 10, 64, counts=True)
        assert np.array_equal(io, ig.cpu().numpy().astype(np.uint32)), f"round {r}: result ids"
        assert np.array_equal(do, dgp.cpu().numpy()), f"round {r}: result distances"
        assert np.array_equal(eo, cg[:, 0].cpu().numpy().astype(np.uint32)), f"round {r}: expansions per query"
        gt, _ = o.bruteforce(q, 10)
        rec = recall_at(io, gt)
        assert rec >= 0.95, f"round {r}: Recall@10 {rec}"
        print(f"[tiny] round {r}: bit-exact, Recall@10 {rec:.4f}", flush=True)
    g.close()


def _l2(a, b):
    d = a.astype(np.int64) - b.astype(np.int64)
    return (d * d).sum(-1)


def test_scale_workload_sampled_and_properties():
    torch = _torch()
    from paper_2607_02543_amd import etale

    wl = dg.scale_u8(rounds=2, n_queries=2000)
    st = dg.Stream(wl)
    dev = torch.device("cuda")
    cap = wl.id_capacity()
    g = etale.Index(wl.dim, R=wl.R, L_build=wl.L_build, n_entry=8192, id_capacity=cap,
                    slab_capacity=2 * cap + 10000 * (wl.R + 2), max_batch=10000)
    xs = np.zeros((cap, wl.dim), np.uint8)
    done = 0
    for b in wl.build_batches():
        x = st.base(b)
        xs[done:done + b] = x
        g.insert(torch.from_numpy(x).to(dev))
        done += b
    q = st.queries(wl.n_queries)
    qd = torch.from_numpy(q).to(dev)
    rng = np.random.default_rng(123)
    deleted = set()
    live = np.ones(done, bool)
    for r in range(wl.churn_rounds):
        dl = st.deletes(np.nonzero(live)[0].astype(np.uint32), wl.churn_count())
        status = g.delete(torch.from_numpy(dl.astype(np.int32)).to(dev)).cpu().numpy()
        assert (status == 0).all()
        deleted |= set(dl.tolist())
        x = st.inserts(wl.churn_count())
        xs[done:done + len(x)] = x
        g.insert(torch.from_numpy(x).to(dev))
        live[dl] = False
        live = np.concatenate([live, np.ones(len(x), bool)])
        done += len(x)
        g.reclaim()
        e = g.export()
        n = done
        nbr, rho, deg, de, hs = e["nbr"], e["rho"], e["deg"], e["deleted"], e["has_slab"]
        s = g.stats()
        # flags: exactly the deleted ids; after reclaim no tombstone holds a slab
        assert np.array_equal(np.nonzero(de)[0], np.array(sorted(deleted)))
        assert not hs[de].any() and hs[~de].all()
        assert s["resident_slabs"] == s["live"] == int((~de).sum())
        # degree bound, padding, no self loops, no edge into a tombstone
        assert (deg <= wl.R).all()
        cols = np.arange(wl.R)[None, :]
        valid = cols < deg[:, None]
        assert (nbr[~valid] == 0xFFFFFFFF).all()
        assert not (nbr == np.arange(n, dtype=np.uint32)[:, None])[valid].any()
        assert not de[nbr[valid].astype(np.int64)].any()
        # sampled nodes: stored distances exact, lists sorted by (distance, id), no duplicates
        for u in rng.choice(np.nonzero(~de)[0], size=2000, replace=False):
            d = int(deg[u])
            ids = nbr[u, :d].astype(np.int64)
            true = _l2(xs[ids], xs[u])
            assert np.array_equal(rho[u, :d].astype(np.int64), true)
            keys = list(zip(true.tolist(), ids.tolist()))
            assert keys == sorted(keys) and len(set(ids.tolist())) == d
        # searches: deleted ids never returned; returned distances exact; recall
        ids, dist = g.search(qd, 10, 64)
        ids, dist = ids.cpu().numpy().astype(np.int64), dist.cpu().numpy()
        assert not (set(ids.ravel().tolist()) & deleted)
        for i in rng.choice(len(q), size=200, replace=False):
            assert np.array_equal(dist[i].astype(np.int64), _l2(xs[ids[i]], q[i]))
            assert (np.diff(dist[i].astype(np.int64)) >= 0).all()
        gt, gd = g.bruteforce(qd[:200], 10)
        gt, gd = gt.cpu().numpy().astype(np.int64), gd.cpu().numpy()
        # the brute-force kernel itself against numpy on a few queries
        live_ids = np.nonzero(~de)[0]
        for i in range(5):
            dd = _l2(xs[live_ids], q[i])
            order = np.lexsort((live_ids, dd))[:10]
            assert np.array_equal(gt[i], live_ids[order]) and np.array_equal(gd[i], dd[order])
        rec = recall_at(ids[:200], gt)
        assert rec >= 0.95, f"round {r}: Recall@10 {rec}"
        print(f"[scale] round {r}: properties hold, sampled distances exact, Recall@10 {rec:.4f}", flush=True)
    g.close()
