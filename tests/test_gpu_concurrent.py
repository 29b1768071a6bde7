"""Concurrent mode: searches on one stream while rounds publish on another,
with reverse edges applied offer by offer and racing by CAS (Algorithm 1's
retry loop runs).

Nothing here is deterministic, so nothing is compared with the oracle: the
checks are the paper's invariants and what a concurrent reader may see.
- Every result a search returns names a handed-out id with its exact distance,
  in (distance, id) order, and never an id deleted before the search was
  enqueued (deletion monotonicity seen by a reader, Proposition 1).
- Afterwards: the degree bound, no self loop or repeat, every stored distance
  exact, every deleted id still flagged; after the mode ends and a reclaim
  runs, one resident slab per live node (Proposition 3), no live node pointing
  at a tombstone, and the pool whole (nothing leaked while slabs were retired
  and not recycled during the mode).
- The retry path ran: compare-and-swap failures were counted.
"""

import numpy as np
import pytest

from common import index_params, make_gpu, recall_at, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _exact(q, x, ids):
    return ((x[ids.astype(np.int64)].astype(np.int64) - q[:, None, :].astype(np.int64)) ** 2).sum(-1)


def test_concurrent_searches_and_contended_reverse_edges():
    import torch
    wl = small_workload(n_base=20000, clusters=64, seed=61, batch=5000, rounds=0)
    p = index_params(wl, n_entry=256, W=2)
    rounds, churn = 6, 500
    p["id_capacity"] = wl.n_base + rounds * churn + 16
    p["max_batch"] = 5000
    # no slab is recycled while the mode lasts: room for every publication of it
    p["slab_capacity"] = 2 * p["id_capacity"] + rounds * churn * 4 * (wl.R + 2) * 4
    g = make_gpu(p)
    st = dg.Stream(wl)
    xs = [st.base(b) for b in wl.build_batches()]
    for x in xs:
        g.insert(torch.from_numpy(x).cuda())
    q = st.queries(1000)
    qd = torch.from_numpy(q).cuda()
    ids0, _ = g.search(qd, 10, 64)
    ids0 = ids0.cpu().numpy()
    inserts = [st.inserts(churn) for _ in range(rounds)]
    x_all = np.concatenate(xs + inserts)
    live = np.arange(wl.n_base, dtype=np.uint32)
    dels = []
    for _ in range(rounds):
        d = st.deletes(live, churn)
        live = np.setdiff1d(live, d)
        dels.append(d)
    S = torch.cuda.Stream()
    print("[concurrent] 20k uint8: 12 query batches on a side stream, 6 rounds of 500 + 500", flush=True)
    g.set_concurrent(True, S)
    results = []
    deleted_before = [set()]
    with torch.cuda.stream(S):
        for b in range(12):  # enqueued at once: they run while the rounds below publish
            results.append(g.search(qd, 10, 64))
    for r in range(rounds):
        g.delete(torch.from_numpy(dels[r].astype(np.int32)).cuda())
        g.insert(torch.from_numpy(inserts[r]).cuda())
    torch.cuda.synchronize()
    g.set_concurrent(False)
    s1 = g.stats()
    print(f"[concurrent] cas failures {s1['cas_failures']}, dropped {s1['publish_dropped']}, "
          f"reverse publications {s1['pub_reverse']}", flush=True)
    assert s1["cas_failures"] > 0, "no contended publication happened"
    assert s1["publish_dropped"] <= rounds * churn * wl.R // 100
    assert s1["error_bits"] == 0
    # what the concurrent readers saw
    for b, (ids, d) in enumerate(results):
        ids, d = ids.cpu().numpy().astype(np.uint32), d.cpu().numpy().astype(np.int64)
        ok = ids != 0xFFFFFFFF
        assert ok.all(), f"batch {b}: a query returned fewer than k results"
        assert (ids < wl.n_base + rounds * churn).all()
        assert np.array_equal(d, _exact(q, x_all, ids)), f"batch {b}: a distance is not the exact one"
        keys = d * (1 << 32) + ids
        assert (np.diff(keys, axis=1) > 0).all(), f"batch {b}: results not in (distance, id) order"
        assert recall_at(ids, ids0) >= 0.8, f"batch {b}: recall against the quiescent results collapsed"
    # the state after the mode
    e = g.export()
    n = e["nbr"].shape[0]
    gone = np.concatenate(dels)
    assert e["deleted"][gone].all() and e["deleted"].sum() == gone.size
    for u in range(n):
        k = int(e["deg"][u])
        nb = e["nbr"][u, :k].astype(np.int64)
        assert k <= wl.R and u not in nb and len(set(nb.tolist())) == k
        if k:
            ex = ((x_all[nb].astype(np.int64) - x_all[u].astype(np.int64)) ** 2).sum(1)
            assert np.array_equal(e["rho"][u, :k].astype(np.int64), ex), f"stored distances of {u}"
    g.reclaim()
    s2 = g.stats()
    e = g.export()
    assert s2["resident_slabs"] == s2["live"], "a slab leaked or a live node lost its slab"
    assert s2["free_slabs"] + s2["resident_slabs"] == p["slab_capacity"]
    for u in np.nonzero(~e["deleted"])[0]:
        assert not e["deleted"][e["nbr"][u, :e["deg"][u]].astype(np.int64)].any()
    # the index still answers like before (quality, not parity)
    ids2, _ = g.search(qd, 10, 64)
    gt, _ = g.bruteforce(qd, 10)
    assert recall_at(ids2.cpu().numpy(), gt.cpu().numpy()) >= 0.9
    g.close()
