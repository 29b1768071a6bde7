"""Reclaim on the GPU over graphs of Proposition 4's uniform-placement model:
the same hand-built graph (see test_reclaim_model.py) imported into the GPU
index and the oracle, the tombstones deleted, one reclaim; the dirty and
dead-edge counts, the compaction's publications and the whole state after
it must be identical, and the dirty count must be that of the model's
construction (distinct in-edge sources)."""

import numpy as np
import pytest

from test_reclaim_model import DIM, R, model_graph, model_rows, run_oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_live,t,dbar,seed", [(2000, 250, 8, 3), (3000, 1500, 8, 4), (700, 60, 2, 5)])
def test_reclaim_counts_match_the_oracle(n_live, t, dbar, seed):
    import torch

    from paper_2607_02543_amd import etale
    n = n_live + t
    print(f"[reclaim-model] L={n_live} t={t} dbar={dbar} seed={seed}", flush=True)
    m, lists, pairs, _, o = run_oracle(n_live, t, dbar, seed)
    g = etale.Index(DIM, R=R, L_build=32, alpha=(6, 5), n_entry=8, id_capacity=n + 16,
                    slab_capacity=(R + 4) * n + 1000, max_batch=n)
    g.insert(torch.from_numpy(model_rows(n, seed)).cuda())
    nbr = np.full((n, R), 0xFFFFFFFF, np.uint32)
    deg = np.zeros(n, np.uint32)
    for u, lst in enumerate(lists):
        nbr[u, :len(lst)] = lst
        deg[u] = len(lst)
    g.set_lists(np.arange(n, dtype=np.uint32), nbr, deg)
    st = g.delete(torch.arange(n_live, n, dtype=torch.int32).cuda()).cpu().numpy()
    assert (st == 0).all()
    c0 = g.stats()["pub_compact"]
    g.reclaim()
    s = g.stats()
    assert s["error_bits"] == 0
    dirty = sum(1 for w in range(n_live) if any(u >= n_live for u in lists[w]))
    assert s["dirty_last"] == m["dirty_last"] == dirty
    assert s["dead_edges_last"] == m["dead_last"] == len(pairs)
    assert s["pub_compact"] - c0 == dirty
    assert s["resident_slabs"] == m["resident"] == n_live
    eo, eg = o.export(), g.export()
    for f in ("deg", "deleted", "has_slab", "nbr"):
        assert np.array_equal(eo[f], eg[f]), f"{f} differs after reclaim"
    assert np.array_equal(eo["rho"].astype(np.int64), eg["rho"].astype(np.int64))
    g.close()
