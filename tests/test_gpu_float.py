"""Float embeddings (inner product) on the GPU against the FP64 oracle.

Three traversal copies: FP32, bf16, and FP8 e4m3 with a per-row scale, each
accumulating in FP32; stored lists, their distances and RobustPrune use the
FP32 rows. Tolerance: 1e-5 relative distance; result ids may differ only
where the oracle's own distances tie within that tolerance.
"""

import numpy as np
import pytest

import oracle
from common import (exact_ip_dist, float_workload, index_params, make_gpu_f, make_oracle_f)
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def _torch():
    import torch
    return torch


def _vectors(n, dim, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x = x.astype(np.float32)
    # edge rows: zero row, one-hot, tiny and large magnitudes (non-unit on purpose)
    x[0] = 0.0
    x[1] = 0.0
    x[1, 3] = 1.0
    x[2] *= 1e-6
    x[3] *= 3.0
    return x


@pytest.mark.parametrize("trav", [1, 2])
def test_traversal_codes_match_oracle(trav):
    torch = _torch()
    wl = float_workload(n_base=300, batch=300, rounds=0)
    p = index_params(wl, n_entry=16)
    x = _vectors(300, 96, 5)
    o = make_oracle_f(p, traversal=trav)
    g = make_gpu_f(p, traversal=trav)
    o.insert(x)
    g.insert(torch.from_numpy(x).cuda())
    if trav == 1:
        got = g.rows(0, 300, 1)
        exp = np.stack([o.codes(u)[0] for u in range(300)])
        assert np.array_equal(got, exp)
    else:
        codes, scales = g.rows(0, 300, 2), g.rows(0, 300, 3)
        exp_c = np.stack([o.codes(u)[1] for u in range(300)])
        exp_s = np.array([o.codes(u)[2] for u in range(300)], np.float32)
        assert np.array_equal(scales, exp_s)
        assert np.array_equal(codes, exp_c)
    g.close()


def _compare_results(q, x, ids_o, d_o, ids_g, d_g, where):
    """Distances within RTOL; a differing id must tie (within RTOL) with the oracle's at that rank."""
    ids_o = ids_o.astype(np.int64)
    ids_g = ids_g.astype(np.int64)
    ok = np.isfinite(d_o)
    assert np.array_equal(np.isfinite(d_g), ok), f"{where}: result counts differ"
    rel = np.abs(d_g[ok] - d_o[ok]) / np.maximum(np.abs(d_o[ok]), 1e-3)
    assert rel.max(initial=0) <= RTOL, f"{where}: distance error {rel.max()}"
    diff = (ids_o != ids_g) & ok
    n_diff = 0
    for r, c in zip(*np.nonzero(diff)):
        n_diff += 1
        dg_exact = exact_ip_dist(q[r], x, ids_g[r, c:c + 1])[0]
        assert abs(dg_exact - d_o[r, c]) <= RTOL * max(abs(d_o[r, c]), 1e-3), (
            f"{where}: query {r} rank {c}: gpu id {ids_g[r, c]} ({dg_exact}) vs oracle id {ids_o[r, c]} ({d_o[r, c]})")
    return n_diff


@pytest.mark.parametrize("trav", [0, 1, 2])
def test_search_parity_on_identical_graph(trav):
    torch = _torch()
    wl = float_workload(n_base=2000, batch=500, rounds=0, seed=7)
    p = index_params(wl, n_entry=32)
    o = make_oracle_f(p, traversal=trav)
    g = make_gpu_f(p, traversal=trav)
    st = dg.Stream(wl)
    xs = []
    for b in wl.build_batches():
        xb = st.base(b)
        xs.append(xb)
        o.insert(xb)
        g.insert(torch.from_numpy(xb).cuda())
    x = np.concatenate(xs)
    e = o.export()
    n = e["meta"]["next_id"]
    g.set_lists(np.arange(n, dtype=np.uint32), e["nbr"], e["deg"])
    ge = g.export()
    assert np.array_equal(np.sort(ge["nbr"], axis=1), np.sort(e["nbr"], axis=1)), "imported graph differs"
    q = st.queries(300)
    total = 0
    for L in (16, 48, 100):
        io, do = o.search(q, 10, L)
        ig, dgp = g.search(torch.from_numpy(q).cuda(), 10, L)
        total += _compare_results(q, x, io, do, ig.cpu().numpy(), dgp.cpu().numpy().astype(np.float64),
                                  f"trav={trav} L={L}")
    print(f"[float parity] trav={trav}: {total} near-tie swaps", flush=True)
    g.close()


def _hops(sources, nbr_a, deg_a, nbr_b, deg_b, depth):
    """Nodes within `depth` hops of `sources` in the union of two graphs, edges
    taken in both directions."""
    n = nbr_a.shape[0]
    adj = [set() for _ in range(n)]
    for nbr, deg in ((nbr_a, deg_a), (nbr_b, deg_b)):
        for u in range(n):
            for v in nbr[u, :deg[u]].tolist():
                adj[u].add(v)
                adj[v].add(u)
    seen = set(int(s) for s in sources)
    frontier = set(seen)
    for _ in range(depth):
        frontier = {v for u in frontier for v in adj[u]} - seen
        seen |= frontier
    return seen


@pytest.mark.parametrize("trav", [0, 1, 2])
def test_float_maintenance_matches_oracle(trav):
    """End-to-end protocol on the float path. After every call the maintained
    lists are compared as neighbor sets. Until they first differ, they must be
    identical, with the same flags, pool counts and publications; at the call
    where they first differ, the oracle must have logged near-ties (float
    comparisons decided by less than 1e-5 relative) in that call, and every
    differing list must lie within three hops of a logged node in the union of
    the two graphs (a tie in node v's search or prune changes v's list, then
    the reverse offers v makes, then the same-batch refine of nodes two hops
    from v). From then on the two runs are different graphs, and only flags,
    stored distances against FP64 and the degree bound are compared."""
    torch = _torch()
    wl = float_workload(n_base=1500, batch=500, rounds=2, seed=11)
    p = index_params(wl, n_entry=32)
    o = make_oracle_f(p, traversal=trav)
    g = make_gpu_f(p, traversal=trav)
    st = dg.Stream(wl)
    xs = np.zeros((p["id_capacity"], wl.dim), np.float32)
    state = {"diverged": None, "n": 0}

    def compare(where):
        tie_margin = o.near_ties(clear=True)
        ties = set(tie_margin)
        eo, eg = o.export(), g.export()
        n = eo["meta"]["next_id"]
        assert np.array_equal(eo["deleted"], eg["deleted"]), where
        differ = [u for u in range(n) if set(eo["nbr"][u, :eo["deg"][u]].tolist()) !=
                  set(eg["nbr"][u, :eg["deg"][u]].tolist())]
        # the GPU's lists are valid whatever happened before: degree bound, no
        # self loop or repeat, stored distances within 1e-5 of FP64
        for u in range(n):
            d = int(eg["deg"][u])
            ids = eg["nbr"][u, :d].astype(np.int64)
            assert d <= wl.R and u not in ids and len(set(ids.tolist())) == d, f"{where}: list of {u}"
            if d:
                ex = 1.0 - xs[ids].astype(np.float64) @ xs[u].astype(np.float64)
                rel = np.abs(eg["rho"][u, :d] - ex) / np.maximum(np.abs(ex), 1e-3)
                assert rel.max() <= RTOL, f"{where}: stored distance of {u}"
        if state["diverged"] is None:
            if differ:
                assert ties, f"{where}: {len(differ)} lists differ and the oracle logged no near-tie"
                near = _hops(ties, eo["nbr"], eo["deg"], eg["nbr"], eg["deg"], 3)
                far = [u for u in differ if u not in near]
                assert not far, f"{where}: lists of {far[:10]} differ, none within 3 hops of a near-tie {sorted(ties)[:10]}"
                state["diverged"] = where
                tight = {u for u, m in tie_margin.items() if m < 1e-6}
                near_t = _hops(tight, eo["nbr"], eo["deg"], eg["nbr"], eg["deg"], 3) if tight else set()
                print(f"[float maint] trav={trav} {where}: first divergence, {len(differ)} lists; "
                      f"{sum(u in ties for u in differ)} of them own a near-tie, "
                      f"{sum(u in near_t for u in differ)} lie within 3 hops of a tie below 1e-6 "
                      f"({len(tight)} such nodes)", flush=True)
            else:
                sg, mo = g.stats(), eo["meta"]
                assert sg["resident_slabs"] == mo["resident"] and sg["free_slabs"] == mo["free"], where
                for k in ("pub_forward", "pub_repair", "pub_reverse", "pub_refine", "pub_compact", "freed"):
                    assert mo[k] == sg[k], f"{where}: {k}"
        print(f"[float maint] trav={trav} {where}: {len(differ)} lists differ, {len(ties)} nodes with near-ties, "
              f"first divergence: {state['diverged']}", flush=True)

    def insert(xb):
        n0 = state["n"]
        xs[n0:n0 + xb.shape[0]] = xb
        state["n"] += xb.shape[0]
        o.insert(xb)
        g.insert(torch.from_numpy(xb).cuda())

    for bi, b in enumerate(wl.build_batches()):
        insert(st.base(b))
        compare(f"build batch {bi}")
    for r in range(wl.churn_rounds):
        live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
        dl = st.deletes(live, wl.churn_count())
        o.delete(dl)
        g.delete(torch.from_numpy(dl.astype(np.int32)).cuda())
        compare(f"round {r} delete")
        insert(st.inserts(wl.churn_count()))
        compare(f"round {r} insert")
        o.reclaim()
        g.reclaim()
        compare(f"round {r} reclaim")
        if state["diverged"] is None:
            sg, mo = g.stats(), o.meta()
            assert sg["resident_slabs"] == mo["resident"] and sg["free_slabs"] == mo["free"]
    g.close()
