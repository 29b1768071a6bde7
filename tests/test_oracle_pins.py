"""More pins of the CPU oracle, on the parts the first pins left open.

Each test checks the oracle against something other than itself:
- the float metric d = 1 - <q, x> and its (distance, id) order against numpy in
  FP64;
- the bf16 and FP8-e4m3 traversal distances against numpy over vectors
  decoded by torch's own casts (FP8 with the per-row scale max|x| / 448);
- the exact re-rank of the first rerank_mult * k live candidates, on a hand
  case where the traversal order and the exact order disagree;
- beam search with W = 2 (two entries expanded per step) on a hand-worked
  chain, with and without the visit cap, and with W = 2 and W = 4 on a list
  longer than the index, where it must return the exact kNN of the reachable
  set;
- the prune_cap truncation of RobustPrune's candidate set by hand;
- the bootstrap (first batch into an empty index): with a slack that prunes
  nothing, every list is the exact R nearest other batch members;
- the near-tie log: a float comparison decided by less than the tie margin is
  logged for the node whose list it decides, and none is logged where every
  margin is wide.
"""

import numpy as np
import pytest

import oracle
from common import index_params, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg
from test_oracle import _reachable, np_knn, tiny_oracle

NONE = 0xFFFFFFFF


def float_oracle(dim, n_cap, R=4, L=8, traversal=oracle.TRAV_NATIVE, rerank_mult=4, alpha=(6, 5), **kw):
    return oracle.Oracle(oracle.METRIC_IP_F32, dim, R, L, n_cap, 10 * n_cap + 100, alpha=alpha,
                         traversal=traversal, rerank_mult=rerank_mult, **kw)


def np_ip(q, x):
    """d = 1 - <q, x> in FP64 from FP32 values."""
    return 1.0 - q.astype(np.float64) @ x.astype(np.float64).T


def float_rows(n, dim, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x = x.astype(np.float32)
    x[0] = 0.0          # zero row
    x[1, :] = 0.0
    x[1, 2] = 1.0       # one-hot
    x[2] *= 3.0         # not unit length
    x[3] *= 1e-3
    return x


# ---- float distances ------------------------------------------------------------------

def test_ip_distance_and_order_match_numpy():
    x = float_rows(400, 24, 0)
    x[9] = x[5]  # exact tie: broken by id
    rng = np.random.default_rng(1)
    q = rng.standard_normal((30, 24)).astype(np.float32)
    q = np.concatenate([q, x[5:6]])
    o = float_oracle(24, 500, R=8, L=16)
    o.insert(x)
    ids, d = o.bruteforce(q, 12)
    D = np_ip(q, x)
    for r in range(q.shape[0]):
        order = np.lexsort((np.arange(400), D[r]))[:12]
        assert ids[r].tolist() == order.tolist()
        assert np.allclose(d[r], D[r][order], rtol=0, atol=1e-12)
    assert ids[-1, 0] == 5 and ids[-1, 1] == 9


def _trav_dists(o, q, n):
    """The oracle's traversal distance to every node: all nodes are entries and
    the list is longer than the index, so the initial list holds them all."""
    o.set_entries(np.arange(n, dtype=np.uint32))
    r = o.beam_search(q, L=n + 4, visit_cap=0)
    out = np.full(n, np.nan)
    out[r["list_ids"]] = r["list_d"]
    return out


def test_bf16_traversal_distance_matches_torch_decoded_rows():
    torch = pytest.importorskip("torch")
    x = float_rows(200, 32, 2)
    o = float_oracle(32, 300, traversal=oracle.TRAV_BF16)
    o.insert(x)
    dec = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    rng = np.random.default_rng(3)
    for _ in range(3):
        q = rng.standard_normal(32).astype(np.float32)
        got = _trav_dists(o, q, 200)
        exp = 1.0 - dec @ q.astype(np.float64)
        assert np.allclose(got, exp, rtol=0, atol=1e-12)
        # and not the exact distance (the copy is lossy)
        assert np.abs(got - np_ip(q[None], x)[0]).max() > 1e-6


def test_fp8_traversal_distance_matches_torch_decoded_rows_times_scale():
    torch = pytest.importorskip("torch")
    x = float_rows(200, 32, 4)
    o = float_oracle(32, 300, traversal=oracle.TRAV_FP8)
    o.insert(x)
    amax = np.abs(x).max(axis=1)
    s = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    codes = torch.from_numpy((x / s[:, None]).astype(np.float32)).to(torch.float8_e4m3fn)
    dec = codes.to(torch.float64).numpy() * s.astype(np.float64)[:, None]
    # the stored codes and scales are those torch produces
    assert np.array_equal(np.stack([o.codes(u)[1] for u in range(200)]), codes.view(torch.uint8).numpy())
    assert np.array_equal(np.array([o.codes(u)[2] for u in range(200)], np.float32), s)
    rng = np.random.default_rng(5)
    for _ in range(3):
        q = rng.standard_normal(32).astype(np.float32)
        got = _trav_dists(o, q, 200)
        exp = 1.0 - dec @ q.astype(np.float64)
        assert np.allclose(got, exp, rtol=0, atol=1e-12)


# ---- exact re-rank of the first rerank_mult * k live candidates ----------------------------

@pytest.mark.parametrize("trav,rows", [
    # FP8: x0[0] / s0 = 258.7 and x1[0] / s1 = 265.7 both round to the code 256, so
    # the traversal distances are 1 - 256 s0 = 0.5051 and 1 - 256 s1 = 0.5086
    # (node 0 first) while the exact ones are 0.5 and 0.49 (node 1 first)
    (oracle.TRAV_FP8, [[0.5, 0.8660254, 0, 0], [0.51, 0.86, 0, 0]]),
    # bf16: 0.501 rounds to 0.5, so both traversal distances are 0.5 and the tie
    # goes to the smaller id (node 0), while node 1 is exactly nearer
    (oracle.TRAV_BF16, [[0.5, 0, 0, 0], [0.501, 0, 0, 0]]),
])
def test_rerank_by_hand_when_traversal_order_is_wrong(trav, rows):
    x = np.array(rows, np.float32)
    q = np.array([[1, 0, 0, 0]], np.float32)
    exact = np_ip(q, x)[0]
    assert exact[1] < exact[0]
    res = {}
    for mult in (0, 1, 2):
        o = float_oracle(4, 10, R=2, L=2, traversal=trav, rerank_mult=mult)
        o.insert(x)
        o.set_entries([0, 1])
        t = _trav_dists(o, q[0], 2)
        assert t[0] <= t[1]  # traversal order: node 0 first
        o.set_entries([0, 1])
        res[mult] = o.search(q, 1, 2)
        if mult == 0:
            assert res[0][0][0, 0] == 0 and res[0][1][0, 0] == t[0]  # traversal distance itself
    # re-rank of the first candidate only: node 0 with its exact distance
    assert res[1][0][0, 0] == 0 and res[1][1][0, 0] == exact[0]
    # re-rank of the first two: node 1 wins on the exact distance
    assert res[2][0][0, 0] == 1 and res[2][1][0, 0] == exact[1]


# ---- beam search with several expansions per step ----------------------------------------

def _chain(W):
    # ids 0..9 at 0, 10, ..., 90 on a line; edges i -> i-1, i+1
    x = (np.arange(10) * 10).astype(np.uint8).reshape(-1, 1)
    o = tiny_oracle(1, 20, R=2, L=3, W=W)
    o.insert(x)
    for i in range(10):
        o.set_list(i, [j for j in (i - 1, i + 1) if 0 <= j < 10])
    o.set_entries([0, 9])
    return o


def test_beam_search_two_expansions_per_step_by_hand():
    # Query 47, L = 3, entries {0, 9}: start [(1849,9), (2209,0)].
    # step 1 expands 9 and 0: 8 (1089) in; 1 (1369) in, 0 evicted
    #   -> [(1089,8), (1369,1), (1849,9)]
    # step 2 expands 8 and 1: 7 (529) in, 9 evicted; 2 (729) in, 1 evicted
    # step 3 expands 7 and 2: 6 (169), 3 (289) in
    # step 4 expands 6 and 3: 5 (9), 4 (49) in -> [(9,5), (49,4), (169,6)]
    # step 5 expands 5 and 4: every neighbor seen; nothing open: stop.
    o = _chain(2)
    r = o.beam_search(np.array([47], np.uint8), L=3, visit_cap=100)
    assert r["visited_ids"].tolist() == [9, 0, 8, 1, 7, 2, 6, 3, 5, 4]
    assert r["list_ids"].tolist() == [5, 4, 6]
    assert r["list_d"].tolist() == [9.0, 49.0, 169.0]
    assert r["list_expanded"].all()
    assert r["distances"] == 10
    # the visit cap counts single expansions: after step 1 (two), step 2 may
    # expand only one more (8), whose neighbor 7 still enters the list
    r3 = o.beam_search(np.array([47], np.uint8), L=3, visit_cap=3)
    assert r3["visited_ids"].tolist() == [9, 0, 8]
    assert r3["list_ids"].tolist() == [7, 8, 1]
    # one expansion per step walks only from the nearer end
    o1 = _chain(1)
    r1 = o1.beam_search(np.array([47], np.uint8), L=3, visit_cap=100)
    assert r1["visited_ids"].tolist() == [9, 8, 7, 6, 5, 4]
    assert r1["list_ids"].tolist() == [5, 4, 6]
    assert r1["distances"] == 8


@pytest.mark.parametrize("W", [2, 4])
def test_search_with_full_list_is_exact_knn_of_reachable_several_expansions(W):
    wl = small_workload(n_base=600, clusters=4, seed=11 + W, batch=200, rounds=0)
    p = index_params(wl, n_entry=4, W=W)
    o = make_oracle(p)
    st = dg.Stream(wl)
    xs = [st.base(b) for b in wl.build_batches()]
    for x in xs:
        o.insert(x)
    x = np.concatenate(xs)
    e = o.export()
    reach = _reachable(e["nbr"], e["deg"], o.entries())
    q = st.queries(25)
    ids, d = o.search(q, 10, 1024)
    ei, ed = np_knn(q, x[reach], reach, 10)
    assert np.array_equal(ids, ei)
    assert np.array_equal(d.astype(np.int64), ed)


# ---- RobustPrune's candidate cap -----------------------------------------------------------

def test_prune_cap_truncates_after_order_duplicates_and_tombstones():
    # 1-d points 0..5 (ids 0..5), owner 0; slack 1000 prunes only coincident
    # points, so without a cap every admissible candidate is kept in order.
    x = np.arange(6, dtype=np.uint8).reshape(-1, 1)
    cand = [5, 4, 3, 3, 2, 1, 0]  # a duplicate and the owner itself
    full = tiny_oracle(1, 10, R=5, L=4, alpha=(1000, 1), prune_cap=256)
    full.insert(x)
    assert full.robust_prune(0, cand)[0].tolist() == [1, 2, 3, 4, 5]
    capped = tiny_oracle(1, 10, R=5, L=4, alpha=(1000, 1), prune_cap=3)
    capped.insert(x)
    ids, d = capped.robust_prune(0, cand)
    assert ids.tolist() == [1, 2, 3] and d.tolist() == [1.0, 4.0, 9.0]
    # the cap counts admissible candidates: a tombstone does not use a place
    capped.delete(np.array([2], np.uint32))
    assert capped.robust_prune(0, cand)[0].tolist() == [1, 3, 4]


# ---- bootstrap: the first batch into an empty index ----------------------------------------

def test_bootstrap_lists_are_exact_r_nearest_with_a_slack_that_prunes_nothing():
    # Slack 1000 makes RobustPrune keep the R nearest admissible candidates; the
    # bootstrap offers each node its visit_cap (= 4 L_build = 32) nearest batch
    # members, and reverse offers cannot displace an exact R-NN list, so every
    # list must equal the brute-force 8 nearest other members by (distance, id).
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, size=(300, 16), dtype=np.uint8)
    o = tiny_oracle(16, 400, R=8, L=8, alpha=(1000, 1))
    o.insert(x)
    e = o.export()
    D = ((x.astype(np.int64)[:, None, :] - x.astype(np.int64)[None, :, :]) ** 2).sum(-1)
    for u in range(300):
        order = [v for v in np.lexsort((np.arange(300), D[u])).tolist() if v != u][:8]
        assert e["nbr"][u].tolist() == order, u
        assert e["rho"][u].astype(np.int64).tolist() == D[u, order].tolist()


def test_float_bootstrap_lists_are_exact_r_nearest():
    x = float_rows(250, 16, 10)[4:]  # unit rows only
    o = float_oracle(16, 300, R=6, L=8, alpha=(1000, 1))
    o.insert(x)
    e = o.export()
    D = np_ip(x, x)
    n = x.shape[0]
    for u in range(n):
        order = [v for v in np.lexsort((np.arange(n), D[u])).tolist() if v != u][:6]
        assert e["nbr"][u].tolist() == order, u
        assert np.allclose(e["rho"][u], D[u, order], rtol=0, atol=1e-12)


# ---- the near-tie log ------------------------------------------------------------------------

def test_near_tie_logged_for_the_node_whose_prune_it_decides():
    # owner 0 at e0; candidates 1 and 2 at exactly the same distance from it
    # (mirror images), and 3 well apart: the order of 1 and 2 is decided by
    # less than the margin, so pruning for 0 logs 0.
    x = np.zeros((5, 4), np.float32)
    x[0] = [1, 0, 0, 0]
    x[1] = [0.6, 0.8, 0, 0]
    x[2] = [0.6, -0.8, 0, 0]
    x[3] = [0, 0, 1, 0]
    x[4] = [0, 0, 0, 1]
    o = float_oracle(4, 10, R=4, L=4)
    o.insert(x)
    o.near_ties(clear=True)
    ids, _ = o.robust_prune(0, [1, 2, 3])
    assert len(o.near_ties()) == 0  # a prune outside a call has no owner
    # within an insert call the new node's forward prune is logged for it
    o2 = float_oracle(4, 10, R=4, L=8, n_entry=4)
    o2.insert(x[1:5])            # ids 0..3: bootstrap
    o2.near_ties(clear=True)
    o2.insert(x[0:1])            # id 4 sees ids 0 and 1 at the same distance
    ties = o2.near_ties()
    assert 4 in ties and ties[4] == 0.0  # the two distances are equal


def test_no_near_tie_on_the_integer_path():
    wl = small_workload(n_base=800, clusters=4, seed=5, batch=400, rounds=0)
    o = make_oracle(index_params(wl, n_entry=16))
    st = dg.Stream(wl)
    for b in wl.build_batches():
        o.insert(st.base(b))
    assert len(o.near_ties()) == 0
