"""Pins of the oracle's round call (deletes, inserts and queries in one epoch).

A round runs the phases of Definition 2 in one launch epoch: tombstones and ids
first, then the insert searches and the queries on the state those tombstones
left, then forward prunes, repairs, reverse edges, refine and the recycle. The
tests pin it against the separate calls it must reduce to, and against an
index that only tombstones (so its state after a delete call is exactly the
state a round's searches see).
"""

import numpy as np
import pytest

import oracle
from common import index_params, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg
from test_oracle import check_invariants

NONE = 0xFFFFFFFF


def _built(wl, **kw):
    p = index_params(wl, n_entry=32, **kw)
    o = make_oracle(p)
    st = dg.Stream(wl)
    rows = [st.base(b) for b in wl.build_batches()]
    for x in rows:
        o.insert(x)
    return o, st, np.concatenate(rows)


def _same_export(a, b, where):
    ea, eb = a.export(), b.export()
    for f in ("nbr", "deg", "deleted", "has_slab"):
        assert np.array_equal(ea[f], eb[f]), f"{where}: {f} differs"
    assert np.array_equal(ea["rho"], eb["rho"]), where
    for k in ("next_id", "free", "resident", "retired", "pub_forward", "pub_repair", "pub_reverse", "pub_refine",
              "pub_compact", "freed"):
        assert ea["meta"][k] == eb["meta"][k], f"{where}: {k}"
    assert np.array_equal(a.entries(), b.entries()), where


def test_round_with_only_deletes_is_the_delete_call():
    wl = small_workload(n_base=1500, seed=31, rounds=1)
    a, st, _ = _built(wl)
    b, _, _ = _built(wl)
    live = np.nonzero(~a.export()["deleted"])[0].astype(np.uint32)
    dl = st.deletes(live, 60)
    dl = np.concatenate([dl, dl[:3], [10**6]]).astype(np.uint32)  # duplicates and an unknown id
    sa, _, _, _ = a.round(del_ids=dl, reclaim=True)
    sb = b.delete(dl)
    b.reclaim()
    assert np.array_equal(sa, sb)
    _same_export(a, b, "delete-only round")


def test_round_with_only_inserts_is_the_insert_call():
    wl = small_workload(n_base=1500, seed=32, rounds=1)
    a, st, _ = _built(wl)
    b, _, _ = _built(wl)
    x = st.inserts(75)
    _, ia, _, _ = a.round(x=x)
    ib = b.insert(x)
    assert np.array_equal(ia, ib)
    _same_export(a, b, "insert-only round")


def test_round_into_an_empty_index_bootstraps():
    wl = small_workload(n_base=500, seed=33, rounds=1)
    p = index_params(wl, n_entry=16)
    a, b = make_oracle(p), make_oracle(p)
    x = dg.Stream(wl).base(500)
    a.round(x=x)
    b.insert(x)
    _same_export(a, b, "bootstrap round")


@pytest.mark.parametrize("seed", [34, 35])
def test_round_searches_see_the_tombstoned_state(seed):
    # An index that only tombstones holds, after a delete call, exactly the
    # state a round's searches read. So the round's query results equal that
    # index's search results, and (without refine, which is the only phase
    # that rewrites a new node's list) its new nodes' lists equal the ones
    # that index's insert call gives them.
    wl = small_workload(n_base=1500, seed=seed, rounds=1)
    a, st, _ = _built(wl, refine=False)
    b, _, _ = _built(wl, refine=False, tombstone_only=True)
    live = np.nonzero(~a.export()["deleted"])[0].astype(np.uint32)
    dl = st.deletes(live, 75)
    x = st.inserts(75)
    q = st.queries(60)
    _, ids_a, qi, qd = a.round(del_ids=dl, x=x, q=q, k=10, L=48)
    b.delete(dl)
    qi_b, qd_b = b.search(q, 10, 48)
    assert np.array_equal(qi, qi_b) and np.array_equal(qd, qd_b)
    assert not (set(qi.ravel().tolist()) & set(dl.tolist()))
    ids_b = b.insert(x)
    assert np.array_equal(ids_a, ids_b)
    ea, eb = a.export(), b.export()
    new = ids_a.astype(np.int64)
    assert np.array_equal(ea["nbr"][new], eb["nbr"][new])
    assert np.array_equal(ea["rho"][new], eb["rho"][new])


def test_round_repairs_and_keeps_invariants():
    wl = small_workload(n_base=1500, seed=36, rounds=1)
    a, st, base = _built(wl)
    before = a.export()
    live = np.nonzero(~before["deleted"])[0].astype(np.uint32)
    dl = st.deletes(live, 75)
    x = st.inserts(75)
    m0 = a.meta()
    _, ids, _, _ = a.round(del_ids=dl, x=x, q=st.queries(5), k=5, L=32)
    m1 = a.meta()
    assert m1["pub_forward"] - m0["pub_forward"] == len(x)
    e = a.export()
    dset = set(dl.tolist())
    # every live out-neighbor of a deleted node was repaired: it lists no tombstone
    targets = {int(t) for u in dl for t in before["nbr"][u, :before["deg"][u]] if not e["deleted"][t]}
    assert m1["pub_repair"] - m0["pub_repair"] == len(targets)
    for t in targets:
        assert not (set(e["nbr"][t, :e["deg"][t]].tolist()) & dset)
    # new nodes never list a tombstone
    for v in ids:
        assert not (set(e["nbr"][v, :e["deg"][v]].tolist()) & dset)
    xs = np.concatenate([base, x])
    check_invariants(a, xs, dset, wl.R, since_reclaim=len(dl))


def test_round_pool_check_leaves_state_unchanged():
    wl = small_workload(n_base=800, seed=37, rounds=1, batch=100)
    p = index_params(wl, n_entry=16)
    # room for the build (calls of 100 need 100 (R + 2) free slabs) and 1,000 more:
    # a round of 100 inserts and 40 deletes needs 100 (R + 2) + 40 R
    p["id_capacity"] = 1000
    p["slab_capacity"] = 800 + 100 * (wl.R + 2) + 1000
    o = make_oracle(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        o.insert(st.base(b))
    before = o.export()
    live = np.nonzero(~before["deleted"])[0].astype(np.uint32)
    with pytest.raises(oracle.OracleError) as ei:
        o.round(del_ids=st.deletes(live, 40), x=st.inserts(100))
    assert ei.value.rc == -3
    after = o.export()
    for f in ("nbr", "deg", "deleted", "has_slab"):
        assert np.array_equal(before[f], after[f])
    assert before["meta"] == after["meta"]
