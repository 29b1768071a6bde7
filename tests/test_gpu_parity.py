"""GPU path vs the CPU oracle through the C ABI: bit-exact on the uint8 path.

Every insert / delete / reclaim call is followed by a full comparison of the
exported state (neighbor lists with their distances, degrees, deletion flags,
slab presence, pool counts, publication counters, entry set), and every
search by a comparison of ids and distances.
"""

import numpy as np
import pytest

from common import assert_same_state, index_params, make_gpu, make_oracle, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def run_parity(wl, n_entry=64, refine=True, tombstone_only=False, search_L=(64,), k=10, n_queries=200,
               reclaim=True, W=1, visit_mult=4, **gpu_kw):
    torch = _torch()
    p = index_params(wl, n_entry=n_entry, refine=refine, tombstone_only=tombstone_only, W=W, visit_mult=visit_mult)
    o = make_oracle(p)
    g = make_gpu(p, **gpu_kw)
    st = dg.Stream(wl)
    dev = torch.device("cuda")
    print(f"[parity] {wl.name} n={wl.n_base} rounds={wl.churn_rounds} n_entry={n_entry} refine={refine} "
          f"tombstone_only={tombstone_only} gpu_kw={gpu_kw}", flush=True)
    for bi, b in enumerate(wl.build_batches()):
        x = st.base(b)
        ido = o.insert(x)
        idg = g.insert(torch.from_numpy(x).to(dev)).cpu().numpy().astype(np.uint32)
        assert np.array_equal(ido, idg)
        assert_same_state(o, g, f"build batch {bi}")
    q = st.queries(n_queries)
    qd = torch.from_numpy(q).to(dev)

    def check_search(where):
        for L in search_L:
            io, do = o.search(q, k, L)
            ig, dgpu = g.search(qd, k, L)
            ig = ig.cpu().numpy().astype(np.uint32)
            dgpu = dgpu.cpu().numpy()
            assert np.array_equal(io, ig), f"{where} L={L}: result ids differ"
            assert np.array_equal(do, dgpu), f"{where} L={L}: result distances differ"

    check_search("after build")
    for r in range(wl.churn_rounds):
        live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
        dl = st.deletes(live, wl.churn_count())
        so = o.delete(dl)
        sg = g.delete(torch.from_numpy(dl.astype(np.int32)).to(dev)).cpu().numpy()
        assert np.array_equal(so, sg)
        assert_same_state(o, g, f"round {r} delete")
        x = st.inserts(wl.churn_count())
        o.insert(x)
        g.insert(torch.from_numpy(x).to(dev))
        assert_same_state(o, g, f"round {r} insert")
        if reclaim:
            o.reclaim()
            g.reclaim()
            assert_same_state(o, g, f"round {r} reclaim")
        check_search(f"round {r}")
    g.close()


def test_parity_small_default():
    run_parity(small_workload())


def test_parity_small_no_refine_two_L():
    # L = 200 takes the start-set path that writes the distance matrix
    run_parity(small_workload(seed=2), refine=False, search_L=(16, 32, 100, 200))


def test_parity_short_build_list_filtered_bootstrap():
    # L_build = 32: the bootstrap's candidate lists (4 L_build = 128) take the
    # filtered start-set path with the batch itself as the start set, where each
    # row skips itself
    wl = dg.Workload("small_lb32", dg.Mixture(128, 8, 18.0, dg.METRIC_L2_U8), 1500, 32, 32, 6, 5,
                     1, 0.05, 200, 10, (32,), 13, 700, 700)
    run_parity(wl, search_L=(16, 32))


def test_parity_many_entries_filtered_start_set():
    # 1,000 entries: four spans of start rows, so the bounded keys of a query
    # come from several spans and are merged before the sort
    run_parity(small_workload(seed=12, rounds=1), n_entry=1000, search_L=(10, 64, 128))


def test_parity_row_lengths():
    # 64-, 256- and 512-byte rows: start-set scoring with slices past the row,
    # four slices held in registers, and rows scored in two chunks (smaller R
    # and L_build keep the longer rows' staged prunes within one workgroup's LDS,
    # which index creation checks)
    for dim, R, L_build in ((64, 16, 32), (256, 16, 32), (512, 8, 16)):
        wl = dg.Workload(f"rows{dim}", dg.Mixture(dim, 8, 18.0, dg.METRIC_L2_U8), 1200, R, L_build, 6, 5,
                         1, 0.05, 200, 10, (32,), 30 + dim, 400, 400)
        run_parity(wl, n_entry=300, search_L=(16, 48))


def test_parity_tombstone_only():
    run_parity(small_workload(seed=3), tombstone_only=True)


def test_parity_ragged_batches():
    # batch sizes that are not multiples of the wave width or of 4 waves
    wl = small_workload(n_base=1237, seed=4, batch=301, rounds=2, churn=0.03)
    run_parity(wl, n_entry=37, search_L=(10, 64))


def test_parity_knob_invariance():
    # visited-table size, waves per block and lanes per row must not change any result
    wl = small_workload(seed=5, n_base=1500, rounds=1)
    run_parity(wl, vt_slots=64, waves_per_block=1)
    run_parity(wl, vt_slots=4096, waves_per_block=2)
    run_parity(wl, row_lanes=4, W=2, search_L=(32, 64, 100))


def test_autotune_choice_leaves_results_unchanged():
    # the autotuner only picks result-invariant knobs: results before and after
    # are identical, and identical to the oracle's
    torch = _torch()
    wl = small_workload(seed=14, n_base=6000, clusters=16, batch=2000, rounds=0)
    p = index_params(wl, n_entry=512, W=2)
    o, g = make_oracle(p), make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        x = st.base(b)
        o.insert(x)
        g.insert(torch.from_numpy(x).cuda())
    q = st.queries(3000)
    qd = torch.from_numpy(q).cuda()
    before = [g.search(qd, 10, L) for L in (32, 64, 128)]
    tune = g.autotune(qd, 10, 64)
    print(f"[autotune] {tune}", flush=True)
    assert tune["row_lanes"] in (4, 8) and tune["ms"] <= tune["ms_default"] * 1.05
    for L, (i0, d0) in zip((32, 64, 128), before):
        i1, d1 = g.search(qd, 10, L)
        assert torch.equal(i0, i1) and torch.equal(d0, d1), f"L={L}: results changed with the tuned knobs"
        io, do = o.search(q, 10, L)
        assert np.array_equal(io, i1.cpu().numpy().astype(np.uint32)) and np.array_equal(do, d1.cpu().numpy())
    g.close()


def test_parity_two_slot_register_list():
    # lists of 65..128 entries held as two slots per lane: one entry in the
    # second slot (L = 65), a full second slot (L = 128), an initial list
    # shorter than one slot (37 entries), and a crowded visited table at W = 2
    run_parity(small_workload(seed=15, rounds=1), n_entry=37, search_L=(65, 127))
    run_parity(small_workload(seed=16, rounds=1), n_entry=200, W=2, search_L=(65, 128), vt_slots=64)
    # insert searches on the two-slot list (L_build = 96; a visit cap of 2 L_build
    # keeps the maintenance kernels' LDS within a workgroup's)
    wl = dg.Workload("lbuild96", dg.Mixture(128, 8, 18.0, dg.METRIC_L2_U8), 1200, 32, 96, 6, 5,
                     1, 0.05, 200, 10, (96,), 17, 400, 400)
    run_parity(wl, search_L=(96,), visit_mult=2)


def test_parity_two_expansions_per_iteration():
    # W = 2: two slabs read side by side by one wavefront
    run_parity(small_workload(seed=6, rounds=2), W=2, search_L=(16, 64, 101))


def test_parity_two_expansions_crowded_visited_table():
    # W = 2 with a visited table far too small: ids listed in both slabs pass
    # the crowded table twice and must reach the merge once
    run_parity(small_workload(seed=9, rounds=2), W=2, search_L=(16, 64, 101), vt_slots=64)


def test_parity_heavy_ties():
    # Two distinct vectors repeated (a tenth of the rows nudged by one or two
    # units): most distances tie, so more start rows lie at or below the
    # selection bound than fit in LDS, and the initial lists come from the
    # bisection and tie paths of the start-set selection.
    torch = _torch()
    wl = small_workload(n_base=3000, seed=8, batch=1500, rounds=1, dim=32)
    p = index_params(wl, n_entry=2048)
    o, g = make_oracle(p), make_gpu(p)
    rng = np.random.default_rng(8)
    pats = rng.integers(0, 256, size=(2, 32), dtype=np.uint8)

    def rows(n):
        x = pats[rng.integers(0, 2, size=n)].copy()
        m = rng.random(n) < 0.1
        x[m, 0] ^= rng.integers(1, 3, size=int(m.sum())).astype(np.uint8)
        return x

    def check_search(where):
        q = rows(100)
        for L in (16, 64):
            io, do = o.search(q, 10, L)
            ig, dgpu = g.search(torch.from_numpy(q).cuda(), 10, L)
            assert np.array_equal(io, ig.cpu().numpy().astype(np.uint32)), f"{where} L={L}: ids"
            assert np.array_equal(do, dgpu.cpu().numpy()), f"{where} L={L}: distances"

    print("[parity] heavy ties", flush=True)
    for bi in range(2):
        x = rows(1500)
        ido = o.insert(x)
        idg = g.insert(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.uint32)
        assert np.array_equal(ido, idg)
        assert_same_state(o, g, f"ties batch {bi}")
    check_search("ties after build")
    live = np.nonzero(~o.export()["deleted"])[0].astype(np.uint32)
    dl = rng.choice(live, size=150, replace=False).astype(np.uint32)
    assert np.array_equal(o.delete(dl), g.delete(torch.from_numpy(dl.astype(np.int32)).cuda()).cpu().numpy())
    x = rows(150)
    o.insert(x)
    g.insert(torch.from_numpy(x).cuda())
    o.reclaim()
    g.reclaim()
    assert_same_state(o, g, "ties after churn")
    check_search("ties after churn")
    g.close()


def test_parity_four_expansions_per_step():
    # W = 4: four slabs per step, scored in one batch (two halves of 64 lanes)
    # for L <= 64, in two merges for longer lists
    run_parity(small_workload(seed=10, rounds=2), W=4, search_L=(16, 64, 101))


def test_parity_four_expansions_crowded_visited_table():
    run_parity(small_workload(seed=11, rounds=1), W=4, search_L=(32, 100), vt_slots=64)
