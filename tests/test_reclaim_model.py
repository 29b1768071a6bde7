"""The oracle's reclaim counters against Proposition 4's uniform-placement model.

Proposition 4 counts the dirty nodes (live nodes with at least one edge into a
tombstone) after t tombstones, when each tombstone's mean-in-degree worth of
in-edges sits on live nodes drawn independently and uniformly:
D(t) = L (1 - (1 - 1/L)^(d t)) ~ L (1 - exp(-t / tau)), tau = L / d.

Here the graph is built to be exactly that model: L live nodes, t further
nodes that will be deleted, and for each of those d in-edges from live nodes
drawn uniformly with replacement (a repeated draw adds no new edge). The
deleted nodes get empty lists, so the delete call has no repair target
(repair rebuilds the out-neighbors of a deleted node, Algorithm 3) and the
stranded in-edges stay until reclaim. Then:
- exactly: the oracle's dirty count is the number of distinct drawing nodes,
  its dead-edge count the number of distinct (live, tombstone) pairs, and the
  compaction publishes once per dirty node (Algorithm 4);
- in distribution: the dirty count lies within a few standard deviations of
  the closed form (the occupancy count's exact mean and variance), and the
  mean over seeds follows the saturating curve.
"""

import math

import numpy as np

import oracle

R = 32
DIM = 16


def model_graph(n_live, t, dbar, seed, k_live=2):
    """Lists of the uniform-placement model: for each tombstone-to-be u (ids
    n_live .. n_live + t - 1), dbar in-edge sources drawn uniformly from the
    live ids; besides, each live node points at k_live other live nodes
    (edges that compaction must keep, and that change no dirty count).
    Returns (lists per id, set of distinct (live, tombstone) pairs)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n_live, size=(t, dbar))
    lists = [set() for _ in range(n_live + t)]
    for w in range(n_live):
        for v in rng.integers(0, n_live, size=k_live):
            if int(v) != w:
                lists[w].add(int(v))
    for j in range(t):
        for w in src[j]:
            lists[int(w)].add(n_live + j)
    pairs = {(w, u) for w in range(n_live) for u in lists[w] if u >= n_live}
    return [sorted(x) for x in lists], pairs


def model_rows(n, seed):
    return np.random.default_rng(seed + 7).integers(0, 256, size=(n, DIM), dtype=np.uint8)


def occupancy_moments(L, m):
    """Mean and variance of the number of distinct bins hit by m uniform draws into L bins."""
    q1 = (1.0 - 1.0 / L) ** m
    q2 = (1.0 - 2.0 / L) ** m
    mean = L * (1.0 - q1)
    var = L * q1 + L * (L - 1) * q2 - (L * q1) ** 2
    return mean, max(var, 0.0)


def run_oracle(n_live, t, dbar, seed):
    n = n_live + t
    o = oracle.Oracle(oracle.METRIC_L2_U8, DIM, R, 32, n + 16, (R + 4) * n + 1000, n_entry=8)
    o.insert(model_rows(n, seed))  # one bootstrap batch
    lists, pairs = model_graph(n_live, t, dbar, seed)
    for u in range(n):
        o.set_list(u, lists[u])
    st = o.delete(np.arange(n_live, n, dtype=np.uint32))
    assert (st == 0).all()
    pub0 = o.meta()["pub_compact"]
    o.reclaim()
    m = o.meta()
    return m, lists, pairs, pub0, o


def test_counters_are_the_distinct_sources_and_pairs():
    for n_live, t, dbar, seed in ((300, 40, 4, 0), (500, 200, 8, 1), (200, 300, 3, 2)):
        m, lists, pairs, pub0, o = run_oracle(n_live, t, dbar, seed)
        dirty = sum(1 for w in range(n_live) if any(u >= n_live for u in lists[w]))
        assert m["dirty_last"] == dirty
        assert m["dead_last"] == len(pairs)
        assert m["pub_compact"] - pub0 == dirty
        assert m["resident"] == n_live  # every tombstone's slab freed, one per live node
        e = o.export()
        for w in range(n_live):  # the live edges stay, in (distance, id) order
            kept = [u for u in lists[w] if u < n_live]
            assert sorted(e["nbr"][w, :e["deg"][w]].tolist()) == kept


def test_dirty_count_follows_the_closed_form():
    n_live, dbar = 2000, 8
    tau = n_live / dbar
    means = []
    for t in (25, 100, 250, 600, 1500):
        obs = []
        for seed in range(3):
            m = run_oracle(n_live, t, dbar, 100 * t + seed)[0]
            obs.append(m["dirty_last"])
        mu, var = occupancy_moments(n_live, dbar * t)
        sd = math.sqrt(var)
        for d in obs:
            assert abs(d - mu) <= 5.0 * sd + 1.0, f"t={t}: dirty {d}, model {mu:.1f} +- {sd:.1f}"
        mean = float(np.mean(obs))
        # the exponential form of the proposition is within a fraction of a node of the exact one here
        assert abs(n_live * (1.0 - math.exp(-t / tau)) - mu) < 0.01 * n_live
        assert abs(mean - mu) <= 3.0 * sd / math.sqrt(len(obs)) + 1.0
        means.append(mean)
    # sublinear: each added tombstone dirties fewer new nodes than the previous ones did
    ts = (25, 100, 250, 600, 1500)
    slopes = [(means[i + 1] - means[i]) / (ts[i + 1] - ts[i]) for i in range(len(ts) - 1)]
    assert all(a > b for a, b in zip(slopes, slopes[1:]))
    assert means[-1] < n_live
