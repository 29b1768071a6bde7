"""Shared helpers of the test suite: configurations and state comparison."""

import numpy as np

import oracle
from paper_2607_02543_amd import datagen as dg


def small_workload(n_base=2000, clusters=8, seed=1, batch=500, rounds=2, churn=0.05, dim=128):
    return dg.Workload("small", dg.Mixture(dim, clusters, 18.0, dg.METRIC_L2_U8), n_base, 32, 64, 6, 5,
                       rounds, churn, 200, 10, (64,), seed, batch, batch)


def index_params(wl, n_entry=64, refine=True, tombstone_only=False, max_batch=None, slack=2, W=1, visit_mult=4):
    cap = wl.id_capacity()
    mb = max_batch or max(wl.build_batch_max, wl.churn_count(), 1)
    return dict(dim=wl.dim, R=wl.R, L_build=wl.L_build, alpha=(wl.alpha_num, wl.alpha_den), n_entry=n_entry,
                refine=refine, tombstone_only=tombstone_only, id_capacity=cap,
                slab_capacity=slack * cap + mb * (wl.R + 2), max_batch=mb, W=W, visit_mult=visit_mult)


def make_oracle(p):
    return oracle.Oracle(oracle.METRIC_L2_U8, p["dim"], p["R"], p["L_build"], p["id_capacity"], p["slab_capacity"],
                         alpha=p["alpha"], n_entry=p["n_entry"], refine=p["refine"],
                         tombstone_only=p["tombstone_only"], W=p["W"], visit_mult=p.get("visit_mult", 4))


def make_gpu(p, **kw):
    from paper_2607_02543_amd import etale
    return etale.Index(p["dim"], R=p["R"], L_build=p["L_build"], alpha=p["alpha"], n_entry=p["n_entry"],
                       refine=p["refine"], tombstone_only=p["tombstone_only"], id_capacity=p["id_capacity"],
                       slab_capacity=p["slab_capacity"], max_batch=p["max_batch"], W=p["W"],
                       visit_mult=p.get("visit_mult", 4), **kw)


def assert_same_state(o, g, where=""):
    eo, eg = o.export(), g.export()
    n = eo["meta"]["next_id"]
    assert eg["nbr"].shape[0] == n, where
    for field in ("deg", "deleted", "has_slab"):
        bad = np.nonzero(eo[field] != eg[field])[0]
        assert bad.size == 0, f"{where}: {field} differs at ids {bad[:10]}"
    bad = np.nonzero((eo["nbr"] != eg["nbr"]).any(axis=1))[0]
    assert bad.size == 0, (f"{where}: lists differ at {bad.size} ids, first {bad[:5]}; "
                           f"oracle {eo['nbr'][bad[0]]} gpu {eg['nbr'][bad[0]]}")
    ro = eo["rho"].astype(np.int64)
    rg = eg["rho"].astype(np.int64)
    assert np.array_equal(ro, rg), f"{where}: list distances differ"
    mo, sg = eo["meta"], g.stats()
    assert sg["error_bits"] == 0, where
    assert mo["free"] == sg["free_slabs"], f"{where}: free {mo['free']} vs {sg['free_slabs']}"
    assert mo["resident"] == sg["resident_slabs"], where
    for k in ("pub_forward", "pub_repair", "pub_reverse", "pub_refine", "pub_compact", "freed"):
        assert mo[k] == sg[k], f"{where}: {k} {mo[k]} vs {sg[k]}"
    assert np.array_equal(o.entries(), g.entries()), f"{where}: entry sets differ"


def recall_at(ids, gt, k=10):
    ids, gt = np.asarray(ids), np.asarray(gt)
    return float(np.mean([len(set(ids[i, :k].tolist()) & set(gt[i, :k].tolist())) / k for i in range(ids.shape[0])]))


def float_workload(n_base=1500, clusters=16, seed=1, batch=500, rounds=2, churn=0.03, dim=96, sigma=0.3):
    return dg.Workload("small_f32", dg.Mixture(dim, clusters, sigma, dg.METRIC_IP_F32), n_base, 24, 48, 6, 5,
                       rounds, churn, 200, 10, (48,), seed, batch, batch)


def make_oracle_f(p, traversal=0, rerank_mult=4):
    return oracle.Oracle(oracle.METRIC_IP_F32, p["dim"], p["R"], p["L_build"], p["id_capacity"], p["slab_capacity"],
                         alpha=p["alpha"], n_entry=p["n_entry"], refine=p["refine"],
                         tombstone_only=p["tombstone_only"], traversal=traversal, rerank_mult=rerank_mult,
                         W=p["W"])


def make_gpu_f(p, traversal=0, rerank_mult=4, **kw):
    from paper_2607_02543_amd import etale
    return etale.Index(p["dim"], R=p["R"], L_build=p["L_build"], alpha=p["alpha"], n_entry=p["n_entry"],
                       refine=p["refine"], tombstone_only=p["tombstone_only"], id_capacity=p["id_capacity"],
                       slab_capacity=p["slab_capacity"], max_batch=p["max_batch"], metric=etale.METRIC_IP_F32,
                       traversal=traversal, rerank_mult=rerank_mult, W=p["W"], **kw)


def exact_ip_dist(q, x, ids):
    """FP64 d = 1 - <q, x_id> for rows of ids (NONE -> inf)."""
    ids = np.asarray(ids, dtype=np.int64)
    out = np.full(ids.shape, np.inf)
    ok = ids != 0xFFFFFFFF
    out[ok] = 1.0 - np.einsum("...d,...d->...", np.broadcast_to(q.astype(np.float64)[..., None, :], ids.shape + (q.shape[-1],))[ok], x.astype(np.float64)[ids[ok]])
    return out
