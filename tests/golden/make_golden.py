"""Writes the stored digests of the oracle at the benchmark's own settings.

The benchmark runs the uint8 path with an entry set of 8,192 ids, two
expansions per search step (W = 2), a 1,024-slot visited table and insert
batches of up to 10,000 vectors. The GPU parity tests at small sizes never
reach that regime (32 spans of start rows, crowded visited tables, 10,000
insert searches per launch), so this script runs the oracle, and only the
oracle, through the same call sequence on a mid-size instance of the same
mixture and stores a digest of the state after every call and of every query
batch's results: `scale_u8_100k.json`. `tests/test_gpu_golden.py` replays the
sequence on the GPU and compares digests.

Recipe (all draws from paper_2607_02543_amd.datagen, seed 0):
- 100,000 vectors of 128-d uint8 from the 1,024-cluster mixture (sigma 18),
  inserted in the build batches 1,000, 2,000, 4,000, 8,000, 10,000, ...;
- R = 32, L_build = 64, alpha = 6/5, visit cap 4L, entry set 8,192, W = 2;
- after the build and after each of 3 churn rounds (1% deletes of live ids,
  1% inserts, then reclaim), 1,000 queries with k = 10 at L = 32, 64, 128.

A digest is SHA-256 over a canonical byte form: neighbor ids (uint32), their
distances (int64), degree, deletion flag and slab presence (one byte each) of
ids [0, next id), plus the pool counts and publication counters; per query
batch the result ids (uint32) and distances (int64). Chunk digests (10,000 ids
or 100 queries each) name the region of a first difference.

Run: python tests/golden/make_golden.py  (single-threaded oracle, a few minutes)
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2607_02543_amd import datagen as dg  # noqa: E402

OUT = os.path.join(HERE, "scale_u8_100k.json")

N_BASE = 100_000
ROUNDS = 3
N_QUERIES = 1000
SEARCH_L = (32, 64, 128)
K = 10
KNOBS = dict(R=32, L_build=64, alpha=(6, 5), n_entry=8192, W=2, visit_mult=4, refine=True)
GPU_KNOBS = dict(vt_slots=1024, waves_per_block=4)  # result-invariant launch knobs of the benchmark
ID_CHUNK, Q_CHUNK = 10_000, 100


def workload():
    return dg.scale_u8(n_base=N_BASE, rounds=ROUNDS, n_queries=N_QUERIES)


def capacities(wl):
    cap = wl.id_capacity()
    max_batch = max(wl.build_batch_max, wl.churn_count())
    return cap, 2 * cap + max_batch * (wl.R + 2), max_batch


def _sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def state_digest(nbr, rho, deg, deleted, has_slab, meta, entries) -> dict:
    """nbr uint32 [n, R], rho int64 [n, R], deg / deleted / has_slab [n] bytes."""
    nbr = np.asarray(nbr, np.uint32)
    rho = np.asarray(rho, np.int64)
    deg = np.asarray(deg, np.uint8)
    deleted = np.asarray(deleted, np.uint8)
    has_slab = np.asarray(has_slab, np.uint8)
    n = nbr.shape[0]
    chunks = [_sha(nbr[s:s + ID_CHUNK], rho[s:s + ID_CHUNK], deg[s:s + ID_CHUNK], deleted[s:s + ID_CHUNK],
                   has_slab[s:s + ID_CHUNK]) for s in range(0, n, ID_CHUNK)]
    return {"n": int(n), "lists": _sha(nbr, rho, deg, deleted, has_slab), "chunks": chunks, "meta": meta,
            "entries": _sha(np.asarray(entries, np.uint32)), "n_entries": int(len(entries)),
            "edges": int(deg.astype(np.int64).sum()), "live": int(n - deleted.sum())}


def search_digest(ids, dists) -> dict:
    ids = np.asarray(ids, np.uint32)
    d = np.asarray(dists, np.int64)
    return {"results": _sha(ids, d),
            "chunks": [_sha(ids[s:s + Q_CHUNK], d[s:s + Q_CHUNK]) for s in range(0, ids.shape[0], Q_CHUNK)],
            "first_ids": ids[0].tolist()}


META_KEYS = ("next_id", "free", "resident", "pub_forward", "pub_repair", "pub_reverse", "pub_refine",
             "pub_compact", "freed", "dirty_last", "dead_edges_last")


def drive(ix, log=print):
    """Runs the recipe on `ix` and yields (label, digest). `ix` offers
    insert(x), delete(ids), reclaim(), search(q, k, L) -> (ids, dists) and
    state() -> the arguments of state_digest, all with numpy arrays."""
    wl = workload()
    st = dg.Stream(wl)
    handed, deleted = 0, np.zeros(wl.id_capacity(), bool)
    q = st.queries(N_QUERIES)
    for bi, b in enumerate(wl.build_batches()):
        ix.insert(st.base(b))
        handed += b
        yield f"build {bi}", state_digest(*ix.state())
    for L in SEARCH_L:
        yield f"build search L={L}", search_digest(*ix.search(q, K, L))
    for r in range(wl.churn_rounds):
        live = np.nonzero(~deleted[:handed])[0].astype(np.uint32)
        dl = st.deletes(live, wl.churn_count())
        ix.delete(dl)
        deleted[dl] = True
        yield f"round {r} delete", state_digest(*ix.state())
        x = st.inserts(wl.churn_count())
        ix.insert(x)
        handed += x.shape[0]
        yield f"round {r} insert", state_digest(*ix.state())
        ix.reclaim()
        yield f"round {r} reclaim", state_digest(*ix.state())
        for L in SEARCH_L:
            yield f"round {r} search L={L}", search_digest(*ix.search(q, K, L))
        log(f"round {r} done")


class OracleIndex:
    """The oracle behind drive()'s interface."""

    def __init__(self):
        import oracle

        wl = workload()
        cap, slabs, _ = capacities(wl)
        self.o = oracle.Oracle(oracle.METRIC_L2_U8, wl.dim, KNOBS["R"], KNOBS["L_build"], cap, slabs,
                               alpha=KNOBS["alpha"], W=KNOBS["W"], visit_mult=KNOBS["visit_mult"],
                               n_entry=KNOBS["n_entry"], refine=KNOBS["refine"])

    def insert(self, x):
        self.o.insert(x)

    def delete(self, ids):
        self.o.delete(ids)

    def reclaim(self):
        self.o.reclaim()

    def search(self, q, k, L):
        return self.o.search(q, k, L)

    def state(self):
        e = self.o.export()
        m = e["meta"]
        meta = {k: int(m[{"dead_edges_last": "dead_last"}.get(k, k)]) for k in META_KEYS}
        return (e["nbr"], e["rho"].astype(np.int64), e["deg"], e["deleted"], e["has_slab"], meta,
                self.o.entries())


def main():
    t0 = time.time()
    ix = OracleIndex()
    out = {"recipe": {"n_base": N_BASE, "rounds": ROUNDS, "queries": N_QUERIES, "search_L": list(SEARCH_L),
                      "k": K, **{k: list(v) if isinstance(v, tuple) else v for k, v in KNOBS.items()},
                      "gpu_knobs": GPU_KNOBS},
           "steps": []}
    for label, dig in drive(ix, log=lambda s: print(f"[{time.time() - t0:.0f}s] {s}", flush=True)):
        out["steps"].append({"label": label, **dig})
        print(f"[{time.time() - t0:.0f}s] {label}", flush=True)
    out["oracle_seconds"] = round(time.time() - t0, 1)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
