"""GPU path at the benchmark's own settings against the oracle's stored digests.

The benchmark runs the uint8 path with 8,192 entry points (32 spans of start
rows, so a query's initial list is merged from 32 spans of 32 key slots),
two expansions per search step, a 1,024-slot visited table and insert calls
of 10,000 vectors. `tests/golden/make_golden.py` ran the oracle alone through
a 100,000-vector instance of the same mixture with those settings and stored a
digest of the whole state after every call and of every query batch; this
test replays the same calls on the GPU and requires every digest to match:
neighbor lists with their distances, degrees, deletion flags, slab presence,
pool counts, publication counters and the entry set, and result ids and
distances at L = 32, 64 and 128.
"""

import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden as mg  # noqa: E402

GOLDEN = os.path.join(HERE, "golden", "scale_u8_100k.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_file_matches_recipe():
    g = _load()
    r = g["recipe"]
    assert r["n_base"] == mg.N_BASE and r["rounds"] == mg.ROUNDS and r["queries"] == mg.N_QUERIES
    assert r["search_L"] == list(mg.SEARCH_L) and r["k"] == mg.K
    for k, v in mg.KNOBS.items():
        assert r[k] == (list(v) if isinstance(v, tuple) else v), k
    wl = mg.workload()
    labels = [s["label"] for s in g["steps"]]
    n_build = len(wl.build_batches())
    assert labels[:n_build] == [f"build {i}" for i in range(n_build)]
    assert len(labels) == n_build + len(mg.SEARCH_L) * (1 + mg.ROUNDS) + 3 * mg.ROUNDS
    # the stored states are consistent with the recipe's sizes
    last = g["steps"][n_build - 1]
    assert last["n"] == mg.N_BASE and last["live"] == mg.N_BASE
    assert last["n_entries"] == mg.KNOBS["n_entry"]
    # reclaim leaves exactly one resident slab per live node (Proposition 3)
    for s in g["steps"]:
        if s["label"].endswith("reclaim"):
            assert s["meta"]["resident"] == s["live"]


class GpuIndex:
    def __init__(self, torch):
        from paper_2607_02543_amd import etale

        self.torch = torch
        wl = mg.workload()
        cap, slabs, max_batch = mg.capacities(wl)
        k = mg.KNOBS
        self.g = etale.Index(wl.dim, R=k["R"], L_build=k["L_build"], alpha=k["alpha"], n_entry=k["n_entry"],
                             W=k["W"], visit_mult=k["visit_mult"], refine=k["refine"], id_capacity=cap,
                             slab_capacity=slabs, max_batch=max_batch, **mg.GPU_KNOBS)
        self.qdev = None

    def insert(self, x):
        self.g.insert(self.torch.from_numpy(x).cuda())

    def delete(self, ids):
        self.g.delete(self.torch.from_numpy(ids.astype(np.int32)).cuda())

    def reclaim(self):
        self.g.reclaim()

    def search(self, q, k, L):
        if self.qdev is None:
            self.qdev = self.torch.from_numpy(q).cuda()
        ids, d = self.g.search(self.qdev, k, L)
        return ids.cpu().numpy().astype(np.uint32), d.cpu().numpy().astype(np.int64)

    def state(self):
        e = self.g.export()
        s = self.g.stats()
        assert s["error_bits"] == 0 and s["cas_failures"] == 0
        meta = {"next_id": s["next_id"], "free": s["free_slabs"], "resident": s["resident_slabs"],
                "pub_forward": s["pub_forward"], "pub_repair": s["pub_repair"], "pub_reverse": s["pub_reverse"],
                "pub_refine": s["pub_refine"], "pub_compact": s["pub_compact"], "freed": s["freed"],
                "dirty_last": s["dirty_last"], "dead_edges_last": s["dead_edges_last"]}
        return (e["nbr"], e["rho"].astype(np.int64), e["deg"], e["deleted"], e["has_slab"], meta, self.g.entries())


def _first_diff(a, b):
    return next((i for i, (x, y) in enumerate(zip(a, b)) if x != y), None)


@pytest.mark.gpu
def test_gpu_matches_oracle_digests_at_benchmark_settings():
    import torch

    golden = _load()["steps"]
    ix = GpuIndex(torch)
    print("[golden] 100k uint8, 8192 entries, W=2, 1024 visited slots, batches up to 10k", flush=True)
    n = 0
    for (label, dig), exp in zip(mg.drive(ix, log=lambda s: print(f"[golden] {s}", flush=True)), golden):
        assert label == exp["label"]
        if "lists" in exp:
            for k in ("n", "edges", "live", "n_entries"):
                assert dig[k] == exp[k], f"{label}: {k} {dig[k]} vs oracle {exp[k]}"
            assert dig["meta"] == exp["meta"], f"{label}: pool / publication counts {dig['meta']} vs {exp['meta']}"
            assert dig["entries"] == exp["entries"], f"{label}: entry sets differ"
            c = _first_diff(dig["chunks"], exp["chunks"])
            assert dig["lists"] == exp["lists"], f"{label}: lists differ, first in ids [{c * mg.ID_CHUNK}, ...)"
        else:
            c = _first_diff(dig["chunks"], exp["chunks"])
            assert dig["results"] == exp["results"], (
                f"{label}: results differ, first in queries [{c * mg.Q_CHUNK}, ...); first query "
                f"{dig['first_ids']} vs oracle {exp['first_ids']}")
        n += 1
    assert n == len(golden)
    ix.g.close()
