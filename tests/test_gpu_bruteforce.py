"""Brute-force ground truth (etale_bruteforce) against the oracle's plain
definition: the exact k nearest live rows by (distance, id), bit for bit on
uint8 rows. Rows of 64 to 256 bytes take the matrix-core path (several chunks
of rows per query, merged); the ids include tombstones, reclaimed ids and a
ragged last tile; heavy ties check the (distance, id) order across chunks."""

import numpy as np
import pytest

import oracle
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n", [(128, 30001), (64, 5003), (256, 12007)])
def test_bruteforce_matches_oracle(dim, n):
    import torch
    from paper_2607_02543_amd import etale

    rng = np.random.default_rng(dim)
    mix = dg.Mixture(dim, 32, 18.0, dg.METRIC_L2_U8)
    c = mix.centers(rng)
    x = mix.draw(rng, c, n)
    x[n // 2:n // 2 + 300] = x[:300]  # exact duplicates: equal distances, broken by id
    cap = n + 16
    o = oracle.Oracle(oracle.METRIC_L2_U8, dim, 16, 32, cap, 4 * cap + 100000, n_entry=64)
    g = etale.Index(dim, R=16, L_build=32, n_entry=64, id_capacity=cap, slab_capacity=4 * cap + 100000,
                    max_batch=5000)
    for s in range(0, n, 5000):
        o.insert(x[s:s + 5000])
        g.insert(torch.from_numpy(x[s:s + 5000]).cuda())
    dl = rng.choice(n, size=n // 10, replace=False).astype(np.uint32)
    o.delete(dl)
    g.delete(torch.from_numpy(dl.astype(np.int32)).cuda())
    o.reclaim()
    g.reclaim()
    dl2 = rng.choice(np.setdiff1d(np.arange(n), dl), size=n // 20, replace=False).astype(np.uint32)
    o.delete(dl2)  # tombstones that still hold slabs
    g.delete(torch.from_numpy(dl2.astype(np.int32)).cuda())
    q = np.concatenate([mix.draw(rng, c, 197), x[:3]])
    print(f"[bruteforce] dim={dim} n={n}", flush=True)
    for k in (1, 10, 16):
        io, do = o.bruteforce(q, k)
        ig, dgp = g.bruteforce(torch.from_numpy(q).cuda(), k)
        ig, dgp = ig.cpu().numpy().astype(np.uint32), dgp.cpu().numpy().astype(np.int64)
        assert np.array_equal(io, ig), f"k={k}: ids differ"
        assert np.array_equal(do.astype(np.int64), dgp), f"k={k}: distances differ"
    g.close()
