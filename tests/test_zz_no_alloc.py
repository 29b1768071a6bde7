"""The allocation-free search entry point (etale_search_batch_noalloc) against
etale_search_batch on the same index: identical ids, distances and per-query
counts, bit for bit, on two calls in a row, the second one smaller.

The first call (4,000 queries, 8,192 entry points, L = 64) runs in three
chunks of the static scratch where the library's own scratch takes it in one;
the second (700 queries, L = 200) takes the start-set path that writes the
distance rows, in one chunk, over an array that still holds the first call's
contents. A float index repeats the check on its own start-set kernels.
"""

import numpy as np
import pytest

from common import float_workload, index_params, make_gpu, make_gpu_f, small_workload
from paper_2607_02543_amd import datagen as dg

pytestmark = pytest.mark.gpu


def _same(a, b, where):
    for x, y, name in zip(a, b, ("ids", "distances", "counts")):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.array_equal(x, y), f"{where}: {name} differ at {np.argwhere(x != y)[:5].tolist()}"


def test_noalloc_search_matches_search_batch_u8():
    import torch

    wl = small_workload(n_base=20000, clusters=64, seed=21, batch=5000, rounds=0)
    p = index_params(wl, n_entry=8192, W=2)
    g = make_gpu(p)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        g.insert(torch.from_numpy(st.base(b)).cuda())
    print("[no-alloc] uint8 20k, 8192 entries: 4000 queries at L=64, then 700 at L=200", flush=True)
    q1 = torch.from_numpy(st.queries(4000)).cuda()
    a1 = g.search(q1, 10, 64, counts=True)
    b1 = g.search_noalloc(q1, 10, 64, counts=True)
    _same(a1, b1, "first call")
    q2 = torch.from_numpy(st.queries(700)).cuda()
    a2 = g.search(q2, 16, 200, counts=True)
    b2 = g.search_noalloc(q2, 16, 200, counts=True)
    _same(a2, b2, "second call")
    # the library's path is unchanged by the calls through the static scratch
    _same(a1, g.search(q1, 10, 64, counts=True), "search after the static-scratch calls")
    assert g.stats()["error_bits"] == 0
    g.close()


def test_noalloc_search_matches_search_batch_float():
    import torch

    wl = float_workload(n_base=6000, batch=2000, rounds=0, seed=3)
    p = index_params(wl, n_entry=1024, W=2)
    g = make_gpu_f(p, traversal=1, copies=2)
    st = dg.Stream(wl)
    for b in wl.build_batches():
        g.insert(torch.from_numpy(st.base(b)).cuda())
    print("[no-alloc] float 6k x 96, 1024 entries: bf16 then FP8 traversal", flush=True)
    q1 = torch.from_numpy(st.queries(3000)).cuda()
    _same(g.search(q1, 10, 48, counts=True), g.search_noalloc(q1, 10, 48, counts=True), "float first call")
    g.set_query_traversal(2, 4)
    q2 = torch.from_numpy(st.queries(500)).cuda()
    _same(g.search(q2, 10, 100, counts=True), g.search_noalloc(q2, 10, 100, counts=True), "float second call")
    g.close()
