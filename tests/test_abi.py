"""The C-ABI library loads and exports every function include/etale.h declares,
and the binding's structures have the header's layout (no GPU needed)."""

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "etale.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:etale_status|const char\*)\s+(etale_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("etale_create", "etale_destroy", "etale_insert_batch", "etale_delete_batch", "etale_search_batch",
              "etale_reclaim", "etale_round", "etale_get_stats", "etale_export", "etale_sync", "etale_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_02543_amd import etale
    lib = etale.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _c_layout():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "etale.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(etale_config), offsetof(etale_config, id_capacity),
         offsetof(etale_config, hip_stream), sizeof(etale_stats), offsetof(etale_stats, error_bits),
         sizeof(etale_round_desc), offsetof(etale_round_desc, max_q), offsetof(etale_round_desc, counts),
         offsetof(etale_round_desc, graph));
  printf("%zu %zu %zu %zu\n", sizeof(etale_request), sizeof(etale_serve_config), sizeof(etale_serve_stats),
         offsetof(etale_serve_stats, wall_seconds));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        return [int(v) for v in subprocess.check_output([exe]).split()]


def test_struct_layout_matches_header():
    from paper_2607_02543_amd import etale
    size, off_cap, off_stream, ssize, off_err, rsize, off_mq, off_cnt, off_graph, qsize, scsize, sssize, off_ts = \
        _c_layout()
    assert C.sizeof(etale.Config) == size
    assert etale.Config.id_capacity.offset == off_cap
    assert etale.Config.hip_stream.offset == off_stream
    assert C.sizeof(etale.Stats) == ssize
    assert etale.Stats.error_bits.offset == off_err
    assert C.sizeof(etale.RoundDesc) == rsize
    assert etale.RoundDesc.max_q.offset == off_mq
    assert etale.RoundDesc.counts.offset == off_cnt
    assert etale.RoundDesc.graph.offset == off_graph
    assert C.sizeof(etale.Request) == qsize
    assert C.sizeof(etale.ServeConfig) == scsize
    assert C.sizeof(etale.ServeStats) == sssize
    assert etale.ServeStats.wall_seconds.offset == off_ts
    assert etale.ServeConfig.realtime.offset == 28


def test_create_rejects_bad_configs_without_touching_a_device():
    # argument validation happens before any HIP call
    from paper_2607_02543_amd import etale
    lib = etale.load()
    good = dict(dim=128, R=32, L_build=64, alpha_num=6, alpha_den=5, visit_mult=4, prune_cap=256, n_entry=64,
                refine=1, tombstone_only=0, publish_attempts=8, max_batch=100, vt_slots=1024, waves_per_block=4,
                metric=0, traversal=0, rerank_mult=4, copies=0, W=1, reserved=0, id_capacity=1000, slab_capacity=5000,
                hip_stream=None)
    bad = [dict(dim=96), dict(R=0), dict(R=65), dict(L_build=0), dict(alpha_den=0), dict(prune_cap=8),
           dict(vt_slots=1000), dict(waves_per_block=3), dict(metric=7), dict(max_batch=5000), dict(n_entry=0),
           dict(id_capacity=0xFFFFFFFF), dict(metric=1, dim=128), dict(metric=1, dim=96, traversal=3),
           dict(metric=1, dim=96, traversal=1, rerank_mult=65), dict(metric=1, dim=96, copies=4), dict(W=0),
           dict(W=3), dict(W=2, R=48)]
    for change in bad:
        cfg = etale.Config(**{**good, **change})
        h = C.c_void_p()
        assert lib.etale_create(C.byref(cfg), C.byref(h)) == etale.EINVAL, change
    assert lib.etale_destroy(None) == etale.OK
