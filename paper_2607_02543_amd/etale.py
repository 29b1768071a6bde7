"""Python binding of the ETALE C ABI (include/etale.h).

Argument marshalling only: every step of insert / delete / search / reclaim
runs in the HIP kernels of libetale.so. torch supplies device memory and the
current HIP stream. The binding refuses to run without the built library.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetale.so")

OK, EINVAL, ENOMEM, EPOOL, ECAPACITY, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5, -6
METRIC_L2_U8, METRIC_IP_F32 = 0, 1
TRAV_NATIVE, TRAV_BF16, TRAV_FP8 = 0, 1, 2
DEL_OK, DEL_NOT_LIVE, DEL_OUT_OF_RANGE, DEL_DUPLICATE = 0, 1, 2, 3
NONE = 0xFFFFFFFF

_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EPOOL: "EPOOL", ECAPACITY: "ECAPACITY", EDEVICE: "EDEVICE",
             ESTATE: "ESTATE"}


class EtaleError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_ERRNAMES.get(code, code)} ({msg})")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_uint32), ("R", C.c_uint32), ("L_build", C.c_uint32),
        ("alpha_num", C.c_uint32), ("alpha_den", C.c_uint32), ("visit_mult", C.c_uint32),
        ("prune_cap", C.c_uint32), ("n_entry", C.c_uint32), ("refine", C.c_uint32),
        ("tombstone_only", C.c_uint32), ("publish_attempts", C.c_uint32), ("max_batch", C.c_uint32),
        ("vt_slots", C.c_uint32), ("waves_per_block", C.c_uint32), ("metric", C.c_int32),
        ("traversal", C.c_int32), ("rerank_mult", C.c_uint32), ("copies", C.c_uint32),
        ("W", C.c_uint32), ("reserved", C.c_uint32),
        ("id_capacity", C.c_uint64), ("slab_capacity", C.c_uint64),
        ("hip_stream", C.c_void_p),
    ]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "next_id", "live", "tombstones", "slab_capacity", "free_slabs", "resident_slabs", "n_entries",
        "pub_forward", "pub_repair", "pub_reverse", "pub_refine", "pub_compact", "freed", "dirty_last",
        "dead_edges_last", "search_expansions", "search_distances", "cas_failures", "publish_dropped",
        "device_bytes", "error_bits")]


class TuneResult(C.Structure):
    _fields_ = [("waves_per_block", C.c_uint32), ("vt_slots", C.c_uint32), ("row_lanes", C.c_uint32),
                ("ms", C.c_float), ("ms_default", C.c_float)]


class Request(C.Structure):
    _fields_ = [("t_arrive", C.c_double), ("kind", C.c_uint32), ("arg", C.c_uint32)]


class ServeConfig(C.Structure):
    _fields_ = [("k", C.c_uint32), ("L", C.c_uint32), ("max_tick", C.c_uint32), ("reclaim_every", C.c_uint32),
                ("hbm_budget_bytes", C.c_uint64), ("graph", C.c_int32), ("realtime", C.c_int32)]


class ServeStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "ticks", "searches", "inserts", "deletes", "rejected_inserts", "deferred", "reclaims", "failed_ticks",
        "peak_resident_slabs", "final_resident_slabs", "ids_handed_out", "graphs")] + \
        [("wall_seconds", C.c_double), ("device_busy_seconds", C.c_double)]


REQ_SEARCH, REQ_INSERT, REQ_DELETE = 0, 1, 2


class RoundDesc(C.Structure):
    _fields_ = [
        ("del_ids", C.c_void_p), ("del_status", C.c_void_p), ("max_del", C.c_uint32),
        ("ins_vecs", C.c_void_p), ("ins_ids", C.c_void_p), ("max_ins", C.c_uint32),
        ("queries", C.c_void_p), ("q_ids", C.c_void_p), ("q_dists", C.c_void_p), ("max_q", C.c_uint32),
        ("k", C.c_uint32), ("L", C.c_uint32), ("counts", C.c_void_p), ("status", C.c_void_p),
        ("reclaim", C.c_int32), ("graph", C.c_int32),
    ]


_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> C.CDLL:
    """Load libetale.so; raise if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_02543_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
    sigs = {
        "etale_create": ([C.POINTER(Config), C.POINTER(vp)], i32),
        "etale_destroy": ([vp], i32),
        "etale_set_stream": ([vp, vp], i32),
        "etale_insert_batch": ([vp, vp, u64, vp], i32),
        "etale_delete_batch": ([vp, vp, u64, vp], i32),
        "etale_search_batch": ([vp, vp, u64, u32, u32, vp, vp, vp], i32),
        "etale_search_batch_noalloc": ([vp, vp, u64, u32, u32, vp, vp, vp], i32),
        "etale_reclaim": ([vp], i32),
        "etale_round": ([vp, C.POINTER(RoundDesc)], i32),
        "etale_bruteforce": ([vp, vp, u64, u32, vp, vp], i32),
        "etale_get_stats": ([vp, C.POINTER(Stats)], i32),
        "etale_export": ([vp, u64, vp, vp, vp, vp, vp], i32),
        "etale_get_entries": ([vp, vp, u64, C.POINTER(u64)], i32),
        "etale_set_lists": ([vp, u64, vp, vp, vp], i32),
        "etale_set_query_traversal": ([vp, i32, u32], i32),
        "etale_export_rows": ([vp, u64, u64, i32, vp], i32),
        "etale_set_search_knobs": ([vp, u32, u32], i32),
        "etale_serve": ([vp, C.POINTER(ServeConfig), vp, u64, vp, u64, vp, vp, vp, vp, C.POINTER(ServeStats)], i32),
        "etale_autotune": ([vp, vp, u64, u32, u32, C.POINTER(TuneResult)], i32),
        "etale_set_search_lanes": ([vp, u32], i32),
        "etale_set_search_timing": ([vp, i32], i32),
        "etale_get_search_timing": ([vp, vp, u64, C.POINTER(u64)], i32),
        "etale_set_concurrent": ([vp, i32, vp], i32),
        "etale_sync": ([vp], i32),
        "etale_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Index:
    """One ETALE index on the current GPU."""

    def __init__(self, dim: int, R: int = 32, L_build: int = 64, alpha=(6, 5), visit_mult: int = 4,
                 prune_cap: Optional[int] = None, n_entry: int = 128, refine: bool = True,
                 tombstone_only: bool = False, publish_attempts: int = 8, max_batch: int = 10000,
                 vt_slots: int = 1024, waves_per_block: int = 4, id_capacity: int = 100000,
                 slab_capacity: Optional[int] = None, metric: int = METRIC_L2_U8, traversal: int = TRAV_NATIVE,
                 rerank_mult: int = 4, copies: int = 0, W: int = 1, stream=None, row_lanes: int = 0):
        import torch

        self.torch = torch
        self.lib = load()
        if prune_cap is None:
            prune_cap = max(visit_mult * L_build, 2 * R + 2)
        if slab_capacity is None:
            slab_capacity = 2 * id_capacity + max_batch * (R + 2)
        self.dim, self.R, self.metric = dim, R, metric
        self.traversal = traversal
        self.cfg = Config(dim, R, L_build, alpha[0], alpha[1], visit_mult, prune_cap, n_entry, int(refine),
                          int(tombstone_only), publish_attempts, max_batch, vt_slots, waves_per_block, metric,
                          traversal, rerank_mult, copies, W, 0, id_capacity, slab_capacity, None)
        s = stream if stream is not None else torch.cuda.current_stream()
        self.cfg.hip_stream = s.cuda_stream
        self.stream = s
        h = C.c_void_p()
        rc = self.lib.etale_create(C.byref(self.cfg), C.byref(h))
        if rc != OK:
            raise EtaleError(rc, "etale_create", "configuration rejected or allocation failed")
        self.h = h
        if row_lanes:
            self.set_search_lanes(row_lanes)

    def close(self):
        if getattr(self, "h", None):
            self.lib.etale_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, where: str):
        if rc != OK:
            msg = self.lib.etale_last_error(self.h)
            raise EtaleError(rc, where, msg.decode() if msg else "")

    def _dev(self, t, dtype):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise TypeError("expected a CUDA (HIP) tensor")
        return t.contiguous().to(dtype)

    @property
    def _vdtype(self):
        return self.torch.uint8 if self.metric == METRIC_L2_U8 else self.torch.float32

    @property
    def _ddtype(self):
        return self.torch.int32 if self.metric == METRIC_L2_U8 else self.torch.float32

    def insert(self, x):
        torch = self.torch
        x = self._dev(x, self._vdtype)
        n = x.shape[0]
        ids = torch.empty(n, dtype=torch.int32, device=x.device)
        self._check(self.lib.etale_insert_batch(self.h, _ptr(x), n, _ptr(ids)), "insert_batch")
        return ids

    def delete(self, ids):
        torch = self.torch
        ids = self._dev(ids, torch.int32)
        st = torch.empty(ids.numel(), dtype=torch.uint8, device=ids.device)
        self._check(self.lib.etale_delete_batch(self.h, _ptr(ids), ids.numel(), _ptr(st)), "delete_batch")
        return st

    def search(self, q, k: int, L: int, counts: bool = False):
        torch = self.torch
        q = self._dev(q, self._vdtype)
        nq = q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        d = torch.empty((nq, k), dtype=self._ddtype, device=q.device)
        cnt = torch.empty((nq, 2), dtype=torch.int32, device=q.device) if counts else None
        self._check(self.lib.etale_search_batch(self.h, _ptr(q), nq, k, L, _ptr(ids), _ptr(d), _ptr(cnt)),
                    "search_batch")
        return (ids, d, cnt) if counts else (ids, d)

    def search_noalloc(self, q, k: int, L: int, counts: bool = False):
        """search() through the allocation-free entry point (static scratch);
        the output tensors are the caller's, allocated here by torch."""
        torch = self.torch
        q = self._dev(q, self._vdtype)
        nq = q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        d = torch.empty((nq, k), dtype=self._ddtype, device=q.device)
        cnt = torch.empty((nq, 2), dtype=torch.int32, device=q.device) if counts else None
        self._check(self.lib.etale_search_batch_noalloc(self.h, _ptr(q), nq, k, L, _ptr(ids), _ptr(d), _ptr(cnt)),
                    "search_batch_noalloc")
        return (ids, d, cnt) if counts else (ids, d)

    def reclaim(self):
        self._check(self.lib.etale_reclaim(self.h), "reclaim")

    def round(self, del_ids=None, x=None, q=None, k: int = 10, L: int = 64, reclaim: bool = False) -> dict:
        """One round (deletes, inserts, queries in one epoch) with the counts
        given by the inputs. Returns device tensors; `status` holds the round
        and reclaim status words once the stream has reached them."""
        torch = self.torch
        dev = torch.device("cuda")
        dl = self._dev(del_ids, torch.int32) if del_ids is not None else None
        xv = self._dev(x, self._vdtype) if x is not None else None
        qv = self._dev(q, self._vdtype) if q is not None else None
        nd = 0 if dl is None else dl.numel()
        ni = 0 if xv is None else xv.shape[0]
        nq = 0 if qv is None else qv.shape[0]
        out = {"status": torch.zeros(2, dtype=torch.int32, device=dev),
               "del_status": torch.empty(nd, dtype=torch.uint8, device=dev),
               "ids": torch.empty(ni, dtype=torch.int32, device=dev),
               "q_ids": torch.empty((nq, k), dtype=torch.int32, device=dev),
               "q_dists": torch.empty((nq, k), dtype=self._ddtype, device=dev)}
        desc = RoundDesc(_ptr(dl), _ptr(out["del_status"]), nd, _ptr(xv), _ptr(out["ids"]), ni, _ptr(qv),
                         _ptr(out["q_ids"]), _ptr(out["q_dists"]), nq, k, L, None, _ptr(out["status"]),
                         int(reclaim), 0)
        self._keep = (dl, xv, qv)  # inputs stay alive until the next call
        self._check(self.lib.etale_round(self.h, C.byref(desc)), "round")
        return out

    def bruteforce(self, q, k: int):
        torch = self.torch
        q = self._dev(q, self._vdtype)
        ids = torch.empty((q.shape[0], k), dtype=torch.int32, device=q.device)
        d = torch.empty((q.shape[0], k), dtype=self._ddtype, device=q.device)
        self._check(self.lib.etale_bruteforce(self.h, _ptr(q), q.shape[0], k, _ptr(ids), _ptr(d)), "bruteforce")
        return ids, d

    def sync(self):
        self._check(self.lib.etale_sync(self.h), "sync")

    def set_concurrent(self, enable: bool, search_stream=None):
        """Concurrent mode: searches on `search_stream` (a torch.cuda.Stream)
        alongside rounds on the index's stream; leaving it drains both."""
        ptr = search_stream.cuda_stream if search_stream is not None else None
        self._check(self.lib.etale_set_concurrent(self.h, int(enable), ptr), "set_concurrent")

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.etale_get_stats(self.h, C.byref(s)), "get_stats")
        return {name: int(getattr(s, name)) for name, _ in Stats._fields_}

    def export(self, n_ids: Optional[int] = None) -> dict:
        if n_ids is None:
            n_ids = self.stats()["next_id"]
        R = self.R
        nbr = np.zeros((max(n_ids, 1), R), np.uint32)
        rho = np.zeros((max(n_ids, 1), R), np.uint32)
        deg = np.zeros(max(n_ids, 1), np.uint8)
        de = np.zeros(max(n_ids, 1), np.uint8)
        hs = np.zeros(max(n_ids, 1), np.uint8)
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(self.lib.etale_export(self.h, n_ids, p(nbr), p(rho), p(deg), p(de), p(hs)), "export")
        rv = rho[:n_ids].view(np.int32 if self.metric == METRIC_L2_U8 else np.float32)
        return dict(nbr=nbr[:n_ids], rho=rv, deg=deg[:n_ids],
                    deleted=de[:n_ids].astype(bool), has_slab=hs[:n_ids].astype(bool))

    def entries(self) -> np.ndarray:
        cap = int(self.cfg.n_entry)
        out = np.zeros(cap, np.uint32)
        n = C.c_uint64(0)
        self._check(self.lib.etale_get_entries(self.h, out.ctypes.data_as(C.c_void_p), cap, C.byref(n)), "entries")
        return out[:n.value].copy()

    def set_query_traversal(self, traversal: int, rerank_mult: int = 4):
        self._check(self.lib.etale_set_query_traversal(self.h, traversal, rerank_mult), "set_query_traversal")

    def set_lists(self, ids, nbr, deg):
        """Install neighbor lists (import): row i of nbr (R wide) holds deg[i] neighbors of ids[i]."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        nbr = np.ascontiguousarray(nbr, dtype=np.uint32).reshape(ids.size, self.R)
        deg = np.ascontiguousarray(deg, dtype=np.uint32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(self.lib.etale_set_lists(self.h, ids.size, p(ids), p(nbr), p(deg)), "set_lists")

    def rows(self, first: int, n: int, which: int = 0) -> np.ndarray:
        """Stored rows: 0 as inserted, 1 bf16 copy (uint16), 2 FP8 codes, 3 FP8 scales."""
        if which == 0:
            out = np.zeros((n, self.dim), np.uint8 if self.metric == METRIC_L2_U8 else np.float32)
        elif which == 1:
            out = np.zeros((n, self.dim), np.uint16)
        elif which == 2:
            out = np.zeros((n, self.dim), np.uint8)
        else:
            out = np.zeros(n, np.float32)
        self._check(self.lib.etale_export_rows(self.h, first, n, which, out.ctypes.data_as(C.c_void_p)), "export_rows")
        return out

    def serve(self, t_arrive: np.ndarray, kind: np.ndarray, arg: np.ndarray, rows, k: int = 10, L: int = 64,
              max_tick: int = 4096, reclaim_every: int = 0, hbm_budget_bytes: int = 0, graph: bool = True,
              realtime: bool = False, results: bool = False):
        """Run a request stream through the library's serving loop (continuous
        batching into ticks whose searches and updates overlap on the device).
        Returns (per-request latency in ms, per-request tick, stats) and, with
        results=True, the device tensors (ids, distances), n x k, written for
        the search requests."""
        torch = self.torch
        n = int(t_arrive.size)
        reqs = np.zeros(n, dtype=np.dtype([("t", np.float64), ("kind", np.uint32), ("arg", np.uint32)]))
        reqs["t"], reqs["kind"], reqs["arg"] = t_arrive, kind, arg
        rows = self._dev(rows, self._vdtype)
        lat = np.zeros(n, np.float32)
        ticks = np.zeros(n, np.uint32)
        res_i = res_d = None
        if results:
            res_i = torch.full((n, k), -1, dtype=torch.int32, device=rows.device)
            res_d = torch.zeros((n, k), dtype=self._ddtype, device=rows.device)
        cfg = ServeConfig(k, L, max_tick, reclaim_every, hbm_budget_bytes, int(graph), int(realtime))
        st = ServeStats()
        p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._check(self.lib.etale_serve(self.h, C.byref(cfg), p(reqs), n, _ptr(rows), rows.shape[0], p(lat), p(ticks),
                                         _ptr(res_i), _ptr(res_d), C.byref(st)), "serve")
        stats = {name: getattr(st, name) for name, _ in ServeStats._fields_}
        if results:
            return lat, ticks, stats, (res_i, res_d)
        return lat, ticks, stats

    def set_search_knobs(self, waves_per_block: int, vt_slots: int):
        self._check(self.lib.etale_set_search_knobs(self.h, waves_per_block, vt_slots), "set_search_knobs")

    def autotune(self, q, k: int, L: int) -> dict:
        """Pick the fastest result-invariant search knobs on this query batch."""
        q = self._dev(q, self._vdtype)
        r = TuneResult()
        self._check(self.lib.etale_autotune(self.h, _ptr(q), q.shape[0], k, L, C.byref(r)), "autotune")
        return {"waves_per_block": r.waves_per_block, "vt_slots": r.vt_slots, "row_lanes": r.row_lanes, "ms": r.ms,
                "ms_default": r.ms_default}

    def set_search_lanes(self, lanes_per_row: int):
        self._check(self.lib.etale_set_search_lanes(self.h, lanes_per_row), "set_search_lanes")

    def set_search_timing(self, enable: bool = True):
        self._check(self.lib.etale_set_search_timing(self.h, int(enable)), "set_search_timing")

    def search_timing(self, cap: int = 4096) -> np.ndarray:
        """(scan, select, search) milliseconds of each timed search launch since the last read."""
        ms = np.zeros((cap, 3), np.float32)
        n = C.c_uint64(0)
        self._check(self.lib.etale_get_search_timing(self.h, ms.ctypes.data_as(C.c_void_p), cap, C.byref(n)),
                    "get_search_timing")
        return ms[:min(n.value, cap)].copy()


class RoundRunner:
    """Rounds of uneven sizes through fixed device buffers, so that one
    captured HIP graph serves every round: the counts are written into device
    memory before each replay and the kernels read them when they run.

    Inputs are copied into the buffers on the index's stream; outputs are
    views of the buffers, valid until the next call."""

    def __init__(self, index: Index, max_del: int, max_ins: int, max_q: int, k: int = 10, L: int = 64,
                 reclaim: bool = False, graph: bool = True, buckets: bool = False):
        torch = index.torch
        self.ix, self.torch = index, torch
        dev = torch.device("cuda")
        self.max_del, self.max_ins, self.max_q, self.k = max_del, max_ins, max_q, k
        self.del_ids = torch.zeros(max(max_del, 1), dtype=torch.int32, device=dev)
        self.del_status = torch.zeros(max(max_del, 1), dtype=torch.uint8, device=dev)
        self.vecs = torch.zeros((max(max_ins, 1), index.dim), dtype=index._vdtype, device=dev)
        self.ids = torch.zeros(max(max_ins, 1), dtype=torch.int32, device=dev)
        self.q = torch.zeros((max(max_q, 1), index.dim), dtype=index._vdtype, device=dev)
        self.q_ids = torch.zeros((max(max_q, 1), k), dtype=torch.int32, device=dev)
        self.q_dists = torch.zeros((max(max_q, 1), k), dtype=index._ddtype, device=dev)
        self.counts = torch.zeros(3, dtype=torch.int32, device=dev)
        self.status = torch.zeros(2, dtype=torch.int32, device=dev)
        self.L, self.reclaim, self.graph, self.buckets = L, reclaim, graph, buckets
        self.desc = self._desc(max_del, max_ins, max_q)
        self.descs = {}

    def _desc(self, md: int, mi: int, mq: int) -> RoundDesc:
        return RoundDesc(_ptr(self.del_ids), _ptr(self.del_status), md, _ptr(self.vecs), _ptr(self.ids), mi,
                         _ptr(self.q), _ptr(self.q_ids), _ptr(self.q_dists), mq, self.k, self.L, _ptr(self.counts),
                         _ptr(self.status), int(self.reclaim), int(self.graph))

    @staticmethod
    def _bucket(n: int, floor: int, cap: int) -> int:
        if n == 0:
            return 0
        b = floor
        while b < n:
            b *= 2
        return min(b, cap)

    def captured(self, nd: int, ni: int, nq: int) -> bool:
        """Whether a round of these counts replays an already captured graph."""
        if not self.buckets:
            return bool(self.descs) or getattr(self, "_ran", False)
        key = (self._bucket(nd, 1024, self.max_del), self._bucket(ni, 1024, self.max_ins),
               self._bucket(nq, 64, self.max_q))
        return key in self.descs

    def desc_for(self, nd: int, ni: int, nq: int) -> RoundDesc:
        """Launch shapes of a round: the largest ones, or (buckets) the next
        power of two above each count, so that every bucket is one graph."""
        if not self.buckets:
            return self.desc
        key = (self._bucket(nd, 1024, self.max_del), self._bucket(ni, 1024, self.max_ins),
               self._bucket(nq, 64, self.max_q))
        if key not in self.descs:
            self.descs[key] = self._desc(*key)
        return self.descs[key]

    def prepare(self, sizes):
        """Capture the graphs of the size buckets of `sizes` ((nd, ni, nq)
        triples) ahead of time by running rounds with zero counts, which
        change no index state."""
        for nd, ni, nq in sizes:
            if self.captured(nd, ni, nq):
                continue
            self.counts.zero_()
            self.n = (0, 0, 0)
            desc = self.desc_for(nd, ni, nq)
            self.ix._check(self.ix.lib.etale_round(self.ix.h, C.byref(desc)), "round")
            self._ran = True

    def load(self, del_ids=None, x=None, q=None, counts=None):
        """Copy a round's inputs into the buffers and set its counts (stream
        ordered). `counts` (nd, ni, nq) may override the input lengths, e.g.
        to pass counts above the maximum on purpose."""
        nd = 0 if del_ids is None else del_ids.numel()
        ni = 0 if x is None else x.shape[0]
        nq = 0 if q is None else q.shape[0]
        if nd:
            self.del_ids[:nd].copy_(del_ids.reshape(-1))
        if ni:
            self.vecs[:ni].copy_(x)
        if nq:
            self.q[:nq].copy_(q)
        c = counts if counts is not None else (nd, ni, nq)
        for i in range(3):
            self.counts[i].fill_(int(c[i]))
        self.n = (nd, ni, nq)

    def run(self) -> dict:
        """Run the round on the loaded inputs (replays the graph after the first call)."""
        nd, ni, nq = self.n
        self.ix._check(self.ix.lib.etale_round(self.ix.h, C.byref(self.desc_for(nd, ni, nq))), "round")
        self._ran = True
        return {"status": self.status, "del_status": self.del_status[:nd], "ids": self.ids[:ni],
                "q_ids": self.q_ids[:nq], "q_dists": self.q_dists[:nq]}

    def __call__(self, del_ids=None, x=None, q=None, counts=None) -> dict:
        self.load(del_ids, x, q, counts)
        return self.run()
