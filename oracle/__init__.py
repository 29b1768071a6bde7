"""CPU oracle for the dynamic graph index -- TEST INFRASTRUCTURE ONLY.

Python handle over ``etale_oracle.cpp`` (single-threaded C++17, built with g++).
Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it; the product path never imports it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "etale_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

METRIC_L2_U8 = 0
METRIC_IP_F32 = 1
TRAV_NATIVE, TRAV_BF16, TRAV_FP8 = 0, 1, 2
NONE = 0xFFFFFFFF

META_FIELDS = ("next_id", "n_entries", "P", "free", "resident", "retired", "pub_forward", "pub_repair",
               "pub_reverse", "pub_refine", "pub_compact", "freed", "dirty_last", "dead_last",
               "search_expansions", "search_distances")


def build(force: bool = True) -> str:
    """Compile the oracle (-O2, no intrinsics, no OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        vp, u32, u64, i32, i64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_int64
        lib.oracle_create.restype = vp
        lib.oracle_create.argtypes = [i32, i32, u32, u32, u32, u32, u32, u32, u32, u32, u32, u32, u64, u64, i32, i32]
        lib.oracle_destroy.argtypes = [vp]
        lib.oracle_insert.argtypes = [vp, vp, u64, vp]
        lib.oracle_delete.argtypes = [vp, vp, u64, vp]
        lib.oracle_reclaim.argtypes = [vp]
        lib.oracle_round.argtypes = [vp, vp, u64, vp, vp, u64, vp, vp, u64, u32, u32, vp, vp, i32]
        lib.oracle_search.argtypes = [vp, vp, u64, u32, u32, vp, vp, vp, vp]
        lib.oracle_beam_search.argtypes = [vp, vp, u32, u32, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_robust_prune.argtypes = [vp, u32, vp, u64, vp, vp, vp]
        lib.oracle_bruteforce.argtypes = [vp, vp, u64, u32, vp, vp]
        lib.oracle_set_list.argtypes = [vp, u32, vp, u32]
        lib.oracle_set_entries.argtypes = [vp, vp, u32]
        lib.oracle_get_entries.argtypes = [vp, vp]
        lib.oracle_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_get_codes.argtypes = [vp, u32, vp, vp, vp]
        lib.oracle_near_ties.restype = i64
        lib.oracle_near_ties.argtypes = [vp, vp, vp, u64, i32]
        lib.oracle_bf16_encode.argtypes = [vp, u64, vp]
        lib.oracle_fp8_encode.argtypes = [vp, u64, vp]
        lib.oracle_fp8_decode.argtypes = [vp, u64, vp]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} failed: {rc}")
        self.rc = rc


class Oracle:
    """The index, as a plain CPU model. Same call semantics as the C-ABI."""

    def __init__(self, metric: int, dim: int, R: int, L_build: int, id_capacity: int, slab_capacity: int,
                 alpha=(6, 5), W: int = 1, visit_mult: int = 4, prune_cap: Optional[int] = None,
                 traversal: int = TRAV_NATIVE, rerank_mult: int = 4, n_entry: int = 1, refine: bool = True,
                 tombstone_only: bool = False):
        self.lib = _load()
        self.metric, self.dim, self.R = metric, dim, R
        if prune_cap is None:
            prune_cap = max(visit_mult * L_build, 2 * R + 2)
        self.h = self.lib.oracle_create(metric, traversal, dim, R, L_build, W, visit_mult, prune_cap,
                                        alpha[0], alpha[1], rerank_mult, n_entry, id_capacity, slab_capacity,
                                        int(refine), int(tombstone_only))
        if not self.h:
            raise ValueError("oracle_create rejected the configuration")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_destroy(h)
            self.h = None

    def _vecs(self, x: np.ndarray) -> np.ndarray:
        dt = np.uint8 if self.metric == METRIC_L2_U8 else np.float32
        x = np.ascontiguousarray(x, dtype=dt)
        assert x.ndim == 2 and x.shape[1] == self.dim
        return x

    def insert(self, x: np.ndarray) -> np.ndarray:
        x = self._vecs(x)
        ids = np.zeros(x.shape[0], np.uint32)
        rc = self.lib.oracle_insert(self.h, _p(x), x.shape[0], _p(ids))
        if rc:
            raise OracleError(rc, "insert")
        return ids

    def delete(self, ids) -> np.ndarray:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        st = np.zeros(ids.size, np.uint8)
        rc = self.lib.oracle_delete(self.h, _p(ids), ids.size, _p(st))
        if rc:
            raise OracleError(rc, "delete")
        return st

    def reclaim(self) -> None:
        rc = self.lib.oracle_reclaim(self.h)
        if rc:
            raise OracleError(rc, "reclaim")

    def round(self, del_ids=None, x: Optional[np.ndarray] = None, q: Optional[np.ndarray] = None, k: int = 10,
              L: int = 64, reclaim: bool = False):
        """One round: deletes, inserts and queries in one epoch (queries and
        insert searches see the state after this round's tombstones), then an
        optional reclaim. Returns (delete statuses, new ids, result ids, result
        distances)."""
        dl = np.ascontiguousarray(np.zeros(0) if del_ids is None else del_ids, dtype=np.uint32)
        x = self._vecs(np.zeros((0, self.dim)) if x is None else x)
        q = self._vecs(np.zeros((0, self.dim)) if q is None else q)
        st = np.zeros(dl.size, np.uint8)
        ids = np.zeros(x.shape[0], np.uint32)
        qi = np.zeros((q.shape[0], k), np.uint32)
        qd = np.zeros((q.shape[0], k), np.int32 if self.metric == METRIC_L2_U8 else np.float64)
        rc = self.lib.oracle_round(self.h, _p(dl), dl.size, _p(st), _p(x), x.shape[0], _p(ids), _p(q), q.shape[0],
                                   k, L, _p(qi), _p(qd), int(reclaim))
        if rc:
            raise OracleError(rc, "round")
        return st, ids, qi, qd

    def search(self, q: np.ndarray, k: int, L: int, counts: bool = False):
        q = self._vecs(q)
        nq = q.shape[0]
        ids = np.zeros((nq, k), np.uint32)
        d = np.zeros((nq, k), np.int32 if self.metric == METRIC_L2_U8 else np.float64)
        ex = np.zeros(nq, np.uint32)
        nd = np.zeros(nq, np.uint32)
        rc = self.lib.oracle_search(self.h, _p(q), nq, k, L, _p(ids), _p(d), _p(ex), _p(nd))
        if rc:
            raise OracleError(rc, "search")
        return (ids, d, ex, nd) if counts else (ids, d)

    def beam_search(self, q: np.ndarray, L: int, visit_cap: int):
        q = self._vecs(q.reshape(1, -1))
        li = np.zeros(L, np.uint32)
        ld = np.zeros(L, np.float64)
        le = np.zeros(L, np.uint8)
        ln = C.c_uint32(0)
        vi = np.zeros(max(1, visit_cap), np.uint32)
        vd = np.zeros(max(1, visit_cap), np.float64)
        vn = C.c_uint32(0)
        nd = C.c_uint64(0)
        self.lib.oracle_beam_search(self.h, _p(q), L, visit_cap, _p(li), _p(ld), _p(le), C.byref(ln), _p(vi),
                                    _p(vd), C.byref(vn), C.byref(nd))
        n, m = ln.value, vn.value
        return dict(list_ids=li[:n].copy(), list_d=ld[:n].copy(), list_expanded=le[:n].astype(bool),
                    visited_ids=vi[:m].copy(), visited_d=vd[:m].copy(), distances=nd.value)

    def robust_prune(self, p: int, cand) -> tuple:
        cand = np.ascontiguousarray(cand, dtype=np.uint32)
        oi = np.zeros(self.R, np.uint32)
        od = np.zeros(self.R, np.float64)
        on = C.c_uint32(0)
        rc = self.lib.oracle_robust_prune(self.h, p, _p(cand), cand.size, _p(oi), _p(od), C.byref(on))
        if rc:
            raise OracleError(rc, "robust_prune")
        return oi[:on.value].copy(), od[:on.value].copy()

    def bruteforce(self, q: np.ndarray, k: int):
        q = self._vecs(q)
        ids = np.zeros((q.shape[0], k), np.uint32)
        d = np.zeros((q.shape[0], k), np.float64)
        self.lib.oracle_bruteforce(self.h, _p(q), q.shape[0], k, _p(ids), _p(d))
        return ids, d

    def set_list(self, u: int, ids) -> None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        rc = self.lib.oracle_set_list(self.h, u, _p(ids), ids.size)
        if rc:
            raise OracleError(rc, "set_list")

    def set_entries(self, ids) -> None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        rc = self.lib.oracle_set_entries(self.h, _p(ids), ids.size)
        if rc:
            raise OracleError(rc, "set_entries")

    def entries(self) -> np.ndarray:
        out = np.zeros(max(1, self.meta()["n_entries"]), np.uint32)
        n = self.lib.oracle_get_entries(self.h, _p(out))
        return out[:n].copy()

    def meta(self) -> dict:
        m = np.zeros(16, np.int64)
        self.lib.oracle_export(self.h, None, None, None, None, None, _p(m))
        return dict(zip(META_FIELDS, (int(v) for v in m)))

    def export(self) -> dict:
        meta = self.meta()
        n = meta["next_id"]
        nbr = np.zeros((max(n, 1), self.R), np.uint32)
        rho = np.zeros((max(n, 1), self.R), np.float64)
        deg = np.zeros(max(n, 1), np.uint8)
        de = np.zeros(max(n, 1), np.uint8)
        hs = np.zeros(max(n, 1), np.uint8)
        m = np.zeros(16, np.int64)
        self.lib.oracle_export(self.h, _p(nbr), _p(rho), _p(deg), _p(de), _p(hs), _p(m))
        return dict(meta=meta, nbr=nbr[:n], rho=rho[:n], deg=deg[:n], deleted=de[:n].astype(bool),
                    has_slab=hs[:n].astype(bool))

    def near_ties(self, clear: bool = True) -> dict:
        """{node: smallest relative margin} of the float comparisons within the
        tie margin (1e-5 relative) that decided a node's list since the last
        clear (see the C source)."""
        n = int(self.lib.oracle_near_ties(self.h, None, None, 0, 0))
        own = np.zeros(max(n, 1), np.uint32)
        mar = np.zeros(max(n, 1), np.float64)
        self.lib.oracle_near_ties(self.h, _p(own), _p(mar), n, int(clear))
        out = {}
        for u, m in zip(own[:n].tolist(), mar[:n].tolist()):
            out[u] = min(m, out.get(u, m))
        return out

    def codes(self, u: int):
        bf = np.zeros(self.dim, np.uint16)
        q8 = np.zeros(self.dim, np.uint8)
        sc = np.zeros(1, np.float32)
        rc = self.lib.oracle_get_codes(self.h, u, _p(bf), _p(q8), _p(sc))
        if rc:
            raise OracleError(rc, "codes")
        return bf, q8, float(sc[0])


def bf16_encode(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    out = np.zeros(x.size, np.uint16)
    _load().oracle_bf16_encode(_p(x), x.size, _p(out))
    return out


def fp8_encode(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    out = np.zeros(x.size, np.uint8)
    _load().oracle_fp8_encode(_p(x), x.size, _p(out))
    return out


def fp8_decode(c: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.uint8).ravel()
    out = np.zeros(c.size, np.float64)
    _load().oracle_fp8_decode(_p(c), c.size, _p(out))
    return out
