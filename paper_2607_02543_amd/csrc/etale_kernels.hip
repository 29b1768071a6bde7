// HIP kernels of the ETALE index for gfx950 (uint8 vectors, squared L2).
//
// Execution model (Definition 2): every kernel is one launch; the host
// serializes them on one stream. Within a maintenance phase each target node
// is owned by exactly one wavefront, so the reference CAS of a publication is
// uncontended and the phase result does not depend on scheduling.
#include "etale_dev.h"
#include "etale_float.h"
#include "etale_launch.h"

#include <map>
#include <mutex>
#include <type_traits>

namespace etale {

__host__ __device__ inline uint64_t pair_key(uint32_t target, uint32_t source) {
  return ((uint64_t)target << 32) | source;
}

// ---- pool / state initialisation ----------------------------------------------

__global__ void k_init(Index ix) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ix.cap; i += stride)
    ix.refs[i] = REF_UNBORN;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ix.P; i += stride)
    ix.free_stack[i] = (uint32_t)(ix.P - 1 - i);
  if (blockIdx.x == 0)
    for (uint32_t i = threadIdx.x; i < CTR_WORDS; i += blockDim.x) ix.ctr[i] = i == C_FREE_TOP ? ix.P : 0ull;
}

// End of a launch epoch: the retired stack joins the free stack (Lemma 1).
// The epoch's end (Lemma 1): retired slabs rejoin the free stack. Many
// workgroups copy; a one-thread launch after them moves the counters.
__global__ void __launch_bounds__(256) k_recycle(Index ix) {
  const uint64_t n = ix.ctr[C_RETIRED_TOP];
  const uint64_t f = ix.ctr[C_FREE_TOP];
  if (f + n > ix.P) return;  // reported by k_recycle_commit
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    ix.free_stack[f + i] = ix.retired_stack[i];
}

__global__ void k_recycle_commit(Index ix) {
  const uint64_t n = ix.ctr[C_RETIRED_TOP];
  const uint64_t f = ix.ctr[C_FREE_TOP];
  if (f + n > ix.P) {
    atomicOr(&ix.ctr[C_ERROR], (unsigned long long)ERR_POOL_OVERFLOW);
    return;
  }
  ix.ctr[C_FREE_TOP] = f + n;
  ix.ctr[C_RETIRED_TOP] = 0;
}

// ---- round control --------------------------------------------------------------------
// A round's counts come from a device array (a replayed graph) or from the
// launch arguments. Counts above the launch shapes fail the round.
constexpr int32_t ST_EINVAL = -1, ST_EPOOL = -3, ST_ECAPACITY = -4;

__global__ void k_round_begin(Index ix, const uint32_t* counts, uint32_t nd, uint32_t ni, uint32_t nq,
                              uint32_t max_d, uint32_t max_i, uint32_t max_q, int32_t* status) {
  if (threadIdx.x != 0) return;
  if (counts) {
    nd = counts[0];
    ni = counts[1];
    nq = counts[2];
  }
  uint64_t gate = 0;
  int32_t st = 0;
  if (nd > max_d || ni > max_i || nq > max_q) {
    gate = G_FAIL;
    st = ST_EINVAL;
    nd = ni = nq = 0;
  }
  ix.ctr[C_R_NDEL] = nd;
  ix.ctr[C_R_NINS] = ni;
  ix.ctr[C_R_NQ] = nq;
  ix.ctr[C_R_GATE] = gate;
  ix.ctr[C_DEL_OK] = 0;
  ix.ctr[C_R_FIRST] = ix.ctr[C_NEXT_ID];
  if (status) {
    status[0] = st;
    status[1] = 0;
  }
}

// After the deletes are classified and before any mutation: id space and
// the worst-case slab demand |I|(R+2) + |D|R (|I|(R+2) without repair); a
// bootstrap (no live node left once this round's tombstones are set) takes at
// most boot_max new vectors. On success the new ids are handed out.
__global__ void k_round_gate(Index ix, uint32_t tombstone_only, uint32_t boot_max, int32_t* status) {
  if (threadIdx.x != 0) return;
  uint64_t gate = ix.ctr[C_R_GATE];
  if (gate & G_FAIL) return;
  const uint64_t dok = ix.ctr[C_DEL_OK], ni = ix.ctr[C_R_NINS];
  const uint64_t next = ix.ctr[C_NEXT_ID], live = ix.ctr[C_LIVE];
  const uint64_t need = ni * (ix.R + 2ull) + (tombstone_only ? 0ull : dok * ix.R);
  const bool boot = ni > 0 && live == dok;
  int32_t st = 0;
  if (next + ni > ix.cap)
    st = ST_ECAPACITY;
  else if (ix.ctr[C_FREE_TOP] < need)
    st = ST_EPOOL;
  else if (boot && ni > boot_max)
    st = ST_EINVAL;
  if (st) {
    gate |= G_FAIL;
  } else {
    gate |= boot ? G_BOOT : G_NOBOOT;
    ix.ctr[C_R_FIRST] = next;
    ix.ctr[C_NEXT_ID] = next + ni;
    ix.ctr[C_LIVE] = live - dok + ni;
  }
  ix.ctr[C_R_GATE] = gate;
  if (status) status[0] = st;
}

// reclaim: compaction republishes every dirty node, so it needs that many slabs
__global__ void k_reclaim_gate(Index ix, int32_t* status) {
  if (threadIdx.x != 0) return;
  const uint64_t gate = ix.ctr[C_R_GATE];
  if (gate & G_FAIL) return;
  const bool ok = ix.ctr[C_FREE_TOP] >= ix.ctr[C_DIRTY];
  if (!ok) ix.ctr[C_R_GATE] = gate | G_RFAIL;
  if (status) status[1] = ok ? 0 : ST_EPOOL;
}

// new rows at ids [first, first + n) (16-byte words), and the ids handed out
__global__ void k_store_rows(Index ix, const uint4* src, uint32_t* ids_out, uint32_t first, uint32_t n, Dyn d) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  first = dyn_first(ix, d, first);
  const uint32_t words = ix.metric == 0 ? ix.dim / 16u : ix.dim / 4u;
  uint4* dst = reinterpret_cast<uint4*>(ix.metric == 0 ? (void*)ix.x : (void*)ix.xf) + (size_t)first * words;
  const uint64_t total = (uint64_t)n * words;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    dst[t] = src[t];
    if (ids_out && t % words == 0) ids_out[t / words] = first + (uint32_t)(t / words);
  }
}

// uint8 rows of at most 256 bytes: the squared norm of each new row goes into
// its (still unborn) reference word, where every later publication carries it
__global__ void __launch_bounds__(256) k_row_norms(Index ix, uint32_t first, uint32_t n, Dyn d) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  first = dyn_first(ix, d, first);
  const uint32_t words = ix.dim / 16u;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint4* row = reinterpret_cast<const uint4*>(ix.x + (size_t)(first + i) * ix.dim);
    uint32_t nn = 0;
    for (uint32_t w = 0; w < words; ++w) {
      const uint4 v = row[w];
      nn = dot16(v, v, nn);
    }
    ix.refs[first + i] = REF_UNBORN | ((uint64_t)nn << 32);
  }
}

// ---- entry set: the S smallest live ids ---------------------------------------------
// Old members stay unless deleted; the gap is filled with the next live ids
// above the old largest member (every live id below it is already a member).
__device__ inline uint32_t block_prefix(bool keep, uint32_t* wcnt, uint32_t* total) {
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t m = ballot(keep);
  if (lane_id() == 0) wcnt[w] = __popcll(m);
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    if (i < w) before += wcnt[i];
    tot += wcnt[i];
  }
  *total = tot;
  return before + lanes_below(m);
}

// The uint8 entry set's shifted copy, each byte XOR 0x80 (a signed value, as
// the matrix cores take it), stored in the order the scoring kernel's lanes
// take their operands: for each block of 16 entries and each 64-byte slice of
// the rows, 1 KiB holding lane l's 16 bytes at 16 l (entry 16 b + l % 16,
// bytes 64 s + 16 (l / 16) .. + 15), so that one operand load of a wave reads
// 1 KiB of consecutive bytes. Slices past dim are zero; entry e's negated
// squared norm (the form the scoring epilogue adds) is at e.
__global__ void __launch_bounds__(256) k_entry_rows(Index ix, uint32_t S, Dyn d) {
  if (gated(ix, d)) return;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= min<uint64_t>(S, ix.ctr[C_N_ENTRIES])) return;
  const uint4* src = reinterpret_cast<const uint4*>(ix.x + (size_t)ix.entries[e] * ix.dim);
  const uint32_t nsl = (ix.dim + 63) / 64, nc = ix.dim / 16;
  uint8_t* blk = ix.ent_x + (size_t)(e >> 4) * nsl * 1024u + (e & 15u) * 16u;
  int sq = 0;
  for (uint32_t c = 0; c < nsl * 4u; ++c) {
    uint4 w = make_uint4(0u, 0u, 0u, 0u);
    if (c < nc) {
      w = src[c];
      w.x ^= 0x80808080u;
      w.y ^= 0x80808080u;
      w.z ^= 0x80808080u;
      w.w ^= 0x80808080u;
      sq = __builtin_amdgcn_sdot4((int)w.x, (int)w.x, sq, false);
      sq = __builtin_amdgcn_sdot4((int)w.y, (int)w.y, sq, false);
      sq = __builtin_amdgcn_sdot4((int)w.z, (int)w.z, sq, false);
      sq = __builtin_amdgcn_sdot4((int)w.w, (int)w.w, sq, false);
    }
    // slice c / 4, lane (c % 4) * 16 + e % 16
    *reinterpret_cast<uint4*>(blk + (c >> 2) * 1024u + (c & 3u) * 256u) = w;
  }
  ix.ent_norm[e] = -sq;
}

__global__ void __launch_bounds__(1024) k_refresh_entries(Index ix, uint32_t next_id, uint32_t S, Dyn d) {
  __shared__ uint32_t wcnt[16];
  if (gated(ix, d)) return;
  next_id = dyn_first(ix, d, next_id);  // ids at or above the bound are not yet live
  const uint32_t m_old = (uint32_t)ix.ctr[C_N_ENTRIES];
  const uint32_t start = m_old ? ix.entries[m_old - 1] + 1u : 0u;
  uint32_t out = 0;
  for (uint32_t base = 0; base < m_old; base += blockDim.x) {
    const uint32_t t = base + threadIdx.x;
    const uint32_t id = t < m_old ? ix.entries[t] : NONE;
    const bool keep = id != NONE && !ref_del(load_ref(ix, id));
    __syncthreads();
    uint32_t tot;
    const uint32_t pos = block_prefix(keep, wcnt, &tot);
    if (keep) ix.entries[out + pos] = id;
    out += tot;
    __syncthreads();
  }
  for (uint32_t base = start; base < next_id && out < S; base += blockDim.x) {
    const uint32_t id = base + threadIdx.x;
    const bool keep = id < next_id && !ref_del(load_ref(ix, id));
    uint32_t tot;
    const uint32_t pos = block_prefix(keep, wcnt, &tot);
    if (keep && out + pos < S) ix.entries[out + pos] = id;
    out = min(S, out + tot);
    __syncthreads();
  }
  if (threadIdx.x == 0) ix.ctr[C_N_ENTRIES] = out;
}

// ---- start-set scoring: the L best start nodes of every query --------------------------
// The start set (the entry set, or the batch itself for a bootstrap) is the
// same for every query of a launch, so scoring it is one dense block of
// distances. Float rows: k_scan_dist_f (64 queries x 256 start rows per
// workgroup, staged through LDS) writes the distance matrix and k_scan_select
// takes, with one wave per query, the exact L smallest (distance, id) keys.
// Uint8 rows are scored on the matrix cores twice instead (first for bounds,
// then for the few keys under them), so the matrix never reaches memory.
// Start rows are in ascending id order, so the row index breaks distance ties
// exactly as the id does.
constexpr int SD_Q = 64, SD_E = 256, SD_KW = 4, SD_STRIDE = SD_KW + 1;  // in 16-byte words
constexpr uint32_t D_INVALID = 0xFFFFFFFFu;

__device__ inline uint32_t start_id(const Index& ix, const ScanArgs& a, uint32_t e) {
  return a.mode == MODE_BOOT ? a.first + e : ix.entries[e];
}

// launch-time counts: queries of this launch, start-set size, first id
__device__ inline void resolve(const Index& ix, ScanArgs& a) {
  a.nq = dyn_count(ix, a.d, a.nq);
  // insert searches: query i of the launch is stored row first + c0 + i; a
  // bootstrap's start set is the whole batch, so its first id is the batch's
  if (a.d.first_ctr != NO_CTR) a.first = (uint32_t)ix.ctr[a.d.first_ctr] + (a.mode == MODE_BOOT ? 0u : a.d.c0);
  if (a.ns_ctr != NO_CTR) a.ns = (uint32_t)min<uint64_t>(a.ns, ix.ctr[a.ns_ctr]);
}

// uint8 rows on the matrix cores: every byte is shifted to a signed value
// (x - 128, an XOR with 0x80), which leaves every difference and so every
// squared distance unchanged, and d = |q'|^2 + |e'|^2 - 2 q'.e' is exact in
// int32. One wave scores 32 start rows x 64 queries at a time as 2 x 4 tiles
// of v_mfma_i32_16x16x64_i8 (start rows as the M operand, queries as N), one
// 64-byte slice of the rows per step; the operands are read straight from
// memory (the start rows stay in L2 across the query tiles). In the result
// tile lane l holds query l % 16 and the four start rows 4 (l / 16) + i, so
// each lane stores 16 contiguous bytes of its query's distance row.
typedef int v4i32 __attribute__((ext_vector_type(4)));
constexpr int SD_WT = 64;  // queries per wave task (and start rows per group-count tile)

__device__ inline v4i32 signed_frag(const uint8_t* row, uint32_t off, uint32_t dim) {
  v4i32 f = {0, 0, 0, 0};
  if (row && off < dim) {
    const uint4 w = *reinterpret_cast<const uint4*>(row + off);
    f = v4i32{(int)(w.x ^ 0x80808080u), (int)(w.y ^ 0x80808080u), (int)(w.z ^ 0x80808080u),
              (int)(w.w ^ 0x80808080u)};
  }
  return f;
}

// a fragment of a row stored already shifted
__device__ inline v4i32 shifted_frag(const uint8_t* row, uint32_t off, uint32_t dim) {
  v4i32 f = {0, 0, 0, 0};
  if (row && off < dim) {
    const uint4 w = *reinterpret_cast<const uint4*>(row + off);
    f = v4i32{(int)w.x, (int)w.y, (int)w.z, (int)w.w};
  }
  return f;
}

__device__ inline int frag_sq(v4i32 f) {
  int s = __builtin_amdgcn_sdot4(f.x, f.x, 0, false);
  s = __builtin_amdgcn_sdot4(f.y, f.y, s, false);
  s = __builtin_amdgcn_sdot4(f.z, f.z, s, false);
  return __builtin_amdgcn_sdot4(f.w, f.w, s, false);
}

// One wave scores 64 queries against a span of SCAN_SPAN start rows, 32 rows
// (one group) at a time, in KS 64-byte slices (KS * 64 >= dim). The query
// tile's operands and squared norms are loaded once per span and stay in
// registers; query slices past dim are zero, so whatever a start row's slice
// holds there adds nothing. In the result tile lane l holds query 16n + l % 16
// against start rows 16m + 4k + i (k = l / 16), and each value is kept as
// u = 2 q'.e' - |e'|^2, one shift-add from the accumulator, so that the
// distance is |q'|^2 - u and the smallest distance is the largest u.
// SCAN_MIN writes each query's group minima; SCAN_DENSE writes them and the
// distances (each lane 16 contiguous bytes of its query's row). SCAN_FILTER
// writes the (distance, row) key of every row at or below the query's bound:
// the four lanes that hold one query fill interleaved slots of the query's span
// region (lane k takes slots k, k + 4, ...), so no lane needs another's count,
// and the four counts go to one word, a byte each; keys past a lane's slots are
// left to the dense fallback. No atomics: each (query, span) pair belongs to
// one wave.
enum ScanPass { SCAN_MIN = 0, SCAN_FILTER = 1, SCAN_DENSE = 2 };

// key slots per (query, span): the per-query key buffer split over the spans
__device__ inline uint32_t scan_slots(uint32_t n_span) { return SCAN_KEYS_Q / max(1u, n_span); }
// slots of one lane of a (query, span) region: below 255, where the byte count saturates
__device__ inline uint32_t scan_lane_slots(uint32_t n_span) { return min(scan_slots(n_span) / 4u, 254u); }

// uint8 group minima, tiled: for each 64-query tile and span of start rows, the
// eight groups of each of the tile's queries side by side (64 x 8 words); the
// first slot of query qi in span s
__device__ inline size_t gmin_tile_slot(uint32_t qi, uint32_t s, uint32_t n_span) {
  return (((size_t)(qi >> 6) * n_span + s) * 64u + (qi & 63u)) * 8u;
}

// the two values a lane and its partner l ^ 16 (SWAP16) or l ^ 32 hold in a
// and b: after the swap a lane of an even 16-lane row holds its own a and its
// partner's a, a lane of an odd row its partner's b and its own b
template <bool SWAP16>
__device__ inline void swap_rows(uint32_t& a, uint32_t& b) {
  const auto p = SWAP16 ? __builtin_amdgcn_permlane16_swap(a, b, false, false)
                        : __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = p[0];
  b = p[1];
}
__device__ inline uint32_t quad_sum(uint32_t v) {
  uint32_t w = v;
  swap_rows<true>(v, w);
  v += w;
  w = v;
  swap_rows<false>(v, w);
  return v + w;
}
// the largest of v[n] over the four lanes l % 16 + 16k, left in lane
// l % 16 + 16n (a reduce-scatter: three swaps for four values)
__device__ inline int quad_max_scatter(const int v[4]) {
  uint32_t a = (uint32_t)v[0], b = (uint32_t)v[1], c = (uint32_t)v[2], d = (uint32_t)v[3];
  swap_rows<true>(a, b);  // even rows: (own v0, partner v0); odd rows: (partner v1, own v1)
  swap_rows<true>(c, d);
  uint32_t x = (uint32_t)max((int)a, (int)b), y = (uint32_t)max((int)c, (int)d);
  swap_rows<false>(x, y);  // rows 0, 1: (own, partner) of v0 / v1; rows 2, 3: of v2 / v3
  return max((int)x, (int)y);
}

constexpr int U_INVALID = (int)0x80000000;  // u of a row that is not scored

// PRE: the start set is the entry set, read from its shifted, operand-ordered
// copy (16-entry blocks in entry order, zero past dim, the blocks padded to a
// multiple of two; norms beside them) instead of through the id list. CHUNKED (rows longer than
// 64 KS bytes, a whole number of KS-slice chunks): the query operands are
// reloaded per chunk instead of staying in registers.
template <int PASS, bool PRE, int KS, bool CHUNKED>
__device__ inline void scan_dist_wave_span(const Index& ix, const ScanArgs& a, uint32_t span, uint32_t q0) {
  constexpr uint32_t CW = 64u * KS;  // bytes of a row per chunk
  const int l = lane_id();
  const uint32_t ns = a.ns, dim = ix.dim, r = (uint32_t)(l & 15), k4 = (uint32_t)(l >> 4), kc = k4 * 16u;
  const uint32_t rb = k4 * 4u;  // first of this lane's four start rows within a 16-row block
  const uint32_t n_span = (ns + SCAN_SPAN - 1) / SCAN_SPAN;
  const uint32_t e_begin = span * SCAN_SPAN, e_end = min(ns, e_begin + SCAN_SPAN);
  const uint32_t nsl = (dim + 63) / 64;  // 64-byte slices per row of the entry copy
  // the query tile: rows q0 + 16n + r; a row past the launch's queries reads
  // the last query, and its results are not written
  const uint8_t* qbase = a.mode == MODE_QUERY ? (const uint8_t*)a.q : ix.x + (size_t)(a.first + a.qoff) * dim;
  const uint8_t* qrow[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) qrow[n] = qbase + (size_t)min(q0 + (uint32_t)n * 16u + r, a.nq - 1u) * dim;
  v4i32 qf[KS][4];
  auto load_q = [&](uint32_t c0) {
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) qf[ks][n] = signed_frag(qrow[n], c0 + (uint32_t)ks * 64u + kc, dim);
  };
  int qn[4] = {0, 0, 0, 0};
  for (uint32_t c0 = 0; c0 < (CHUNKED ? dim : 1u); c0 += CW) {
    load_q(c0);
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) qn[n] += frag_sq(qf[ks][n]);
  }
#pragma unroll
  for (int n = 0; n < 4; ++n) qn[n] = (int)quad_sum((uint32_t)qn[n]);
  // this lane's own query after a reduce-scatter: q0 + 16k + r
  const uint32_t q_own = q0 + k4 * 16u + r;
  const int qn_own = k4 == 0 ? qn[0] : k4 == 1 ? qn[1] : k4 == 2 ? qn[2] : qn[3];
  // a bootstrap row never scores itself: row qoff + q0 + 16n + r of the start
  // set (elsewhere a value no row offset takes)
  const int self_base = a.mode == MODE_BOOT ? (int)(a.qoff + q0 + r) : -0x40000000;
  int nthr[4];      // SCAN_FILTER: a row is kept when u >= nthr
  uint32_t cnt[4];  // SCAN_FILTER: this lane's keys per query
  uint64_t* outp = nullptr;
  uint32_t lane_cap = 0;
  if constexpr (PASS == SCAN_FILTER) {
    lane_cap = scan_lane_slots(n_span);
    outp = a.cand + (size_t)span * scan_slots(n_span) + k4;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const uint32_t qi = q0 + (uint32_t)n * 16u + r;
      const uint32_t b = qi < a.nq ? a.bound[qi] : 0u;
      // distances stay below 2^25: a bound of 2^31 or more admits every row
      nthr[n] = qi >= a.nq ? 0x7FFFFFFF : b >= 0x80000000u ? U_INVALID + 1 : qn[n] - (int)b;
      cnt[n] = 0;
    }
  }
  uint32_t gb[8];  // SCAN_MIN / SCAN_DENSE: the span's group minima of this lane's own query
#pragma unroll
  for (int j = 0; j < 8; ++j) gb[j] = D_INVALID;
  // one group of 32 start rows: its products and results; the group's minimum
  // for each query, one query per lane (SCAN_MIN / SCAN_DENSE)
  auto group = [&](uint32_t e0) -> uint32_t {
    // this lane's rows of the two 16-row blocks: 16m + r, and 16m + rb + i in the result
    const uint8_t* erow[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if constexpr (PRE) {
        // block (e0 + 16m) / 16 of the operand-ordered copy, this lane's 16 bytes
        erow[m] = ix.ent_x + (size_t)((e0 >> 4) + (uint32_t)m) * nsl * 1024u + (uint32_t)l * 16u;
      } else {
        const uint32_t e = e0 + (uint32_t)m * 16u + r;
        erow[m] = e < e_end ? ix.x + (size_t)start_id(ix, a, e) * dim : nullptr;
      }
    }
    v4i32 acc[2][4];
    int es[2] = {0, 0};  // !PRE: partial squared norms of rows 16m + r
    for (uint32_t c0 = 0; c0 < (CHUNKED ? dim : 1u); c0 += CW) {
      if constexpr (CHUNKED) load_q(c0);
      v4i32 ef[KS][2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if constexpr (PRE) {
            const uint4 w = *reinterpret_cast<const uint4*>(erow[m] + ((c0 >> 6) + (uint32_t)ks) * 1024u);
            ef[ks][m] = v4i32{(int)w.x, (int)w.y, (int)w.z, (int)w.w};
          } else {
            ef[ks][m] = signed_frag(erow[m], c0 + (uint32_t)ks * 64u + kc, dim);
            es[m] += frag_sq(ef[ks][m]);
          }
        }
      const bool first = !CHUNKED || c0 == 0;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ef[0][m], qf[0][n], first ? v4i32{0, 0, 0, 0} : acc[m][n],
                                                            0, 0, 0);
#pragma unroll
      for (int ks = 1; ks < KS; ++ks)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 4; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ef[ks][m], qf[ks][n], acc[m][n], 0, 0, 0);
    }
    int ner[2][4];  // minus the squared norms of this lane's start rows 16m + rb + i
    if constexpr (PRE) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        // the (negated) norm array is padded to whole 64-row tiles
        const int4 v = *reinterpret_cast<const int4*>(ix.ent_norm + e0 + (uint32_t)m * 16u + rb);
        ner[m][0] = v.x;
        ner[m][1] = v.y;
        ner[m][2] = v.z;
        ner[m][3] = v.w;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int en = (int)quad_sum((uint32_t)es[m]);  // lane l: row 16m + l % 16
#pragma unroll
        for (int i = 0; i < 4; ++i) ner[m][i] = -__shfl(en, (int)rb + i, 64);
      }
    }
    // rows of the group past the start set, and a bootstrap row itself, are not scored
    const bool check = a.mode == MODE_BOOT || e0 + 32u > ns;
    const int lim = (int)ns - (int)e0;  // rows 16m + rb + i below lim exist
    int gmax[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const uint32_t qi = q0 + (uint32_t)n * 16u + r;
      int u[2][4];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) u[m][i] = (acc[m][n][i] << 1) + ner[m][i];
      if (check) {
        const int self = self_base + n * 16 - (int)e0;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = m * 16 + (int)rb + i;
            if (o >= lim || o == self) u[m][i] = U_INVALID;
          }
      }
      if constexpr (PASS != SCAN_FILTER) {
        if constexpr (PASS == SCAN_DENSE) {
          if (qi < a.nq) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
              uint32_t d[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) d[i] = u[m][i] == U_INVALID ? D_INVALID : (uint32_t)(qn[n] - u[m][i]);
              const uint32_t e = e0 + (uint32_t)m * 16u + rb;
              uint32_t* out = a.dist + (size_t)qi * ns + e;
              if ((ns & 3u) == 0 && e + 3 < ns) {
                *reinterpret_cast<uint4*>(out) = make_uint4(d[0], d[1], d[2], d[3]);
              } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  if (e + (uint32_t)i < ns) out[i] = d[i];
              }
            }
          }
        }
        int v = u[0][0];
#pragma unroll
        for (int j = 1; j < 8; ++j) v = max(v, u[j >> 2][j & 3]);
        gmax[n] = v;
      } else {
        uint64_t* out = outp + (size_t)qi * SCAN_KEYS_Q;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (u[m][i] >= nthr[n]) {
              out[4u * min(cnt[n], lane_cap - 1u)] =
                  make_key((uint32_t)(qn[n] - u[m][i]), e0 + (uint32_t)m * 16u + rb + (uint32_t)i);
              ++cnt[n];
            }
      }
    }
    if constexpr (PASS != SCAN_FILTER) {
      const int g = quad_max_scatter(gmax);
      return g == U_INVALID ? D_INVALID : (uint32_t)(qn_own - g);
    }
    return D_INVALID;
  };
  if constexpr (PASS == SCAN_FILTER) {
    for (uint32_t e0 = e_begin; e0 < e_end; e0 += 32u) group(e0);
  } else {
    // unrolled, so that each minimum has a register of its own
#pragma unroll
    for (int j = 0; j < SCAN_SPAN / 32; ++j) {
      const uint32_t e0 = e_begin + (uint32_t)j * 32u;
      if (e0 >= e_end) break;
      gb[j] = group(e0);
    }
  }
  if constexpr (PASS != SCAN_FILTER) {
    // the span's eight minima of each query side by side: the wave's two
    // stores fill 2 KiB of whole lines (groups past the start set stay invalid)
    if (q_own < a.nq) {
      uint4* gp = reinterpret_cast<uint4*>(a.gmin + gmin_tile_slot(q_own, span, n_span));
      gp[0] = make_uint4(gb[0], gb[1], gb[2], gb[3]);
      gp[1] = make_uint4(gb[4], gb[5], gb[6], gb[7]);
    }
  }
  if constexpr (PASS == SCAN_FILTER) {
    // the four lanes' counts of query r, a byte each (lane k's in byte k)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const uint32_t qi = q0 + (uint32_t)n * 16u + r;
      const uint32_t packed = quad_sum(min(cnt[n], 255u) << (8u * k4));
      if (l < 16 && qi < a.nq) a.ncand[(size_t)qi * n_span + span] = packed;
    }
  }
}

template <int PASS, bool PRE, int KS, bool CHUNKED>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(KS <= 2 ? (PASS == SCAN_MIN ? 4 : 3) : 2))) k_scan_dist(Index ix, ScanArgs a) {
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t n_span = (a.ns + SCAN_SPAN - 1) / SCAN_SPAN, n_tasks = n_span * ((a.nq + SD_WT - 1) / SD_WT);
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  // consecutive waves take consecutive spans of one query tile
  for (uint32_t t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < n_tasks; t += waves)
    scan_dist_wave_span<PASS, PRE, KS, CHUNKED>(ix, a, t % n_span, (t / n_span) * SD_WT);
}

// Float rows: the same 64 x 256 tiling over 16-element slices, in FP32; start
// rows come from the traversal copy (FP8 rows as value/256, their scale
// applied once per pair at the end).
template <int TRAV>
__device__ inline void scan_dist_f_tile(const Index& ix, const ScanArgs& a, uint32_t e0, uint32_t q0, float4* qt,
                                        float4* et, float* es) {
  const int t = (int)threadIdx.x;
  const uint32_t ns = a.ns, dim = ix.dim;
  const int qg = t / 32, eg = t % 32;
  float acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.f;
  const uint32_t my_e = e0 + (uint32_t)t;
  const uint32_t my_eid = my_e < ns ? start_id(ix, a, my_e) : NONE;
  es[t] = (TRAV == TRAV_FP8 && my_eid != NONE) ? ix.xs[my_eid] * 256.0f : 1.0f;
  const uint32_t my_q = q0 + (uint32_t)(t & 63);
  const float* qrow = nullptr;
  if (my_q < a.nq)
    qrow = a.mode == MODE_QUERY ? (const float*)a.q + (size_t)my_q * dim : ix.xf + (size_t)(a.first + a.qoff + my_q) * dim;
  for (uint32_t k0 = 0; k0 < dim; k0 += 16) {
    __syncthreads();
    {
      const int r = t & 63, c = t >> 6;
      qt[r * SD_STRIDE + c] = qrow ? reinterpret_cast<const float4*>(qrow + k0)[c] : make_float4(0, 0, 0, 0);
    }
    float4 ev4[4] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0),
                     make_float4(0, 0, 0, 0)};
    if (my_eid != NONE) {
      if (TRAV == TRAV_NATIVE) {
        const float4* rw = reinterpret_cast<const float4*>(ix.xf + (size_t)my_eid * dim + k0);
#pragma unroll
        for (int c = 0; c < 4; ++c) ev4[c] = rw[c];
      } else if (TRAV == TRAV_BF16) {
        const uint4* rw = reinterpret_cast<const uint4*>(ix.xb + (size_t)my_eid * dim + k0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint4 w = rw[h];
          const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
          float f[8];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            f[2 * e] = __builtin_bit_cast(float, wd[e] << 16);
            f[2 * e + 1] = __builtin_bit_cast(float, wd[e] & 0xFFFF0000u);
          }
          ev4[2 * h] = make_float4(f[0], f[1], f[2], f[3]);
          ev4[2 * h + 1] = make_float4(f[4], f[5], f[6], f[7]);
        }
      } else {
        const uint4 w = *reinterpret_cast<const uint4*>(ix.x8 + (size_t)my_eid * dim + k0);
        const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ev4[e] = make_float4(e4m3_div256(wd[e] & 0xFFu), e4m3_div256((wd[e] >> 8) & 0xFFu),
                               e4m3_div256((wd[e] >> 16) & 0xFFu), e4m3_div256(wd[e] >> 24));
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) et[t * SD_STRIDE + c] = ev4[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float4 qv[8], ev[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) qv[i] = qt[(qg * 8 + i) * SD_STRIDE + c];
#pragma unroll
      for (int j = 0; j < 8; ++j) ev[j] = et[(eg + 32 * j) * SD_STRIDE + c];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float x = acc[i][j];
          x = __builtin_fmaf(qv[i].x, ev[j].x, x);
          x = __builtin_fmaf(qv[i].y, ev[j].y, x);
          x = __builtin_fmaf(qv[i].z, ev[j].z, x);
          acc[i][j] = __builtin_fmaf(qv[i].w, ev[j].w, x);
        }
    }
  }
  __syncthreads();
  // group minima: the 32 start rows e0 + 4 (eg / 4) + {0..3} + 32 j form group
  // e0 / 32 + eg / 4 (8 group slots per 256-row tile), reduced over the four
  // adjacent threads that hold them
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t qi = q0 + (uint32_t)(qg * 8 + i);
    const uint32_t self = a.mode == MODE_BOOT ? a.qoff + qi : NONE;
    uint32_t g = D_INVALID;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t e = e0 + (uint32_t)(eg + 32 * j);
      const float d = 1.0f - es[eg + 32 * j] * acc[i][j];
      const uint32_t key = e == self || e >= ns ? D_INVALID : fkey(d);
      g = min(g, key);
      if (qi < a.nq && e < ns) a.dist[(size_t)qi * ns + e] = key;
    }
    g = min(g, (uint32_t)__shfl_xor((int)g, 1, 64));
    g = min(g, (uint32_t)__shfl_xor((int)g, 2, 64));
    if (qi < a.nq && (eg & 3) == 0) a.gmin[(size_t)qi * a.g_stride + (e0 >> 5) + (uint32_t)(eg >> 2)] = g;
  }
}

template <int TRAV>
__global__ void __launch_bounds__(256) k_scan_dist_f(Index ix, ScanArgs a) {
  __shared__ float4 qt[SD_Q * SD_STRIDE];
  __shared__ float4 et[SD_E * SD_STRIDE];
  __shared__ float es[SD_E];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t n_et = (a.ns + SD_E - 1) / SD_E, n_tiles = n_et * ((a.nq + SD_Q - 1) / SD_Q);
  for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    __syncthreads();
    scan_dist_f_tile<TRAV>(ix, a, (tile % n_et) * SD_E, (tile / n_et) * SD_Q, qt, et, es);
  }
}

// One wave per query: the exact L smallest (distance, row) pairs of its
// distance row. The scoring kernels leave, per query, the smallest distance of
// every group of 32 start rows. If at least L groups hold a valid row, the L-th
// smallest group minimum b bounds the L-th smallest distance from above (the L
// groups at or below b each hold a row at or below it). One pass over the row
// compacts every row at or below b, as a (distance, row) key, to LDS; a
// bitonic sort then puts the answer first. Should more than `cap` rows lie at
// or below b (ties, or no bound), bisection over the row, counting with
// ballots, lowers the bound until they fit; if more than `cap` rows tie at the
// L-th value itself, the rows below it plus the first ones (in row order)
// equal to it are taken. Rows ascend with ids, so (distance, row) sorts as
// (distance, id); ids are looked up at the end.
constexpr uint32_t SEL_COMPACT = 512;  // rows compacted per query
constexpr int SEL_GPL = 8;             // group minima per lane: up to 512 groups (16,384 start rows)
constexpr int SEL_CH = 8;              // row values per lane per step of a pass

// rows of D at or below hi, counted
__device__ inline uint32_t sel_count(const uint32_t* D, uint32_t ns, uint32_t hi) {
  const int l = lane_id();
  uint32_t c = 0;
  for (uint32_t base = 0; base < ns; base += 64 * SEL_CH) {
    uint32_t v[SEL_CH];
#pragma unroll
    for (int t = 0; t < SEL_CH; ++t) {
      const uint32_t i = base + (uint32_t)(t * 64 + l);
      v[t] = i < ns ? D[i] : D_INVALID;
    }
#pragma unroll
    for (int t = 0; t < SEL_CH; ++t) c += (uint32_t)__popcll(ballot(v[t] <= hi));
  }
  return c;
}

// keys of the rows at or below hi, in row order, the first `cap` of them
// written; returns their number (may exceed cap)
__device__ inline uint32_t sel_compact(const uint32_t* D, uint32_t ns, uint32_t hi, uint64_t* sel, uint32_t cap,
                                       uint32_t* lmin) {
  const int l = lane_id();
  uint32_t n = 0, mn = D_INVALID;
  for (uint32_t base = 0; base < ns; base += 64 * SEL_CH) {
    uint32_t v[SEL_CH];
#pragma unroll
    for (int t = 0; t < SEL_CH; ++t) {
      const uint32_t i = base + (uint32_t)(t * 64 + l);
      v[t] = i < ns ? D[i] : D_INVALID;
    }
#pragma unroll
    for (int t = 0; t < SEL_CH; ++t) {
      mn = min(mn, v[t]);
      const bool in = v[t] <= hi;
      const uint64_t m = ballot(in);
      const uint32_t pos = n + lanes_below(m);
      if (in && pos < cap) sel[pos] = make_key(v[t], base + (uint32_t)(t * 64 + l));
      n += (uint32_t)__popcll(m);
    }
  }
  *lmin = mn;
  return n;
}

// rows a query selects: L, or every valid start row if fewer
__device__ inline uint32_t scan_need(const ScanArgs& a, uint32_t qi) {
  const bool self_in = a.mode == MODE_BOOT && a.qoff + qi < a.ns;  // the one row scored D_INVALID
  return min(a.L, a.ns - (self_in ? 1u : 0u));
}

// The need_all-th smallest of the group minima held GPL per lane (the rest
// unused): at least need_all groups, and so at least need_all rows, lie at or
// below it. With fewer valid groups than that, every valid row (D_INVALID - 1).
template <int GPL>
__device__ inline uint32_t bound_bisect(const uint32_t (&gv)[SEL_GPL], uint32_t need_all) {
  uint32_t glo = D_INVALID, ghi = 0, gvalid = 0;
#pragma unroll
  for (int t = 0; t < GPL; ++t) {
    if (gv[t] != D_INVALID) {
      glo = min(glo, gv[t]);
      ghi = max(ghi, gv[t]);
      ++gvalid;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    glo = min(glo, (uint32_t)__shfl_xor((int)glo, o, 64));
    ghi = max(ghi, (uint32_t)__shfl_xor((int)ghi, o, 64));
    gvalid += (uint32_t)__shfl_xor((int)gvalid, o, 64);
  }
  if (bcast(gvalid) < need_all) return D_INVALID - 1;
  uint32_t lo = bcast(glo), hi = bcast(ghi);
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    uint32_t c = 0;
#pragma unroll
    for (int t = 0; t < GPL; ++t) c += (uint32_t)__popcll(ballot(gv[t] <= mid));
    if (c >= need_all) hi = mid;
    else lo = mid + 1;
  }
  return hi;
}

// query qi's bound from its group minima
__device__ inline uint32_t scan_bound_one(const ScanArgs& a, uint32_t qi, uint32_t need_all) {
  const int l = lane_id();
  uint32_t gv[SEL_GPL];
  uint32_t ng;
  if (a.g_rows == (uint32_t)SD_WT) {
    // uint8 rows: the tiled layout, eight slots per span (all written); lane l
    // takes groups 4 (64 u + l) .. + 3, one 16-byte load each
    const uint32_t n_span = (a.ns + SCAN_SPAN - 1) / SCAN_SPAN;
    ng = n_span * 8u;
#pragma unroll
    for (int u = 0; u < SEL_GPL / 4; ++u) {
      const uint32_t i = (uint32_t)(u * 64 + l) * 4u;
      uint4 v = make_uint4(D_INVALID, D_INVALID, D_INVALID, D_INVALID);
      if (i < ng) v = *reinterpret_cast<const uint4*>(a.gmin + gmin_tile_slot(qi, i >> 3, n_span) + (i & 7u));
      gv[4 * u] = v.x;
      gv[4 * u + 1] = v.y;
      gv[4 * u + 2] = v.z;
      gv[4 * u + 3] = v.w;
    }
  } else {
    // float rows: each query's row of g_stride slots (a 256-row tile's eight groups interleave its rows)
    ng = (a.ns + a.g_rows - 1) / a.g_rows * (a.g_rows / 32);
    const uint32_t* G = a.gmin + (size_t)qi * a.g_stride;
#pragma unroll
    for (int t = 0; t < SEL_GPL; ++t) {
      const uint32_t i = (uint32_t)(t * 64 + l);
      gv[t] = i < ng ? G[i] : D_INVALID;
    }
  }
  // up to 256 groups fill four values per lane in both layouts
  return ng <= 256 ? bound_bisect<4>(gv, need_all) : bound_bisect<SEL_GPL>(gv, need_all);
}

__device__ inline void scan_select_one(const Index& ix, const ScanArgs& a, uint32_t qi, uint64_t* sel, uint32_t cap) {
  const int l = lane_id();
  const uint32_t ns = a.ns;
  const uint32_t* D = a.dist + (size_t)qi * ns;
  const uint32_t need_all = scan_need(a, qi);
  uint32_t cnt = 0;
  if (need_all > 0) {
    uint32_t hi = scan_bound_one(a, qi, need_all);
    uint32_t lmin;
    cnt = sel_compact(D, ns, hi, sel, cap, &lmin);
    if (cnt > cap) {
      // invariant: #{v < lo} < need_all <= #{v <= hi} = cnt
      for (int o = 32; o > 0; o >>= 1) lmin = min(lmin, (uint32_t)__shfl_xor((int)lmin, o, 64));
      uint32_t lo = bcast(lmin);
      while (cnt > cap && lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        const uint32_t c = sel_count(D, ns, mid);
        if (c >= need_all) {
          hi = mid;
          cnt = c;
        } else {
          lo = mid + 1;
        }
      }
      wave_sync();
      if (cnt <= cap) {
        cnt = sel_compact(D, ns, hi, sel, cap, &lmin);
      } else {
        // more than cap rows share the value tau = lo = hi
        const uint32_t need = need_all - (lo ? sel_count(D, ns, lo - 1) : 0u);
        uint32_t eq_seen = 0;
        cnt = 0;
        for (uint32_t base = 0; base < ns; base += 64) {
          const uint32_t i = base + (uint32_t)l;
          const uint32_t v = i < ns ? D[i] : D_INVALID;
          const bool eq = v == lo;
          const uint64_t meq = ballot(eq);
          const bool take = v < lo || (eq && eq_seen + lanes_below(meq) < need);
          const uint64_t mt = ballot(take);
          if (take) sel[cnt + lanes_below(mt)] = make_key(v, i);
          cnt += (uint32_t)__popcll(mt);
          eq_seen += (uint32_t)__popcll(meq);
        }
      }
    }
  }
  const int np = next_pow2_ge64((int)cnt);
  for (int i = (int)cnt + l; i < np; i += 64) sel[i] = KEY_NONE;
  wave_sync();
  wave_bitonic_sort(sel, np);
  cnt = min(cnt, need_all);
  for (uint32_t i = (uint32_t)l; i < cnt; i += 64) {
    const uint64_t k = sel[i];
    a.out_keys[(size_t)qi * a.out_stride + i] = make_key(key_dist(k), start_id(ix, a, key_id(k)));
  }
  if (l == 0) a.out_n[qi] = cnt;
}

__global__ void __launch_bounds__(256) k_scan_select(Index ix, ScanArgs a, uint32_t sel_cap) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t qi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (qi >= a.nq) return;
  scan_select_one(ix, a, qi, reinterpret_cast<uint64_t*>(smem + (size_t)(threadIdx.x >> 6) * 8 * sel_cap), sel_cap);
}

// uint8 rows, in four launches that never write the distance matrix: group
// minima (k_scan_dist<SCAN_MIN>), each query's bound (k_scan_bound), the keys
// at or below it (k_scan_dist<SCAN_FILTER>), and their sort (k_scan_final).
// A query whose keys overflow its list (heavy ties at the bound) has its
// distance row written out and takes the general selection above.
__global__ void __launch_bounds__(256) k_scan_bound(Index ix, ScanArgs a) {
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t qi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (qi >= a.nq) return;
  const uint32_t need_all = scan_need(a, qi);
  const uint32_t b = need_all ? scan_bound_one(a, qi, need_all) : 0u;
  if (lane_id() == 0) a.bound[qi] = b;
}

// query qi's distances to every start row (exact in int32, as on the matrix cores)
__device__ inline void scan_dense_row_u8(const Index& ix, const ScanArgs& a, uint32_t qi) {
  const uint32_t dim = ix.dim, ns = a.ns;
  const uint8_t* q = a.mode == MODE_QUERY ? (const uint8_t*)a.q + (size_t)qi * dim
                                          : ix.x + (size_t)(a.first + a.qoff + qi) * dim;
  const uint32_t self = a.mode == MODE_BOOT ? a.qoff + qi : NONE;
  uint32_t* D = a.dist + (size_t)qi * ns;
  for (uint32_t e = (uint32_t)lane_id(); e < ns; e += 64) {
    const uint8_t* row = ix.x + (size_t)start_id(ix, a, e) * dim;
    int s = 0;
    for (uint32_t k = 0; k < dim; k += 16) {
      const uint4 qa = *reinterpret_cast<const uint4*>(q + k), ea = *reinterpret_cast<const uint4*>(row + k);
      const uint32_t qw[4] = {qa.x, qa.y, qa.z, qa.w}, ew[4] = {ea.x, ea.y, ea.z, ea.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int qs = (int)(qw[j] ^ 0x80808080u), es = (int)(ew[j] ^ 0x80808080u);
        s = __builtin_amdgcn_sdot4(qs, qs, s, false);
        s = __builtin_amdgcn_sdot4(es, es, s, false);
        s -= 2 * __builtin_amdgcn_sdot4(qs, es, 0, false);
      }
    }
    D[e] = e == self ? D_INVALID : (uint32_t)s;
  }
  __threadfence_block();
  wave_sync();
}

__global__ void __launch_bounds__(256) k_scan_final(Index ix, ScanArgs a, uint32_t sel_cap) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t qi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (qi >= a.nq) return;
  uint64_t* sel = reinterpret_cast<uint64_t*>(smem + (size_t)(threadIdx.x >> 6) * 8 * sel_cap);
  const int l = lane_id();
  const uint32_t n_span = (a.ns + SCAN_SPAN - 1) / SCAN_SPAN;  // one span per lane
  const uint32_t lane_cap = scan_lane_slots(n_span);
  // a span's region interleaves the keys of its four scoring lanes (lane k's
  // j-th key in slot 4j + k, at least 4 slots per lane) and its count word
  // holds their counts, a byte each. The first two keys of every scoring lane
  // are read together with the counts; slots past a count hold stale keys
  // that are never used
  constexpr uint32_t EARLY = 8;
  const uint64_t* src = a.cand + (size_t)qi * SCAN_KEYS_Q + (uint32_t)l * scan_slots(n_span);
  uint64_t early[EARLY];
#pragma unroll
  for (uint32_t j = 0; j < EARLY; ++j) early[j] = (uint32_t)l < n_span ? src[j] : KEY_NONE;
  const uint32_t packed = (uint32_t)l < n_span ? a.ncand[(size_t)qi * n_span + (uint32_t)l] : 0u;
  uint32_t ck[4], c = 0;
  bool over = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ck[k] = (packed >> (8 * k)) & 0xFFu;
    over |= ck[k] > lane_cap;
    c += ck[k];
  }
  uint32_t off = c;  // inclusive prefix over the spans
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)off, (unsigned)o, 64);
    if (l >= o) off += v;
  }
  const uint32_t n = (uint32_t)__shfl((int)off, 63, 64);
  if (ballot(over) || n > sel_cap) {
    scan_dense_row_u8(ix, a, qi);
    scan_select_one(ix, a, qi, sel, sel_cap);
    return;
  }
  off -= c;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (uint32_t j = 0; j < EARLY / 4; ++j)
      if (j < ck[k]) sel[off + j] = early[4 * j + (uint32_t)k];
    for (uint32_t j = EARLY / 4; j < ck[k]; ++j) sel[off + j] = src[4 * j + (uint32_t)k];
    off += ck[k];
  }
  const int np = next_pow2_ge64((int)n);
  for (int i = (int)n + l; i < np; i += 64) sel[i] = KEY_NONE;
  wave_sync();
  const uint32_t cnt = min(n, scan_need(a, qi));
  uint64_t* out = a.out_keys + (size_t)qi * a.out_stride;
  if (np <= 128) {
    // up to 128 keys: sorted in registers, two per lane
    uint64_t v[2] = {sel[l], np > 64 ? sel[64 + l] : KEY_NONE};
    if (np > 64) {
      wave_sort_regs<2>(v);
    } else {
      uint64_t (&v1)[1] = *reinterpret_cast<uint64_t(*)[1]>(&v[0]);
      wave_sort_regs<1>(v1);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if ((uint32_t)(s * 64 + l) < cnt) out[s * 64 + l] = make_key(key_dist(v[s]), start_id(ix, a, key_id(v[s])));
  } else if (np <= 512) {
    // up to 512 keys: sorted in registers, four or eight per lane
    uint64_t v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = s * 64 < np ? sel[s * 64 + l] : KEY_NONE;
    if (np <= 256) {
      uint64_t (&v4)[4] = *reinterpret_cast<uint64_t(*)[4]>(&v[0]);
      wave_sort_regs<4>(v4);
    } else {
      wave_sort_regs<8>(v);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s)
      if ((uint32_t)(s * 64 + l) < cnt) out[s * 64 + l] = make_key(key_dist(v[s]), start_id(ix, a, key_id(v[s])));
  } else {
    wave_bitonic_sort(sel, np);
    for (uint32_t i = (uint32_t)l; i < cnt; i += 64) {
      const uint64_t k = sel[i];
      out[i] = make_key(key_dist(k), start_id(ix, a, key_id(k)));
    }
  }
  if (l == 0) a.out_n[qi] = cnt;
}

// keys per wave: the compacted rows, or the L selected ones
uint32_t scan_select_keys(uint32_t L) { return (uint32_t)max((int)SEL_COMPACT, next_pow2_ge64((int)L)); }
uint32_t scan_select_lds_per_wave(uint32_t L) { return 8u * scan_select_keys(L); }

// ---- traversal policies ------------------------------------------------------------
// uint8 rows: G lanes per row, C 16-byte chunks each (G * C * 16 = dim)
template <int G, int C = 1>
struct TravU8 {
  static constexpr bool FLOAT = false;
  struct Q {
    uint4 f[C];
    uint32_t qq;
  };
  __device__ static Q load_query(const void* row) {
    Q q;
    const uint4* r = reinterpret_cast<const uint4*>(row);
    const int c = lane_id() % G;
    uint32_t qq = 0;
#pragma unroll
    for (int t = 0; t < C; ++t) {
      q.f[t] = r[t * G + c];
      qq = dot16(q.f[t], q.f[t], qq);
    }
    q.qq = group_sum<G>(qq);
    return q;
  }
  __device__ static const void* stored_row(const Index& ix, uint32_t id) { return ix.x + (size_t)id * ix.dim; }
  __device__ static size_t query_bytes(const Index& ix) { return ix.dim; }
  __device__ static void dist_batch(const Index& ix, const Q& q, const uint32_t* ids, int cnt, uint64_t* ck,
                                    uint64_t* cr) {
    if constexpr (C == 1)
      dist_batch_u8<G>(ix, q.f[0], q.qq, ids, cnt, ck, cr);
    else
      dist_batch_u8c<G, C, true>(ix, q.f, q.qq, ids, cnt, ck, cr);
  }
  // distances only: no reference words read (one line request per row)
  __device__ static void dist_only(const Index& ix, const Q& q, const uint32_t* ids, int cnt, uint64_t* ck) {
    if constexpr (C == 1)
      dist_batch_u8<G, false>(ix, q.f[0], q.qq, ids, cnt, ck, nullptr);
    else
      dist_batch_u8c<G, C, false>(ix, q.f, q.qq, ids, cnt, ck, nullptr);
  }
  __device__ static uint32_t out_bits(uint32_t kd) { return kd; }            // int32 distance
  __device__ static uint32_t pad_bits() { return 0x7FFFFFFFu; }              // INT32_MAX
};

// float rows: traversal copy TRAV, G lanes per row; FP32 re-rank for non-FP32 copies
template <int G, int TRAV>
struct TravFloat {
  static constexpr bool FLOAT = true;
  static constexpr int MODE = TRAV;
  using T = TravF<G, TRAV>;
  using Q = typename T::Q;
  static constexpr int GF = G * T::EPC / 4;  // lanes per row of the FP32 copy
  using Exact = TravF<GF, TRAV_NATIVE>;
  __device__ static Q load_query(const void* row) { return T::load_query(reinterpret_cast<const float*>(row)); }
  __device__ static const void* stored_row(const Index& ix, uint32_t id) { return ix.xf + (size_t)id * ix.dim; }
  __device__ static size_t query_bytes(const Index& ix) { return (size_t)ix.dim * 4; }
  __device__ static void dist_batch(const Index& ix, const Q& q, const uint32_t* ids, int cnt, uint64_t* ck,
                                    uint64_t* cr) {
    T::dist_batch(ix, q, ids, cnt, ck, cr);
  }
  __device__ static void dist_only(const Index& ix, const Q& q, const uint32_t* ids, int cnt, uint64_t* ck) {
    T::dist_batch(ix, q, ids, cnt, ck, nullptr);
  }
  __device__ static uint32_t out_bits(uint32_t kd) { return __builtin_bit_cast(uint32_t, fkey_inv(kd)); }
  __device__ static uint32_t pad_bits() { return 0x7F800000u; }              // +inf
};

// ---- greedy beam search (queries and insert searches) ---------------------------------
// Candidates of one expansion batch after the visited table: lane l holds id
// nid, vr its table result, fresh whether it is to be scored. Only ids that
// met a crowded table (VT_CROWDED) can repeat an id of another lane or of the
// list, so each crowded lane is checked with one ballot: it gives way to a
// lane that stored the same id, to a lower crowded lane with it and (with a
// list in registers, lanes below n holding keys lk) to a listed entry.
__device__ inline bool drop_crowded_twins(uint32_t nid, uint32_t vr, bool fresh, uint64_t lk = KEY_NONE,
                                          int n = 0) {
  const int l = lane_id();
  const uint64_t crowded = ballot(vr == VT_CROWDED);
  if (!crowded) return fresh;
  const uint64_t fr = ballot(fresh);
  bool keep = fresh;
  for (uint64_t cm = crowded & fr; cm; cm &= cm - 1) {
    const int c = (int)__builtin_ctzll(cm);
    const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)nid, c);
    const uint64_t others = ballot(nid == id) & fr & ~(1ull << c);
    bool drop = (others & ((1ull << c) - 1ull)) != 0 || (others & ~crowded) != 0;
    if (n > 0) drop = drop || ballot(l < n && key_id(lk) == id) != 0;
    if (drop && l == c) keep = false;
  }
  return keep;
}

// a wave's running totals of expansions and distance evaluations over its
// queries (added to the index's counters once per workgroup)
struct SearchTally {
  uint32_t exp = 0, dist = 0;  // a wave's share of one launch stays below 2^32
};

// The search's results from its final list (keys lk, reference words lr, n
// entries): a query's k nearest non-deleted listed nodes (re-ranked from the
// FP32 rows for a bf16 / FP8 traversal), or an insert search's visit count;
// then the per-query counters. ci and ck are the wave's 64-entry scratch.
template <class TP>
__device__ inline void search_finish(const Index& ix, const SearchArgs& a, uint32_t qi, const void* qrow,
                                     const uint64_t* lk, const uint64_t* lr, int n, uint32_t* ci, uint64_t* ck,
                                     uint32_t nexp, uint32_t ndist, SearchTally& tally) {
  const int l = lane_id();
  if (a.mode == MODE_QUERY) {
    // the first `want` listed nodes whose reference has flag 0: k of them, or
    // rerank*k for a bf16 / FP8 traversal, which are then re-scored from the
    // FP32 rows and cut to k
    bool rerank = false;
    if constexpr (TP::FLOAT) rerank = TP::MODE != TRAV_NATIVE;
    if (a.rerank == 0) rerank = false;
    const uint32_t want = rerank ? min(64u, a.rerank * a.k) : a.k;
    uint32_t got = 0;
    for (int b = 0; b < n && got < want; b += 64) {
      const int i = b + l;
      bool live = false;
      uint64_t key = 0;
      if (i < n) {
        key = lk[i];
        live = !ref_del(lr[i]);
      }
      const uint64_t m = ballot(live);
      const uint32_t idx = got + lanes_below(m);
      if (live && idx < want) {
        if (rerank) {
          ci[idx] = key_id(key);
        } else {
          a.out_ids[(size_t)qi * a.k + idx] = key_id(key);
          a.out_d[(size_t)qi * a.k + idx] = TP::out_bits(key_dist(key));
        }
      }
      got += (uint32_t)__popcll(m);
    }
    got = min(got, want);
    if constexpr (TP::FLOAT) {
      if (rerank) {
        wave_sync();
        using E = typename TP::Exact;
        E::dist_batch(ix, E::load_query(reinterpret_cast<const float*>(qrow)), ci, (int)got, ck, nullptr);
        for (int i = (int)got + l; i < 64; i += 64) ck[i] = KEY_NONE;
        wave_sync();
        wave_bitonic_sort(ck, 64);
        got = min(got, a.k);
        for (uint32_t i = (uint32_t)l; i < got; i += 64) {
          a.out_ids[(size_t)qi * a.k + i] = key_id(ck[i]);
          a.out_d[(size_t)qi * a.k + i] = TP::out_bits(key_dist(ck[i]));
        }
      }
    }
    for (uint32_t i = got + (uint32_t)l; i < a.k; i += 64) {
      a.out_ids[(size_t)qi * a.k + i] = NONE;
      a.out_d[(size_t)qi * a.k + i] = TP::pad_bits();
    }
  } else if (l == 0) {
    a.vis_cnt[qi] = nexp;
  }
  if (a.mode == MODE_QUERY) {
    tally.exp += nexp;
    tally.dist += ndist;
  }
  if (l == 0) {
    if (a.counts) {
      a.counts[2 * (size_t)qi] = nexp;
      a.counts[2 * (size_t)qi + 1] = ndist;
    }
  }
}

// The ids in the slabs of one or two list entries (reference words r0, r1),
// side by side: lanes [0, R) read the first slab, lanes [R, 2R) the second.
__device__ inline uint32_t expansion_ids(const Index& ix, uint64_t r0, uint64_t r1, bool two) {
  const uint32_t l = (uint32_t)lane_id(), R = ix.R;
  const bool second = l >= R;
  const uint64_t r = second ? r1 : r0;
  const uint32_t slot = second ? l - R : l;
  const uint32_t deg = (second && !two) ? 0u : ref_deg(r), s = ref_slab(r);
  uint32_t nid = NONE;
  if (slot < deg && s < ix.P) {
    const uint32_t* w = ix.slabs + (size_t)s * 2u * R + slot;
    // with writers running alongside, the slab may have been written on
    // another XCD after this one cached its previous use: read it coherently
    nid = ix.concurrent ? __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *w;
  }
  return nid < ix.cap ? nid : NONE;
}

// One wavefront per query, starting from the initial list the start-set scan
// left (the L best members of the entry set). This variant (L > 64) keeps the
// list in LDS. Per-wave LDS: the double-buffered candidate list (keys,
// reference words, expanded flags), one batch of candidates, the merge
// scratch and the visited table.
template <class TP>
__device__ inline void search_one(const Index& ix, const SearchArgs& a, char* base, uint32_t qi, SearchTally& tally) {
  const int l = lane_id();
  CandList cl;
  uint64_t* p64 = reinterpret_cast<uint64_t*>(base);
  cl.k0 = p64;
  cl.k1 = p64 + a.L;
  cl.r0 = p64 + 2 * a.L;
  cl.r1 = p64 + 3 * a.L;
  uint64_t* ck = p64 + 4 * a.L;
  uint64_t* cr = ck + 64;
  cl.acck = cr + 64;
  cl.accr = cl.acck + 64;
  uint32_t* ci = reinterpret_cast<uint32_t*>(cl.accr + 64);
  cl.accp = ci + 64;
  uint32_t* vt = cl.accp + 64;
  uint8_t* flags = reinterpret_cast<uint8_t*>(vt + a.vt_mask + 1);
  cl.x0 = flags;
  cl.x1 = flags + a.L;
  cl.cur = 0;
  cl.n = 0;
  cl.L = (int)a.L;
  const void* qrow = a.mode == MODE_QUERY ? (const void*)((const uint8_t*)a.q + (size_t)qi * TP::query_bytes(ix))
                                          : TP::stored_row(ix, a.first + qi);
  const typename TP::Q qv = TP::load_query(qrow);
  for (uint32_t i = (uint32_t)l; i <= a.vt_mask; i += 64) vt[i] = NONE;
  // the initial list: the L best start nodes, with their reference words
  const uint32_t n0 = a.init_n[qi];
  for (uint32_t i = (uint32_t)l; i < n0; i += 64) {
    const uint64_t key = a.init_keys[(size_t)qi * a.init_stride + i];
    cl.k0[i] = key;
    cl.r0[i] = load_ref(ix, key_id(key));
    cl.x0[i] = 0;
  }
  cl.n = (int)n0;
  wave_sync();
  for (int i = l; i < cl.n; i += 64) (void)vt_insert(vt, a.vt_mask, key_id(cl.k0[i]));
  wave_sync();
  uint32_t ndist = (uint32_t)ix.ctr[C_N_ENTRIES];  // scored by the start-set scan
  uint32_t nexp = 0;
  {
    while (nexp < a.vcap) {
      // up to W best unexpanded entries, within the visit cap, all picked
      // before any neighbor is merged; their slabs are read two at a time side
      // by side (lanes [w*R, (w+1)*R) read the w-th), each pair scored and
      // merged in turn (the merge keeps the L smallest of the union, so the
      // result is that of one merge of all)
      uint64_t pk[4], pr[4];
      uint32_t np = 0;
      int from = 0;
      for (uint32_t k = 0; k < 4; ++k) {
        pk[k] = KEY_NONE;
        pr[k] = 0;
        if (k > 0 && (k >= a.W || nexp + k >= a.vcap)) continue;
        const int j = list_first_open(cl, from);
        if (j < 0) break;
        from = j + 1;
        pk[k] = cl.keys()[j];
        pr[k] = cl.refs()[j];
        if (l == 0) {
          cl.flags()[j] = 1;
          if (a.mode == MODE_INSERT) a.vis_keys[(size_t)qi * a.vcap + nexp + k] = pk[k];
        }
        ++np;
      }
      if (np == 0) break;
      wave_sync();
      nexp += np;
      for (uint32_t h = 0; 2 * h < np; ++h) {
        const uint32_t nid = expansion_ids(ix, pr[2 * h], pr[2 * h + 1], 2 * h + 1 < np);
        const uint32_t vr = nid != NONE ? vt_insert(vt, a.vt_mask, nid) : VT_SEEN;
        bool fresh = vr != VT_SEEN;
        // a crowded table can pass an id listed in both slabs twice; the merge
        // needs distinct candidates
        fresh = drop_crowded_twins(nid, vr, fresh);
        const uint64_t m = ballot(fresh);
        if (fresh) ci[lanes_below(m)] = nid;
        const int cnt = __popcll(m);
        wave_sync();
        if (cnt) {
          TP::dist_batch(ix, qv, ci, cnt, ck, cr);
          wave_sync();
          list_merge(cl, ck, cr, cnt);
          ndist += (uint32_t)cnt;
        }
      }
    }
  }

  search_finish<TP>(ix, a, qi, qrow, cl.keys(), cl.refs(), cl.n, ci, ck, nexp, ndist, tally);
}

// Crowded-table twins of a step with H halves of 64 slab entries (half h
// holds the slabs of the step's entries 2h and 2h + 1, in rank order). A
// crowded lane drops its id when an earlier half, a lane of its own half that
// stored it or a lower crowded lane of its own half offers it too, or when it
// is listed (list entry 64s + l, for entries below n, is lane l's lk[s]).
template <int H, int NL>
__device__ inline void drop_crowded_twins_h(const uint32_t (&nid)[H], const uint32_t (&vr)[H], bool (&fresh)[H],
                                            const uint64_t (&lk)[NL], int n) {
  const int l = lane_id();
  uint64_t crowded[H], fr[H];
  uint64_t any = 0;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    crowded[h] = ballot(vr[h] == VT_CROWDED);
    fr[h] = ballot(fresh[h]);
    any |= crowded[h];
  }
  if (!any) return;
#pragma unroll
  for (int h = 0; h < H; ++h) {
    for (uint64_t cm = crowded[h] & fr[h]; cm; cm &= cm - 1) {
      const int c = (int)__builtin_ctzll(cm);
      const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)nid[h], c);
      const uint64_t others = ballot(nid[h] == id) & fr[h] & ~(1ull << c);
      bool drop = (others & ((1ull << c) - 1ull)) != 0 || (others & ~crowded[h]) != 0;
#pragma unroll
      for (int e = 0; e < h; ++e) drop = drop || (ballot(nid[e] == id) & fr[e]) != 0;
#pragma unroll
      for (int s = 0; s < NL; ++s) drop = drop || ballot(64 * s + l < n && key_id(lk[s]) == id) != 0;
      if (drop && l == c) fresh[h] = false;
    }
  }
}

// A list entry's reference word is read when the entry is expanded (or read
// ahead for expansion), not when its distance is computed: most scored nodes
// never reach expansion, and a reference word read costs a line request of its
// own. Entries not read yet hold REF_LAZY (degree 127, impossible for a real
// word); the output stage reads the words of the entries that still have none.
constexpr uint64_t REF_LAZY = ~0ull;

// List slots in registers: entry 64s + l of the list is lane l's slot s.
// The open (unexpanded) entries are one ballot per slot; entries are taken
// lowest first.
template <int NL>
__device__ inline bool open_any(const uint64_t (&o)[NL]) {
  bool any = false;
#pragma unroll
  for (int s = 0; s < NL; ++s) any = any || o[s] != 0;
  return any;
}

// the lowest entry of a non-empty open set (its list index), taken out of it
template <int NL>
__device__ inline int open_take(uint64_t (&o)[NL]) {
  if constexpr (NL == 1) {
    const int j = (int)__builtin_ctzll(o[0]);
    o[0] &= o[0] - 1;
    return j;
  } else {
    int e = -1;
#pragma unroll
    for (int s = 0; s < NL; ++s)
      if (e < 0 && o[s]) {
        e = 64 * s + (int)__builtin_ctzll(o[s]);
        o[s] &= o[s] - 1;
      }
    return e;
  }
}

// the value of list entry e (wave-uniform) held in slots v
template <int NL>
__device__ inline uint64_t list_at(const uint64_t (&v)[NL], int e) {
  if constexpr (NL == 1) {
    return bcast_lane64(v[0], e);
  } else {
    uint64_t r = 0;
#pragma unroll
    for (int s = 0; s < NL; ++s)
      if ((e >> 6) == s) r = bcast_lane64(v[s], e & 63);
    return r;
  }
}

// The same search with the list in registers, for L <= 64 NL: lane l holds
// entries l, 64 + l, ... (key, reference word or REF_LAZY, expanded flag),
// entries at or past n hold KEY_NONE. The next entries to expand are the
// lowest of one ballot per slot. A step expands up to W entries (H = 2 halves
// of 64 slab entries when W = 4), scores all their fresh neighbors in one
// batch and merges them by rank: every list entry and accepted candidate
// counts the keys of the other side below it (one broadcast per accepted
// candidate), the first L of the union are scattered to LDS at their ranks and
// read back in order. Per-wave LDS: a scratch of 64 max(H, NL) entries (one
// batch of candidates, the merged list) and the visited table.
template <class TP, int H, int NL>
__device__ inline void search_one_rl(const Index& ix, const SearchArgs& a, char* base, uint32_t qi,
                                     SearchTally& tally) {
  constexpr int WMAX = 2 * H;
  constexpr int CAP = 64 * (H > NL ? H : NL);
  const int l = lane_id();
  uint64_t* ck = reinterpret_cast<uint64_t*>(base);
  uint64_t* cr = ck + CAP;
  uint32_t* ci = reinterpret_cast<uint32_t*>(cr + CAP);
  uint32_t* vt = ci + CAP;
  const int L = (int)a.L;
  const void* qrow = a.mode == MODE_QUERY ? (const void*)((const uint8_t*)a.q + (size_t)qi * TP::query_bytes(ix))
                                          : TP::stored_row(ix, a.first + qi);
  const typename TP::Q qv = TP::load_query(qrow);
  for (uint32_t i = (uint32_t)l; i <= a.vt_mask; i += 64) vt[i] = NONE;
  // the initial list: the L best start nodes, with their reference words
  int n = (int)a.init_n[qi];
  uint64_t lk[NL], lr[NL];
  uint32_t lx[NL];
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    lk[s] = KEY_NONE;
    lr[s] = 0;
    lx[s] = 0;
    if (64 * s + l < n) {
      lk[s] = a.init_keys[(size_t)qi * a.init_stride + 64 * s + l];
      lr[s] = REF_LAZY;
    }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < NL; ++s)
    if (64 * s + l < n) (void)vt_insert(vt, a.vt_mask, key_id(lk[s]));
  wave_sync();
  uint32_t ndist = (uint32_t)ix.ctr[C_N_ENTRIES];  // scored by the start-set scan
  uint32_t nexp = 0;
  // slab ids of the entries the next step is expected to expand, read while
  // this step's vectors are in flight; used when the merge leaves those
  // entries first (their keys identify them)
  uint32_t pre_nid[H];
  uint64_t pre_k[WMAX];
#pragma unroll
  for (int h = 0; h < H; ++h) pre_nid[h] = NONE;
#pragma unroll
  for (int k = 0; k < WMAX; ++k) pre_k[k] = KEY_NONE;
  while (nexp < a.vcap) {
    // up to W best unexpanded entries, within the visit cap
    uint64_t open[NL];
#pragma unroll
    for (int s = 0; s < NL; ++s) open[s] = ballot(64 * s + l < n && lx[s] == 0);
    if (!open_any(open)) break;
    uint64_t key[WMAX], ref[WMAX];
    uint32_t np = 0;
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      key[k] = KEY_NONE;
      ref[k] = 0;
      if (open_any(open) && (k == 0 || ((uint32_t)k < a.W && nexp + (uint32_t)k < a.vcap))) {
        const int e = open_take(open);  // then the open entries after the picked ones
        key[k] = list_at(lk, e);
        ref[k] = list_at(lr, e);
#pragma unroll
        for (int s = 0; s < NL; ++s)
          if (64 * s + l == e) lx[s] = 1;
        if (l == 0 && a.mode == MODE_INSERT) a.vis_keys[(size_t)qi * a.vcap + nexp + (uint32_t)k] = key[k];
        ++np;
      }
    }
    nexp += np;
    // the slabs of entries 2h, 2h + 1 side by side in half h: lanes
    // [w*R, (w+1)*R) read the w-th
    uint32_t nid[H];
    bool hit = true;
#pragma unroll
    for (int k = 0; k < WMAX; ++k) hit = hit && key[k] == pre_k[k];
    if (!hit) {  // the slabs were not read ahead: the reference words first, where not read yet
#pragma unroll
      for (int k = 0; k < WMAX; ++k)
        if (key[k] != KEY_NONE && ref[k] == REF_LAZY) ref[k] = load_ref(ix, key_id(key[k]));
    }
#pragma unroll
    for (int h = 0; h < H; ++h)
      nid[h] = hit ? pre_nid[h] : expansion_ids(ix, ref[2 * h], ref[2 * h + 1], key[2 * h + 1] != KEY_NONE);
#pragma unroll
    for (int k = 0; k < WMAX; ++k) pre_k[k] = KEY_NONE;
#pragma unroll
    for (int h = 0; h < H; ++h) pre_nid[h] = NONE;
    // read-ahead, first half: the entries the next step should expand and the
    // reference words they still lack; the words are consumed only after the
    // visited-table pass, so their latency overlaps it
    const bool ahead = nexp < a.vcap && open_any(open);
    uint64_t pref[WMAX];
    int pj[WMAX];
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      pref[k] = 0;
      pj[k] = -1;
    }
    if (ahead) {
      uint64_t o[NL];
#pragma unroll
      for (int s = 0; s < NL; ++s) o[s] = open[s];
#pragma unroll
      for (int k = 0; k < WMAX; ++k) {
        if (open_any(o) && (k == 0 || ((uint32_t)k < a.W && nexp + (uint32_t)k < a.vcap))) {
          const int e = open_take(o);
          pre_k[k] = list_at(lk, e);
          pref[k] = list_at(lr, e);
          if (pref[k] == REF_LAZY) {
            pref[k] = load_ref(ix, key_id(pre_k[k]));
            pj[k] = e;
          }
        }
      }
    }
    uint32_t vr[H];
    bool fresh[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      vr[h] = nid[h] != NONE ? vt_insert(vt, a.vt_mask, nid[h]) : VT_SEEN;
      fresh[h] = vr[h] != VT_SEEN;
    }
    // a crowded table can pass an id twice (two slabs list it) or one already
    // listed; the insertion below needs distinct, unlisted candidates
    drop_crowded_twins_h<H, NL>(nid, vr, fresh, lk, n);
    int cnt = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint64_t m = ballot(fresh[h]);
      if (fresh[h]) ci[cnt + (int)lanes_below(m)] = nid[h];
      cnt += __popcll(m);
    }
    // read-ahead, second half: the slabs' ids, in flight with this step's rows
    if (ahead) {
#pragma unroll
      for (int k = 0; k < WMAX; ++k)
#pragma unroll
        for (int s = 0; s < NL; ++s)
          if (64 * s + l == pj[k]) lr[s] = pref[k];  // the word travels with its entry through the merge
#pragma unroll
      for (int h = 0; h < H; ++h)
        pre_nid[h] = expansion_ids(ix, pref[2 * h], pref[2 * h + 1], pre_k[2 * h + 1] != KEY_NONE);
    }
    wave_sync();
    if (!cnt) continue;
    TP::dist_only(ix, qv, ci, cnt, ck);  // reference words are read when an entry is expanded
    wave_sync();
    ndist += (uint32_t)cnt;
    // merge: the list becomes the L smallest of itself and the candidates
    // below its current worst entry (no other candidate can enter). Every
    // entry's place is its rank in that union: one broadcast per accepted
    // candidate counts, for each list entry and each candidate, the accepted
    // candidates below it, and for each candidate the list entries below it.
    // The wave then scatters the union's first L entries to the scratch (free
    // after the distances) and reads them back in order.
    const uint64_t worst = n == L ? list_at(lk, L - 1) : KEY_NONE;
    uint64_t cand[H], accm[H];
    int na = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      cand[h] = 64 * h + l < cnt ? ck[64 * h + l] : KEY_NONE;
      accm[h] = ballot(cand[h] < worst);
      na += __popcll(accm[h]);
    }
    if (!na) continue;
    // Per accepted candidate: one compare against each list slot gives both
    // each list entry's count of candidates below it and (its ballot, as list
    // keys and candidates are distinct) the candidate's count of list entries
    // below it; entries at or past n hold KEY_NONE and are never written back.
    uint64_t nmask[NL];
    uint32_t below_l[NL], below_c[H], list_c[H];
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      nmask[s] = ballot(64 * s + l < n);
      below_l[s] = 0;
    }
#pragma unroll
    for (int h = 0; h < H; ++h) below_c[h] = list_c[h] = 0;
#pragma unroll
    for (int hh = 0; hh < H; ++hh)
      for (uint64_t m = accm[hh]; m; m &= m - 1) {
        const int c = (int)__builtin_ctzll(m);
        const uint64_t kc = bcast_lane64(cand[hh], c);
        uint32_t nl = 0;
#pragma unroll
        for (int s = 0; s < NL; ++s) {
          const bool above = kc < lk[s];
          below_l[s] += above ? 1u : 0u;
          nl += (uint32_t)__popcll(nmask[s] & ~ballot(above));
        }
#pragma unroll
        for (int h = 0; h < H; ++h) below_c[h] += kc < cand[h] ? 1u : 0u;
        if (l == c) list_c[hh] = nl;
      }
    wave_sync();
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const uint32_t e = 64u * (uint32_t)s + (uint32_t)l;
      if ((int)e < n && e + below_l[s] < (uint32_t)L) {
        ck[e + below_l[s]] = lk[s];
        cr[e + below_l[s]] = lr[s];
        ci[e + below_l[s]] = lx[s];
      }
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const uint32_t p = list_c[h] + below_c[h];
      if (((accm[h] >> l) & 1ull) && p < (uint32_t)L) {
        ck[p] = cand[h];
        cr[p] = REF_LAZY;
        ci[p] = 0;
      }
    }
    wave_sync();
    n = min(n + na, L);
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      lk[s] = KEY_NONE;
      if (64 * s + l < n) {
        lk[s] = ck[64 * s + l];
        lr[s] = cr[64 * s + l];
        lx[s] = ci[64 * s + l];
      }
    }
    wave_sync();
  }
  // the list to LDS for the shared result stage (the candidate scratch is
  // free), every entry with its reference word: the output keeps flag-0 nodes
#pragma unroll
  for (int s = 0; s < NL; ++s) {
    if (64 * s + l < n && lr[s] == REF_LAZY) lr[s] = load_ref(ix, key_id(lk[s]));
    ck[64 * s + l] = lk[s];
    cr[64 * s + l] = lr[s];
  }
  wave_sync();
  search_finish<TP>(ix, a, qi, qrow, ck, cr, n, ci, ck, nexp, ndist, tally);
}

template <class TP, bool RL, int H, int NL = 1>
__device__ inline void search_kernel(const Index& ix, SearchArgs& a, char* smem) {
  __shared__ unsigned long long tsum[2];
  if (gated(ix, a.d)) return;
  if (threadIdx.x == 0) tsum[0] = tsum[1] = 0;
  __syncthreads();
  a.nq = dyn_count(ix, a.d, a.nq);
  a.first = dyn_first(ix, a.d, a.first);
  char* base = smem + (size_t)(threadIdx.x >> 6) * a.lds_per_wave;
  const int l = lane_id();
  SearchTally tally;
  if (!a.persistent) {  // one wave per query
    const uint32_t qi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (qi < a.nq) {
      if constexpr (RL) search_one_rl<TP, H, NL>(ix, a, base, qi, tally);
      else search_one<TP>(ix, a, base, qi, tally);
    }
  } else {
    unsigned long long* queue = &ix.ctr[C_QUEUE];
    for (uint32_t qi = wave_ticket(queue); qi < a.nq; qi = wave_ticket(queue)) {
      wave_sync();
      if constexpr (RL) search_one_rl<TP, H, NL>(ix, a, base, qi, tally);
      else search_one<TP>(ix, a, base, qi, tally);
    }
    const uint32_t done = wave_ticket(&ix.ctr[C_QDONE]);
    if (l == 0 && done + 1 == total_waves()) {
      atomicExch(queue, 0ull);
      atomicExch(&ix.ctr[C_QDONE], 0ull);
    }
  }
  // the workgroup's totals, one pair of atomics
  if (l == 0 && (tally.exp | tally.dist)) {
    atomicAdd(&tsum[0], (unsigned long long)tally.exp);
    atomicAdd(&tsum[1], (unsigned long long)tally.dist);
  }
  __syncthreads();
  if (threadIdx.x == 0 && (tsum[0] | tsum[1])) {
    atomicAdd(&ix.ctr[C_SEARCH_EXP], tsum[0]);
    atomicAdd(&ix.ctr[C_SEARCH_DIST], tsum[1]);
  }
}

// list in registers; uint8 rows hold their registers to 7 waves per SIMD (the
// LDS of 7 four-wave blocks fits a CU at the default visited-table size),
// float rows keep theirs (they would spill). Q: query searches (results out)
// or insert searches (expanded sets out), compiled apart so that each keeps
// only its own output code and each has a kernel name of its own.
template <class TP, unsigned WPE, int H, bool Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_search_rl(Index ix, SearchArgs a) {
  extern __shared__ __align__(16) char smem[];
  a.mode = Q ? MODE_QUERY : MODE_INSERT;
  search_kernel<TP, true, H>(ix, a, smem);
}

// two list slots per lane (64 < L <= 128, up to two expansions per step);
// uint8 rows at 6 waves per SIMD
template <class TP, unsigned WPE, bool Q>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) k_search_rl2(Index ix, SearchArgs a) {
  extern __shared__ __align__(16) char smem[];
  a.mode = Q ? MODE_QUERY : MODE_INSERT;
  search_kernel<TP, true, 1, 2>(ix, a, smem);
}

template <class TP, bool Q>
__global__ void __launch_bounds__(256) k_search(Index ix, SearchArgs a) {
  extern __shared__ __align__(16) char smem[];
  a.mode = Q ? MODE_QUERY : MODE_INSERT;
  search_kernel<TP, false, 1>(ix, a, smem);
}

// ---- LDS carving for the maintenance kernels ------------------------------------------
// words of the matrix-core prune's distance table (64 x 63 / 2 pairs, plus the
// diagonal's index one past them), rounded up to 16 bytes
constexpr uint32_t MX_M_WORDS = (64u * 63u / 2u + 1u + 3u) & ~3u;

struct MaintLds {
  PruneLds pr;
  uint32_t* cand;   // [nmax]
  uint32_t* nl_id;  // [R + 1] current list of the target
  uint32_t* nl_d;   // [R + 1]
  uint32_t* tmp;    // [R + 1]
};

__device__ inline MaintLds carve(char* base, const MaintArgs& a, uint32_t R) {
  MaintLds m;
  char* p = base;
  m.pr.nsort = a.nsort;
  m.pr.rows = a.prune_cap;
  m.pr.vstride = a.vstride;
  m.pr.keys = reinterpret_cast<uint64_t*>(p);
  p += (size_t)a.nsort * 8;
  m.pr.keys2 = reinterpret_cast<uint64_t*>(p);
  p += (size_t)a.prune_cap * 8;
  m.pr.M = m.pr.tn = m.pr.kn = nullptr;
  m.pr.vec = nullptr;
  m.pr.norm = m.pr.idx = nullptr;
  if (a.mx) {  // the matrix-core selection: a distance table instead of staged rows
    p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 15u) & ~(uintptr_t)15u);
    m.pr.M = reinterpret_cast<uint32_t*>(p);
    p += (size_t)MX_M_WORDS * 4;
    m.pr.tn = reinterpret_cast<uint32_t*>(p);
    p += 64 * 4;
    m.pr.kn = reinterpret_cast<uint32_t*>(p);
    p += 64 * 4;
  } else {
    m.pr.vec = reinterpret_cast<uint8_t*>(p);
    p += (size_t)a.prune_cap * a.vstride;
    m.pr.norm = reinterpret_cast<uint32_t*>(p);
    p += (size_t)a.prune_cap * 4;
    m.pr.idx = reinterpret_cast<uint32_t*>(p);
    p += (size_t)a.prune_cap * 4;
  }
  m.pr.out_ids = reinterpret_cast<uint32_t*>(p);
  p += (size_t)(R + 1) * 4;
  m.pr.out_d = reinterpret_cast<uint32_t*>(p);
  p += (size_t)(R + 1) * 4;
  m.cand = reinterpret_cast<uint32_t*>(p);
  p += (size_t)a.nmax * 4;
  m.nl_id = reinterpret_cast<uint32_t*>(p);
  p += (size_t)(R + 1) * 4;
  m.nl_d = reinterpret_cast<uint32_t*>(p);
  p += (size_t)(R + 1) * 4;
  m.tmp = reinterpret_cast<uint32_t*>(p);
  p += (size_t)(R + 1) * 4;
  m.pr.kill = reinterpret_cast<uint8_t*>(p);
  return m;
}

__device__ inline uint32_t wave_index() { return blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); }
__device__ inline char* wave_lds(char* smem, const MaintArgs& a) {
  return smem + (size_t)(threadIdx.x >> 6) * a.lds_per_wave;
}

// load node u's current list into (ids, d); returns its degree
__device__ inline uint32_t load_list(const Index& ix, uint32_t u, uint32_t* ids, uint32_t* d) {
  const uint64_t r = bcast64(load_ref(ix, u));
  const uint32_t deg = ref_deg(r), s = ref_slab(r);
  const int l = lane_id();
  if ((uint32_t)l < deg && s != NONE) {
    ids[l] = ix.slabs[(size_t)s * 2u * ix.R + (uint32_t)l];
    d[l] = ix.slabs[(size_t)s * 2u * ix.R + ix.R + (uint32_t)l];
  }
  wave_sync();
  return s == NONE ? 0u : deg;
}

__device__ inline void copy_out(const MaintLds& m, uint32_t n) {
  const int l = lane_id();
  if ((uint32_t)l < n) {
    m.nl_id[l] = m.pr.out_ids[l];
    m.nl_d[l] = m.pr.out_d[l];
  }
  wave_sync();
}

// ---- RobustPrune's ordered selection over cached distances ----------------------------
// The alpha test a^2 D(kept, x) <= b^2 D(p, x) on exact integer distances:
// 24-bit multiplies into 32 bits where every uint8 distance and both
// products fit (Index::cmp32, checked at create), 64-bit products otherwise.
template <bool C32>
struct AlphaT {
  using T = typename std::conditional<C32, uint32_t, uint64_t>::type;
  __device__ static T scale(uint32_t c, uint32_t d) {
    if constexpr (C32)
      return __umul24(c, d);
    else
      return (uint64_t)c * (uint64_t)d;
  }
};

// Lane x holds candidate x (candidates in rank order) with thr = b^2 D(p, x).
// The candidates of `rest` are decided in order, four at a time: dist(j)
// gives this lane's cached D(j, x) (read for the four together), and a
// candidate covered by an earlier one of the four is skipped; a kept j
// (keep(j, rank, true); keep(.., false) for one that is not) drops every
// later candidate it covers. Returns the kept count, at most R: the result of
// the one-at-a-time selection. The four decisions are made without branches
// (scalar selects), and reading eight rows at a time, decided or not,
// measured slower: most candidates are covered early and their rows need not
// be read. When a candidate is decided every candidate ranked before it has
// left `rest` (kept, or covered), so a kept one's cover mask needs no
// masking to the later ranks, and after the four nothing up to the last of
// them remains.
template <bool C32, class Dist, class Keep>
__device__ inline uint32_t select_in_order(uint64_t rest, uint32_t R, uint32_t a2, typename AlphaT<C32>::T thr,
                                           Dist dist, Keep keep) {
  uint32_t cnt = 0;
  while (cnt < R && rest) {
    int j[4];
    uint64_t bit[4];
    uint32_t d[4];
    // past the last candidate: bit 0 and index 63 (its distance is read and
    // never used: every caller's table has a row for every lane)
    uint64_t m = rest;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      j[k] = (int)__builtin_ctzll(m | (1ull << 63));
      const uint64_t next = m & (m - 1ull);
      bit[k] = m ^ next;
      m = next;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = dist(j[k]);
    // the four in order; with room for all four kept, liveness alone decides
    // (no count test per candidate)
    auto decide = [&](auto check_count) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t tk = rest & bit[k];  // live, not covered by an earlier one of the four
        uint32_t t = (uint32_t)((tk | (0ull - tk)) >> 63);  // tk != 0, in scalar arithmetic
        if constexpr (decltype(check_count)::value) t = cnt < R ? t : 0u;
        keep(j[k], cnt, t != 0);
        const uint64_t kill = ballot(AlphaT<C32>::scale(a2, d[k]) <= thr);
        rest &= t ? ~(kill | tk) : ~0ull;
        cnt += t;
      }
    };
    if (cnt + 4u <= R)
      decide(std::false_type{});
    else
      decide(std::true_type{});
  }
  return cnt;
}

// ---- RobustPrune on the matrix cores (uint8 rows, dim <= 128, R <= 32) ------------------
// The ranked candidates (prune_rank_u8) are decided in tiles of 64, in rank
// order, without staging their rows in LDS:
//   - the distances between the tile's candidates come from
//     v_mfma_i32_16x16x64_i8 tiles over the rows shifted to signed bytes
//     (exact int32, as everywhere: the shift leaves every difference
//     unchanged), the diagonal tiles giving the shifted norms; they go to a
//     triangular table in LDS;
//   - the candidates already kept (all ranked before the tile) are tested
//     against the whole tile at once, from the same kind of tiles (kept rows x
//     tile rows): a candidate that one of them covers is dropped;
//   - the survivors are then decided in order as in the staged selection
//     (four at a time, reading the table), the kept ones appended.
// The kept set, its order and the stored distances are exactly those of the
// one-at-a-time selection.
__device__ inline v4i32 mx_frag(const Index& ix, uint32_t id, uint32_t off) {
  v4i32 f = {0, 0, 0, 0};
  if (id != NONE && off < ix.dim) {
    const uint4 w = *reinterpret_cast<const uint4*>(ix.x + (size_t)id * ix.dim + off);
    f = v4i32{(int)(w.x ^ 0x80808080u), (int)(w.y ^ 0x80808080u), (int)(w.z ^ 0x80808080u),
              (int)(w.w ^ 0x80808080u)};
  }
  return f;
}

// index of the pair (x, y), x < y, in a triangular table
__device__ inline uint32_t tri_lt(uint32_t x, uint32_t y) { return y * (y - 1u) / 2u + x; }

template <int G>
__device__ inline int prune_select_mx(const Index& ix, int m, PruneLds& s) {
  constexpr uint32_t KS = (16u * G + 63u) / 64u;  // 64-byte steps of a row
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u, rb = (uint32_t)(l >> 4) * 4u;
  const uint64_t a2 = ix.a2, b2 = ix.b2;
  const int R = (int)ix.R;  // at most 32: two blocks of kept rows
  int cnt = 0;
  for (int t0 = 0; t0 < m && cnt < R; t0 += 64) {
    const int tm = min(64, m - t0);
    // lane l's candidate (selection), and the tile's rows as matrix operands:
    // block h, row 16h + l % 16, bytes 64 ks + 16 (l / 16) .. + 15
    const uint64_t lk = l < tm ? s.keys2[t0 + l] : KEY_NONE;
    const uint64_t dpl = (uint64_t)key_dist(lk);
    v4i32 f[4][KS];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int i = h * 16 + (int)r;
      const uint32_t id = i < tm ? key_id(s.keys2[t0 + i]) : NONE;
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) f[h][ks] = mx_frag(ix, id, ks * 64u + kc);
    }
    // 1. the tile against itself. Lane l holds rows 16g + 4 (l / 16) + i
    // against column 16h + l % 16; the diagonal blocks' diagonals are the
    // shifted squared norms, stored first
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      v4i32 acc = {0, 0, 0, 0};
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[g][ks], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (rb + (uint32_t)i == r) s.tn[g * 16 + (int)r] = (uint32_t)acc[i];
    }
    wave_sync();
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const uint4 nr = *reinterpret_cast<const uint4*>(s.tn + g * 16 + (int)rb);
      const uint32_t nrow[4] = {nr.x, nr.y, nr.z, nr.w};
#pragma unroll
      for (int h = g; h < 4; ++h) {
        v4i32 acc = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[h][ks], acc, 0, 0, 0);
        const uint32_t col = (uint32_t)h * 16u + r;
        if ((int)col >= tm) continue;
        const uint32_t nc = s.tn[col];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t row = (uint32_t)g * 16u + rb + (uint32_t)i;
          if (row < col) s.M[tri_lt(row, col)] = nrow[i] + nc - 2u * (uint32_t)acc[i];
        }
      }
    }
    uint64_t rest = tm == 64 ? ~0ull : ((1ull << tm) - 1ull);
    // 2. the kept candidates (blocks of 16 rows) against the tile
    if (cnt) {
      const int KB = (cnt + 15) / 16;
      v4i32 kf[2][KS];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int k = g * 16 + (int)r;
        const uint32_t id = g < KB && k < cnt ? s.out_ids[k] : NONE;
#pragma unroll
        for (uint32_t ks = 0; ks < KS; ++ks) kf[g][ks] = mx_frag(ix, id, ks * 64u + kc);
      }
      uint32_t nkv[2][4];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const uint4 nk = *reinterpret_cast<const uint4*>(s.kn + g * 16 + (int)rb);
        nkv[g][0] = nk.x;
        nkv[g][1] = nk.y;
        nkv[g][2] = nk.z;
        nkv[g][3] = nk.w;
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        v4i32 ka[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          if (g >= KB) break;
#pragma unroll
          for (uint32_t ks = 0; ks < KS; ++ks) ka[g] = __builtin_amdgcn_mfma_i32_16x16x64_i8(kf[g][ks], f[h][ks], ka[g], 0, 0, 0);
        }
        const uint32_t col = (uint32_t)h * 16u + r;
        bool cov = false;
        if ((int)col < tm) {
          const uint32_t nc = s.tn[col];
          const uint64_t dpc = (uint64_t)key_dist(s.keys2[t0 + (int)col]);
#pragma unroll
          for (int g = 0; g < 2; ++g) {
            if (g >= KB) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int k = g * 16 + (int)rb + i;
              if (k < cnt && a2 * (uint64_t)(nkv[g][i] + nc - 2u * (uint32_t)ka[g][i]) <= b2 * dpc) cov = true;
            }
          }
        }
        // the four row groups of a column: bits r, r + 16, r + 32, r + 48
        uint64_t cm = ballot(cov);
        cm |= cm >> 32;
        cm |= cm >> 16;
        rest &= ~((cm & 0xFFFFull) << (16 * h));
      }
    }
    wave_sync();
    // 3. the survivors in order, four at a time
    const uint32_t tnl = l < tm ? s.tn[l] : 0u;
    auto dist = [&](int j) { return l > j ? s.M[tri_lt((uint32_t)j, (uint32_t)l)] : 0u; };
    auto keep = [&](int j, uint32_t rank, bool take) {
      const uint64_t kj = bcast_lane64(lk, j);
      const uint32_t nj = (uint32_t)__builtin_amdgcn_readlane((int)tnl, j);
      if (take && l == 0) {
        s.out_ids[cnt + (int)rank] = key_id(kj);
        s.out_d[cnt + (int)rank] = key_dist(kj);
        s.kn[cnt + (int)rank] = nj;
      }
    };
    const uint32_t left = (uint32_t)(R - cnt);
    if (ix.cmp32)
      cnt += (int)select_in_order<true>(rest, left, ix.a2, AlphaT<true>::scale(ix.b2, (uint32_t)dpl), dist, keep);
    else
      cnt += (int)select_in_order<false>(rest, left, ix.a2, AlphaT<false>::scale(ix.b2, (uint32_t)dpl), dist, keep);
    wave_sync();
  }
  return cnt;
}

// ---- per-metric maintenance policy --------------------------------------------------------
// prune: RobustPrune; dist1: the exact stored distance between two rows (the
// bit pattern kept in a slab); kd: a stored distance as the distance half of a
// (distance, id) key.
template <int G>
struct MaintU8 {
  __device__ static int prune(const Index& ix, uint32_t p, const uint32_t* cand, int n, PruneLds& s) {
    if constexpr (G <= 8) {
      if (s.M) return prune_select_mx<G>(ix, prune_rank_u8<G>(ix, p, cand, n, s), s);
    }
    return robust_prune_u8<G>(ix, p, cand, n, s);
  }
  __device__ static uint32_t dist1(const Index& ix, uint32_t w, uint32_t v, uint32_t* tmp, uint64_t* ck) {
    const uint4 wf = load_frag<G>(ix.x + (size_t)w * ix.dim);
    const uint32_t ww = group_sum<G>(dot16(wf, wf, 0u));
    if (lane_id() == 0) tmp[0] = v;
    wave_sync();
    dist_batch_u8<G>(ix, wf, ww, tmp, 1, ck);
    wave_sync();
    return key_dist(ck[0]);
  }
  __device__ static uint32_t kd(uint32_t rho) { return rho; }
  static constexpr bool CHAIN = true;  // reverse edges keep a cached candidate state
  static constexpr int GL = G;
};

template <int G>
struct MaintF32 {
  __device__ static int prune(const Index& ix, uint32_t p, const uint32_t* cand, int n, PruneLds& s) {
    return robust_prune_f32<G>(ix, p, cand, n, s);
  }
  __device__ static uint32_t dist1(const Index& ix, uint32_t w, uint32_t v, uint32_t*, uint64_t*) {
    return dist1_f32<G>(ix, w, v);
  }
  __device__ static uint32_t kd(uint32_t rho) { return fkey(__builtin_bit_cast(float, rho)); }
  static constexpr bool CHAIN = false;
  static constexpr int GL = G;
};

__device__ inline void resolve(const Index& ix, MaintArgs& a) {
  a.n = dyn_count(ix, a.d, a.n);
  a.first = dyn_first(ix, a.d, a.first);
  if (a.np_ctr != NO_CTR) a.npairs = (uint32_t)min<uint64_t>(a.npairs, ix.ctr[a.np_ctr] * a.np_mult);
}

// Item loops of the maintenance kernels: persistent waves, item i, i + waves, ...
#define FOR_EACH_WAVE_ITEM(i, n) for (uint32_t i = wave_index(); i < (n); i += total_waves())

// items the calling wave takes in FOR_EACH_WAVE_ITEM over n items
__device__ inline uint32_t wave_items(uint32_t n) {
  const uint32_t w = wave_index(), W = total_waves();
  return n > w ? (n - 1u - w) / W + 1u : 0u;
}

// ---- insert: forward prune + own publication (Algorithm 2, first lines) --------------
template <class P>
__device__ inline void forward_one(const Index& ix, const MaintArgs& a, MaintLds& m, uint32_t qi, SlabCursor& cur) {
  const int l = lane_id();
  const uint32_t v = a.first + qi;
  const uint32_t nc = a.vis_cnt[qi];
  for (uint32_t j = (uint32_t)l; j < nc; j += 64) m.cand[j] = key_id(a.vis_keys[(size_t)qi * a.vcap + j]);
  wave_sync();
  const int cnt = P::prune(ix, v, m.cand, (int)nc, m.pr);
  publish(ix, v, m.pr.out_ids, m.pr.out_d, (uint32_t)cnt, C_PUB_FORWARD, &cur);
  for (uint32_t j = (uint32_t)l; j < ix.R; j += 64) a.F[(size_t)qi * ix.R + j] = j < (uint32_t)cnt ? m.pr.out_ids[j] : NONE;
}

template <class P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_forward(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  SlabCursor cur = reserve_slabs_block(ix, wave_items(a.n), 0);  // new nodes hold no slab yet
  FOR_EACH_WAVE_ITEM(qi, a.n) {
    wave_sync();
    forward_one<P>(ix, a, m, qi, cur);
  }
  finish_slabs_block(ix, cur, C_PUB_FORWARD);
}

__global__ void k_reverse_pairs(Index ix, MaintArgs a) {
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) ix.ctr[C_NSEG] = 0;
  if (t >= (uint64_t)a.n * ix.R) return;
  const uint32_t w = a.F[t];
  const uint32_t v = a.first + (uint32_t)(t / ix.R);
  a.pairs[t] = w == NONE ? KEY_NONE : pair_key(w, v);
}

// Runs of one target in the sorted pair list: the start index of each run is
// appended to seg (in no particular order; each run is applied by one wave,
// and runs touch distinct targets).
constexpr uint32_t SEG_CHUNK = 2048;  // sorted pairs per workgroup

__global__ void __launch_bounds__(256) k_segments(Index ix, const uint64_t* pairs, uint32_t n, Dyn d, uint32_t* seg) {
  __shared__ uint32_t buf[SEG_CHUNK];
  __shared__ uint32_t cnt_s, base_s;
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  const uint32_t c0 = blockIdx.x * SEG_CHUNK;
  if (c0 >= n) return;
  if (threadIdx.x == 0) cnt_s = 0;
  __syncthreads();
  // run starts of the workgroup's pairs gather in LDS, then take their place
  // in the list with one atomic per workgroup
  for (uint32_t step = 0; step < SEG_CHUNK / 256u; ++step) {
    const uint32_t t = c0 + step * 256u + threadIdx.x;
    bool start = false;
    if (t < n) {
      const uint64_t k = pairs[t];
      start = k != KEY_NONE && (t == 0 || (uint32_t)(pairs[t - 1] >> 32) != (uint32_t)(k >> 32));
    }
    const uint64_t m = ballot(start);
    uint32_t at = 0;
    if (lane_id() == 0 && m) at = atomicAdd(&cnt_s, (uint32_t)__popcll(m));
    at = bcast(at);
    if (start) buf[at + lanes_below(m)] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt_s) base_s = (uint32_t)atomicAdd(&ix.ctr[C_NSEG], (unsigned long long)cnt_s);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < cnt_s; i += blockDim.x) seg[base_s + i] = buf[i];
}

// ---- insert: reverse edges in (target, source) order, one publication per target ------
template <class P>
__device__ inline void reverse_one(const Index& ix, const MaintArgs& a, MaintLds& m, uint32_t t, SlabCursor& cur) {
  const uint32_t w = (uint32_t)(a.pairs[t] >> 32);
  const int l = lane_id();
  const uint32_t R = ix.R;
  uint32_t n = load_list(ix, w, m.nl_id, m.nl_d);
  uint64_t* ck = m.pr.keys;  // scratch for one distance
  for (uint32_t u = t; u < a.npairs && a.pairs[u] != KEY_NONE && (uint32_t)(a.pairs[u] >> 32) == w; ++u) {
    const uint32_t v = (uint32_t)a.pairs[u];
    const bool present = ballot((uint32_t)l < n && m.nl_id[l] == v) != 0ull;
    if (present) continue;  // a set union: nothing to add
    if (n < R) {
      const uint32_t rho = P::dist1(ix, w, v, m.tmp, ck);
      const uint64_t kv = make_key(P::kd(rho), v);
      const bool before = (uint32_t)l < n && make_key(P::kd(m.nl_d[l]), m.nl_id[l]) < kv;
      const uint32_t pos = (uint32_t)__popcll(ballot(before));
      uint32_t id_l = 0, d_l = 0;
      if ((uint32_t)l < n) {
        id_l = m.nl_id[l];
        d_l = m.nl_d[l];
      }
      wave_sync();
      if ((uint32_t)l < n && (uint32_t)l >= pos) {
        m.nl_id[l + 1] = id_l;
        m.nl_d[l + 1] = d_l;
      }
      if (l == 0) {
        m.nl_id[pos] = v;
        m.nl_d[pos] = rho;
      }
      wave_sync();
      ++n;
    } else {
      if ((uint32_t)l < n) m.cand[l] = m.nl_id[l];
      if (l == 0) m.cand[n] = v;
      wave_sync();
      n = (uint32_t)P::prune(ix, w, m.cand, (int)n + 1, m.pr);
      copy_out(m, n);
    }
  }
  publish(ix, w, m.nl_id, m.nl_d, n, C_PUB_REVERSE, &cur);
}


// ---- reverse edges with a cached candidate state (uint8 rows, R <= 32) --------------
// A target w takes its offers v in ascending source order: a listed v changes
// nothing, below R the offer is inserted in (distance, id) order, at R the list
// is re-pruned with v. Consecutive prunes of one target share all but one
// candidate, so the wave keeps, per slot (R + 1 of them), the candidate's row,
// norm, id, distance to w and deletion flag, and the matrix of squared
// distances between the slots' rows. An offer then costs one row load and at
// most R distances from LDS instead of a full RobustPrune. The distances are
// exact integers, so the result is the one RobustPrune gives.
// Index of the pair {x, y} of distinct slots in a triangular distance cache
// of S slots (S (S - 1) / 2 + 1 words: x = y lands inside, on a word that is
// never read for a decision).
__device__ inline uint32_t tri(uint32_t x, uint32_t y) {
  const uint32_t hi = max(x, y), lo = min(x, y);
  return hi * (hi - 1u) / 2u + lo;
}

struct ChainLds {
  uint8_t* rows;    // [S][vstride]
  uint32_t* norm;   // [S]
  uint32_t* M;      // [S (S - 1) / 2 + 1] squared distances between slots, by tri()
  uint32_t* id;     // [S]
  uint32_t* dw;     // [S] squared distance to the target
  uint32_t* dead;   // [S] deletion flag of the candidate
  uint32_t* order;  // [S] list position -> slot
  uint32_t* out_id; // [S]
  uint32_t* out_d;  // [S]
  uint32_t S, vstride;
};

__host__ __device__ inline uint32_t chain_lds_bytes(uint32_t R, uint32_t vstride) {
  const uint32_t S = R + 1;
  const uint32_t b = S * vstride + S * 4 + ((S * (S - 1u) / 2u + 1u + 3u) & ~3u) * 4 + 7 * S * 4;
  return (b + 15u) & ~15u;
}

__device__ inline ChainLds carve_chain(char* base, uint32_t R, uint32_t vstride) {
  ChainLds c;
  c.S = R + 1;
  c.vstride = vstride;
  c.rows = reinterpret_cast<uint8_t*>(base);
  uint32_t* p = reinterpret_cast<uint32_t*>(base + (size_t)c.S * vstride);
  c.norm = p;
  p += c.S;
  c.M = p;
  p += (c.S * (c.S - 1u) / 2u + 1u + 3u) & ~3u;
  c.id = p;
  p += c.S;
  c.dw = p;
  p += c.S;
  c.dead = p;
  p += c.S;
  c.order = p;
  p += c.S;
  c.out_id = p;
  p += c.S;
  c.out_d = p;
  return c;
}

// stage the rows of `cnt` slots (listed in slots[0..cnt)) with their norms
template <int G>
__device__ inline void chain_stage_rows(const Index& ix, const ChainLds& c, const uint32_t* slots, int cnt) {
  constexpr int VPP = 64 / G;
  const int l = lane_id();
  const int ch = l % G, grp = l / G;
  for (int base = 0; base < cnt; base += 4 * VPP) {
    uint4 v[4];
    int sl[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = base + u * VPP + grp;
      sl[u] = k < cnt ? (int)slots[k] : -1;
      v[u] = make_uint4(0, 0, 0, 0);
      if (sl[u] >= 0) v[u] = reinterpret_cast<const uint4*>(ix.x + (size_t)c.id[sl[u]] * ix.dim)[ch];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t nn = group_sum<G>(dot16(v[u], v[u], 0u));
      if (sl[u] >= 0) {
        *reinterpret_cast<uint4*>(c.rows + (size_t)sl[u] * c.vstride + ch * 16) = v[u];
        if (ch == 0) c.norm[sl[u]] = nn;
      }
    }
  }
  wave_sync();
}

// M[a][b] = M[b][a] = squared distance, for slot a against slots[0..cnt)
template <int G>
__device__ inline void chain_fill_row(const ChainLds& c, uint32_t a, const uint32_t* slots, int cnt) {
  constexpr int VPP = 64 / G;
  const int l = lane_id();
  const int ch = l % G, grp = l / G;
  const uint4 av = *reinterpret_cast<const uint4*>(c.rows + (size_t)a * c.vstride + ch * 16);
  const uint32_t na = c.norm[a];
  for (int base = 0; base < cnt; base += VPP) {
    const int k = base + grp;
    const uint32_t b = k < cnt ? slots[k] : a;
    const uint4 bv = *reinterpret_cast<const uint4*>(c.rows + (size_t)b * c.vstride + ch * 16);
    const uint32_t dot = group_sum<G>(dot16(av, bv, 0u));
    if (k < cnt && ch == 0 && b != a) {  // the diagonal's word belongs to another pair
      const uint32_t d = na + c.norm[b] - 2u * dot;
      c.M[tri(a, b)] = d;
    }
  }
  wave_sync();
}

// All of M at once, on the matrix cores: every pair of slots below S (S <= 64)
// from the staged rows (slots that hold no row give values never read). The
// bytes are shifted to signed values (an XOR with 0x80), which leaves every
// squared distance unchanged: d = |r'|^2 + |c'|^2 - 2 r'.c', exact in int32.
// The shifted squared norms come from the diagonal tiles first (into nrm,
// S words of scratch), then each tile pair (a <= b) of 16 x 16 slots fills
// M[r][c] and M[c][r].
__device__ inline v4i32 chain_frag(const ChainLds& c, uint32_t slot, uint32_t off, uint32_t dim) {
  v4i32 f = {0, 0, 0, 0};
  if (slot < c.S && off < dim) {
    const uint4 w = *reinterpret_cast<const uint4*>(c.rows + (size_t)slot * c.vstride + off);
    f = v4i32{(int)(w.x ^ 0x80808080u), (int)(w.y ^ 0x80808080u), (int)(w.z ^ 0x80808080u),
              (int)(w.w ^ 0x80808080u)};
  }
  return f;
}

__device__ inline v4i32 chain_tile(const ChainLds& c, uint32_t ta, uint32_t tb, uint32_t dim) {
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u;
  v4i32 acc = {0, 0, 0, 0};
  for (uint32_t k0 = 0; k0 < dim; k0 += 64)
    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(chain_frag(c, ta * 16u + r, k0 + kc, dim),
                                               chain_frag(c, tb * 16u + r, k0 + kc, dim), acc, 0, 0, 0);
  return acc;
}

__device__ inline void chain_fill_mfma(const Index& ix, const ChainLds& c, uint32_t* nrm) {
  const int l = lane_id();
  const uint32_t S = c.S, T = (S + 15u) / 16u, dim = ix.dim;
  const uint32_t r = (uint32_t)(l & 15), rb = (uint32_t)(l >> 4) * 4u;
  // lane l holds rows rb + i, column r of a tile: the diagonal is row == column
  for (uint32_t ta = 0; ta < T; ++ta) {
    const v4i32 acc = chain_tile(c, ta, ta, dim);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (rb + (uint32_t)i == r && ta * 16u + r < S) nrm[ta * 16u + r] = (uint32_t)acc[i];
  }
  wave_sync();
  for (uint32_t ta = 0; ta < T; ++ta)
    for (uint32_t tb = ta; tb < T; ++tb) {
      const v4i32 acc = chain_tile(c, ta, tb, dim);
      const uint32_t col = tb * 16u + r;
      if (col >= S) continue;
      const uint32_t nc = nrm[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t row = ta * 16u + rb + (uint32_t)i;
        if (row < S) {
          const uint32_t d = nrm[row] + nc - 2u * (uint32_t)acc[i];
          if (row != col) c.M[tri(row, col)] = d;
        }
      }
    }
  wave_sync();
}

// OR of a 64-bit word over the wave, in every lane
__device__ inline uint64_t wave_or64(uint64_t v) {
  v |= lane_xor<1>(v);
  v |= lane_xor<2>(v);
  v |= lane_xor<4>(v);
  v |= lane_xor<8>(v);
  v |= lane_xor<16>(v);
  v |= lane_xor<32>(v);
  return v;
}

// M entries of slot a (row fragment av in the G-lane layout, squared norm na)
// against slots[0..cnt), their rows read from memory
template <int G>
__device__ inline void chain_fill_row_g(const Index& ix, const ChainLds& c, uint32_t a, uint4 av, uint32_t na,
                                        const uint32_t* slots, int cnt) {
  constexpr int VPP = 64 / G;
  const int l = lane_id();
  const int ch = l % G, grp = l / G;
  for (int base = 0; base < cnt; base += 4 * VPP) {
    uint4 v[4];
    uint32_t sl[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = base + u * VPP + grp;
      sl[u] = k < cnt ? slots[k] : a;
      v[u] = make_uint4(0, 0, 0, 0);
      if (sl[u] != a) v[u] = reinterpret_cast<const uint4*>(ix.x + (size_t)c.id[sl[u]] * ix.dim)[ch];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t dot = group_sum<G>(dot16(av, v[u], 0u));
      const uint32_t nb = group_sum<G>(dot16(v[u], v[u], 0u));
      if (ch == 0 && sl[u] != a) c.M[tri(a, sl[u])] = na + nb - 2u * dot;  // the diagonal's word is another pair's
    }
  }
  wave_sync();
}

// A target's first prune with rows up to 128 bytes: slots 0..S-1 (the list,
// then the offer) are read once as matrix operands and every pair's distance
// is computed and stored once (tiles g <= h; shifted bytes, the diagonal
// tiles giving the norms); the flags of the list entries not known yet
// (`known`: slots of this launch's offers, all live) are read alongside.
template <int G>
__device__ inline void chain_first_mx(const Index& ix, const ChainLds& c, uint32_t S, uint64_t known) {
  constexpr uint32_t KS = (16u * G + 63u) / 64u;
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u, rb = (uint32_t)(l >> 4) * 4u;
  const bool need = (uint32_t)l < S && !((known >> l) & 1ull);
  const uint64_t ref = need ? load_ref(ix, c.id[l]) : 0ull;
  v4i32 f[3][KS];
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    const uint32_t sl = (uint32_t)h * 16u + r;
    const uint32_t id = sl < S ? c.id[sl] : NONE;
#pragma unroll
    for (uint32_t ks = 0; ks < KS; ++ks) f[h][ks] = mx_frag(ix, id, ks * 64u + kc);
  }
  uint32_t* nrm = c.out_d;  // S words of scratch
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    v4i32 acc = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[g][ks], acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (rb + (uint32_t)i == r && (uint32_t)g * 16u + r < S) nrm[g * 16 + (int)r] = (uint32_t)acc[i];
  }
  wave_sync();
#pragma unroll
  for (int g = 0; g < 3; ++g) {
#pragma unroll
    for (int h = g; h < 3; ++h) {
      if ((uint32_t)h * 16u >= S) break;
      v4i32 acc = {0, 0, 0, 0};
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[h][ks], acc, 0, 0, 0);
      const uint32_t col = (uint32_t)h * 16u + r;
      if (col >= S) continue;
      const uint32_t nc = nrm[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t row = (uint32_t)g * 16u + rb + (uint32_t)i;
        if (row < col) c.M[tri_lt(row, col)] = nrm[row] + nc - 2u * (uint32_t)acc[i];
      }
    }
  }
  if (need) c.dead[l] = ref_del(ref);
  wave_sync();
}

template <int G>
__device__ inline void reverse_chain_u8(const Index& ix, const MaintArgs& a, const ChainLds& c, uint32_t t,
                                        SlabCursor& cur) {
  // rows up to 128 bytes: distances from matrix operands and rows in memory,
  // no row staged in LDS
  constexpr bool MX = G <= 8;
  const int l = lane_id();
  const int ch = l % G;
  const uint32_t R = ix.R;
  const uint32_t w = (uint32_t)(a.pairs[t] >> 32);
  const uint4 wf = load_frag<G>(ix.x + (size_t)w * ix.dim);
  const uint32_t ww = group_sum<G>(dot16(wf, wf, 0u));
  // the target's list; slot i holds position i
  const uint64_t r = bcast64(load_ref(ix, w));
  uint32_t n = ref_slab(r) == NONE ? 0u : ref_deg(r);
  if ((uint32_t)l < n) {
    const uint32_t s = ref_slab(r);
    c.id[l] = ix.slabs[(size_t)s * 2u * R + (uint32_t)l];
    c.dw[l] = ix.slabs[(size_t)s * 2u * R + R + (uint32_t)l];
    c.order[l] = (uint32_t)l;
  }
  wave_sync();
  uint64_t used = (1ull << n) - 1ull;  // slots holding a list entry (n <= 32)
  uint64_t staged = 0;                 // slots whose row, norm and flag are in LDS
  bool cached = false;                 // M holds every pair of used slots
  const uint32_t cap = ix.prune_cap < 64u ? ix.prune_cap : 64u;
  for (uint32_t u = t; u < a.npairs && a.pairs[u] != KEY_NONE && (uint32_t)(a.pairs[u] >> 32) == w; ++u) {
    const uint32_t v = (uint32_t)a.pairs[u];
    if (ballot((uint32_t)l < n && c.id[c.order[l]] == v) != 0ull) continue;  // a set union
    // the offer takes a free slot: its row, norm, flag and distance to w
    const uint32_t f = (uint32_t)__builtin_ctzll(~used);
    const uint4 vv = reinterpret_cast<const uint4*>(ix.x + (size_t)v * ix.dim)[ch];
    const uint32_t vn = group_sum<G>(dot16(vv, vv, 0u));
    {
      const uint32_t dot = group_sum<G>(dot16(wf, vv, 0u));
      if (!MX && l < G) *reinterpret_cast<uint4*>(c.rows + (size_t)f * c.vstride + ch * 16) = vv;
      if (l == 0) {
        c.id[f] = v;
        c.dead[f] = 0u;  // the round's new nodes are live
        c.norm[f] = vn;
        c.dw[f] = ww + vn - 2u * dot;
      }
    }
    wave_sync();
    staged |= 1ull << f;
    const uint64_t kv = make_key(c.dw[f], v);
    const uint32_t sl = (uint32_t)l < n ? c.order[l] : 0u;
    const uint32_t pos = (uint32_t)__popcll(ballot((uint32_t)l < n && make_key(c.dw[sl], c.id[sl]) < kv));
    if (n < R) {
      // below R: insert in (distance, id) order
      wave_sync();
      if ((uint32_t)l < n && (uint32_t)l >= pos) c.order[l + 1] = sl;
      if (l == 0) c.order[pos] = f;
      wave_sync();
      if (cached) {  // M stays complete
        if constexpr (MX)
          chain_fill_row_g<G>(ix, c, f, vv, vn, c.order, (int)n + 1);
        else
          chain_fill_row<G>(c, f, c.order, (int)n + 1);
      }
      used |= 1ull << f;
      ++n;
      continue;
    }
    // at R: RobustPrune(w, list + v) over the cached state
    if (!cached) {
      if constexpr (MX) {
        // slots 0..n: the list entries and offers kept so far fill slots in
        // order until the first prune, and the offer takes slot n
        chain_first_mx<G>(ix, c, n + 1u, staged);
      } else {
        // first prune of this target: rows and flags of the list entries, then all of M
        const bool need = (uint32_t)l < n && !((staged >> sl) & 1ull);
        const uint64_t nm = ballot(need);
        if (need) {
          c.out_id[lanes_below(nm)] = sl;
          c.dead[sl] = ref_del(load_ref(ix, c.id[sl]));
        }
        wave_sync();
        chain_stage_rows<G>(ix, c, c.out_id, __popcll(nm));
        staged |= used;
        chain_fill_mfma(ix, c, c.out_d);  // every staged pair, v's row included
      }
      cached = true;
    } else {
      if constexpr (MX)
        chain_fill_row_g<G>(ix, c, f, vv, vn, c.order, (int)n);
      else
        chain_fill_row<G>(c, f, c.order, (int)n);
    }
    // candidates in (distance, id) order: the list with v at position pos
    uint32_t cs = f;
    if ((uint32_t)l < pos) cs = sl;
    else if ((uint32_t)l > pos && (uint32_t)l <= n) cs = c.order[l - 1];
    const bool is_cand = (uint32_t)l <= n;
    const uint32_t cdw = is_cand ? c.dw[cs] : 0u;
    uint64_t alive = ballot(is_cand && c.dead[cs] == 0u);
    {  // at most prune_cap candidates are considered, the first in order
      uint64_t rest = alive;
      for (uint32_t k = 0; k < cap && rest; ++k) rest &= rest - 1ull;
      alive &= ~rest;
    }
    // the selection in order, four live candidates per step (their distances
    // read together, then decided in order; one killed by an earlier one of
    // the four is skipped)
    uint32_t ns = 0;
    // the triangular table's entry for slots (sj, cs), the larger one's row:
    // computed per lane without a branch (the selection is bound by scalar issue)
    auto dist = [&](int j) {
      const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)cs, j);
      const uint32_t hi = max(sj, cs), lo = min(sj, cs);
      return c.M[__umul24(hi, hi - 1u) / 2u + lo];
    };
    auto keep = [&](int j, uint32_t rank, bool take) {
      const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)cs, j);
      if (take && (uint32_t)l == rank) ns = sj;
    };
    const uint32_t cnt = ix.cmp32 ? select_in_order<true>(alive, R, ix.a2, AlphaT<true>::scale(ix.b2, cdw), dist, keep)
                                  : select_in_order<false>(alive, R, ix.a2, AlphaT<false>::scale(ix.b2, cdw), dist, keep);
    // the kept candidates, in order, are the new list
    wave_sync();
    if ((uint32_t)l < cnt) c.order[l] = ns;
    used = wave_or64((uint32_t)l < cnt ? 1ull << ns : 0ull);
    n = cnt;
    wave_sync();
  }
  if ((uint32_t)l < n) {
    const uint32_t sl = c.order[l];
    c.out_id[l] = c.id[sl];
    c.out_d[l] = c.dw[sl];
  }
  wave_sync();
  publish(ix, w, c.out_id, c.out_d, n, C_PUB_REVERSE, &cur, r);  // only this wave writes w
}

// one wave per run of the sorted (target, source) pairs
template <class P>
__global__ void __launch_bounds__(256) k_reverse_apply(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t nseg = (uint32_t)ix.ctr[C_NSEG];
  // every target is a live node with a slab: one fresh slab and one retired slab each
  SlabCursor cur = reserve_slabs_block(ix, wave_items(nseg), wave_items(nseg));
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  FOR_EACH_WAVE_ITEM(si, nseg) {
    wave_sync();
    reverse_one<P>(ix, a, m, a.seg[si], cur);
  }
  finish_slabs_block(ix, cur, C_PUB_REVERSE);
}

// the same with the cached candidate state (uint8 rows, R <= 32): a kernel of
// its own so that its registers are not those of the generic path
// Reverse edges in the concurrent mode (Algorithm 2's loop as the paper runs
// it): the (target, source) offers are not sorted or grouped; each wave takes
// single offers and applies each to the target's list as it stands, with a
// compare-and-swap against the snapshot it read. Offers to one target from
// different waves race; a lost CAS rebuilds the list from a fresh snapshot
// and tries again, up to the attempt budget (then the offer is dropped and
// counted). The order in which a target's offers land is not fixed.
template <class P>
__global__ void __launch_bounds__(256) k_reverse_fast(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  const int l = lane_id();
  const uint32_t R = ix.R;
  uint64_t* ck = m.pr.keys;
  const uint32_t np = a.n * R;
  FOR_EACH_WAVE_ITEM(t, np) {
    const uint64_t key = a.pairs[t];
    if (key == KEY_NONE) continue;
    const uint32_t w = (uint32_t)(key >> 32), v = (uint32_t)key;
    bool done = false;
    for (uint32_t attempt = 0; attempt < ix.publish_attempts && !done; ++attempt) {
      const uint64_t snap = bcast64(load_ref(ix, w));
      const uint32_t s = ref_slab(snap);
      uint32_t n = s == NONE ? 0u : ref_deg(snap);
      if ((uint32_t)l < n) {
        m.nl_id[l] = __hip_atomic_load(ix.slabs + (size_t)s * 2u * R + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        m.nl_d[l] = __hip_atomic_load(ix.slabs + (size_t)s * 2u * R + R + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      wave_sync();
      if (ballot((uint32_t)l < n && m.nl_id[l] == v) != 0ull) {
        done = true;  // already listed: a set union changes nothing
        break;
      }
      if (n < R) {
        const uint32_t rho = P::dist1(ix, w, v, m.tmp, ck);
        const uint64_t kv = make_key(P::kd(rho), v);
        const bool before = (uint32_t)l < n && make_key(P::kd(m.nl_d[l]), m.nl_id[l]) < kv;
        const uint32_t pos = (uint32_t)__popcll(ballot(before));
        uint32_t id_l = 0, d_l = 0;
        if ((uint32_t)l < n) {
          id_l = m.nl_id[l];
          d_l = m.nl_d[l];
        }
        wave_sync();
        if ((uint32_t)l < n && (uint32_t)l >= pos) {
          m.nl_id[l + 1] = id_l;
          m.nl_d[l + 1] = d_l;
        }
        if (l == 0) {
          m.nl_id[pos] = v;
          m.nl_d[pos] = rho;
        }
        wave_sync();
        ++n;
      } else {
        if ((uint32_t)l < n) m.cand[l] = m.nl_id[l];
        if (l == 0) m.cand[n] = v;
        wave_sync();
        n = (uint32_t)P::prune(ix, w, m.cand, (int)n + 1, m.pr);
        copy_out(m, n);
      }
      done = publish_once(ix, w, snap, m.nl_id, m.nl_d, n, C_PUB_REVERSE);
    }
    if (!done && l == 0) atomicAdd(&ix.ctr[C_PUB_DROPPED], 1ull);
  }
}

template <int G>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_reverse_chain(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t nseg = (uint32_t)ix.ctr[C_NSEG];
  SlabCursor cur = reserve_slabs_block(ix, wave_items(nseg), wave_items(nseg));
  const ChainLds c = carve_chain(wave_lds(smem, a), ix.R, a.vstride);
  FOR_EACH_WAVE_ITEM(si, nseg) {
    wave_sync();
    reverse_chain_u8<G>(ix, a, c, a.seg[si], cur);
  }
  finish_slabs_block(ix, cur, C_PUB_REVERSE);
}

// ---- insert: refine -- same-batch nodes two hops away are offered ----------------------
template <class P>
__device__ inline void refine_one(const Index& ix, const MaintArgs& a, MaintLds& m, uint32_t qi) {
  const int l = lane_id();
  const uint32_t v = a.first + qi;
  const uint32_t end = a.first + a.n;
  const uint32_t own = load_list(ix, v, m.nl_id, m.nl_d);
  if ((uint32_t)l < own) m.cand[l] = m.nl_id[l];
  uint32_t nc = own;
  const uint32_t R = ix.R;
  if (2u * R <= 64u) {
    // every entry's reference word at once (lane j: entry j), then all their
    // slabs' ids, two entries per load (lanes [0, R): entry 2i, [R, 2R):
    // entry 2i + 1), before any is used; same-batch ids appended in entry order
    const uint64_t rj = (uint32_t)l < own ? load_ref(ix, m.nl_id[l]) : 0ull;
    const bool hi = (uint32_t)l >= R;
    const uint32_t slot = hi ? (uint32_t)l - R : (uint32_t)l;
    uint32_t b[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      b[i] = NONE;
      if (2u * (uint32_t)i >= own) continue;
      const uint64_t r0 = bcast_lane64(rj, 2 * i), r1 = bcast_lane64(rj, 2 * i + 1);
      const uint64_t r = hi ? r1 : r0;
      const uint32_t dw = 2u * (uint32_t)i + (hi ? 1u : 0u) < own ? ref_deg(r) : 0u, s = ref_slab(r);
      if ((uint32_t)l < 2u * R && slot < dw && s != NONE) b[i] = ix.slabs[(size_t)s * 2u * R + slot];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (2u * (uint32_t)i >= own) break;
      const bool extra = b[i] >= a.first && b[i] < end && b[i] != v;
      const uint64_t e0 = ballot(extra && !hi), e1 = ballot(extra && hi);
      if (extra && !hi) m.cand[nc + lanes_below(e0)] = b[i];
      nc += (uint32_t)__popcll(e0);
      if (extra && hi) m.cand[nc + lanes_below(e1)] = b[i];
      nc += (uint32_t)__popcll(e1);
    }
  } else {
    for (uint32_t j = 0; j < own; ++j) {
      const uint32_t w = m.nl_id[j];
      const uint64_t r = bcast64(load_ref(ix, w));
      const uint32_t dw = ref_deg(r), s = ref_slab(r);
      uint32_t b = NONE;
      if ((uint32_t)l < dw && s != NONE) b = ix.slabs[(size_t)s * 2u * R + (uint32_t)l];
      const bool extra = b >= a.first && b < end && b != v;
      const uint64_t bm = ballot(extra);
      if (extra) m.cand[nc + lanes_below(bm)] = b;
      nc += (uint32_t)__popcll(bm);
    }
  }
  wave_sync();
  uint32_t cnt = NONE;  // unchanged
  if (nc != own) {      // some same-batch node within two hops
    const int c = P::prune(ix, v, m.cand, (int)nc, m.pr);
    const bool diff = (uint32_t)c != own || ballot((uint32_t)l < own && m.pr.out_ids[l] != m.nl_id[l]) != 0ull;
    if (diff) {
      cnt = (uint32_t)c;
      if ((uint32_t)l < cnt) a.vis_keys[(size_t)qi * a.vcap + l] = make_key(m.pr.out_d[l], m.pr.out_ids[l]);
    }
  }
  if (l == 0) a.vis_cnt[qi] = cnt;
}

// Refine reads every list as it stands when the pass starts: the new lists
// are computed into the insert searches' scratch first (k_refine), then
// published (k_refine_publish).
template <class P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_refine(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  FOR_EACH_WAVE_ITEM(qi, a.n) {
    wave_sync();
    refine_one<P>(ix, a, m, qi);
  }
}

__global__ void __launch_bounds__(256) k_refine_publish(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  uint32_t* ids = reinterpret_cast<uint32_t*>(smem + (size_t)(threadIdx.x >> 6) * 512u);
  uint32_t* d = ids + 64;
  const int l = lane_id();
  const uint32_t w = wave_index(), W = total_waves();
  // the wave's changed lists (items w, w + W, ...) are counted first, so the
  // workgroup reserves their slabs with one atomic per stack
  uint32_t np = 0;
  for (uint32_t r0 = w; r0 < a.n; r0 += 64u * W) {
    const uint32_t my = r0 + (uint32_t)l * W;
    np += (uint32_t)__popcll(ballot(my < a.n && a.vis_cnt[my] != NONE));
  }
  SlabCursor cur = reserve_slabs_block(ix, np, np);
  for (uint32_t r0 = w; r0 < a.n; r0 += 64u * W) {
    for (uint32_t qi = r0; qi < a.n && qi < r0 + 64u * W; qi += W) {
      const uint32_t cnt = a.vis_cnt[qi];
      if (cnt == NONE) continue;
      wave_sync();
      if ((uint32_t)l < cnt) {
        const uint64_t k = a.vis_keys[(size_t)qi * a.vcap + l];
        ids[l] = key_id(k);
        d[l] = key_dist(k);
      }
      wave_sync();
      publish(ix, a.first + qi, ids, d, cnt, C_PUB_REFINE, &cur);
    }
  }
  finish_slabs_block(ix, cur, C_PUB_REFINE);
}

// ---- install given neighbor lists (import / test hook) -----------------------------------
// One wave per listed node: its neighbors' stored distances are computed from
// the rows, the list is ordered by (distance, id) and published.
template <class P>
__global__ void __launch_bounds__(256) k_set_lists(Index ix, MaintArgs a, const uint32_t* ids, const uint32_t* nbr,
                                                   const uint32_t* deg) {
  extern __shared__ __align__(16) char smem[];
  const uint32_t i = wave_index();
  if (i >= a.n) return;
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  const int l = lane_id();
  const uint32_t u = ids[i];
  const uint32_t d = min(deg[i], ix.R);
  uint64_t* keys = m.pr.keys;  // nsort >= 64
  for (uint32_t j = 0; j < d; ++j) {
    const uint32_t v = nbr[(size_t)i * ix.R + j];
    const uint32_t rho = P::dist1(ix, u, v, m.tmp, m.pr.keys2);
    if (l == 0) {
      keys[j] = make_key(P::kd(rho), v);
      m.nl_d[j] = rho;  // temporary: rho by input position
      m.nl_id[j] = v;
    }
  }
  for (int j = (int)d + l; j < 64; j += 64) keys[j] = KEY_NONE;
  wave_sync();
  // order by key; carry rho by looking its input position back up
  uint64_t myk = (uint32_t)l < d ? keys[l] : KEY_NONE;
  uint32_t myrho = (uint32_t)l < d ? m.nl_d[l] : 0u;
  wave_sync();
  uint32_t rank = 0;
  for (uint32_t j = 0; j < d; ++j) rank += keys[j] < myk;
  wave_sync();
  if ((uint32_t)l < d) {
    m.pr.out_ids[rank] = key_id(myk);
    m.pr.out_d[rank] = myrho;
  }
  wave_sync();
  publish(ix, u, m.pr.out_ids, m.pr.out_d, d, C_PUB_FORWARD);
}

// ---- delete: classify, tombstone, repair (Algorithm 3) ----------------------------------
__global__ void k_del_keys(Index ix, const uint32_t* ids, uint32_t n, Dyn d, uint64_t* keys) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) keys[t] = pair_key(ids[t], t);
}

// ids at or above the id count at the round's start are out of range
__global__ void k_del_classify(Index ix, const uint64_t* sorted, uint32_t n, Dyn d, uint8_t* status,
                               uint32_t* dlist) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  const uint64_t next_id = ix.ctr[C_NEXT_ID];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint8_t st = DEL_DUPLICATE;
  uint32_t id = 0;
  if (t < n) {
    const uint64_t k = sorted[t];
    id = (uint32_t)(k >> 32);
    const uint32_t pos = (uint32_t)k;
    const bool first = t == 0 || (uint32_t)(sorted[t - 1] >> 32) != id;
    if (!first)
      st = DEL_DUPLICATE;
    else if ((uint64_t)id >= next_id)
      st = DEL_OUT_OF_RANGE;
    else if (ref_del(load_ref(ix, id)))
      st = DEL_NOT_LIVE;
    else
      st = DEL_OK;
    if (status) status[pos] = st;
  }
  // dlist keeps the sorted order: position t holds the id when it is
  // accepted and NONE otherwise, so the deleted ids appear in ascending order
  // (pairs generated from them come out in source order); the accepted count,
  // one atomic per wave
  const bool ok = t < n && st == DEL_OK;
  if (t < n) dlist[t] = ok ? id : NONE;
  const uint64_t m = ballot(ok);
  if (m) wave_atomic_add(&ix.ctr[C_DEL_OK], (unsigned long long)__popcll(m));
}

// <0,d,s> -> <1,d,s>: the flag is set, degree and slab are kept
__global__ void k_tombstone(Index ix, const uint32_t* dlist, uint32_t n, Dyn d) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  bool done = false;
  const uint32_t u = t < n ? dlist[t] : NONE;
  if (u != NONE) {
    uint64_t r = load_ref(ix, u);
    for (int attempt = 0; attempt < 1024 && !ref_del(r); ++attempt) {
      const uint64_t prev = atomicCAS(&ix.refs[u], (unsigned long long)r, (unsigned long long)(r | (1ull << 63)));
      if (prev == r) {
        done = true;
        break;
      }
      r = prev;
    }
  }
  const uint64_t m = ballot(done);  // one count per wave
  if (m) wave_atomic_add(&ix.ctr[C_TOMBSTONED], (unsigned long long)__popcll(m));
}

__global__ void k_repair_pairs(Index ix, MaintArgs a) {
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t i = wave_index();
  if (i == 0 && lane_id() == 0) ix.ctr[C_NSEG] = 0;
  if (i >= a.n) return;
  const int l = lane_id();
  const uint32_t u = a.dlist[i];  // NONE where the delete was not accepted
  const uint64_t r = u != NONE ? bcast64(load_ref(ix, u)) : 0ull;
  const uint32_t deg = u != NONE ? ref_deg(r) : 0u, s = ref_slab(r);
  if ((uint32_t)l >= ix.R) return;
  uint64_t key = KEY_NONE;
  if ((uint32_t)l < deg && s != NONE) {
    const uint32_t an = ix.slabs[(size_t)s * 2u * ix.R + (uint32_t)l];
    if (!ref_del(load_ref(ix, an))) key = pair_key(an, u);
  }
  a.pairs[(size_t)i * ix.R + (uint32_t)l] = key;
}

template <class P>
__device__ inline void repair_one(const Index& ix, const MaintArgs& a, MaintLds& m, uint32_t t, SlabCursor& cur) {
  const uint32_t an = (uint32_t)(a.pairs[t] >> 32);
  const int l = lane_id();
  const uint32_t R = ix.R;
  uint32_t n = load_list(ix, an, m.nl_id, m.nl_d);
  for (uint32_t q = t; q < a.npairs && a.pairs[q] != KEY_NONE && (uint32_t)(a.pairs[q] >> 32) == an; ++q) {
    const uint32_t u = (uint32_t)a.pairs[q];
    // K = RobustPrune(a, N(u) \ {a})
    const uint64_t r = bcast64(load_ref(ix, u));
    const uint32_t du = ref_deg(r), s = ref_slab(r);
    uint32_t b = NONE;
    if ((uint32_t)l < du && s != NONE) b = ix.slabs[(size_t)s * 2u * R + (uint32_t)l];
    const bool ok = b != NONE && b != an;
    const uint64_t bm = ballot(ok);
    if (ok) m.cand[lanes_below(bm)] = b;
    wave_sync();
    const int kc = P::prune(ix, an, m.cand, __popcll(bm), m.pr);
    // N = RobustPrune(a, (N(a) \ {u}) U K)
    const bool keep = (uint32_t)l < n && m.nl_id[l] != u;
    const uint64_t km = ballot(keep);
    const uint32_t nk = (uint32_t)__popcll(km);
    uint32_t kid = (l < kc) ? m.pr.out_ids[l] : NONE;
    wave_sync();
    if (keep) m.cand[lanes_below(km)] = m.nl_id[l];
    if (l < kc) m.cand[nk + (uint32_t)l] = kid;
    wave_sync();
    n = (uint32_t)P::prune(ix, an, m.cand, (int)(nk + (uint32_t)kc), m.pr);
    copy_out(m, n);
  }
  publish(ix, an, m.nl_id, m.nl_d, n, C_PUB_REPAIR, &cur);
}


// ---- repair with a wave-local candidate pool (uint8 rows, R <= 32) ------------------
// Algorithm 3 for one target a: for each deleted u in ascending order,
// K = RobustPrune(a, N(u) \ {a}), then N(a) = RobustPrune(a, (N(a) \ {u}) U K).
// A pool of 64 slots holds the ids, distances to a and deletion flags of a's
// list and of one N(u), and the squared distances between every two occupied
// slots (a triangular cache). a's list is staged once; per u only the members
// of N(u) that are not already pooled are fetched, and their distances to the
// occupied slots are filled on the matrix cores. Both prunes then run from
// LDS: candidates are ranked by (distance, id) with duplicates, a and
// tombstones dropped, at most prune_cap are considered, and every distance
// between a kept candidate and a later one is one cache read.
struct PoolLds {
  uint32_t* M;       // [64 * 63 / 2 + 1] squared distances, tri(x, y) = max(x,y)(max-1)/2 + min(x,y)
  uint32_t* norm;    // [64] squared norm of the row shifted to signed bytes
  uint32_t* id;      // [64]
  uint32_t* dw;      // [64] squared distance to the target (< 2^27), bit 31: deletion flag
  uint32_t* list;    // [64] list position -> slot
  uint32_t* cand;    // [64] candidate slots of a prune
  uint32_t* sorted;  // [64] candidate slots in (distance, id) order
  uint32_t* kept;    // [64] output slots of a prune
};

constexpr uint32_t POOL = 64;

// the distances of distinct slots (the diagonal is never read for a decision;
// its index, at most one past the last pair, stays inside the array), sized
// so that 16 waves fit a CU's LDS
constexpr uint32_t POOL_M = POOL * (POOL - 1u) / 2u + 1u;

__host__ __device__ inline uint32_t pool_lds_bytes(uint32_t) {
  return ((POOL_M * 4u + 7u * POOL * 4u) + 15u) & ~15u;
}
constexpr uint32_t DW_DEAD = 0x80000000u;

__device__ inline PoolLds carve_pool(char* base, uint32_t) {
  PoolLds p;
  p.M = reinterpret_cast<uint32_t*>(base);
  uint32_t* q = p.M + ((POOL_M + 3u) & ~3u);
  p.norm = q;
  p.id = q + POOL;
  p.dw = q + 2 * POOL;
  p.list = q + 3 * POOL;
  p.cand = q + 4 * POOL;
  p.sorted = q + 5 * POOL;
  p.kept = q + 6 * POOL;
  return p;
}


// shifted squared norms, deletion flags and distances to the target (fragment
// wf, norm ww) of slots[0..cnt), all loads issued before any is used
template <int G>
__device__ inline void pool_stage(const Index& ix, const PoolLds& p, const uint32_t* slots, int cnt, uint4 wf,
                                  uint32_t ww) {
  constexpr int VPP = 64 / G;
  // rows per lane in flight together
  constexpr int U = G < 4 ? G : 4;
  const int l = lane_id();
  const int ch = l % G, grp = l / G;
  const uint4 ones = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
  uint64_t ref = 0;
  const uint32_t my = l < cnt ? slots[l] : 0u;
  if (l < cnt) ref = load_ref(ix, p.id[my]);
  for (int base = 0; base < cnt; base += U * VPP) {
    uint4 v[U];
    int sl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * VPP + grp;
      sl[u] = k < cnt ? (int)slots[k] : -1;
      v[u] = make_uint4(0, 0, 0, 0);
      if (sl[u] >= 0) v[u] = reinterpret_cast<const uint4*>(ix.x + (size_t)p.id[sl[u]] * ix.dim)[ch];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t nn = group_sum<G>(dot16(v[u], v[u], 0u));
      const uint32_t sm = group_sum<G>(dot16(v[u], ones, 0u));
      const uint32_t dt = group_sum<G>(dot16(wf, v[u], 0u));
      if (sl[u] >= 0 && ch == 0) {
        // |x - 128|^2 = |x|^2 - 256 sum(x) + 128^2 dim
        p.norm[sl[u]] = nn - 256u * sm + 16384u * ix.dim;
        p.dw[sl[u]] = ww + nn - 2u * dt;
      }
    }
  }
  wave_sync();
  if (l < cnt && ref_del(ref)) p.dw[my] |= DW_DEAD;
  wave_sync();
}

// The cache entries between the nf slots fresh[0..nf) and every slot of the
// mask occ (fresh ones included), on the matrix cores: 16 fresh rows x 16
// slots per v_mfma_i32_16x16x64_i8 tile over the rows shifted to signed bytes
// (exact in int32), the rows read from memory. Needs the shifted norms.
__device__ inline v4i32 pool_frag(const Index& ix, const PoolLds& p, uint32_t slot, bool valid, uint32_t off) {
  v4i32 f = {0, 0, 0, 0};
  if (valid && off < ix.dim) {
    const uint4 w = *reinterpret_cast<const uint4*>(ix.x + (size_t)p.id[slot] * ix.dim + off);
    f = v4i32{(int)(w.x ^ 0x80808080u), (int)(w.y ^ 0x80808080u), (int)(w.z ^ 0x80808080u),
              (int)(w.w ^ 0x80808080u)};
  }
  return f;
}

// lane l holds fresh rows f0 + 4 (l / 16) + i against slot 16 st + l % 16
__device__ inline void pool_store(const PoolLds& p, const uint32_t* fresh, uint32_t nf, uint64_t occ, uint32_t f0,
                                  const v4i32 (&acc)[4]) {
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), rb = (uint32_t)(l >> 4) * 4u;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const uint32_t sb = (uint32_t)st * 16u + r;
    if (!((occ >> sb) & 1ull)) continue;
    const uint32_t nb = p.norm[sb];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t fi = f0 + rb + (uint32_t)i;
      if (fi < nf) {
        const uint32_t fs = fresh[fi];
        if (fs != sb) p.M[tri(fs, sb)] = p.norm[fs] + nb - 2u * (uint32_t)acc[st][i];
      }
    }
  }
}

template <int G>
__device__ inline void pool_fill(const Index& ix, const PoolLds& p, const uint32_t* fresh, uint32_t nf, uint64_t occ) {
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u;
  constexpr uint32_t KS = (16u * G + 63u) / 64u;  // 64-byte steps of a row
  if constexpr (KS <= 2) {
    // rows up to 128 bytes: the slot operands are the same for every block of
    // 16 fresh rows, so they are read once, all at once, and each block's
    // fresh operands are read while the previous block's results are stored
    v4i32 sf[4][KS], ff[KS];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const uint32_t sb = (uint32_t)st * 16u + r;
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) sf[st][ks] = pool_frag(ix, p, sb, (occ >> sb) & 1ull, ks * 64u + kc);
    }
    {
      const uint32_t fa = r < nf ? fresh[r] : 0u;
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) ff[ks] = pool_frag(ix, p, fa, r < nf, ks * 64u + kc);
    }
    for (uint32_t f0 = 0; f0 < nf; f0 += 16) {
      v4i32 acc[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        acc[st] = v4i32{0, 0, 0, 0};
#pragma unroll
        for (uint32_t ks = 0; ks < KS; ++ks)
          acc[st] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ff[ks], sf[st][ks], acc[st], 0, 0, 0);
      }
      if (f0 + 16u < nf) {  // the next block's operands travel while this block's results are stored
        const uint32_t nx = f0 + 16u + r;
        const uint32_t fa = nx < nf ? fresh[nx] : 0u;
#pragma unroll
        for (uint32_t ks = 0; ks < KS; ++ks) ff[ks] = pool_frag(ix, p, fa, nx < nf, ks * 64u + kc);
      }
      pool_store(p, fresh, nf, occ, f0, acc);
    }
  } else {
    for (uint32_t f0 = 0; f0 < nf; f0 += 16) {
      const uint32_t fa = f0 + r < nf ? fresh[f0 + r] : 0u;
      v4i32 acc[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) acc[st] = v4i32{0, 0, 0, 0};
      for (uint32_t k0 = 0; k0 < ix.dim; k0 += 64) {
        const v4i32 fa_frag = pool_frag(ix, p, fa, f0 + r < nf, k0 + kc);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const uint32_t sb = (uint32_t)st * 16u + r;
          acc[st] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa_frag, pool_frag(ix, p, sb, (occ >> sb) & 1ull, k0 + kc),
                                                          acc[st], 0, 0, 0);
        }
      }
      pool_store(p, fresh, nf, occ, f0, acc);
    }
  }
  wave_sync();
}

// The first (target, deleted neighbor) pair of a chain fills the whole pool
// at once: slots 0..n-1 hold the target's list (lane x: entry x, whose stored
// distance to the target is rho), slots n..nf-1 the new members of B. All
// slots' rows are read once as matrix operands (with the target's row), and
// the matrix cores give every slot's shifted norm (diagonal tiles), its
// distance to the target where no stored one exists (target row x slot
// tiles), and each pair's distance once (tiles g <= h), for the same table
// the general fill writes.
template <int G>
__device__ inline void pool_first(const Index& ix, const PoolLds& p, uint32_t n, uint32_t nf, uint32_t an,
                                  uint32_t rho) {
  constexpr uint32_t KS = (16u * G + 63u) / 64u;
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u, rb = (uint32_t)(l >> 4) * 4u;
  const uint64_t ref = (uint32_t)l < nf ? load_ref(ix, p.id[l]) : 0ull;
  v4i32 f[4][KS], fa[KS];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint32_t sl = (uint32_t)h * 16u + r;
    const uint32_t id = sl < nf ? p.id[sl] : NONE;
#pragma unroll
    for (uint32_t ks = 0; ks < KS; ++ks) f[h][ks] = mx_frag(ix, id, ks * 64u + kc);
  }
#pragma unroll
  for (uint32_t ks = 0; ks < KS; ++ks) fa[ks] = mx_frag(ix, an, ks * 64u + kc);
  // shifted norms of the slots and of the target
  v4i32 aa = {0, 0, 0, 0};
#pragma unroll
  for (uint32_t ks = 0; ks < KS; ++ks) aa = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[ks], fa[ks], aa, 0, 0, 0);
  const uint32_t na = (uint32_t)aa[0];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    v4i32 acc = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[g][ks], acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (rb + (uint32_t)i == r) p.norm[g * 16 + (int)r] = (uint32_t)acc[i];
  }
  wave_sync();
  // distances to the target: stored for the list, from the tiles for the rest
  // (every row of the target's tile is the target: lanes 0..15 hold column r)
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    v4i32 acc = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[ks], f[h][ks], acc, 0, 0, 0);
    const uint32_t sl = (uint32_t)h * 16u + r;
    if (l < 16 && sl >= n && sl < nf) p.dw[sl] = na + p.norm[sl] - 2u * (uint32_t)acc[0];
  }
  if ((uint32_t)l < n) p.dw[l] = rho;
  // every pair once
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const uint4 nr = *reinterpret_cast<const uint4*>(p.norm + g * 16 + (int)rb);
    const uint32_t nrow[4] = {nr.x, nr.y, nr.z, nr.w};
#pragma unroll
    for (int h = g; h < 4; ++h) {
      if ((uint32_t)h * 16u >= nf) break;
      v4i32 acc = {0, 0, 0, 0};
#pragma unroll
      for (uint32_t ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(f[g][ks], f[h][ks], acc, 0, 0, 0);
      const uint32_t col = (uint32_t)h * 16u + r;
      if (col >= nf) continue;
      const uint32_t nc = p.norm[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t row = (uint32_t)g * 16u + rb + (uint32_t)i;
        if (row < col) p.M[tri_lt(row, col)] = nrow[i] + nc - 2u * (uint32_t)acc[i];
      }
    }
  }
  wave_sync();
  if ((uint32_t)l < nf && ref_del(ref)) p.dw[l] |= DW_DEAD;
  wave_sync();
}

// 64-lane bitonic sort of (key, value) pairs held one per lane, ascending
template <int K, int J>
__device__ inline void lane_bitonic_step(uint64_t& key, uint32_t& val) {
  const int l = lane_id();
  const uint64_t ok = lane_xor<J>(key);
  const uint32_t ov = lane_xor<J>(val);
  const bool up = (l & K) == 0, lower = (l & J) == 0;
  const bool take = lower == up ? ok < key : ok > key;
  if (take) {
    key = ok;
    val = ov;
  }
  if constexpr (J > 1) lane_bitonic_step<K, J / 2>(key, val);
}

template <int K>
__device__ inline void lane_bitonic_stage(uint64_t& key, uint32_t& val) {
  lane_bitonic_step<K, K / 2>(key, val);
  if constexpr (K < 64) lane_bitonic_stage<K * 2>(key, val);
}

__device__ inline void lane_bitonic_sort(uint64_t& key, uint32_t& val) { lane_bitonic_stage<2>(key, val); }

// stages 2 .. KMAX only: each run of KMAX lanes sorted (the first ascending)
template <int K, int KMAX>
__device__ inline void lane_bitonic_stages(uint64_t& key, uint32_t& val) {
  lane_bitonic_step<K, K / 2>(key, val);
  if constexpr (K < KMAX) lane_bitonic_stages<K * 2, KMAX>(key, val);
}

// How pool_prune ranks its candidates: any order (a full sort), at most 32
// candidates (a sort of 32 lanes), or two runs each already in (distance, id)
// order (one bitonic merge: the first run ascending from lane 0, the second
// descending into the top lanes).
enum PoolRank { RANK_SORT = 0, RANK_SORT32 = 1, RANK_MERGE = 2 };
constexpr uint32_t DROP = 0x80000000u;  // a ranked slot that takes no part (itself or flagged)

// RobustPrune(self, candidate slots cs[0..m)) into out[0..return); m <= 64;
// with RANK_MERGE, cs[0..m1) and cs[m1..m) are the two ordered runs.
// Candidates are ranked in registers (one per lane); during the selection each
// lane reads the distance from the kept candidate to its own from the cache.
template <int MODE>
__device__ inline uint32_t pool_prune(const Index& ix, const PoolLds& p, const uint32_t* cs, uint32_t m, uint32_t m1,
                                      uint32_t self, uint32_t* out) {
  const int l = lane_id();
  uint32_t slot = 0;
  uint64_t key = KEY_NONE;
  if constexpr (MODE == RANK_MERGE) {
    // the runs keep their order whatever is dropped: a dropped candidate keeps
    // its key for the merge and carries DROP in its slot word
    const int src = (uint32_t)l < m1 ? l : (int)m1 + (63 - l);
    if ((uint32_t)l < m1 || (l >= 64 - (int)(m - m1) && src < (int)m)) {
      slot = cs[src];
      const uint32_t id = p.id[slot];
      const uint32_t w = p.dw[slot];
      key = make_key(w & ~DW_DEAD, id);
      if (id == self || (w & DW_DEAD)) slot |= DROP;
    }
    lane_bitonic_stages<64, 64>(key, slot);
  } else {
    if ((uint32_t)l < m) {
      slot = cs[l];
      const uint32_t id = p.id[slot];
      const uint32_t w = p.dw[slot];
      if (id != self && !(w & DW_DEAD)) key = make_key(w, id);
    }
    if constexpr (MODE == RANK_SORT32)
      lane_bitonic_stages<2, 32>(key, slot);
    else
      lane_bitonic_sort(key, slot);
  }
  // repeated ids are adjacent with equal keys: one copy stays
  const uint64_t prev_lo = (uint32_t)__shfl_up((int)(uint32_t)key, 1, 64);
  const uint64_t prev_hi = (uint32_t)__shfl_up((int)(uint32_t)(key >> 32), 1, 64);
  const bool keep = key != KEY_NONE && !(slot & DROP) && (l == 0 || ((prev_hi << 32) | prev_lo) != key);
  // the candidates stay in their ranked lanes (the lanes of the others are
  // skipped); at most prune_cap of them, the first in rank order
  uint64_t alive = ballot(keep);
  const uint32_t cap = ix.prune_cap < POOL ? ix.prune_cap : POOL;
  if ((uint32_t)__popcll(alive) > cap) {
    uint64_t rest = alive;
    for (uint32_t k = 0; k < cap; ++k) rest &= rest - 1ull;
    alive &= ~rest;
  }
  const uint32_t csl = slot & ~DROP;
  const uint32_t cdw = keep ? key_dist(key) : 0u;
  uint32_t keep_slot = 0;
  // the selection in order of rank over the cached distances (the slot of
  // the k-th kept candidate lands in lane k)
  // the triangular table's entry for slots (sj, csl), the larger one's row:
  // computed per lane without a branch (the selection is bound by scalar issue)
  auto dist = [&](int j) {
    const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)csl, j);
    const uint32_t hi = max(sj, csl), lo = min(sj, csl);
    return p.M[__umul24(hi, hi - 1u) / 2u + lo];
  };
  auto take = [&](int j, uint32_t rank, bool kept) {
    const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)csl, j);
    if (kept && (uint32_t)l == rank) keep_slot = sj;
  };
  const uint32_t cnt = ix.cmp32 ? select_in_order<true>(alive, ix.R, ix.a2, AlphaT<true>::scale(ix.b2, cdw), dist, take)
                                : select_in_order<false>(alive, ix.R, ix.a2, AlphaT<false>::scale(ix.b2, cdw), dist, take);
  wave_sync();
  if ((uint32_t)l < cnt) out[l] = keep_slot;
  wave_sync();
  return cnt;
}

// The words a repair target starts from, read for a batch of targets at once
// (lane k: the batch's k-th target): its first pair (a, u), the pair after
// it, and the reference words of a and u.
struct RepairHead {
  uint64_t pair, next;
  uint64_t ra, ru;
};

__device__ inline RepairHead repair_heads(const Index& ix, const MaintArgs& a, uint32_t b0, uint32_t nb) {
  const uint32_t l = (uint32_t)lane_id();
  RepairHead h{KEY_NONE, KEY_NONE, 0, 0};
  if (l < nb) {
    const uint32_t t = a.seg[b0 + l];
    h.pair = a.pairs[t];
    h.next = t + 1 < a.npairs ? a.pairs[t + 1] : KEY_NONE;
    h.ra = load_ref(ix, (uint32_t)(h.pair >> 32));
    h.ru = load_ref(ix, (uint32_t)h.pair);
  }
  return h;
}

// lane k < nb: the batch's k-th segment start
__device__ inline uint32_t l_seg(const MaintArgs& a, uint32_t b0, uint32_t nb) {
  const uint32_t l = (uint32_t)lane_id();
  return l < nb ? a.seg[b0 + l] : 0u;
}

template <int G>
__device__ inline void repair_chain_u8(const Index& ix, const MaintArgs& a, const PoolLds& p, uint32_t t,
                                       const RepairHead& hd, int k, SlabCursor& cur) {
  const int l = lane_id();
  const uint32_t R = ix.R;
  const uint64_t pair0 = bcast_lane64(hd.pair, k);
  const uint32_t an = (uint32_t)(pair0 >> 32);
  const uint4 wf = load_frag<G>(ix.x + (size_t)an * ix.dim);
  const uint32_t ww = group_sum<G>(dot16(wf, wf, 0u));
  // a's list and the first N(u), read side by side; the list lives in slots
  // 0..n-1 and in registers (lane x: slot and id of list entry x)
  uint32_t u = (uint32_t)pair0;
  const uint64_t ra = bcast_lane64(hd.ra, k);
  uint64_t ru = bcast_lane64(hd.ru, k);
  const uint64_t pair1 = bcast_lane64(hd.next, k);
  uint32_t n = ref_slab(ra) == NONE ? 0u : ref_deg(ra);
  uint32_t du = ref_slab(ru) == NONE ? 0u : ref_deg(ru);
  uint32_t lid = NONE, b = NONE, rho = 0;
  if ((uint32_t)l < n) {
    lid = ix.slabs[(size_t)ref_slab(ra) * 2u * R + (uint32_t)l];
    rho = ix.slabs[(size_t)ref_slab(ra) * 2u * R + R + (uint32_t)l];
  }
  if ((uint32_t)l < du) b = ix.slabs[(size_t)ref_slab(ru) * 2u * R + (uint32_t)l];
  uint32_t lslot = (uint32_t)l;
  if ((uint32_t)l < n) {
    p.id[l] = lid;
    p.list[l] = (uint32_t)l;
  }
  uint64_t used = n == 64 ? ~0ull : ((1ull << n) - 1ull);
  bool first = true;
  for (uint32_t q = t; q < a.npairs; ++q) {
    if (!first) {
      const uint64_t pq = q == t + 1 ? pair1 : a.pairs[q];
      if (pq == KEY_NONE || (uint32_t)(pq >> 32) != an) break;
      u = (uint32_t)pq;
      ru = bcast64(load_ref(ix, u));
      du = ref_slab(ru) == NONE ? 0u : ref_deg(ru);
      b = NONE;
      if ((uint32_t)l < du) b = ix.slabs[(size_t)ref_slab(ru) * 2u * R + (uint32_t)l];
    }
    // B = N(u) \ {a}: members on the list keep their slot, the others take free slots
    const bool ok = b != NONE && b != an;
    int at = -1;
    for (uint32_t x = 0; x < n; ++x)
      if ((uint32_t)__builtin_amdgcn_readlane((int)lid, (int)x) == b)
        at = __builtin_amdgcn_readlane((int)lslot, (int)x);
    if (!ok) at = -1;
    const bool fresh = ok && at < 0;
    const uint64_t fm = ballot(fresh);
    // the k-th fresh member takes the k-th free slot (for the first pair the
    // free slots are n, n + 1, ...)
    if (first) {
      if (fresh) at = (int)(n + lanes_below(fm));
    } else {
      uint64_t fr = ~used;
      for (uint64_t m2 = fm; m2; m2 &= m2 - 1ull) {
        if (l == (int)__builtin_ctzll(m2)) at = (int)__builtin_ctzll(fr);
        fr &= fr - 1ull;
      }
    }
    if (fresh) p.id[at] = b;
    const uint64_t om = ballot(ok);
    if (ok) p.cand[lanes_below(om)] = (uint32_t)at;
    // slots to stage: the fresh members (and, for the first u, a's list)
    uint32_t* fs = p.kept;
    const uint32_t nl = first ? n : 0u;
    if ((uint32_t)l < nl) fs[l] = (uint32_t)l;
    if (fresh) fs[nl + lanes_below(fm)] = (uint32_t)at;
    wave_sync();
    const uint32_t nf = nl + (uint32_t)__popcll(fm);
    uint64_t occ = used;
    if (first)
      occ = nf == 64 ? ~0ull : ((1ull << nf) - 1ull);
    else
      for (uint64_t m2 = fm; m2; m2 &= m2 - 1ull)
        occ |= 1ull << (uint32_t)__builtin_amdgcn_readlane(at, (int)__builtin_ctzll(m2));
    bool filled = false;
    if constexpr (G <= 8) {  // rows up to 128 bytes: operands in registers
      if (first) {  // slots 0..nf-1 in order: the list, then B's new members
        pool_first<G>(ix, p, n, nf, an, rho);
        filled = true;
      }
    }
    if (!filled && nf) {
      pool_stage<G>(ix, p, fs, (int)nf, wf, ww);
      pool_fill<G>(ix, p, fs, nf, occ);
    }
    first = false;
    // K = RobustPrune(a, B): at most R <= 32 candidates
    const uint32_t kc = pool_prune<RANK_SORT32>(ix, p, p.cand, (uint32_t)__popcll(om), 0u, an, p.kept);
    // N = RobustPrune(a, (N \ {u}) U K)
    const uint32_t ks = (uint32_t)l < kc ? p.kept[l] : 0u;
    const bool stay = (uint32_t)l < n && lid != u;
    const uint64_t sm = ballot(stay);
    const uint32_t ns = (uint32_t)__popcll(sm);
    wave_sync();
    if (stay) p.cand[lanes_below(sm)] = lslot;
    if ((uint32_t)l < kc) p.cand[ns + (uint32_t)l] = ks;
    wave_sync();
    // the list (without u) and K are each in (distance, id) order already
    n = pool_prune<RANK_MERGE>(ix, p, p.cand, ns + kc, ns, an, p.list);
    lslot = (uint32_t)l < n ? p.list[l] : 0u;
    lid = (uint32_t)l < n ? p.id[lslot] : NONE;
    // slots not on the new list become free
    used = wave_or64((uint32_t)l < n ? 1ull << lslot : 0ull);
  }
  // publish (ids and distances in list order)
  const uint32_t od = (uint32_t)l < n ? p.dw[lslot] : 0u;
  wave_sync();
  if ((uint32_t)l < n) {
    p.cand[l] = lid;
    p.sorted[l] = od;
  }
  wave_sync();
  publish(ix, an, p.cand, p.sorted, n, C_PUB_REPAIR, &cur, ra);  // only this wave writes a
}

template <class P>
__global__ void __launch_bounds__(256) k_repair_apply(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t nseg = (uint32_t)ix.ctr[C_NSEG];
  SlabCursor cur = reserve_slabs_block(ix, wave_items(nseg), wave_items(nseg));
  MaintLds m = carve(wave_lds(smem, a), a, ix.R);
  FOR_EACH_WAVE_ITEM(si, nseg) {
    wave_sync();
    repair_one<P>(ix, a, m, a.seg[si], cur);
  }
  finish_slabs_block(ix, cur, C_PUB_REPAIR);
}

// the same with the wave-local candidate pool (uint8 rows, R <= 32), a kernel
// of its own. Targets differ in cost (one to a dozen deleted out-neighbors),
// so waves take them from queues in batches of four. Every target publishes
// once, so the launch's slabs (one fresh and one retired slot per target) are
// reserved beforehand by one thread (k_reserve_launch) and batch b takes the
// b-th four of each: no per-batch atomics. The batches are split over N_RQ
// queues on lines of their own, a workgroup starting at its own queue and
// moving on when it is empty, and the publication count is summed per
// workgroup: same-address atomics from thousands of waves serialize.
__global__ void k_reserve_launch(Index ix, Dyn d) {
  if (gated(ix, d)) return;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t n = ix.ctr[C_NSEG];
  unsigned long long f = ~0ull, r = ~0ull;
  if (n) {
    const unsigned long long top = atomicAdd(&ix.ctr[C_FREE_TOP], (unsigned long long)(-(long long)n));
    if (top >= n && top <= ix.P)
      f = top;
    else
      atomicAdd(&ix.ctr[C_FREE_TOP], (unsigned long long)n);  // a shortage: each publication allocates alone
    const unsigned long long at = atomicAdd(&ix.ctr[C_RETIRED_TOP], (unsigned long long)n);
    if (at + n <= ix.P)
      r = at;
    else
      atomicAdd(&ix.ctr[C_RETIRED_TOP], (unsigned long long)(-(long long)n));
  }
  ix.ctr[C_RES_FREE] = f;
  ix.ctr[C_RES_RET] = r;
}

template <int G>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_repair_pool(Index ix, MaintArgs a) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, a.d)) return;
  resolve(ix, a);
  const uint32_t nseg = (uint32_t)ix.ctr[C_NSEG];
  const uint64_t fbase = ix.ctr[C_RES_FREE], rbase = ix.ctr[C_RES_RET];
  constexpr uint32_t BATCH = 4;
  const uint32_t nbat = (nseg + BATCH - 1) / BATCH;
  const PoolLds p = carve_pool(wave_lds(smem, a), a.vstride);
  uint32_t pubs = 0;
  for (uint32_t qq = 0; qq < N_RQ; ++qq) {
    const uint32_t q = (blockIdx.x + qq) % N_RQ;
    unsigned long long* queue = &ix.ctr[rq_word(q)];
    const uint32_t lo = (uint32_t)((uint64_t)nbat * q / N_RQ), hi = (uint32_t)((uint64_t)nbat * (q + 1) / N_RQ);
    // an empty queue is passed over with a plain read
    if (lo + (uint32_t)__hip_atomic_load(queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= hi) continue;
    for (;;) {
      const uint32_t bi = lo + (uint32_t)wave_atomic_add(queue, 1ull);
      if (bi >= hi) break;
      const uint32_t b0 = bi * BATCH;
      const uint32_t nb = min(BATCH, nseg - b0);
      SlabCursor cur;
      if (fbase != ~0ull) {
        cur.free_hi = fbase - b0;
        cur.free_left = nb;
      }
      if (rbase != ~0ull) {
        cur.ret_next = rbase + b0;
        cur.ret_left = nb;
      }
      const RepairHead hd = repair_heads(ix, a, b0, nb);
      const uint32_t ts = l_seg(a, b0, nb);
      for (uint32_t k = 0; k < nb; ++k) {
        wave_sync();
        repair_chain_u8<G>(ix, a, p, (uint32_t)__builtin_amdgcn_readlane((int)ts, (int)k), hd, (int)k, cur);
      }
      return_slabs(ix, cur);
      pubs += cur.pubs;
    }
  }
  SlabCursor tally;
  tally.pubs = pubs;
  finish_slabs_block(ix, tally, C_PUB_REPAIR);  // ends with a workgroup barrier
  // the last workgroup out resets the queues for the next launch
  if (threadIdx.x == 0) {
    const unsigned long long done = atomicAdd(&ix.ctr[C_QDONE], 1ull);
    if (done + 1 == gridDim.x) {
      for (uint32_t q = 0; q < N_RQ; ++q) atomicExch(&ix.ctr[rq_word(q)], 0ull);
      atomicExch(&ix.ctr[C_QDONE], 0ull);
    }
  }
}

// ---- stable LSD radix sort with a launch-time count --------------------------------------
// 8-bit digits over a bit range. Per pass: digit counts per tile of 1,024
// keys, an exclusive scan of each digit's counts over the tiles (one block
// per digit), then a stable scatter: a tile is read in 4 rounds of 256 keys
// in input order; a key's rank among equal digits is its rank within its wave
// (ballots on the digit bits) plus the counts of the earlier waves and rounds.
// Pair keys are produced in ascending source order, so sorting on the target
// half alone gives (target, source) order.
constexpr uint32_t RS_TILE = 1024;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

__global__ void __launch_bounds__(256) k_rs_count(Index ix, const uint64_t* in, uint32_t cap, Dyn d, int shift,
                                                  uint32_t mask, uint32_t* hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  if (gated(ix, d)) return;
  const uint32_t n = dyn_count(ix, d, cap);
  const uint32_t t = threadIdx.x, tile = blockIdx.x;
  h[t] = 0;
  __syncthreads();
  const uint32_t b0 = tile * RS_TILE, b1 = min(n, b0 + RS_TILE);
  for (uint32_t i = b0 + t; i < b1; i += 256) atomicAdd(&h[(uint32_t)(in[i] >> shift) & mask], 1u);
  __syncthreads();
  hist[(size_t)t * ntiles + tile] = h[t];
}

__global__ void __launch_bounds__(256) k_rs_scan(Index ix, uint32_t* hist, uint32_t ntiles, uint32_t* tot, Dyn d) {
  __shared__ uint32_t ws[4];
  if (gated(ix, d)) return;
  uint32_t* row = hist + (size_t)blockIdx.x * ntiles;
  const uint32_t t = threadIdx.x, w = t >> 6;
  uint32_t carry = 0;
  for (uint32_t c = 0; c < ntiles; c += 256) {
    const uint32_t i = c + t;
    const uint32_t v = i < ntiles ? row[i] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (lane_id() == 63) ws[w] = incl;
    __syncthreads();
    uint32_t before = carry;
    for (uint32_t k = 0; k < w; ++k) before += ws[k];
    if (i < ntiles) row[i] = before + incl - v;
    carry += ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
  }
  if (t == 0) tot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(256) k_rs_scatter(Index ix, const uint64_t* in, uint64_t* out, uint32_t cap, Dyn d,
                                                    int shift, uint32_t mask, const uint32_t* hist,
                                                    const uint32_t* tot, uint32_t ntiles) {
  __shared__ uint32_t base[256], run[256], wh[4][256], ws[4];
  if (gated(ix, d)) return;
  const uint32_t n = dyn_count(ix, d, cap);
  const uint32_t t = threadIdx.x, w = t >> 6, tile = blockIdx.x;
  const uint32_t b0 = tile * RS_TILE;
  if (b0 >= n) return;
  {
    const uint32_t v = tot[t];
    const uint32_t incl = wave_incl_scan(v);
    if (lane_id() == 63) ws[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; ++k) before += ws[k];
    base[t] = before + incl - v + hist[(size_t)t * ntiles + tile];
    run[t] = 0;
    wh[0][t] = wh[1][t] = wh[2][t] = wh[3][t] = 0;
  }
  __syncthreads();
  for (uint32_t r = 0; r < RS_TILE / 256 && b0 + r * 256 < n; ++r) {
    const uint32_t i = b0 + r * 256 + t;
    const bool valid = i < n;
    uint64_t key = 0;
    uint32_t dg = 0;
    if (valid) {
      key = in[i];
      dg = (uint32_t)(key >> shift) & mask;
    }
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t bb = ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = lanes_below(peers);
    if (valid && rank == 0) wh[w][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = run[dg] + rank;
      for (uint32_t k = 0; k < w; ++k) off += wh[k][dg];
      out[base[dg] + off] = key;
    }
    __syncthreads();
    run[t] += wh[0][t] + wh[1][t] + wh[2][t] + wh[3][t];
    wh[0][t] = wh[1][t] = wh[2][t] = wh[3][t] = 0;
    __syncthreads();
  }
}

// ---- reclaim (Algorithm 4) -------------------------------------------------------------
__global__ void k_del_bitmap(Index ix, uint64_t n_ids, Dyn d, uint64_t* bitmap) {
  if (gated(ix, d)) return;
  n_ids = dyn_count(ix, d, (uint32_t)n_ids);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    ix.ctr[C_DIRTY] = 0;
    ix.ctr[C_DEAD] = 0;
  }
  const bool flagged = t < n_ids && ref_del(load_ref(ix, (uint32_t)t));
  const uint64_t m = ballot(flagged);
  if (lane_id() == 0 && t < n_ids) bitmap[t >> 6] = m;
}

__device__ inline bool bit_set(const uint64_t* bm, uint32_t id) { return (bm[id >> 6] >> (id & 63u)) & 1ull; }

// live nodes with an edge into a tombstone ("dirty"), and the count of such
// edges; neighbors are tested against the deletion bitmap.
constexpr uint32_t DIRTY_CHUNK = 1024;  // nodes per workgroup and step

__global__ void __launch_bounds__(256) k_dirty(Index ix, uint64_t n_ids, Dyn d, const uint64_t* bitmap,
                                               uint32_t* dirty) {
  __shared__ uint32_t buf[DIRTY_CHUNK];
  __shared__ uint32_t cnt_s, dead_s, base_s;
  if (gated(ix, d)) return;
  const uint32_t n = dyn_count(ix, d, (uint32_t)n_ids);
  const uint32_t R = ix.R;
  // A workgroup takes 1,024 nodes per step: each wave four runs of 64, lane l
  // owning node base + l. The slabs are read by eight lanes per node, eight
  // nodes at a time (lane c of a group reads ids 4c.. 4c+3, then 32 further
  // on), so a node's id half is one contiguous run; each group's count goes
  // to its node's lane. Dirty ids gather in LDS and take their place in the
  // list with one atomic per workgroup and step.
  const int l = lane_id();
  const uint32_t c = (uint32_t)(l & 7), wv = threadIdx.x >> 6;
  const bool short_lists = R <= 32u && (R & 3u) == 0;
  for (uint32_t chunk = blockIdx.x; chunk * DIRTY_CHUNK < n; chunk += gridDim.x) {
    if (threadIdx.x == 0) {
      cnt_s = 0;
      dead_s = 0;
    }
    __syncthreads();
    for (uint32_t run = 0; run < DIRTY_CHUNK / 256u; ++run) {
      const uint32_t base = chunk * DIRTY_CHUNK + (run * 4u + wv) * 64u;
      uint32_t dead = 0;
      if (short_lists) {
        // R <= 32: one 16-byte read per lane and node covers the list. The
        // run's reference words are read in one coalesced load (lane l: node
        // base + l) and the eight groups' slab reads are all issued before
        // the first bitmap test, so the three dependent reads of a node
        // overlap with those of the others.
        const uint32_t vme = base + (uint32_t)l;
        const uint64_t rme = vme < n ? load_ref(ix, vme) : ~0ull;
        uint4 w[8];
        uint32_t dg[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
          const uint64_t r = __shfl((unsigned long long)rme, (int)(8u * k + (uint32_t)(l >> 3)), 64);
          const uint32_t deg = ref_deg(r), s = ref_slab(r);
          const bool live = !ref_del(r) && s != NONE && 4u * c < deg;
          dg[k] = live ? deg : 0u;
          w[k] = live ? *reinterpret_cast<const uint4*>(ix.slabs + (size_t)s * 2u * R + 4u * c) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
          const uint32_t j = 4u * c;
          uint32_t cn = 0;
          if (j < dg[k]) cn += bit_set(bitmap, w[k].x);
          if (j + 1 < dg[k]) cn += bit_set(bitmap, w[k].y);
          if (j + 2 < dg[k]) cn += bit_set(bitmap, w[k].z);
          if (j + 3 < dg[k]) cn += bit_set(bitmap, w[k].w);
          cn = group_sum<8>(cn);
          const uint32_t got = (uint32_t)__shfl((int)cn, (int)((l & 7) * 8), 64);
          if ((uint32_t)(l >> 3) == k) dead = got;
        }
      } else
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t v = base + 8u * k + (uint32_t)(l >> 3);
        uint32_t cn = 0;
        if (v < n) {
          const uint64_t r = load_ref(ix, v);
          const uint32_t deg = ref_deg(r), s = ref_slab(r);
          if (!ref_del(r) && s != NONE) {
            const uint32_t* ids = ix.slabs + (size_t)s * 2u * R;
            if ((R & 3u) == 0) {
              for (uint32_t j = 4u * c; j < deg; j += 32u) {
                const uint4 w = *reinterpret_cast<const uint4*>(ids + j);
                cn += bit_set(bitmap, w.x);
                if (j + 1 < deg) cn += bit_set(bitmap, w.y);
                if (j + 2 < deg) cn += bit_set(bitmap, w.z);
                if (j + 3 < deg) cn += bit_set(bitmap, w.w);
              }
            } else {
              for (uint32_t j = c; j < deg; j += 8u) cn += bit_set(bitmap, ids[j]);
            }
          }
        }
        cn = group_sum<8>(cn);
        // lane 8k + g takes the count of group g (node base + 8k + g)
        const uint32_t got = (uint32_t)__shfl((int)cn, (int)((l & 7) * 8), 64);
        if ((uint32_t)(l >> 3) == k) dead = got;
      }
      const uint64_t m = ballot(dead != 0);
      uint32_t total = dead;
      for (int o = 32; o > 0; o >>= 1) total += (uint32_t)__shfl_xor((int)total, o, 64);
      uint32_t at = 0;
      if (l == 0 && m) {
        at = atomicAdd(&cnt_s, (uint32_t)__popcll(m));
        atomicAdd(&dead_s, total);
      }
      at = (uint32_t)__shfl((int)at, 0, 64);
      if (dead) buf[at + lanes_below(m)] = base + (uint32_t)l;
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt_s) {
      base_s = (uint32_t)atomicAdd(&ix.ctr[C_DIRTY], (unsigned long long)cnt_s);
      atomicAdd(&ix.ctr[C_DEAD], (unsigned long long)dead_s);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt_s; i += blockDim.x) dirty[base_s + i] = buf[i];
    __syncthreads();
  }
}

// phase 1, compaction: republish each dirty node without its tombstoned entries
// the list of a dirty node (reference word r) as lane l's entry
__device__ inline void compact_read(const Index& ix, uint64_t r, uint32_t& id, uint32_t& dd) {
  const int l = lane_id();
  const uint32_t deg = ref_deg(r), s = ref_slab(r);
  id = NONE;
  dd = 0;
  if ((uint32_t)l < deg && s != NONE) {
    id = ix.slabs[(size_t)s * 2u * ix.R + (uint32_t)l];
    dd = ix.slabs[(size_t)s * 2u * ix.R + ix.R + (uint32_t)l];
  }
}

// A wave's dirty nodes (every total_waves()-th from its index) in batches of
// 64: the batch's ids and reference words are read together (lane k: the
// k-th), each node's list is read while the previous node is published, and
// the publication starts from the word already read (no other wave touches
// a dirty node in this phase).
__global__ void __launch_bounds__(256) k_compact(Index ix, const uint32_t* dirty, uint64_t n, Dyn dn,
                                                 const uint64_t* bitmap, uint32_t lds_per_wave) {
  extern __shared__ __align__(16) char smem[];
  if (gated(ix, dn)) return;
  const uint32_t cnt = dyn_count(ix, dn, (uint32_t)n);
  uint32_t* ids = reinterpret_cast<uint32_t*>(smem + (size_t)(threadIdx.x >> 6) * lds_per_wave);
  uint32_t* d = ids + 64;
  SlabCursor cur = reserve_slabs_block(ix, wave_items(cnt), wave_items(cnt));
  const int l = lane_id();
  const uint32_t w = wave_index(), W = total_waves();
  for (uint32_t base = w; base < cnt; base += 64u * W) {
    const uint32_t my = base + (uint32_t)l * W;
    const uint32_t ul = my < cnt ? dirty[my] : NONE;
    const uint64_t rl = my < cnt ? load_ref(ix, ul) : 0ull;
    const uint32_t nb = (uint32_t)__popcll(ballot(my < cnt));
    uint32_t id, dd;
    compact_read(ix, bcast_lane64(rl, 0), id, dd);
    for (uint32_t k = 0; k < nb; ++k) {
      const uint32_t u = (uint32_t)__builtin_amdgcn_readlane((int)ul, (int)k);
      const uint64_t r = bcast_lane64(rl, (int)k);
      uint32_t nid = NONE, ndd = 0;
      if (k + 1 < nb) compact_read(ix, bcast_lane64(rl, (int)k + 1), nid, ndd);
      const bool keep = id != NONE && !bit_set(bitmap, id);
      const uint64_t m = ballot(keep);
      wave_sync();
      if (keep) {
        ids[lanes_below(m)] = id;
        d[lanes_below(m)] = dd;
      }
      wave_sync();
      publish(ix, u, ids, d, (uint32_t)__popcll(m), C_PUB_COMPACT, &cur, r);
      id = nid;
      dd = ndd;
    }
  }
  finish_slabs_block(ix, cur, C_PUB_COMPACT);
}

// phase 2: <1,d,s> -> <1,0,none> and the slab is retired. A workgroup takes
// 1,024 ids per step; the slabs it frees gather in LDS and take consecutive
// retired-stack slots with one atomic per workgroup and step.
constexpr uint32_t FREE_CHUNK = 1024;

__global__ void __launch_bounds__(256) k_free_tombstones(Index ix, uint64_t n_ids, Dyn d) {
  __shared__ uint32_t buf[FREE_CHUNK];
  __shared__ uint32_t cnt_s;
  __shared__ unsigned long long base_s;
  if (gated(ix, d)) return;
  n_ids = dyn_count(ix, d, (uint32_t)n_ids);
  for (uint64_t c0 = (uint64_t)blockIdx.x * FREE_CHUNK; c0 < n_ids; c0 += (uint64_t)gridDim.x * FREE_CHUNK) {
    if (threadIdx.x == 0) cnt_s = 0;
    __syncthreads();
    for (uint32_t step = 0; step < FREE_CHUNK / 256u; ++step) {
      const uint64_t t = c0 + step * 256u + threadIdx.x;
      uint32_t freed = NONE;
      if (t < n_ids) {
        const uint32_t u = (uint32_t)t;
        uint64_t r = load_ref(ix, u);
        for (int attempt = 0; attempt < 1024 && ref_del(r) && ref_slab(r) != NONE; ++attempt) {
          const uint64_t prev = atomicCAS(&ix.refs[u], (unsigned long long)r,
                                          (unsigned long long)(make_ref(1, 0, NONE) | (r & REF_NORM_MASK)));
          if (prev == r) {
            freed = ref_slab(r);
            break;
          }
          r = prev;
        }
      }
      const uint64_t m = ballot(freed != NONE);
      uint32_t at = 0;
      if (lane_id() == 0 && m) at = atomicAdd(&cnt_s, (uint32_t)__popcll(m));
      at = bcast(at);
      if (freed != NONE) buf[at + lanes_below(m)] = freed;
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt_s) {
      base_s = atomicAdd(&ix.ctr[C_RETIRED_TOP], (unsigned long long)cnt_s);
      atomicAdd(&ix.ctr[C_FREED], (unsigned long long)cnt_s);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt_s; i += blockDim.x) {
      const unsigned long long idx = base_s + i;
      if (idx < ix.P)
        ix.retired_stack[idx] = buf[i];
      else
        atomicOr(&ix.ctr[C_ERROR], (unsigned long long)ERR_POOL_OVERFLOW);
    }
    __syncthreads();
  }
}

// ---- export -----------------------------------------------------------------------------
__global__ void k_export(Index ix, uint64_t n_ids, uint32_t* nbr, uint32_t* rho, uint8_t* deg, uint8_t* del,
                         uint8_t* has_slab) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_ids * ix.R) return;
  const uint32_t u = (uint32_t)(t / ix.R), j = (uint32_t)(t % ix.R);
  const uint64_t r = load_ref(ix, u);
  const uint32_t dg = ref_deg(r), s = ref_slab(r);
  const bool has = s != NONE && j < dg;
  nbr[t] = has ? ix.slabs[(size_t)s * 2u * ix.R + j] : NONE;
  rho[t] = has ? ix.slabs[(size_t)s * 2u * ix.R + ix.R + j] : 0u;
  if (j == 0) {
    deg[u] = s == NONE ? 0 : (uint8_t)dg;
    del[u] = (uint8_t)ref_del(r);
    has_slab[u] = s != NONE;
  }
}

// ---- brute-force ground truth over the live set ---------------------------------------
// One wave per query; each lane scans ids l, l+64, ... keeping its own K best,
// then the 64 lane lists are merged by a sort in LDS.
template <int K>
__global__ void __launch_bounds__(64) k_bruteforce_u8(Index ix, const uint8_t* q, uint32_t nq, uint64_t n_ids,
                                                       uint32_t k, uint32_t* out_ids, int32_t* out_d) {
  __shared__ uint64_t all[64 * K];
  const uint32_t qi = blockIdx.x;
  if (qi >= nq) return;
  const int l = lane_id();
  const uint4* qv = reinterpret_cast<const uint4*>(q + (size_t)qi * ix.dim);
  const int words = (int)ix.dim / 16;
  uint32_t qq = 0;
  for (int w = 0; w < words; ++w) qq = dot16(qv[w], qv[w], qq);
  uint64_t best[K];
#pragma unroll
  for (int i = 0; i < K; ++i) best[i] = KEY_NONE;
  for (uint64_t u = (uint64_t)l; u < n_ids; u += 64) {
    if (ref_del(load_ref(ix, (uint32_t)u)) || ref_slab(load_ref(ix, (uint32_t)u)) == NONE) continue;
    const uint4* xv = reinterpret_cast<const uint4*>(ix.x + u * ix.dim);
    uint32_t qx = 0, xx = 0;
    for (int w = 0; w < words; ++w) {
      const uint4 v = xv[w];
      qx = dot16(qv[w], v, qx);
      xx = dot16(v, v, xx);
    }
    uint64_t key = make_key(qq + xx - 2u * qx, (uint32_t)u);
    if (key < best[K - 1]) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const uint64_t lo = key < best[i] ? key : best[i];
        const uint64_t hi = key < best[i] ? best[i] : key;
        best[i] = lo;
        key = hi;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) all[l * K + i] = best[i];
  __syncthreads();
  wave_bitonic_sort(all, 64 * K);
  for (uint32_t i = (uint32_t)l; i < k; i += 64) {
    const uint64_t kk = all[i];
    out_ids[(size_t)qi * k + i] = kk == KEY_NONE ? NONE : key_id(kk);
    out_d[(size_t)qi * k + i] = kk == KEY_NONE ? 0x7FFFFFFF : (int32_t)key_dist(kk);
  }
}

// ---- brute-force ground truth on the matrix cores (uint8 rows, dim <= 256) -----------
// The exact k nearest live rows of each query by (distance, id), in three passes.
// Rows are shifted to signed bytes (x - 128), which leaves every squared
// difference unchanged, so d = |q'|^2 + |x'|^2 - 2 q'.x' is exact in int32.
//   k_bf_norms:  |x'|^2 of every id, or -1 where the id is not live;
//   k_bf_mfma:   a wave holds 16 queries as the N operand of
//                v_mfma_i32_16x16x64_i8 (their shifted fragments stay in
//                registers) and streams one chunk of rows through the M operand,
//                16 rows per tile; lane l then holds query l % 16 against rows
//                4 (l / 16) + i of the tile and keeps the K best keys of the rows
//                it sees, so a query's K best over the chunk are among its four
//                lanes' lists, which are written out;
//   k_bf_merge:  one wave per query selects the k best of all its candidates.
__global__ void __launch_bounds__(256) k_bf_norms(Index ix, uint64_t n_ids, int32_t* xn) {
  const uint32_t words = ix.dim / 16u;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n_ids; u += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = load_ref(ix, (uint32_t)u);
    int32_t v = -1;
    if (!ref_del(r) && ref_slab(r) != NONE) {
      const uint8_t* row = ix.x + u * ix.dim;
      int sq = 0;
      for (uint32_t w = 0; w < words; ++w) {
        const v4i32 f = signed_frag(row, w * 16u, ix.dim);
        sq += frag_sq(f);
      }
      v = sq;
    }
    xn[u] = v;
  }
}

template <int S, int K>
__global__ void __launch_bounds__(256) k_bf_mfma(Index ix, const uint8_t* q, uint32_t nq, uint64_t n_ids,
                                                 const int32_t* xn, uint32_t n_chunks, uint64_t chunk, uint64_t* cand) {
  const uint32_t wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t qt = wv / n_chunks, c = wv % n_chunks;
  if (qt * 16u >= nq) return;  // whole waves only
  const int l = lane_id();
  const uint32_t r = (uint32_t)(l & 15), kc = (uint32_t)(l >> 4) * 16u, rb = (uint32_t)(l >> 4) * 4u;
  const uint32_t dim = ix.dim, qi = qt * 16u + r;
  const bool qok = qi < nq;
  const uint8_t* qrow = qok ? q + (size_t)qi * dim : nullptr;
  v4i32 qf[S];
  int qn = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    qf[s] = signed_frag(qrow, (uint32_t)s * 64u + kc, dim);
    qn += frag_sq(qf[s]);
  }
  qn += (int)lane_xor<16>((uint32_t)qn);  // the four lanes of query r hold its four 16-byte pieces
  qn += (int)lane_xor<32>((uint32_t)qn);
  uint64_t best[K];
#pragma unroll
  for (int i = 0; i < K; ++i) best[i] = KEY_NONE;
  const uint64_t e_beg = (uint64_t)c * chunk;
  const uint64_t e_end = min(n_ids, e_beg + chunk);
  // fragments of the first tile, then each tile's while the previous one is scored
  v4i32 xf[S];
#pragma unroll
  for (int s = 0; s < S; ++s)
    xf[s] = signed_frag(e_beg + r < e_end ? ix.x + (e_beg + r) * dim : nullptr, (uint32_t)s * 64u + kc, dim);
  for (uint64_t e0 = e_beg; e0 < e_end; e0 += 16) {
    v4i32 acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < S; ++s) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(xf[s], qf[s], acc, 0, 0, 0);
    const uint64_t nx = e0 + 16 + r;
#pragma unroll
    for (int s = 0; s < S; ++s) xf[s] = signed_frag(nx < e_end ? ix.x + nx * dim : nullptr, (uint32_t)s * 64u + kc, dim);
    // the norms of this lane's four rows (e0 is a multiple of 16: one aligned 16-byte load)
    int4 nn = make_int4(-1, -1, -1, -1);
    if (e0 + rb < e_end) {
      if (e0 + rb + 4 <= e_end) {
        nn = *reinterpret_cast<const int4*>(xn + e0 + rb);
      } else {
        nn.x = xn[e0 + rb];
        if (e0 + rb + 1 < e_end) nn.y = xn[e0 + rb + 1];
        if (e0 + rb + 2 < e_end) nn.z = xn[e0 + rb + 2];
      }
    }
    const int nv[4] = {nn.x, nn.y, nn.z, nn.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!qok || nv[i] < 0) continue;
      uint64_t key = make_key((uint32_t)(qn + nv[i] - 2 * acc[i]), (uint32_t)(e0 + rb + (uint32_t)i));
      if (key < best[K - 1]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const uint64_t lo = key < best[j] ? key : best[j];
          const uint64_t hi = key < best[j] ? best[j] : key;
          best[j] = lo;
          key = hi;
        }
      }
    }
  }
  if (qok) {
    uint64_t* out = cand + (((uint64_t)qi * n_chunks + c) * 4u + (uint32_t)(l >> 4)) * K;
#pragma unroll
    for (int i = 0; i < K; ++i) out[i] = best[i];
  }
}

template <int K>
__global__ void __launch_bounds__(64) k_bf_merge(const uint64_t* cand, uint32_t n_cand, uint32_t k, uint32_t* out_ids,
                                                 int32_t* out_d) {
  __shared__ uint64_t all[64 * K];
  const uint32_t qi = blockIdx.x;
  const int l = lane_id();
  uint64_t best[K];
#pragma unroll
  for (int i = 0; i < K; ++i) best[i] = KEY_NONE;
  const uint64_t* c = cand + (uint64_t)qi * n_cand;
  for (uint32_t j = (uint32_t)l; j < n_cand; j += 64) {
    uint64_t key = c[j];
    if (key < best[K - 1]) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const uint64_t lo = key < best[i] ? key : best[i];
        const uint64_t hi = key < best[i] ? best[i] : key;
        best[i] = lo;
        key = hi;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) all[l * K + i] = best[i];
  __syncthreads();
  wave_bitonic_sort(all, 64 * K);
  for (uint32_t i = (uint32_t)l; i < k; i += 64) {
    const uint64_t kk = all[i];
    out_ids[(size_t)qi * k + i] = kk == KEY_NONE ? NONE : key_id(kk);
    out_d[(size_t)qi * k + i] = kk == KEY_NONE ? 0x7FFFFFFF : (int32_t)key_dist(kk);
  }
}

// ---- float rows: traversal copies written on insert ------------------------------------------
// One wave per new row: bf16 copy (round to nearest even) and/or FP8 e4m3
// copy of x / s with s = max|x_i| / 448 (s = 1 for an all-zero row).
__global__ void __launch_bounds__(256) k_encode_f32(Index ix, uint32_t first, uint32_t n, Dyn d, float* xs,
                                                    uint16_t* xb, uint8_t* x8) {
  if (gated(ix, d)) return;
  n = dyn_count(ix, d, n);
  first = dyn_first(ix, d, first);
  const uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int l = lane_id();
  const uint32_t id = first + i;
  const float* row = ix.xf + (size_t)id * ix.dim;
  float amax = 0.f;
  for (uint32_t j = (uint32_t)l; j < ix.dim; j += 64) amax = fmaxf(amax, fabsf(row[j]));
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if (xb)
    for (uint32_t j = (uint32_t)l; j < ix.dim; j += 64) xb[(size_t)id * ix.dim + j] = to_bf16(row[j]);
  if (x8) {
    const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
    for (uint32_t j = (uint32_t)l; j < ix.dim; j += 64) x8[(size_t)id * ix.dim + j] = to_e4m3(row[j] / sc);
    if (l == 0) xs[id] = sc;
  }
}

// exact FP32 k nearest live rows by (distance, id); one wave per query, G lanes
// per row, 64 rows per step, each lane keeping its own K best
template <int G>
__global__ void __launch_bounds__(64) k_bruteforce_f32(Index ix, const float* q, uint32_t nq, uint64_t n_ids,
                                                        uint32_t k, uint32_t* out_ids, uint32_t* out_d) {
  constexpr int K = 16;
  __shared__ uint64_t all[64 * K];
  __shared__ uint64_t ck[64];
  __shared__ uint32_t ids[64];
  const uint32_t qi = blockIdx.x;
  if (qi >= nq) return;
  const int l = lane_id();
  using E = TravF<G, TRAV_NATIVE>;
  const typename E::Q qv = E::load_query(q + (size_t)qi * ix.dim);
  uint64_t best[K];
#pragma unroll
  for (int i = 0; i < K; ++i) best[i] = KEY_NONE;
  for (uint64_t b = 0; b < n_ids; b += 64) {
    const uint64_t u = b + (uint64_t)l;
    bool ok = false;
    if (u < n_ids) {
      const uint64_t r = load_ref(ix, (uint32_t)u);
      ok = !ref_del(r) && ref_slab(r) != NONE;
    }
    const uint64_t m = ballot(ok);
    if (ok) ids[lanes_below(m)] = (uint32_t)u;
    const int cnt = __popcll(m);
    __syncthreads();
    E::dist_batch(ix, qv, ids, cnt, ck, nullptr);
    __syncthreads();
    if (l < cnt) {
      uint64_t key = ck[l];
      if (key < best[K - 1]) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const uint64_t lo = key < best[i] ? key : best[i];
          const uint64_t hi = key < best[i] ? best[i] : key;
          best[i] = lo;
          key = hi;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < K; ++i) all[l * K + i] = best[i];
  __syncthreads();
  wave_bitonic_sort(all, 64 * K);
  for (uint32_t i = (uint32_t)l; i < k; i += 64) {
    const uint64_t kk = all[i];
    out_ids[(size_t)qi * k + i] = kk == KEY_NONE ? NONE : key_id(kk);
    out_d[(size_t)qi * k + i] = kk == KEY_NONE ? 0x7F800000u : __builtin_bit_cast(uint32_t, fkey_inv(key_dist(kk)));
  }
}

// ---- host-side launchers ---------------------------------------------------------------------

static inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

// Item loops run on persistent waves: a launch never needs more workgroups
// than this (the chip holds 256 CUs x a few workgroups; the rest would queue).
constexpr unsigned PERSIST_BLOCKS = 2048;
static inline unsigned persist_grid(uint64_t items, unsigned per_block) {
  const unsigned b = blocks_for(items, per_block);
  return b < PERSIST_BLOCKS ? (b ? b : 1u) : PERSIST_BLOCKS;
}

hipError_t launch_init(const Index& ix, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(1024), dim3(256), 0, s, ix);
  return hipGetLastError();
}

hipError_t launch_recycle(const Index& ix, hipStream_t s) {
  hipLaunchKernelGGL(k_recycle, dim3(256), dim3(256), 0, s, ix);
  hipLaunchKernelGGL(k_recycle_commit, dim3(1), dim3(1), 0, s, ix);
  return hipGetLastError();
}

hipError_t launch_round_begin(const Index& ix, const uint32_t* counts, uint32_t nd, uint32_t ni, uint32_t nq,
                              uint32_t max_d, uint32_t max_i, uint32_t max_q, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(64), 0, s, ix, counts, nd, ni, nq, max_d, max_i, max_q, status);
  return hipGetLastError();
}

hipError_t launch_round_gate(const Index& ix, uint32_t tombstone_only, uint32_t boot_max, int32_t* status,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_round_gate, dim3(1), dim3(64), 0, s, ix, tombstone_only, boot_max, status);
  return hipGetLastError();
}

hipError_t launch_reclaim_gate(const Index& ix, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_reclaim_gate, dim3(1), dim3(64), 0, s, ix, status);
  return hipGetLastError();
}

hipError_t launch_row_norms(const Index& ix, uint32_t first, uint32_t n, Dyn d, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_norms, dim3(blocks_for(n, 256) < 1024u ? blocks_for(n, 256) : 1024u), dim3(256), 0, s, ix,
                     first, n, d);
  return hipGetLastError();
}

hipError_t launch_store_rows(const Index& ix, const void* src, uint32_t* ids_out, uint32_t first, uint32_t n, Dyn d,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t words = (uint64_t)n * (ix.metric == 0 ? ix.dim / 16u : ix.dim / 4u);
  hipLaunchKernelGGL(k_store_rows, dim3(persist_grid(words, 256)), dim3(256), 0, s, ix, (const uint4*)src, ids_out,
                     first, n, d);
  return hipGetLastError();
}

// rows named by index into a contiguous batch (16-byte words)
__global__ void k_gather_rows(const uint4* rows, const uint32_t* idx, uint32_t n, uint32_t words, uint4* out) {
  const uint64_t total = (uint64_t)n * words;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride)
    out[t] = rows[(size_t)idx[t / words] * words + t % words];
}

hipError_t launch_gather_rows(const void* rows, const uint32_t* idx, uint32_t n, uint32_t row_bytes, void* out,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t words = row_bytes / 16u;
  hipLaunchKernelGGL(k_gather_rows, dim3(persist_grid((uint64_t)n * words, 256)), dim3(256), 0, s,
                     (const uint4*)rows, idx, n, words, (uint4*)out);
  return hipGetLastError();
}

// serving: a tick's search results (nq x k) to the rows of the requests they answer
__global__ void k_scatter_results(const uint32_t* ids, const uint32_t* d, const uint32_t* pos, uint32_t nq, uint32_t k,
                                  uint32_t* out_ids, uint32_t* out_d) {
  const uint64_t n = (uint64_t)nq * k;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = (uint64_t)pos[i / k] * k + i % k;
    out_ids[r] = ids[i];
    out_d[r] = d[i];
  }
}

hipError_t launch_scatter_results(const uint32_t* ids, const uint32_t* d, const uint32_t* pos, uint32_t nq, uint32_t k,
                                  uint32_t* out_ids, uint32_t* out_d, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const unsigned b = blocks_for((uint64_t)nq * k, 256);
  hipLaunchKernelGGL(k_scatter_results, dim3(b < 1024u ? b : 1024u), dim3(256), 0, s, ids, d, pos, nq, k, out_ids, out_d);
  return hipGetLastError();
}

hipError_t launch_refresh_entries(const Index& ix, uint32_t bound, uint32_t S, Dyn d, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_entries, dim3(1), dim3(1024), 0, s, ix, bound, S, d);
  if (ix.metric == 0 && ix.ent_x && ix.ent_norm)
    hipLaunchKernelGGL(k_entry_rows, dim3(blocks_for(S ? S : 1u, 256)), dim3(256), 0, s, ix, S, d);
  return hipGetLastError();
}

hipError_t launch_segments(const Index& ix, const uint64_t* pairs, uint32_t nmax, Dyn d, uint32_t* seg,
                           hipStream_t s) {
  if (nmax == 0) return hipSuccess;
  hipLaunchKernelGGL(k_segments, dim3(blocks_for(nmax, SEG_CHUNK)), dim3(256), 0, s, ix, pairs, nmax, d, seg);
  return hipGetLastError();
}

uint32_t sort_hist_words(uint32_t nmax) {
  const uint32_t tiles = nmax ? blocks_for(nmax, RS_TILE) : 1u;
  return 256u * tiles + 256u;
}

hipError_t launch_sort(const Index& ix, uint64_t* a, uint64_t* b, uint32_t nmax, Dyn d, int lo, int nbits,
                       uint32_t* hist, hipStream_t s, uint64_t** result, int low_bits) {
  *result = a;
  if (nmax == 0) return hipSuccess;
  const uint32_t ntiles = blocks_for(nmax, RS_TILE);
  uint32_t* tot = hist + 256u * ntiles;
  uint64_t* src = a;
  uint64_t* dst = b;
  // least significant digits first: bits [0, low_bits), then [lo, lo + nbits)
  for (int part = 0; part < 2; ++part) {
    const int from = part == 0 ? 0 : lo, width_all = part == 0 ? low_bits : nbits;
    for (int sh = 0; sh < width_all; sh += 8) {
      const int width = width_all - sh < 8 ? width_all - sh : 8;
      const uint32_t mask = (1u << width) - 1u;
      hipLaunchKernelGGL(k_rs_count, dim3(ntiles), dim3(256), 0, s, ix, (const uint64_t*)src, nmax, d, from + sh,
                         mask, hist, ntiles);
      hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(256), 0, s, ix, hist, ntiles, tot, d);
      hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(256), 0, s, ix, (const uint64_t*)src, dst, nmax, d,
                         from + sh, mask, (const uint32_t*)hist, (const uint32_t*)tot, ntiles);
      uint64_t* t = src;
      src = dst;
      dst = t;
    }
  }
  *result = src;
  return hipGetLastError();
}

uint32_t search_lds_per_wave(uint32_t L, uint32_t vt_slots, uint32_t W) {
  // L <= 64 (list in registers): candidate keys/refs, ids (64 per two
  // expansions of a step), visited table
  if (L <= 64) return (W > 2 ? 2u : 1u) * (2u * 512u + 256u) + 4u * vt_slots;
  // L <= 128 at W <= 2 (two list slots per lane): the same for 128 entries
  if (L <= 128 && W <= 2) return 2u * (2u * 512u + 256u) + 4u * vt_slots;
  // keys + refs (double-buffered), candidate keys/refs, merge scratch, ids,
  // insertion points, visited table, expanded flags
  return 32u * L + 4u * 512u + 2u * 256u + 4u * vt_slots + ((2u * L + 15u) & ~15u);
}

// lanes per row of a float copy: 3 chunks of 16 bytes per lane
static inline int float_lanes(uint32_t dim, int elem_bytes) { return (int)(dim * (uint32_t)elem_bytes / 16u / 3u); }

// uint8 start-set scoring: 64-byte slices per row fixed at compile time (two
// up to 128 bytes, four up to 256, then chunks of four)
template <int PASS, bool PRE>
static void launch_scan_dist(const Index& ix, const ScanArgs& a, dim3 grid, hipStream_t s) {
  if (ix.dim <= 128)
    hipLaunchKernelGGL((k_scan_dist<PASS, PRE, 2, false>), grid, dim3(256), 0, s, ix, a);
  else if (ix.dim <= 256)
    hipLaunchKernelGGL((k_scan_dist<PASS, PRE, 4, false>), grid, dim3(256), 0, s, ix, a);
  else
    hipLaunchKernelGGL((k_scan_dist<PASS, PRE, 4, true>), grid, dim3(256), 0, s, ix, a);
}

hipError_t launch_scan(const Index& ix, const ScanArgs& args, hipStream_t s, hipEvent_t after_dist) {
  if (args.nq == 0) return hipSuccess;
  ScanArgs a = args;
  a.g_rows = ix.metric == 0 ? (uint32_t)SD_WT : (uint32_t)SD_E;
  a.g_stride = blocks_for(a.ns ? a.ns : 1u, a.g_rows) * (a.g_rows / 32);
  // shapes from the upper bounds; the kernels resolve the launch-time counts
  const uint64_t tiles = (uint64_t)blocks_for(a.ns ? a.ns : 1u, SD_E) * blocks_for(a.nq, SD_Q);
  const dim3 dgrid(tiles < 2 * PERSIST_BLOCKS ? (unsigned)tiles : 2 * PERSIST_BLOCKS);
  const uint32_t cap = scan_select_keys(a.L);
  const dim3 grid(blocks_for(a.nq, 4)), blk(256);
  const size_t lds = 4 * scan_select_lds_per_wave(a.L);
  if (a.ns > SEL_GPL * 64 * 32) return hipErrorInvalidValue;
  if (ix.metric == 0) {
    // one 64-query x SCAN_SPAN-row span per wave, four waves per workgroup
    if (a.ns > SCAN_SPAN * 64) return hipErrorInvalidValue;
    const uint64_t wt = (uint64_t)blocks_for(a.ns ? a.ns : 1u, SCAN_SPAN) * blocks_for(a.nq, SD_WT);
    const uint64_t wg = (wt + 3) / 4;
    const dim3 tgrid(wg < 4 * PERSIST_BLOCKS ? (unsigned)wg : 4 * PERSIST_BLOCKS);
    const bool pre = a.mode != MODE_BOOT && ix.ent_x && ix.ent_norm;
    if (a.L > SCAN_FILTER_L_MAX) {
      // long lists: the bound admits a large share of the rows, so the matrix is written
      if (pre)
        launch_scan_dist<SCAN_DENSE, true>(ix, a, tgrid, s);
      else
        launch_scan_dist<SCAN_DENSE, false>(ix, a, tgrid, s);
      if (after_dist) {
        const hipError_t e = hipEventRecord(after_dist, s);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_scan_select, grid, blk, lds, s, ix, a, cap);
      return hipGetLastError();
    }
    if (!a.bound || !a.ncand || !a.cand) return hipErrorInvalidValue;
    if (pre) {
      launch_scan_dist<SCAN_MIN, true>(ix, a, tgrid, s);
      hipLaunchKernelGGL(k_scan_bound, grid, blk, 0, s, ix, a);
      launch_scan_dist<SCAN_FILTER, true>(ix, a, tgrid, s);
    } else {
      launch_scan_dist<SCAN_MIN, false>(ix, a, tgrid, s);
      hipLaunchKernelGGL(k_scan_bound, grid, blk, 0, s, ix, a);
      launch_scan_dist<SCAN_FILTER, false>(ix, a, tgrid, s);
    }
    if (after_dist) {
      const hipError_t e = hipEventRecord(after_dist, s);
      if (e != hipSuccess) return e;
    }
    // key capacity in LDS: lists up to 64 see about a hundred keys, so a
    // smaller capacity keeps more waves resident
    const uint32_t fcap = max(a.L <= 64 ? SCAN_CAND_CAP / 2 : SCAN_CAND_CAP, cap);
    hipLaunchKernelGGL(k_scan_final, grid, blk, (size_t)4 * 8 * fcap, s, ix, a, fcap);
    return hipGetLastError();
  } else {
    const int trav = a.mode == MODE_BOOT ? TRAV_NATIVE : a.trav;
    if (trav == TRAV_NATIVE)
      hipLaunchKernelGGL(k_scan_dist_f<TRAV_NATIVE>, dgrid, dim3(256), 0, s, ix, a);
    else if (trav == TRAV_BF16)
      hipLaunchKernelGGL(k_scan_dist_f<TRAV_BF16>, dgrid, dim3(256), 0, s, ix, a);
    else
      hipLaunchKernelGGL(k_scan_dist_f<TRAV_FP8>, dgrid, dim3(256), 0, s, ix, a);
  }
  if (after_dist) {
    const hipError_t e = hipEventRecord(after_dist, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_select, grid, blk, lds, s, ix, a, cap);
  return hipGetLastError();
}

// the list lives in registers for L <= 64, and for L <= 128 at W <= 2
#define LSQ(TP, Q)                                                                                              \
  do {                                                                                                          \
    if (a.L <= 64)                                                                                              \
      if (a.W > 2)                                                                                              \
        hipLaunchKernelGGL((k_search_rl<TP, TP::FLOAT ? 1u : 6u, 2, Q>), dim3(grid), dim3(64 * waves_per_block), lds, \
                           s, ix, a);                                                                           \
      else                                                                                                      \
        hipLaunchKernelGGL((k_search_rl<TP, TP::FLOAT ? 1u : 7u, 1, Q>), dim3(grid), dim3(64 * waves_per_block), lds, \
                           s, ix, a);                                                                           \
    else if (a.L <= 128 && a.W <= 2)                                                                            \
      hipLaunchKernelGGL((k_search_rl2<TP, TP::FLOAT ? 1u : 6u, Q>), dim3(grid), dim3(64 * waves_per_block), lds, \
                         s, ix, a);                                                                             \
    else                                                                                                        \
      hipLaunchKernelGGL((k_search<TP, Q>), dim3(grid), dim3(64 * waves_per_block), lds, s, ix, a);             \
  } while (0)
#define LS(TP)                           \
  do {                                   \
    if (a.mode == MODE_QUERY)            \
      LSQ(TP, true);                     \
    else                                 \
      LSQ(TP, false);                    \
  } while (0)

hipError_t launch_search(const Index& ix, const SearchArgs& a, uint32_t waves_per_block, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  const unsigned grid = a.persistent ? persist_grid(a.nq, waves_per_block) : blocks_for(a.nq, waves_per_block);
  const size_t lds = (size_t)a.lds_per_wave * waves_per_block;
  if (ix.metric == 0) {
    // lanes per row: dim / 16 (one chunk each), or half that with two chunks each
    const bool half = a.row_lanes != 0 && a.row_lanes * 32u == ix.dim;
    switch (ix.dim / 16) {
      case 1: { using TP = TravU8<1>; LS(TP); break; }
      case 2: { using TP = TravU8<2>; LS(TP); break; }
      case 4: { using TP = TravU8<4>; LS(TP); break; }
      case 8:
        if (half) { using TP = TravU8<4, 2>; LS(TP); } else { using TP = TravU8<8>; LS(TP); }
        break;
      case 16:
        if (half) { using TP = TravU8<8, 2>; LS(TP); } else { using TP = TravU8<16>; LS(TP); }
        break;
      case 32: { using TP = TravU8<32>; LS(TP); break; }
      case 64: { using TP = TravU8<64>; LS(TP); break; }
      default: return hipErrorInvalidValue;
    }
  } else if (a.trav == TRAV_NATIVE) {
    switch (float_lanes(ix.dim, 4)) {
      case 8: { using TP = TravFloat<8, TRAV_NATIVE>; LS(TP); break; }
      case 16: { using TP = TravFloat<16, TRAV_NATIVE>; LS(TP); break; }
      case 32: { using TP = TravFloat<32, TRAV_NATIVE>; LS(TP); break; }
      case 64: { using TP = TravFloat<64, TRAV_NATIVE>; LS(TP); break; }
      default: return hipErrorInvalidValue;
    }
  } else if (a.trav == TRAV_BF16) {
    switch (float_lanes(ix.dim, 2)) {
      case 4: { using TP = TravFloat<4, TRAV_BF16>; LS(TP); break; }
      case 8: { using TP = TravFloat<8, TRAV_BF16>; LS(TP); break; }
      case 16: { using TP = TravFloat<16, TRAV_BF16>; LS(TP); break; }
      case 32: { using TP = TravFloat<32, TRAV_BF16>; LS(TP); break; }
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (float_lanes(ix.dim, 1)) {
      case 2: { using TP = TravFloat<2, TRAV_FP8>; LS(TP); break; }
      case 4: { using TP = TravFloat<4, TRAV_FP8>; LS(TP); break; }
      case 8: { using TP = TravFloat<8, TRAV_FP8>; LS(TP); break; }
      case 16: { using TP = TravFloat<16, TRAV_FP8>; LS(TP); break; }
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}
#undef LS
#undef LSQ

uint32_t chain_lds_per_wave(uint32_t R, uint32_t vstride) { return chain_lds_bytes(R, vstride); }
uint32_t pool_lds_per_wave(uint32_t vstride) { return pool_lds_bytes(vstride); }

uint32_t maint_lds_per_wave(const MaintArgs& a, uint32_t R) {
  const size_t sel = a.mx ? 16 + (size_t)MX_M_WORDS * 4 + 2 * 64 * 4  // alignment, table, tile and kept norms
                          : (size_t)a.prune_cap * a.vstride + (size_t)a.prune_cap * 8;  // staged rows, norms
  size_t b = (size_t)a.nsort * 8 + (size_t)a.prune_cap * 8 + sel + (size_t)(R + 1) * 8 + (size_t)a.nmax * 4 +
             (size_t)(R + 1) * 12 + (size_t)a.prune_cap;
  return (uint32_t)((b + 15) & ~(size_t)15);
}

// Blocks of kernel f (block size threads, dynamic LDS lds) that are resident
// on the whole device at once: a persistent launch larger than this runs its
// waves in generations, each wave with the same share of the items, so the
// last generation leaves the device partly idle. Cached per (kernel, shape).
template <class F>
static unsigned resident_blocks(F f, unsigned threads, size_t lds) {
  struct Key {
    const void* f;
    unsigned threads;
    size_t lds;
    bool operator<(const Key& o) const {
      return f != o.f ? f < o.f : threads != o.threads ? threads < o.threads : lds < o.lds;
    }
  };
  static std::mutex mu;
  static std::map<Key, unsigned> cache;
  static int cus = 0;
  const Key k{reinterpret_cast<const void*>(f), threads, lds};
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(k);
  if (it != cache.end()) return it->second;
  int dev = 0, per_cu = 0;
  if (cus == 0 && (hipGetDevice(&dev) != hipSuccess ||
                   hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess))
    cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, (int)threads, lds) != hipSuccess) per_cu = 0;
  const unsigned r = cus > 0 && per_cu > 0 ? (unsigned)(per_cu * cus) : 0u;  // 0: unknown
  cache[k] = r;
  return r;
}

// share > 1: only that fraction of the resident blocks (the concurrent mode
// leaves room on every CU for the searches of the other stream)
template <class F>
static dim3 resident_grid(F f, unsigned grid, dim3 blk, size_t lds, unsigned share) {
  unsigned r = resident_blocks(f, blk.x, lds);
  if (r && share > 1) r = r / share ? r / share : 1u;
  return dim3(r && grid > r ? r : grid);
}
template <class F>
static dim3 resident_grid(F f, unsigned grid, dim3 blk, size_t lds) {
  return resident_grid(f, grid, blk, lds, 1u);
}

template <class P>
static void launch_maint_p(MaintKernel which, const Index& ix, const MaintArgs& a, unsigned grid, dim3 blk,
                           size_t lds, hipStream_t s) {
  const unsigned sh = ix.concurrent ? 2u : 1u;  // searches of the other stream need CUs too
  switch (which) {
    case MK_FORWARD:
      hipLaunchKernelGGL(k_forward<P>, resident_grid(k_forward<P>, grid, blk, lds, sh), blk, lds, s, ix, a);
      break;
    case MK_REVERSE:
      if constexpr (P::CHAIN) {
        if (a.chain) {
          hipLaunchKernelGGL(k_reverse_chain<P::GL>, resident_grid(k_reverse_chain<P::GL>, grid, blk, lds, sh), blk, lds,
                             s, ix, a);
          break;
        }
      }
      hipLaunchKernelGGL(k_reverse_apply<P>, resident_grid(k_reverse_apply<P>, grid, blk, lds, sh), blk, lds, s, ix, a);
      break;
    case MK_REVERSE_FAST:
      hipLaunchKernelGGL(k_reverse_fast<P>, resident_grid(k_reverse_fast<P>, grid, blk, lds, sh), blk, lds, s, ix, a);
      break;
    case MK_REFINE:
      hipLaunchKernelGGL(k_refine<P>, resident_grid(k_refine<P>, grid, blk, lds, sh), blk, lds, s, ix, a);
      hipLaunchKernelGGL(k_refine_publish, dim3(grid), blk, 512u * (blk.x / 64u), s, ix, a);
      break;
    case MK_REPAIR:
      if constexpr (P::CHAIN) {
        if (a.chain) {
          hipLaunchKernelGGL(k_reserve_launch, dim3(1), dim3(64), 0, s, ix, a.d);
          hipLaunchKernelGGL(k_repair_pool<P::GL>, resident_grid(k_repair_pool<P::GL>, grid, blk, lds, sh), blk, lds, s,
                             ix, a);
          break;
        }
      }
      hipLaunchKernelGGL(k_repair_apply<P>, resident_grid(k_repair_apply<P>, grid, blk, lds, sh), blk, lds, s, ix, a);
      break;
  }
}

hipError_t launch_maint(MaintKernel which, const Index& ix, const MaintArgs& a, uint32_t nwaves,
                        uint32_t waves_per_block, hipStream_t s) {
  if (nwaves == 0) return hipSuccess;
  const unsigned grid = persist_grid(nwaves, waves_per_block);
  const size_t lds = (size_t)a.lds_per_wave * waves_per_block;
  const dim3 blk(64 * waves_per_block);
  if (ix.metric == 0) {
    switch (ix.dim / 16) {
      case 1: launch_maint_p<MaintU8<1>>(which, ix, a, grid, blk, lds, s); break;
      case 2: launch_maint_p<MaintU8<2>>(which, ix, a, grid, blk, lds, s); break;
      case 4: launch_maint_p<MaintU8<4>>(which, ix, a, grid, blk, lds, s); break;
      case 8: launch_maint_p<MaintU8<8>>(which, ix, a, grid, blk, lds, s); break;
      case 16: launch_maint_p<MaintU8<16>>(which, ix, a, grid, blk, lds, s); break;
      case 32: launch_maint_p<MaintU8<32>>(which, ix, a, grid, blk, lds, s); break;
      case 64: launch_maint_p<MaintU8<64>>(which, ix, a, grid, blk, lds, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (float_lanes(ix.dim, 4)) {
      case 8: launch_maint_p<MaintF32<8>>(which, ix, a, grid, blk, lds, s); break;
      case 16: launch_maint_p<MaintF32<16>>(which, ix, a, grid, blk, lds, s); break;
      case 32: launch_maint_p<MaintF32<32>>(which, ix, a, grid, blk, lds, s); break;
      case 64: launch_maint_p<MaintF32<64>>(which, ix, a, grid, blk, lds, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_set_lists(const Index& ix, const MaintArgs& a, const uint32_t* ids, const uint32_t* nbr,
                            const uint32_t* deg, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const dim3 grid(blocks_for(a.n, 1)), blk(64);
  const size_t lds = a.lds_per_wave;
  if (ix.metric == 0) {
    switch (ix.dim / 16) {
      case 1: hipLaunchKernelGGL(k_set_lists<MaintU8<1>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 2: hipLaunchKernelGGL(k_set_lists<MaintU8<2>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 4: hipLaunchKernelGGL(k_set_lists<MaintU8<4>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 8: hipLaunchKernelGGL(k_set_lists<MaintU8<8>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 16: hipLaunchKernelGGL(k_set_lists<MaintU8<16>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 32: hipLaunchKernelGGL(k_set_lists<MaintU8<32>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 64: hipLaunchKernelGGL(k_set_lists<MaintU8<64>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (float_lanes(ix.dim, 4)) {
      case 8: hipLaunchKernelGGL(k_set_lists<MaintF32<8>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 16: hipLaunchKernelGGL(k_set_lists<MaintF32<16>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 32: hipLaunchKernelGGL(k_set_lists<MaintF32<32>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      case 64: hipLaunchKernelGGL(k_set_lists<MaintF32<64>>, grid, blk, lds, s, ix, a, ids, nbr, deg); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_encode(const Index& ix, uint32_t first, uint32_t n, Dyn d, float* xs, uint16_t* xb, uint8_t* x8,
                         hipStream_t s) {
  if (n == 0 || (!xb && !x8)) return hipSuccess;
  hipLaunchKernelGGL(k_encode_f32, dim3(blocks_for(n, 4)), dim3(256), 0, s, ix, first, n, d, xs, xb, x8);
  return hipGetLastError();
}

hipError_t launch_reverse_pairs(const Index& ix, const MaintArgs& a, hipStream_t s) {
  const uint64_t n = (uint64_t)a.n * ix.R;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reverse_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, s, ix, a);
  return hipGetLastError();
}

hipError_t launch_repair_pairs(const Index& ix, const MaintArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;  // a.n: upper bound; the kernel reads the accepted count
  hipLaunchKernelGGL(k_repair_pairs, dim3(blocks_for(a.n, 4)), dim3(256), 0, s, ix, a);
  return hipGetLastError();
}

hipError_t launch_del_keys(const Index& ix, const uint32_t* ids, uint32_t n, Dyn d, uint64_t* keys, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_del_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, ix, ids, n, d, keys);
  return hipGetLastError();
}

hipError_t launch_del_classify(const Index& ix, const uint64_t* sorted, uint32_t n, Dyn d, uint8_t* status,
                               uint32_t* dlist, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_del_classify, dim3(blocks_for(n, 256)), dim3(256), 0, s, ix, sorted, n, d, status, dlist);
  return hipGetLastError();
}

hipError_t launch_tombstone(const Index& ix, const uint32_t* dlist, uint32_t n, Dyn d, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tombstone, dim3(blocks_for(n, 256)), dim3(256), 0, s, ix, dlist, n, d);
  return hipGetLastError();
}

hipError_t launch_del_bitmap(const Index& ix, uint64_t n_ids, Dyn d, uint64_t* bitmap, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  hipLaunchKernelGGL(k_del_bitmap, dim3(blocks_for(n_ids, 256)), dim3(256), 0, s, ix, n_ids, d, bitmap);
  return hipGetLastError();
}

hipError_t launch_dirty(const Index& ix, uint64_t n_ids, Dyn d, const uint64_t* bitmap, uint32_t* dirty,
                        hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  const unsigned blocks = blocks_for(n_ids, DIRTY_CHUNK);
  hipLaunchKernelGGL(k_dirty, dim3(blocks < 4 * PERSIST_BLOCKS ? blocks : 4 * PERSIST_BLOCKS), dim3(256), 0, s, ix,
                     n_ids, d, bitmap, dirty);
  return hipGetLastError();
}

hipError_t launch_compact(const Index& ix, const uint32_t* dirty, uint64_t n, Dyn d, const uint64_t* bitmap,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t per_wave = 512;
  hipLaunchKernelGGL(k_compact, dim3(persist_grid(n, 4)), dim3(256), 4 * per_wave, s, ix, dirty, n, d, bitmap,
                     per_wave);
  return hipGetLastError();
}

hipError_t launch_free_tombstones(const Index& ix, uint64_t n_ids, Dyn d, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  const unsigned blocks = blocks_for(n_ids, FREE_CHUNK);
  hipLaunchKernelGGL(k_free_tombstones, dim3(blocks < 4 * PERSIST_BLOCKS ? blocks : 4 * PERSIST_BLOCKS), dim3(256), 0,
                     s, ix, n_ids, d);
  return hipGetLastError();
}

hipError_t launch_export(const Index& ix, uint64_t n_ids, uint32_t* nbr, uint32_t* rho, uint8_t* deg, uint8_t* del,
                         uint8_t* has_slab, hipStream_t s) {
  if (n_ids == 0) return hipSuccess;
  hipLaunchKernelGGL(k_export, dim3(blocks_for(n_ids * ix.R, 256)), dim3(256), 0, s, ix, n_ids, nbr, rho, deg, del,
                     has_slab);
  return hipGetLastError();
}

uint64_t bruteforce_norm_bytes(uint64_t n_ids) { return (n_ids * 4 + 255) / 256 * 256; }

uint64_t bruteforce_scratch_bytes(const Index& ix, uint32_t nq, uint64_t n_ids) {
  if (ix.metric != 0 || ix.dim < 64 || ix.dim > 256) return 0;
  const uint32_t q_tiles = (nq + 15) / 16;
  const uint64_t n_chunks = std::min<uint64_t>(std::max<uint64_t>(1, (n_ids + 1023) / 1024),
                                               std::max<uint32_t>(1, (4096 + q_tiles - 1) / q_tiles));
  return bruteforce_norm_bytes(n_ids) + (uint64_t)nq * n_chunks * 4 * 16 * 8;
}

hipError_t launch_bruteforce(const Index& ix, const void* q, uint32_t nq, uint64_t n_ids, uint32_t k,
                             uint32_t* out_ids, uint32_t* out_d, hipStream_t s, unsigned char* scratch) {
  if (nq == 0) return hipSuccess;
  if (k > 16) return hipErrorInvalidValue;
  if (ix.metric == 0 && scratch && ix.dim >= 64 && ix.dim <= 256) {
    // on the matrix cores: chunks of rows so that about 4,096 waves run
    const uint32_t q_tiles = blocks_for(nq, 16);
    uint32_t n_chunks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, (n_ids + 1023) / 1024),
                                                     std::max<uint32_t>(1, blocks_for(4096, q_tiles)));
    const uint64_t chunk = ((n_ids + n_chunks - 1) / n_chunks + 15) / 16 * 16;
    n_chunks = (uint32_t)std::max<uint64_t>(1, (n_ids + chunk - 1) / chunk);
    int32_t* xn = reinterpret_cast<int32_t*>(scratch);
    uint64_t* cand = reinterpret_cast<uint64_t*>(scratch + bruteforce_norm_bytes(n_ids));
    hipLaunchKernelGGL(k_bf_norms, dim3(std::min<uint64_t>(4096, blocks_for(n_ids ? n_ids : 1, 256))), dim3(256), 0, s,
                       ix, n_ids, xn);
    const uint64_t waves = (uint64_t)q_tiles * n_chunks;
    const dim3 grid((unsigned)((waves + 3) / 4)), blk(256);
    switch (ix.dim / 64) {
      case 1: hipLaunchKernelGGL((k_bf_mfma<1, 16>), grid, blk, 0, s, ix, (const uint8_t*)q, nq, n_ids, xn, n_chunks, chunk, cand); break;
      case 2: hipLaunchKernelGGL((k_bf_mfma<2, 16>), grid, blk, 0, s, ix, (const uint8_t*)q, nq, n_ids, xn, n_chunks, chunk, cand); break;
      case 4: hipLaunchKernelGGL((k_bf_mfma<4, 16>), grid, blk, 0, s, ix, (const uint8_t*)q, nq, n_ids, xn, n_chunks, chunk, cand); break;
      default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_bf_merge<16>, dim3(nq), dim3(64), 0, s, cand, n_chunks * 4u * 16u, k, out_ids, (int32_t*)out_d);
  } else if (ix.metric == 0) {
    hipLaunchKernelGGL(k_bruteforce_u8<16>, dim3(nq), dim3(64), 0, s, ix, (const uint8_t*)q, nq, n_ids, k, out_ids,
                       (int32_t*)out_d);
  } else {
    switch (float_lanes(ix.dim, 4)) {
      case 8: hipLaunchKernelGGL(k_bruteforce_f32<8>, dim3(nq), dim3(64), 0, s, ix, (const float*)q, nq, n_ids, k, out_ids, out_d); break;
      case 16: hipLaunchKernelGGL(k_bruteforce_f32<16>, dim3(nq), dim3(64), 0, s, ix, (const float*)q, nq, n_ids, k, out_ids, out_d); break;
      case 32: hipLaunchKernelGGL(k_bruteforce_f32<32>, dim3(nq), dim3(64), 0, s, ix, (const float*)q, nq, n_ids, k, out_ids, out_d); break;
      case 64: hipLaunchKernelGGL(k_bruteforce_f32<64>, dim3(nq), dim3(64), 0, s, ix, (const float*)q, nq, n_ids, k, out_ids, out_d); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace etale
