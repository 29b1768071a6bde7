// Device-side building blocks of the ETALE index for gfx950 (wave64).
//
// Layout in HBM (one index):
//   x      : vectors, id-indexed, row = dim bytes (uint8) .
//   refs   : one 64-bit reference word per id (Definition 1):
//              bit 63 deletion flag, bits 62..56 degree, bits 31..0 slab id,
//              slab id 0xFFFFFFFF = no slab. Unborn ids hold <0,0,none>.
//              Bits 55..32 hold the squared norm of the id's uint8 row when
//              dim <= 256 (at most 256 * 255^2 < 2^24), written when the row
//              is stored and carried unchanged by every later change of the
//              word, so a distance needs no second pass over the row; zero
//              for wider or float rows.
//   slabs  : pool of P slabs of 2R words each: R neighbor ids, then R
//            distances (structure of arrays, so a search reads only the ids).
//   free / retired stacks of slab ids with one counter each (Section 3.3).
//   ctr    : 64-bit counters (stack tops, error bits, statistics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etale {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint64_t KEY_NONE = ~0ull;
constexpr uint64_t REF_UNBORN = 0x00000000FFFFFFFFull;

__host__ __device__ inline uint64_t make_ref(uint32_t del, uint32_t deg, uint32_t slab) {
  return ((uint64_t)(del & 1u) << 63) | ((uint64_t)(deg & 0x7Fu) << 56) | (uint64_t)slab;
}
constexpr uint64_t REF_NORM_MASK = 0x00FFFFFF00000000ull;
__host__ __device__ inline uint32_t ref_del(uint64_t r) { return (uint32_t)(r >> 63); }
__host__ __device__ inline uint32_t ref_norm(uint64_t r) { return (uint32_t)(r >> 32) & 0xFFFFFFu; }
// uint8 rows of at most 256 bytes (G = dim / 16 <= 16 lanes) keep their norm in the word
template <int G>
constexpr bool norm_in_ref() { return G <= 16; }
__host__ __device__ inline uint32_t ref_deg(uint64_t r) { return (uint32_t)(r >> 56) & 0x7Fu; }
__host__ __device__ inline uint32_t ref_slab(uint64_t r) { return (uint32_t)r; }

// search / sort key: (distance, id) packed so that integer order is the
// lexicographic order the method uses everywhere.
__host__ __device__ inline uint64_t make_key(uint32_t d, uint32_t id) { return ((uint64_t)d << 32) | id; }
__host__ __device__ inline uint32_t key_id(uint64_t k) { return (uint32_t)k; }
__host__ __device__ inline uint32_t key_dist(uint64_t k) { return (uint32_t)(k >> 32); }

enum Counter {
  C_FREE_TOP = 0,
  C_RETIRED_TOP,
  C_ERROR,
  C_N_ENTRIES,
  C_PUB_FORWARD,
  C_PUB_REPAIR,
  C_PUB_REVERSE,
  C_PUB_REFINE,
  C_PUB_COMPACT,
  C_FREED,
  C_DIRTY,
  C_DEAD,
  C_SEARCH_EXP,
  C_SEARCH_DIST,
  C_CAS_FAIL,
  C_PUB_DROPPED,
  C_DEL_OK,
  C_TOMBSTONED,
  C_NEXT_ID,   // ids handed out so far
  C_LIVE,      // handed-out ids with deletion flag 0
  C_R_NDEL,    // this round's requested deletes, inserts, queries
  C_R_NINS,
  C_R_NQ,
  C_R_FIRST,   // this round's first new id
  C_R_GATE,    // GateBits of this round
  C_NSEG,      // segments (runs of one target) of the last sorted pair list
  C_QUEUE,     // work queue of the running search launch
  C_QDONE,     // waves of that launch that have left the queue
  C_RES_FREE,  // a launch's slab reservation: free-stack top before it (~0: none)
  C_RES_RET,   // and its first retired-stack slot (~0: none)
  C_NCOUNTERS = 32
};
// the repair launch's work queues, each on a line of its own after the
// counters (atomics on one line serialize, whichever word they touch)
constexpr uint32_t N_RQ = 8, RQ_STRIDE = 32;
constexpr uint32_t CTR_WORDS = C_NCOUNTERS + N_RQ * RQ_STRIDE;
__host__ __device__ inline uint32_t rq_word(uint32_t q) { return C_NCOUNTERS + q * RQ_STRIDE; }

// Round gate: set before any mutation of a round; kernels whose skip mask
// meets it do nothing.
enum GateBits : uint64_t { G_FAIL = 1, G_BOOT = 2, G_NOBOOT = 4, G_RFAIL = 8 };

enum ErrorBits : uint64_t { ERR_POOL_EMPTY = 1, ERR_POOL_OVERFLOW = 2, ERR_BAD_LIST = 4 };

struct Index {
  uint32_t dim, R;
  uint32_t a2, b2;  // alpha = a/b, applied squared: a^2 * D1 <= b^2 * D2
  uint32_t cmp32;   // 1: uint8 distances and both products stay below 2^32 (24-bit multiplies suffice)
  uint32_t publish_attempts;
  uint32_t fence;   // 1: a release fence orders a slab's contents before its reference (concurrent readers)
  uint32_t concurrent;  // 1: searches may run alongside writers: slab ids are read with agent-coherent loads
  uint32_t prune_cap;
  int32_t metric;   // 0: uint8 squared L2, 1: FP32 inner product (d = 1 - <a,b>)
  int32_t trav;     // traversal copy for the float metric: 0 FP32, 1 bf16, 2 FP8 e4m3 + scale
  uint32_t rerank;  // float metric, non-FP32 traversal: results re-ranked from rerank*k candidates
  uint64_t cap, P;
  const uint8_t* x;     // uint8 rows
  const float* xf;      // FP32 rows (float metric)
  const uint16_t* xb;   // bf16 rows (bf16 traversal)
  const uint8_t* x8;    // e4m3 rows (FP8 traversal)
  const float* xs;      // per-row FP8 scale
  unsigned long long* refs;
  uint32_t* slabs;
  uint32_t* free_stack;
  uint32_t* retired_stack;
  unsigned long long* ctr;
  uint32_t* entries;
  uint8_t* ent_x;     // uint8 rows: the entry set's rows, each byte XOR 0x80, in matrix-operand order
  int32_t* ent_norm;  // minus their squared norms (as signed bytes), padded to a multiple of 64
};

// ---- counts read at launch time --------------------------------------------------
// A round replayed from a captured graph has launch shapes fixed at capture;
// its item counts live in counters. A kernel resolves them when it starts:
// n = min(cap, counter * mult - c0) items (the cap is the static count of the
// launch), first id from a counter, and nothing at all when the round's gate
// meets the skip mask. NO_CTR keeps the static value.
constexpr uint32_t NO_CTR = 0xFFFFFFFFu;

struct Dyn {
  uint32_t skip = 0;          // GateBits that turn the launch into a no-op
  uint32_t n_ctr = NO_CTR;    // counter with the item count
  uint32_t n_mult = 1;        // items per counted unit
  uint32_t c0 = 0;            // this launch covers items [c0, c0 + cap)
  uint32_t first_ctr = NO_CTR;  // counter with the first id (added to c0)
};

// ---- wave primitives --------------------------------------------------------

__device__ inline int lane_id() { return (int)(threadIdx.x & 63u); }

// Order LDS traffic among the lanes of one wave (waves of a block run
// independent loops, so block barriers are not usable).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint32_t bcast(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t bcast64(uint64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// the value of `lane` (the same lane in every lane of the wave)
__device__ inline uint64_t bcast_lane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// lane i receives lane i - 1's value (lane 0 receives 0): a whole-wave DPP shift
__device__ inline uint32_t lane_shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ inline uint64_t lane_shr1_64(uint64_t v) {
  return ((uint64_t)lane_shr1((uint32_t)(v >> 32)) << 32) | lane_shr1((uint32_t)v);
}

__device__ inline bool gated(const Index& ix, const Dyn& d) {
  return d.skip != 0 && (ix.ctr[C_R_GATE] & (uint64_t)d.skip) != 0;
}
__device__ inline uint32_t dyn_count(const Index& ix, const Dyn& d, uint32_t cap) {
  if (d.n_ctr == NO_CTR) return cap;
  const uint64_t v = ix.ctr[d.n_ctr] * (uint64_t)d.n_mult;
  return v <= d.c0 ? 0u : (uint32_t)(v - d.c0 < cap ? v - d.c0 : cap);
}
__device__ inline uint32_t dyn_first(const Index& ix, const Dyn& d, uint32_t first) {
  return d.first_ctr == NO_CTR ? first : (uint32_t)ix.ctr[d.first_ctr] + d.c0;
}
__device__ inline uint32_t total_waves() { return gridDim.x * (blockDim.x >> 6); }

// One ticket per wave from a counter. Every lane takes part in the atomic
// (lane 0 adds 1, the others 0) so no lane-divergent branch precedes the
// broadcast: inside a loop such a branch lets the compiler split the wave
// into lanes that re-enter the loop without lane 0.
__device__ inline uint32_t wave_ticket(unsigned long long* ctr) {
  const unsigned long long v = atomicAdd(ctr, (threadIdx.x & 63u) == 0 ? 1ull : 0ull);
  return __builtin_amdgcn_readfirstlane((uint32_t)v);
}

__device__ inline uint64_t load_ref(const Index& ix, uint32_t u) {
  return __hip_atomic_load(&ix.refs[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- uint8 squared L2 via 4-wide byte dot products ----------------------------
// |a-b|^2 = |a|^2 + |b|^2 - 2<a,b>, every term exact in 32-bit integers for
// dim <= 1024 (1024 * 255^2 < 2^31).

__device__ inline uint32_t dot16(uint4 a, uint4 b, uint32_t acc) {
  acc = __builtin_amdgcn_udot4(a.x, b.x, acc, false);
  acc = __builtin_amdgcn_udot4(a.y, b.y, acc, false);
  acc = __builtin_amdgcn_udot4(a.z, b.z, acc, false);
  acc = __builtin_amdgcn_udot4(a.w, b.w, acc, false);
  return acc;
}

// The value of lane l ^ J. Distances within a row of 16 lanes move by DPP
// (quad permutes, row shifts and rotates: ALU latency, no LDS crossbar);
// 16 and 32 go through ds_bpermute.
template <int J>
__device__ inline uint32_t lane_xor(uint32_t v) {
  static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16 || J == 32, "lane distance");
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);  // quad_perm 2,3,0,1
  } else if constexpr (J == 4) {
    const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x104, 0xf, 0xf, false);  // row_shl:4
    const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    return (threadIdx.x & 4u) ? dn : up;
  } else if constexpr (J == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);  // row_ror:8
  } else {
    return (uint32_t)__shfl_xor((int)v, J, 64);
  }
}
template <int J>
__device__ inline float lane_xor(float v) {
  return __builtin_bit_cast(float, lane_xor<J>(__builtin_bit_cast(uint32_t, v)));
}
template <int J>
__device__ inline uint64_t lane_xor(uint64_t v) {
  return ((uint64_t)lane_xor<J>((uint32_t)(v >> 32)) << 32) | lane_xor<J>((uint32_t)v);
}

// Bitonic sort of 64 NK keys in registers, ascending: key s * 64 + l in v[s]
// of lane l. Partners within 64 lanes move by lane_xor; at distances of 64
// and more both keys are the lane's own (slots s and s + J / 64).
template <int J, int K, int NK>
__device__ inline void bitonic_step_regs(uint64_t (&v)[NK]) {
  const int l = lane_id();
  if constexpr (J >= 64) {
    constexpr int D = J / 64;
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      if ((s & D) == 0) {
        const bool up = ((s * 64 + l) & K) == 0;  // direction of this pair's run
        const uint64_t lo = min(v[s], v[s + D]), hi = max(v[s], v[s + D]);
        v[s] = up ? lo : hi;
        v[s + D] = up ? hi : lo;
      }
    }
  } else {
    const bool lower = (l & J) == 0;
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const uint64_t p = lane_xor<J>(v[s]);
      const bool up = ((s * 64 + l) & K) == 0;  // direction of this element's run
      v[s] = lower == up ? min(v[s], p) : max(v[s], p);
    }
  }
}
template <int K, int J, int NK>
__device__ inline void bitonic_pass_regs(uint64_t (&v)[NK]) {
  if constexpr (J > 0) {
    bitonic_step_regs<J, K, NK>(v);
    bitonic_pass_regs<K, J / 2, NK>(v);
  }
}
template <int NK, int K = 2>
__device__ inline void wave_sort_regs(uint64_t (&v)[NK]) {
  if constexpr (K <= 64 * NK) {
    bitonic_pass_regs<K, K / 2, NK>(v);
    wave_sort_regs<NK, K * 2>(v);
  }
}

// sum over the G consecutive lanes of a group (G a power of two), every lane
// of the group ending with the same value
template <int G, class T>
__device__ inline T group_sum_t(T v) {
  if constexpr (G > 1) v += lane_xor<1>(v);
  if constexpr (G > 2) v += lane_xor<2>(v);
  if constexpr (G > 4) v += lane_xor<4>(v);
  if constexpr (G > 8) v += lane_xor<8>(v);
  if constexpr (G > 16) v += lane_xor<16>(v);
  if constexpr (G > 32) v += lane_xor<32>(v);
  return v;
}
template <int G>
__device__ inline uint32_t group_sum(uint32_t v) {
  return group_sum_t<G, uint32_t>(v);
}

// ---- visited table: exact ids, open addressing, may forget -----------------------
// Buckets of four slots, each read as one 16-byte LDS load: an id is looked
// for in its bucket and the next one; a miss takes the first empty slot of
// the bucket by compare-and-swap (re-reading the bucket when another id won
// the slot). A lookup that finds the id reports VT_SEEN; a table too crowded
// to take the id reports VT_CROWDED without storing it. Forgetting only costs
// a repeated distance evaluation: the list merge drops keys already listed,
// and a key rejected or evicted earlier is rejected again (the list's worst
// key never increases), so results do not depend on the table size. Two
// lanes that insert the same id in one call cannot both get VT_NEW (they try
// the same slots in the same order), but both can get VT_CROWDED: the caller
// removes such duplicates from its batch.
constexpr int VT_BUCKETS = 2;  // buckets looked at per id (8 slots)
enum VtResult : uint32_t { VT_SEEN = 0, VT_NEW = 1, VT_CROWDED = 2 };

__device__ inline uint32_t vt_insert(uint32_t* vt, uint32_t mask, uint32_t id) {
  const uint32_t bmask = (mask + 1u) / 4u - 1u;
  const uint32_t b = (id * 2654435761u) & bmask;
#pragma unroll 1
  for (int k = 0; k < VT_BUCKETS; ++k) {
    uint32_t* slot = vt + 4u * ((b + (uint32_t)k) & bmask);
#pragma unroll 1
    for (int tries = 0; tries < 4; ++tries) {
      const uint4 w = *reinterpret_cast<const uint4*>(slot);
      // one of the four equals id exactly when the smallest XOR is zero
      if (min(min(w.x ^ id, w.y ^ id), min(w.z ^ id, w.w ^ id)) == 0u) return VT_SEEN;
      // slots fill in order (a miss always takes the first empty one), so the
      // first empty slot is the count of filled ones
      const int e = w.y == NONE ? (w.x == NONE ? 0 : 1) : (w.w == NONE ? (w.z == NONE ? 2 : 3) : -1);
      if (e < 0) break;  // full: the next bucket
      const uint32_t prev = atomicCAS(&slot[e], NONE, id);
      if (prev == NONE) return VT_NEW;
      if (prev == id) return VT_SEEN;
    }
  }
  return VT_CROWDED;
}

// ---- the candidate list (sorted keys + expanded flags, double-buffered) --------
// Each entry also carries the node's reference word, fetched together with
// its vector when it was scored, so an expansion reads the slab directly and
// the output filter needs no further load.
struct CandList {
  uint64_t* k0;
  uint64_t* k1;
  uint64_t* r0;
  uint64_t* r1;
  uint8_t* x0;
  uint8_t* x1;
  int cur;
  int n;
  int L;
  uint64_t* acck;  // [64] accepted keys of one merge
  uint64_t* accr;  // [64] their references
  uint32_t* accp;  // [64] their insertion points
  // the live buffer and the spare one (selects, not indexed arrays, so the
  // pointers stay in registers)
  __device__ uint64_t* keys() const { return cur ? k1 : k0; }
  __device__ uint64_t* refs() const { return cur ? r1 : r0; }
  __device__ uint8_t* flags() const { return cur ? x1 : x0; }
  __device__ uint64_t* spare_keys() const { return cur ? k0 : k1; }
  __device__ uint64_t* spare_refs() const { return cur ? r0 : r1; }
  __device__ uint8_t* spare_flags() const { return cur ? x0 : x1; }
};

// Merge nc <= 64 candidates (keys ck, references cr; keys distinct among
// themselves) into the list, keeping the L smallest keys and dropping keys
// already present.
__device__ inline void list_merge(CandList& cl, const uint64_t* ck, const uint64_t* cr, int nc) {
  const int l = lane_id();
  const uint64_t* lk = cl.keys();
  const uint64_t* lr = cl.refs();
  const uint8_t* lx = cl.flags();
  uint64_t* nk = cl.spare_keys();
  uint64_t* nr = cl.spare_refs();
  uint8_t* nx = cl.spare_flags();
  const int n = cl.n, L = cl.L;
  bool ok = false;
  uint64_t key = KEY_NONE, ref = 0;
  uint32_t pos = 0;
  if (l < nc) {
    key = ck[l];
    ok = key != KEY_NONE && (n < L || key < lk[n - 1]);
    if (ok) {
      uint32_t lo = 0, hi = (uint32_t)n;
      while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (lk[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
      pos = lo;
      if (pos < (uint32_t)n && lk[pos] == key) ok = false;
      ref = cr[l];
    }
  }
  const uint64_t m = ballot(ok);
  const int na = __popcll(m);
  if (na == 0) return;
  if (ok) {
    uint32_t idx = lanes_below(m);
    cl.acck[idx] = key;
    cl.accp[idx] = pos;
  }
  wave_sync();
  uint32_t cpos = 0;
  if (ok) {
    uint32_t r = 0;
    for (int t = 0; t < na; ++t) r += cl.acck[t] < key;
    cpos = pos + r;
  }
  for (int i = l; i < n; i += 64) {
    uint32_t s = 0;
    for (int t = 0; t < na; ++t) s += cl.accp[t] <= (uint32_t)i;
    uint32_t np = (uint32_t)i + s;
    if (np < (uint32_t)L) {
      nk[np] = lk[i];
      nr[np] = lr[i];
      nx[np] = lx[i];
    }
  }
  if (ok && cpos < (uint32_t)L) {
    nk[cpos] = key;
    nr[cpos] = ref;
    nx[cpos] = 0;
  }
  wave_sync();
  cl.cur ^= 1;
  cl.n = min(L, n + na);
}

// index of the first unexpanded entry at or after `from`, or -1
__device__ inline int list_first_open(const CandList& cl, int from = 0) {
  const int l = lane_id();
  const uint8_t* lx = cl.flags();
  for (int base = from & ~63; base < cl.n; base += 64) {
    int i = base + l;
    uint64_t m = ballot(i >= from && i < cl.n && lx[i] == 0);
    if (m) return base + (int)__builtin_ctzll(m);
  }
  return -1;
}

// ---- cooperative distance batch ----------------------------------------------
// G lanes share one vector (16 bytes each); 64/G vectors per pass. qf is this
// lane's 16-byte chunk of the query, qq the query's squared norm.
// Writes ck[i] = (D, id) for ids[0..cnt).
// REFS: read each row's reference word with it (for cr, and for the row's
// norm where the word carries it); without, the norm comes from the row
template <int G, bool REFS = true>
__device__ inline void dist_batch_u8(const Index& ix, uint4 qf, uint32_t qq, const uint32_t* ids, int cnt,
                                     uint64_t* ck, uint64_t* cr = nullptr) {
  constexpr int VPP = 64 / G;
  constexpr bool NR = REFS && norm_in_ref<G>();  // the row's norm comes with its reference word
  const int l = lane_id();
  const int c = l % G, grp = l / G;
  for (int base = 0; base < cnt; base += 4 * VPP) {
    // sub-batches past cnt are skipped (a uniform branch), all loads of the
    // used ones are issued before any is used
    const int used = min(4, (cnt - base + VPP - 1) / VPP);
    uint4 v[4];
    uint32_t id[4];
    uint64_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int vi = base + u * VPP + grp;
      id[u] = NONE;
      v[u] = make_uint4(0, 0, 0, 0);
      r[u] = 0;
      if (u < used) {
        id[u] = vi < cnt ? ids[vi] : NONE;
        if (id[u] != NONE) {
          v[u] = reinterpret_cast<const uint4*>(ix.x + (size_t)id[u] * ix.dim)[c];
          if (REFS && (cr || NR) && c == 0) r[u] = load_ref(ix, id[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= used) break;
      uint32_t qx = group_sum<G>(dot16(qf, v[u], 0u));
      uint32_t xx;
      if constexpr (NR)
        xx = ref_norm(r[u]);  // lane c == 0 holds the word
      else
        xx = group_sum<G>(dot16(v[u], v[u], 0u));
      int vi = base + u * VPP + grp;
      if (c == 0 && vi < cnt) {
        ck[vi] = make_key(qq + xx - 2u * qx, id[u]);
        if (REFS && cr) cr[vi] = r[u];
      }
    }
  }
}

// The same batch with C 16-byte chunks per lane (G lanes per row, G * C * 16 =
// dim): fewer lanes per row, so more rows per pass and shorter group sums.
// 4 / C sub-batches are in flight at a time.
template <int G, int C, bool REFS>
__device__ inline void dist_batch_u8c(const Index& ix, const uint4 (&qf)[C], uint32_t qq, const uint32_t* ids,
                                      int cnt, uint64_t* ck, uint64_t* cr) {
  constexpr int VPP = 64 / G;
  constexpr int U = 4 / C;
  constexpr bool NR = REFS && norm_in_ref<G * C>();
  const int l = lane_id();
  const int c = l % G, grp = l / G;
  for (int base = 0; base < cnt; base += U * VPP) {
    const int used = min(U, (cnt - base + VPP - 1) / VPP);
    uint4 v[U][C];
    uint32_t id[U];
    uint64_t r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int vi = base + u * VPP + grp;
      id[u] = NONE;
      r[u] = 0;
#pragma unroll
      for (int t = 0; t < C; ++t) v[u][t] = make_uint4(0, 0, 0, 0);
      if (u < used) {
        id[u] = vi < cnt ? ids[vi] : NONE;
        if (id[u] != NONE) {
          const uint4* row = reinterpret_cast<const uint4*>(ix.x + (size_t)id[u] * ix.dim);
#pragma unroll
          for (int t = 0; t < C; ++t) v[u][t] = row[t * G + c];
          if (REFS && (cr || NR) && c == 0) r[u] = load_ref(ix, id[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (u >= used) break;
      uint32_t qx = 0;
#pragma unroll
      for (int t = 0; t < C; ++t) qx = dot16(qf[t], v[u][t], qx);
      qx = group_sum<G>(qx);
      uint32_t xx;
      if constexpr (NR) {
        xx = ref_norm(r[u]);
      } else {
        xx = 0;
#pragma unroll
        for (int t = 0; t < C; ++t) xx = dot16(v[u][t], v[u][t], xx);
        xx = group_sum<G>(xx);
      }
      const int vi = base + u * VPP + grp;
      if (c == 0 && vi < cnt) {
        ck[vi] = make_key(qq + xx - 2u * qx, id[u]);
        if (REFS && cr) cr[vi] = r[u];
      }
    }
  }
}

template <int G>
__device__ inline uint4 load_frag(const uint8_t* row) {
  return reinterpret_cast<const uint4*>(row)[lane_id() % G];
}

// ---- pool and publication (Algorithm 1) ---------------------------------------

__device__ inline uint32_t alloc_slab(const Index& ix) {
  unsigned long long old = atomicAdd(&ix.ctr[C_FREE_TOP], ~0ull);  // pop
  if (old == 0ull || old > ix.P) {
    atomicAdd(&ix.ctr[C_FREE_TOP], 1ull);
    atomicOr(&ix.ctr[C_ERROR], (unsigned long long)ERR_POOL_EMPTY);
    return NONE;
  }
  return ix.free_stack[old - 1];
}

__device__ inline void retire_slab(const Index& ix, uint32_t s) {
  unsigned long long idx = atomicAdd(&ix.ctr[C_RETIRED_TOP], 1ull);  // push
  if (idx >= ix.P) {
    atomicOr(&ix.ctr[C_ERROR], (unsigned long long)ERR_POOL_OVERFLOW);
    return;
  }
  ix.retired_stack[idx] = s;
}

// Slabs reserved by one wave for the publications it will make. In the
// deterministic phases every item publishes once with an uncontended CAS, so a
// persistent wave pops all its fresh slabs and reserves all its retired-stack
// slots with one atomic each, and counts its publications locally; the shared
// stack tops and counters then see one atomic per wave instead of several per
// publication. A retry after a lost CAS falls back to single atomics.
struct SlabCursor {
  uint64_t free_hi = 0;  // reserved free-stack entries are [free_hi - free_left, free_hi)
  uint32_t free_left = 0;
  uint64_t ret_next = 0;  // reserved retired-stack entries are [ret_next, ret_next + ret_left)
  uint32_t ret_left = 0;
  uint32_t pubs = 0;
};

// every lane takes part; lane 0's value is the one used (see wave_ticket)
__device__ inline uint64_t wave_atomic_add(unsigned long long* ctr, unsigned long long v) {
  const unsigned long long r = atomicAdd(ctr, (threadIdx.x & 63u) == 0 ? v : 0ull);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)r);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(r >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline SlabCursor reserve_slabs(const Index& ix, uint32_t n_alloc, uint32_t n_retire) {
  SlabCursor c;
  if (n_alloc) {
    const uint64_t top = wave_atomic_add(&ix.ctr[C_FREE_TOP], (unsigned long long)(-(long long)n_alloc));
    if (top >= n_alloc && top <= ix.P) {
      c.free_hi = top;
      c.free_left = n_alloc;
    } else {
      wave_atomic_add(&ix.ctr[C_FREE_TOP], (unsigned long long)n_alloc);  // give back; single allocs report the shortage
    }
  }
  if (n_retire) {
    const uint64_t at = wave_atomic_add(&ix.ctr[C_RETIRED_TOP], (unsigned long long)n_retire);
    if (at + n_retire <= ix.P) {
      c.ret_next = at;
      c.ret_left = n_retire;
    } else {
      wave_atomic_add(&ix.ctr[C_RETIRED_TOP], (unsigned long long)(-(long long)n_retire));
    }
  }
  return c;
}

// reserve_slabs for every wave of a workgroup (all of them call it, with
// their own counts) with one pair of atomics for the workgroup: waves take
// consecutive ranges of the workgroup's reservation. Same-address atomics from
// thousands of waves serialize at the cache, so kernels with many short waves
// reserve this way.
__device__ inline SlabCursor reserve_slabs_block(const Index& ix, uint32_t n_alloc, uint32_t n_retire) {
  __shared__ uint32_t s_na[16], s_nr[16];
  __shared__ unsigned long long s_free, s_ret;
  const uint32_t wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane_id() == 0) {
    s_na[wv] = n_alloc;
    s_nr[wv] = n_retire;
  }
  __syncthreads();
  uint32_t pa = 0, pr = 0, ta = 0, tr = 0;
  for (uint32_t k = 0; k < nw; ++k) {
    if (k < wv) {
      pa += s_na[k];
      pr += s_nr[k];
    }
    ta += s_na[k];
    tr += s_nr[k];
  }
  if (threadIdx.x == 0) {
    unsigned long long f = ~0ull, r = ~0ull;
    if (ta) {
      const unsigned long long top = atomicAdd(&ix.ctr[C_FREE_TOP], (unsigned long long)(-(long long)ta));
      if (top >= ta && top <= ix.P)
        f = top;
      else
        atomicAdd(&ix.ctr[C_FREE_TOP], (unsigned long long)ta);  // give back; single allocs report the shortage
    }
    if (tr) {
      const unsigned long long at = atomicAdd(&ix.ctr[C_RETIRED_TOP], (unsigned long long)tr);
      if (at + tr <= ix.P)
        r = at;
      else
        atomicAdd(&ix.ctr[C_RETIRED_TOP], (unsigned long long)(-(long long)tr));
    }
    s_free = f;
    s_ret = r;
  }
  __syncthreads();
  SlabCursor c;
  if (n_alloc && s_free != ~0ull) {
    c.free_hi = s_free - pa;
    c.free_left = n_alloc;
  }
  if (n_retire && s_ret != ~0ull) {
    c.ret_next = s_ret + pr;
    c.ret_left = n_retire;
  }
  return c;
}

// after a wave's last item: reserved slots left unused go back to the pool
// (every reserved retired slot must name a slab), then the phase counter
__device__ inline void return_slabs(const Index& ix, SlabCursor& c) {
  const int l = lane_id();
  while (c.ret_left) {  // fill with an unused reserved slab, else a freshly popped one
    uint32_t s = NONE;
    if (c.free_left) {
      s = ix.free_stack[c.free_hi - 1];
      --c.free_hi;
      --c.free_left;
    } else {
      const uint64_t top = wave_atomic_add(&ix.ctr[C_FREE_TOP], ~0ull);
      if (top == 0 || top > ix.P) {
        wave_atomic_add(&ix.ctr[C_FREE_TOP], 1ull);
        if (l == 0) atomicOr(&ix.ctr[C_ERROR], (unsigned long long)ERR_POOL_EMPTY);
        break;
      }
      s = ix.free_stack[top - 1];
    }
    if (l == 0) ix.retired_stack[c.ret_next] = s;
    ++c.ret_next;
    --c.ret_left;
  }
  while (c.free_left) {  // popped but unused: retire, they rejoin the pool at the recycle
    const uint32_t s = ix.free_stack[c.free_hi - 1];
    --c.free_hi;
    --c.free_left;
    if (l == 0) retire_slab(ix, s);
  }
}
__device__ inline void finish_slabs(const Index& ix, SlabCursor& c, Counter which) {
  return_slabs(ix, c);
  if (c.pubs) wave_atomic_add(&ix.ctr[which], (unsigned long long)c.pubs);
  c.pubs = 0;
}

// finish_slabs for every wave of a workgroup (all of them call it): the
// publication count goes to the counter with one atomic per workgroup
__device__ inline void finish_slabs_block(const Index& ix, SlabCursor& c, Counter which) {
  __shared__ unsigned int s_pubs;
  return_slabs(ix, c);
  if (threadIdx.x == 0) s_pubs = 0;
  __syncthreads();
  if (lane_id() == 0 && c.pubs) atomicAdd(&s_pubs, c.pubs);
  c.pubs = 0;
  __syncthreads();
  if (threadIdx.x == 0 && s_pubs) atomicAdd(&ix.ctr[which], (unsigned long long)s_pubs);
}

// Copy-on-write publication of list (ids, d)[0..n) for node u by the whole
// wave: snapshot the reference, take a fresh slab, write it, fence, CAS the
// reference from the snapshot to <flag of snapshot, n, fresh slab>; on
// success retire the displaced slab, on failure retire the fresh one and
// retry, up to the attempt budget. Returns true when installed.
// A reference word no node can hold (degree 127): "not read yet".
constexpr uint64_t REF_UNREAD = ~0ull;

// snap0: u's reference word as the caller read it (REF_UNREAD: read it here);
// a failed compare-and-swap reads it afresh for the next attempt.
__device__ inline bool publish(const Index& ix, uint32_t u, const uint32_t* ids, const uint32_t* d, uint32_t n,
                               Counter which, SlabCursor* cur = nullptr, uint64_t snap0 = REF_UNREAD) {
  const int l = lane_id();
  const uint32_t R = ix.R;
  for (uint32_t attempt = 0; attempt < ix.publish_attempts; ++attempt) {
    const uint64_t snap = attempt == 0 && snap0 != REF_UNREAD ? snap0 : bcast64(load_ref(ix, u));
    uint32_t s = 0;
    if (cur && cur->free_left) {
      s = ix.free_stack[cur->free_hi - 1];
      --cur->free_hi;
      --cur->free_left;
    } else {
      if (l == 0) s = alloc_slab(ix);
      s = bcast(s);
    }
    if (s == NONE) return false;
    uint32_t* slab = ix.slabs + (size_t)s * 2u * R;
    for (uint32_t j = (uint32_t)l; j < R; j += 64) {
      slab[j] = j < n ? ids[j] : NONE;
      slab[R + j] = j < n ? d[j] : 0u;
    }
    // Slab contents before the reference that names them, for readers running
    // concurrently with the publication. In the round-synchronous launches no
    // wavefront reads a slab published by another one in the same launch
    // (the launch boundary orders them), so the fence is taken only when
    // concurrent readers are possible.
    if (ix.fence) __threadfence();
    uint32_t won = 0;
    const bool reserved_retire = cur && cur->ret_left && ref_slab(snap) != NONE;
    if (l == 0) {
      const uint64_t want = make_ref(ref_del(snap), n, s) | (snap & REF_NORM_MASK);  // flag and norm carried
      const uint64_t prev = atomicCAS(&ix.refs[u], (unsigned long long)snap, (unsigned long long)want);
      if (prev == snap) {
        won = 1;
        if (reserved_retire)
          ix.retired_stack[cur->ret_next] = ref_slab(snap);
        else if (ref_slab(snap) != NONE)
          retire_slab(ix, ref_slab(snap));
        if (!cur) atomicAdd(&ix.ctr[which], 1ull);
      } else {
        retire_slab(ix, s);
        atomicAdd(&ix.ctr[C_CAS_FAIL], 1ull);
      }
    }
    if (bcast(won)) {
      if (cur) {
        ++cur->pubs;
        if (reserved_retire) {
          ++cur->ret_next;
          --cur->ret_left;
        }
      }
      return true;
    }
  }
  if (l == 0) atomicAdd(&ix.ctr[C_PUB_DROPPED], 1ull);
  return false;
}

// One attempt of Algorithm 1 against an explicit snapshot `snap` of u's
// reference (the list was built from the slab that snapshot names): fresh
// slab, contents, release fence, CAS snap -> <flag of snap, n, fresh>. On
// success the displaced slab is retired; on failure the fresh one is, the
// failure is counted, and the caller rebuilds its list from a new snapshot.
// Whole wave; returns true when installed.
__device__ inline bool publish_once(const Index& ix, uint32_t u, uint64_t snap, const uint32_t* ids, const uint32_t* d,
                                    uint32_t n, Counter which) {
  const int l = lane_id();
  const uint32_t R = ix.R;
  uint32_t s = 0;
  if (l == 0) s = alloc_slab(ix);
  s = bcast(s);
  if (s == NONE) return false;
  uint32_t* slab = ix.slabs + (size_t)s * 2u * R;
  for (uint32_t j = (uint32_t)l; j < R; j += 64) {
    slab[j] = j < n ? ids[j] : NONE;
    slab[R + j] = j < n ? d[j] : 0u;
  }
  __threadfence();  // contents before the reference that names them
  uint32_t won = 0;
  if (l == 0) {
    const uint64_t want = make_ref(ref_del(snap), n, s) | (snap & REF_NORM_MASK);
    const uint64_t prev = atomicCAS(&ix.refs[u], (unsigned long long)snap, (unsigned long long)want);
    if (prev == snap) {
      won = 1;
      if (ref_slab(snap) != NONE) retire_slab(ix, ref_slab(snap));
      atomicAdd(&ix.ctr[which], 1ull);
    } else {
      retire_slab(ix, s);
      atomicAdd(&ix.ctr[C_CAS_FAIL], 1ull);
    }
  }
  return bcast(won) != 0;
}

// ---- RobustPrune (slack alpha), one wave -----------------------------------------
struct PruneLds {
  uint64_t* keys;   // [nsort]
  uint64_t* keys2;  // [rows] survivors in order
  uint8_t* vec;     // [rows * vstride] staged candidate vectors (uint8 rows)
  uint32_t* norm;   // [rows]
  uint32_t* idx;    // [rows] alive-candidate list (FP32 rows)
  uint8_t* kill;    // [rows] per-candidate prune flags (FP32 rows)
  uint32_t* out_ids;  // [R]
  uint32_t* out_d;    // [R] stored distances (uint32 for uint8 rows, FP32 bits for float)
  // matrix-core selection (uint8 rows; vec, norm and idx are then not carved):
  uint32_t* M;   // [64 * 63 / 2 + 1] distances between the candidates of one tile; null: staged rows
  uint32_t* tn;  // [64] shifted squared norms of the tile's candidates
  uint32_t* kn;  // [R] shifted squared norms of the kept candidates
  int nsort;
  int rows;  // keys2 (and, when staged, vec and norm) hold this many candidates
  int vstride;
};

__host__ __device__ inline int next_pow2_ge64(int n) {
  int p = 64;
  while (p < n) p <<= 1;
  return p;
}

// In-LDS bitonic sort of keys[0..np), np a power of two >= 64, by one wave.
__device__ inline void wave_bitonic_sort(uint64_t* keys, int np) {
  const int l = lane_id();
  for (int k = 2; k <= np; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = l; i < np; i += 64) {
        int p = i ^ j;
        if (p > i) {
          uint64_t a = keys[i], b = keys[p];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[p] = a;
          }
        }
      }
      wave_sync();
    }
  }
}

// RobustPrune_alpha(p, cand[0..n), R): drop p, tombstones and duplicates, order
// by (D(p,c), id), keep at most prune_cap, then select in order: keep c unless
// an already kept c' has a^2 * D(c', c) <= b^2 * D(p, c). Result (ids, D) in
// lds.out_ids / lds.out_d, in (D, id) order; returns its length.
// candidate tiles of 64 whose distances a prune's batched selection keeps in
// registers (up to 128 candidates; more take the one-at-a-time selection)
constexpr int PRUNE_TILES = 2;

// Steps 1-2 of RobustPrune on uint8 rows: the admissible candidates (not p,
// not flagged) by (D(p,c), id), duplicates dropped, at most prune_cap, into
// s.keys2; returns their count.
template <int G>
__device__ inline int prune_rank_u8(const Index& ix, uint32_t p, const uint32_t* cand, int n, PruneLds& s) {
  constexpr int VPP = 64 / G;
  const int l = lane_id();
  const int c = l % G, grp = l / G;
  const uint8_t* prow = ix.x + (size_t)p * ix.dim;
  const uint4 pf = load_frag<G>(prow);
  const uint32_t pp = group_sum<G>(dot16(pf, pf, 0u));
  const int np = next_pow2_ge64(n);
  // 1. keys (D(p,c), c) for admissible candidates; a candidate's row and its
  // reference word (for the flag) are read together
  for (int base = 0; base < np; base += 4 * VPP) {
    uint4 v[4];
    uint32_t id[4];
    uint64_t rf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int vi = base + u * VPP + grp;
      id[u] = vi < n ? cand[vi] : NONE;
      if (id[u] == p) id[u] = NONE;
      v[u] = make_uint4(0, 0, 0, 0);
      rf[u] = 0;
      if (id[u] != NONE) {
        rf[u] = load_ref(ix, id[u]);
        v[u] = reinterpret_cast<const uint4*>(ix.x + (size_t)id[u] * ix.dim)[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint32_t px = group_sum<G>(dot16(pf, v[u], 0u));
      uint32_t xx = group_sum<G>(dot16(v[u], v[u], 0u));
      int vi = base + u * VPP + grp;
      const bool none = id[u] == NONE || ref_del(rf[u]);
      if (c == 0 && vi < np) s.keys[vi] = none ? KEY_NONE : make_key(pp + xx - 2u * px, id[u]);
    }
  }
  wave_sync();
  wave_bitonic_sort(s.keys, np);
  // 2. drop duplicates (equal keys are adjacent) and compact
  int m = 0;
  for (int base = 0; base < np; base += 64) {
    int i = base + l;
    uint64_t k = s.keys[i];
    bool keep = k != KEY_NONE && (i == 0 || s.keys[i - 1] != k);
    uint64_t bm = ballot(keep);
    const int at = m + (int)lanes_below(bm);
    if (keep && at < s.rows) s.keys2[at] = k;
    m += __popcll(bm);
  }
  wave_sync();
  if (m > (int)ix.prune_cap) m = (int)ix.prune_cap;
  if (m > s.rows) m = s.rows;
  return m;
}

template <int G>
__device__ inline int robust_prune_u8(const Index& ix, uint32_t p, const uint32_t* cand, int n, PruneLds& s) {
  constexpr int VPP = 64 / G;
  const int l = lane_id();
  const int c = l % G, grp = l / G;
  const int m = prune_rank_u8<G>(ix, p, cand, n, s);
  // 3. stage the survivors' vectors (and norms) in LDS
  for (int base = 0; base < m; base += VPP) {
    int vi = base + grp;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (vi < m) v = reinterpret_cast<const uint4*>(ix.x + (size_t)key_id(s.keys2[vi]) * ix.dim)[c];
    uint32_t nn = group_sum<G>(dot16(v, v, 0u));
    if (vi < m) {
      *reinterpret_cast<uint4*>(s.vec + (size_t)vi * s.vstride + c * 16) = v;
      if (c == 0) s.norm[vi] = nn;
    }
  }
  wave_sync();
  // 4. ordered selection; lane l owns candidates l, l+64, ... The next four
  // live candidates are taken together: each lane computes its candidates'
  // distances to all four in one pass over its rows, then the four are
  // decided in order (one killed by an earlier one of the four is skipped), so
  // the kept set is that of the one-at-a-time selection.
  const int T = (m + 63) >> 6;
  uint32_t alive = 0;
  for (int t = 0; t < T; ++t)
    if (t * 64 + l < m) alive |= 1u << t;
  int cnt = 0, from = 0;
  const uint64_t a2 = ix.a2, b2 = ix.b2;
  const int words = (int)ix.dim / 16;
  if (T > PRUNE_TILES) {  // more candidates than the registers hold: one at a time
    while (cnt < (int)ix.R) {
      int j = -1;
      for (int t = from >> 6; t < T && j < 0; ++t) {
        uint64_t bm = ballot(((alive >> t) & 1u) && (t * 64 + l) >= from);
        if (bm) j = t * 64 + (int)__builtin_ctzll(bm);
      }
      if (j < 0) break;
      const uint64_t kj = s.keys2[j];
      if (l == 0) {
        s.out_ids[cnt] = key_id(kj);
        s.out_d[cnt] = key_dist(kj);
      }
      ++cnt;
      from = j + 1;
      if (cnt == (int)ix.R) break;
      const uint4* vj = reinterpret_cast<const uint4*>(s.vec + (size_t)j * s.vstride);
      const uint32_t nj = s.norm[j];
      for (int t = from >> 6; t < T; ++t) {
        int i = t * 64 + l;
        if (!((alive >> t) & 1u) || i < from) continue;
        const uint4* vi = reinterpret_cast<const uint4*>(s.vec + (size_t)i * s.vstride);
        uint32_t dot = 0;
        for (int w = 0; w < words; ++w) dot = dot16(vi[w], vj[w], dot);
        const uint64_t dji = (uint64_t)(nj + s.norm[i] - 2u * dot);
        const uint64_t dpi = (uint64_t)key_dist(s.keys2[i]);
        if (a2 * dji <= b2 * dpi) alive &= ~(1u << t);
      }
    }
    wave_sync();
    return cnt;
  }
  while (cnt < (int)ix.R) {
    int j[4] = {-1, -1, -1, -1};
    int nj4 = 0;
    for (int t = from >> 6; t < T && nj4 < 4; ++t) {
      uint64_t bm = ballot(((alive >> t) & 1u) && (t * 64 + l) >= from);
      while (bm && nj4 < 4) {
        j[nj4++] = t * 64 + (int)__builtin_ctzll(bm);
        bm &= bm - 1;
      }
    }
    if (nj4 == 0) break;
    // distances from this lane's later live candidates to the (up to) four
    uint32_t dk[4][PRUNE_TILES];
    uint32_t nk[4];
    const uint4* vk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int jj = j[k] >= 0 ? j[k] : j[0];
      vk[k] = reinterpret_cast<const uint4*>(s.vec + (size_t)jj * s.vstride);
      nk[k] = s.norm[jj];
    }
#pragma unroll
    for (int t = 0; t < PRUNE_TILES; ++t) {
      if (t >= T) break;
      const int i = t * 64 + l;
      uint32_t dot[4] = {0, 0, 0, 0};
      if (((alive >> t) & 1u) && i > j[0]) {
        const uint4* vi = reinterpret_cast<const uint4*>(s.vec + (size_t)i * s.vstride);
        for (int w = 0; w < words; ++w) {
          const uint4 x = vi[w];
#pragma unroll
          for (int k = 0; k < 4; ++k) dot[k] = dot16(x, vk[k][w], dot[k]);
        }
      }
      const uint32_t ni = i < m ? s.norm[i] : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) dk[k][t] = nk[k] + ni - 2u * dot[k];
    }
    // decide the four in order
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (j[k] < 0 || cnt >= (int)ix.R) break;
      const uint32_t owner = (uint32_t)__builtin_amdgcn_readlane((int)alive, j[k] & 63);
      if (!((owner >> (j[k] >> 6)) & 1u)) continue;  // killed by an earlier one of the four
      const uint64_t kj = s.keys2[j[k]];
      if (l == 0) {
        s.out_ids[cnt] = key_id(kj);
        s.out_d[cnt] = key_dist(kj);
      }
      ++cnt;
      if (cnt == (int)ix.R) break;
#pragma unroll
      for (int t = 0; t < PRUNE_TILES; ++t) {
        if (t >= T) break;
        const int i = t * 64 + l;
        if (!((alive >> t) & 1u) || i <= j[k]) continue;
        const uint64_t dpi = (uint64_t)key_dist(s.keys2[i]);
        if (a2 * (uint64_t)dk[k][t] <= b2 * dpi) alive &= ~(1u << t);
      }
    }
    // every candidate up to the last of the four is decided
    from = (j[3] >= 0 ? j[3] : (T * 64)) + 1;
    if (j[3] < 0) break;
  }
  wave_sync();
  return cnt;
}

}  // namespace etale
