// C-ABI of the ETALE index: argument checks, device memory, and the order of
// the phase launches of each call. Every numeric step runs in the kernels of
// etale_kernels.hip; this file only moves sizes, pointers and counters.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "etale.h"
#include "etale_dev.h"
#include "etale_launch.h"

using namespace etale;

struct etale_index {
  etale_config cfg;
  hipStream_t stream = nullptr;
  Index dev{};
  uint8_t* x = nullptr;
  float* xf = nullptr;
  uint16_t* xb = nullptr;
  uint8_t* x8 = nullptr;
  float* xs = nullptr;
  unsigned long long* refs = nullptr;
  uint32_t* slabs = nullptr;
  uint32_t* free_stack = nullptr;
  uint32_t* retired_stack = nullptr;
  unsigned long long* ctr = nullptr;
  uint32_t* entries = nullptr;
  uint8_t* ent_x = nullptr;     // uint8 rows: shifted copy of the entry set's rows, in operand order
  int32_t* ent_norm = nullptr;  // and minus their squared norms
  // call scratch
  uint64_t* vis_keys = nullptr;
  uint32_t* vis_cnt = nullptr;
  uint32_t* F = nullptr;
  uint64_t* pairs_a = nullptr;
  uint64_t* pairs_b = nullptr;
  uint32_t* dlist = nullptr;
  uint32_t* dirty = nullptr;
  uint64_t* bitmap = nullptr;
  uint32_t* seg = nullptr;        // run starts of a sorted pair list
  uint32_t* hist = nullptr;       // radix-sort digit counts
  int32_t* status = nullptr;      // round status words of the calls that do not take one
  uint32_t pair_bits = 0;         // bits of an id (the sort range of pair targets)
  bool no_chain = false;          // reverse edges without the cached candidate state
  bool no_mx = false;             // prunes select from staged rows even where the matrix cores could
  uint64_t* scan_keys = nullptr;  // [scan_chunk x 256] initial lists
  uint32_t* scan_n = nullptr;
  uint32_t* scan_dist = nullptr;  // [dist_cap] query x start-set distances
  uint64_t dist_cap = 0;
  uint32_t* scan_gmin = nullptr;  // [gmin_cap] per-query group minima of those distances
  uint64_t gmin_cap = 0;
  uint32_t* scan_bound = nullptr;  // [scan_chunk] per-query bounds (uint8 rows)
  uint32_t* scan_ncand = nullptr;  // [scan_chunk x 64 spans] keys at or below them per span
  uint64_t* scan_cand = nullptr;   // [scan_chunk x SCAN_KEYS_Q] those keys
  uint32_t scan_chunk = 0;
  uint64_t live = 0;
  int32_t qtrav = 0;              // query-side traversal copy
  uint32_t qrerank = 0;
  // opt-in stage timing of search calls: event quadruples per launch
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::array<hipEvent_t, 4>> ev_used;
  // captured rounds, keyed by the descriptor they were captured from
  hipStream_t cap_stream = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;
  uint64_t next_id = 0;           // host mirrors of C_NEXT_ID / C_LIVE, refreshed by read_counters
  uint32_t vcap_build = 0;
  uint64_t bytes = 0;
  bool poisoned = false;
  std::string err;
  std::vector<void*> allocs;
  unsigned char* noalloc = nullptr;  // device address of the static search scratch on the index's device
  uint32_t row_lanes = 0;            // uint8 rows: lanes per row in distance batches (0: dim / 16)
  // concurrent mode: searches on their own stream and scratch while rounds run
  bool concurrent = false;
  hipStream_t search_stream = nullptr;
  std::vector<void*> conc_bufs;
  struct {
    uint64_t* keys = nullptr;
    uint32_t *n = nullptr, *dist = nullptr, *gmin = nullptr, *bound = nullptr, *ncand = nullptr;
    uint64_t* cand = nullptr;
  } cs;
};

namespace {

etale_status fail(etale_index* ix, etale_status code, const std::string& what) {
  if (ix) {
    ix->err = what;
    if (code == ETALE_EDEVICE) ix->poisoned = true;
  }
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ix, ETALE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

// ---- scratch of the allocation-free search (etale_search_batch_noalloc) -------
// A file-scope device array: every device the library runs on holds its own
// copy until the process ends. Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): the address
// is resolved once per device with hipGetSymbolAddress and kept.
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;  // device ordinal -> address of `scratch` there

// address of `scratch` on the current device
hipError_t noalloc_scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_scratch_addr.emplace(dev, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

uint64_t round256(uint64_t b) { return (b + 255) & ~255ull; }

uint32_t pow2_ge64(uint32_t n) {
  uint32_t p = 64;
  while (p < n) p <<= 1;
  return p;
}

template <class T>
hipError_t dalloc(etale_index* ix, T** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
  if (e != hipSuccess) return e;
  ix->allocs.push_back(q);
  ix->bytes += bytes;
  *p = reinterpret_cast<T*>(q);
  return hipSuccess;
}

etale_status read_counters(etale_index* ix, unsigned long long* h) {
  HIP_TRY(hipMemcpyAsync(h, ix->ctr, C_NCOUNTERS * sizeof(unsigned long long), hipMemcpyDeviceToHost, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  if (h[C_ERROR]) {
    ix->poisoned = true;
    return fail(ix, ETALE_ESTATE, "device invariant violated, error bits " + std::to_string(h[C_ERROR]));
  }
  ix->next_id = h[C_NEXT_ID];
  ix->live = h[C_LIVE];
  return ETALE_OK;
}

etale_status refresh_mirror(etale_index* ix) {
  unsigned long long h[C_NCOUNTERS];
  return read_counters(ix, h);
}

// the round's status words, after the stream has drained
etale_status round_status(etale_index* ix, const char* what) {
  int32_t st[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(st, ix->status, sizeof(st), hipMemcpyDeviceToHost, ix->stream));
  if (etale_status e = refresh_mirror(ix)) return e;
  if (st[0] == ETALE_EPOOL) return fail(ix, ETALE_EPOOL, std::string(what) + ": slab pool cannot cover the worst case");
  if (st[0] == ETALE_ECAPACITY) return fail(ix, ETALE_ECAPACITY, std::string(what) + ": id space exhausted");
  if (st[0]) return fail(ix, ETALE_EINVAL, std::string(what) + ": rejected on the device");
  if (st[1] == ETALE_EPOOL) return fail(ix, ETALE_EPOOL, std::string(what) + ": slab pool cannot cover compaction");
  return ETALE_OK;
}

MaintArgs maint_args(const etale_index* ix, uint32_t nmax) {
  MaintArgs a{};
  a.vcap = ix->vcap_build;
  a.nmax = nmax;
  a.nsort = pow2_ge64(nmax);
  a.prune_cap = std::min(ix->cfg.prune_cap, nmax);
  a.vstride = ix->cfg.metric == ETALE_METRIC_L2_U8 ? ix->cfg.dim + 16 : 0;  // uint8 rows are staged in LDS
  a.lds_per_wave = maint_lds_per_wave(a, ix->cfg.R);
  return a;
}

// The prunes of a launch select on the matrix cores (no staged rows) where
// the rows allow it: uint8, at most 128 bytes (the tile's operands stay in
// registers), R <= 32.
void use_mx_prune(const etale_index* ix, MaintArgs& a) {
  if (ix->cfg.metric == ETALE_METRIC_L2_U8 && ix->cfg.dim <= 128 && ix->cfg.R <= 32 && !ix->no_mx) {
    a.mx = 1;
    a.lds_per_wave = maint_lds_per_wave(a, ix->cfg.R);
  }
}

// waves per search workgroup: the configured count, halved until the
// workgroup's LDS fits 64 KiB
uint32_t search_waves_per_block(const etale_index* ix, uint32_t lds_per_wave) {
  uint32_t w = ix->cfg.waves_per_block;
  while (w > 1 && (uint64_t)lds_per_wave * w > 65536u) w >>= 1;
  return w;
}

constexpr uint32_t SCAN_L_MAX = 256;

uint32_t maint_waves_per_block(const MaintArgs& a) {
  uint32_t w = 65536u / a.lds_per_wave;
  return w >= 4 ? 4 : (w >= 2 ? 2 : 1);
}

// queries per launch so that the distance matrix fits its scratch; a whole
// number of 64-query tiles (the uint8 group minima are stored by tile)
uint32_t scan_chunk_for(const etale_index* ix, uint32_t ns) {
  const uint64_t c = std::min<uint64_t>(ix->scan_chunk, ix->dist_cap / std::max(1u, ns));
  return (uint32_t)std::max<uint64_t>(1, c >= 64 ? c / 64 * 64 : c);
}

// group-minimum slots of a chunk of c queries over ns start rows: whole
// 64-query tiles of at most ns / 32 + 8 slots per query
uint64_t gmin_slots(uint64_t c, uint64_t ns) { return (c + 63) / 64 * 64 * (ns / 32 + 8); }

constexpr uint32_t BOOT_MAX = 16384;  // a bootstrap batch is scored as one start set

// Scratch of the start-set scan of one launch chunk: initial lists (out_stride
// L), the query x start-set distance rows, their group minima, bounds, span
// counts and bounded keys. `chunk` queries fit.
struct ScanScratch {
  uint64_t* keys = nullptr;
  uint32_t* n = nullptr;
  uint32_t* dist = nullptr;
  uint32_t* gmin = nullptr;
  uint32_t* bound = nullptr;
  uint32_t* ncand = nullptr;
  uint64_t* cand = nullptr;
  uint32_t chunk = 0;
};

// the library's own scratch, allocated at create
ScanScratch library_scratch(const etale_index* ix, uint32_t ns) {
  ScanScratch s;
  s.keys = ix->scan_keys;
  s.n = ix->scan_n;
  s.dist = ix->scan_dist;
  s.gmin = ix->scan_gmin;
  s.bound = ix->scan_bound;
  s.ncand = ix->scan_ncand;
  s.cand = ix->scan_cand;
  s.chunk = scan_chunk_for(ix, ns);
  return s;
}

// bytes of `scratch` that a chunk of c queries over ns start rows at list
// length L uses (every region 256-byte aligned)
uint64_t noalloc_bytes(uint64_t c, uint64_t ns, uint64_t L) {
  return round256(c * L * 8) + round256(c * 4) + round256(c * ns * 4) + round256(gmin_slots(c, ns) * 4) +
         round256(c * 4) + round256(c * 64 * 4) + round256(c * SCAN_KEYS_Q * 8);
}

// the largest chunk of queries that fits `scratch`, carved at base (0 if none fits)
ScanScratch noalloc_scratch(unsigned char* base, uint32_t ns, uint32_t L) {
  ScanScratch s;
  uint64_t c = std::min<uint64_t>(16384, NOALLOC_SCRATCH_BYTES / std::max<uint64_t>(1, noalloc_bytes(1, ns, L)));
  while (c > 0 && noalloc_bytes(c, ns, L) > NOALLOC_SCRATCH_BYTES) --c;
  if (c == 0) return s;
  unsigned char* p = base;
  auto take = [&](uint64_t bytes) {
    unsigned char* r = p;
    p += round256(bytes);
    return r;
  };
  s.keys = reinterpret_cast<uint64_t*>(take(c * L * 8));
  s.n = reinterpret_cast<uint32_t*>(take(c * 4));
  s.dist = reinterpret_cast<uint32_t*>(take(c * ns * 4));
  s.gmin = reinterpret_cast<uint32_t*>(take(gmin_slots(c, ns) * 4));
  s.bound = reinterpret_cast<uint32_t*>(take(c * 4));
  s.ncand = reinterpret_cast<uint32_t*>(take(c * 64 * 4));
  s.cand = reinterpret_cast<uint64_t*>(take(c * SCAN_KEYS_Q * 8));
  s.chunk = (uint32_t)c;
  return s;
}

// Start-set scoring, then the beam search, over up to nmax queries in chunks.
// `base` gives the launch-time count of the queries (and, for insert
// searches, the counter with the first new id) and the gate bits. With
// counts known only on the device (a replayed graph sized for its maximum),
// persistent search waves take queries from a work queue instead of one wave
// per possible query.
// `view` (default: the index itself) is the state the searches read, e.g. a
// serving snapshot; `stream` (default: the index's) is where they run.
etale_status run_searches(etale_index* ix, int mode, const uint8_t* q, uint64_t nmax, uint32_t k, uint32_t L,
                          uint32_t vcap, uint32_t* out_ids, uint32_t* out_d, uint32_t* counts, Dyn base,
                          bool persistent = false, const ScanScratch* given = nullptr, const Index* view = nullptr,
                          hipStream_t stream = nullptr) {
  const uint32_t ns = ix->cfg.n_entry;  // upper bound; the kernels read the entry count
  const ScanScratch scr = given ? *given : library_scratch(ix, ns);
  const uint32_t chunk = scr.chunk;
  const Index& dev = view ? *view : ix->dev;
  const hipStream_t st = view ? stream : ix->stream;
  const size_t qbytes = (size_t)ix->cfg.dim * (ix->cfg.metric == ETALE_METRIC_L2_U8 ? 1 : 4);
  for (uint64_t c = 0; c < nmax; c += chunk) {
    const uint32_t cn = (uint32_t)std::min<uint64_t>(chunk, nmax - c);
    Dyn d = base;
    d.c0 = (uint32_t)c;
    ScanArgs sc{};
    sc.mode = mode;
    sc.q = mode == MODE_QUERY ? q + c * qbytes : nullptr;
    sc.first = 0;
    sc.nq = cn;
    sc.L = L;
    sc.ns = ns;
    sc.ns_ctr = C_N_ENTRIES;
    sc.dist = scr.dist;
    sc.gmin = scr.gmin;
    sc.bound = scr.bound;
    sc.ncand = scr.ncand;
    sc.cand = scr.cand;
    sc.out_keys = scr.keys;
    sc.out_n = scr.n;
    sc.out_stride = L;
    sc.trav = mode == MODE_QUERY ? ix->qtrav : dev.trav;
    sc.d = d;
    std::array<hipEvent_t, 4> ev{};
    const bool timed = ix->timing && mode == MODE_QUERY && !given;
    if (timed) {
      for (auto& e : ev) {
        if (ix->ev_pool.empty()) {
          // timing only: without the system-scope fence, whose cache
          // write-back stalls the stream for microseconds at every stage
          hipEvent_t ne;
          HIP_TRY(hipEventCreateWithFlags(&ne, hipEventDisableSystemFence));
          ix->ev_pool.push_back(ne);
        }
        e = ix->ev_pool.back();
        ix->ev_pool.pop_back();
      }
      ix->ev_used.push_back(ev);
      HIP_TRY(hipEventRecord(ev[0], st));
    }
    HIP_TRY(launch_scan(dev, sc, st, timed ? ev[1] : nullptr));
    if (timed) HIP_TRY(hipEventRecord(ev[2], st));
    SearchArgs sa{};
    sa.mode = mode;
    sa.q = sc.q;
    sa.first = 0;
    sa.nq = cn;
    sa.L = L;
    sa.k = k;
    sa.vcap = vcap;
    sa.vt_mask = ix->cfg.vt_slots - 1;
    sa.W = ix->cfg.W;
    sa.lds_per_wave = search_lds_per_wave(L, ix->cfg.vt_slots, ix->cfg.W);
    sa.init_keys = scr.keys;
    sa.init_n = scr.n;
    sa.init_stride = L;
    sa.trav = sc.trav;
    sa.rerank = mode == MODE_QUERY ? ix->qrerank : 0;
    sa.d = d;
    sa.persistent = persistent ? 1u : 0u;
    sa.row_lanes = ix->row_lanes;
    if (mode == MODE_QUERY) {
      sa.out_ids = out_ids + c * k;
      sa.out_d = out_d + c * k;
      sa.counts = counts ? counts + 2 * c : nullptr;
    } else {
      sa.vis_keys = ix->vis_keys + c * vcap;
      sa.vis_cnt = ix->vis_cnt + c;
    }
    HIP_TRY(launch_search(dev, sa, search_waves_per_block(ix, sa.lds_per_wave), st));
    if (timed) HIP_TRY(hipEventRecord(ev[3], st));
  }
  return ETALE_OK;
}

// bootstrap: each new node's candidates are the vcap nearest other members
etale_status run_bootstrap(etale_index* ix, uint32_t nmax, uint32_t vcap, Dyn base) {
  const uint32_t ns = std::min(nmax, BOOT_MAX);
  const uint32_t chunk = scan_chunk_for(ix, ns);
  for (uint32_t c = 0; c < ns; c += chunk) {
    Dyn d = base;
    d.c0 = c;
    ScanArgs sc{};
    sc.mode = MODE_BOOT;
    sc.first = 0;
    sc.nq = std::min(chunk, ns - c);
    sc.L = vcap;
    sc.ns = ns;
    sc.ns_ctr = C_R_NINS;
    sc.dist = ix->scan_dist;
    sc.gmin = ix->scan_gmin;
    sc.bound = ix->scan_bound;
    sc.ncand = ix->scan_ncand;
    sc.cand = ix->scan_cand;
    sc.out_keys = ix->vis_keys + (size_t)c * vcap;
    sc.out_n = ix->vis_cnt + c;
    sc.out_stride = vcap;
    sc.qoff = c;
    sc.d = d;
    HIP_TRY(launch_scan(ix->dev, sc, ix->stream));
  }
  return ETALE_OK;
}

// A round's launches (Definition 2), sized by the plan's upper bounds; every
// kernel reads the actual counts from the counters the first kernel sets.
struct RoundPlan {
  uint32_t max_d = 0, max_i = 0, max_q = 0;
  const uint32_t* counts = nullptr;  // device [3]; null: the max_* values are the counts
  const uint32_t* del_ids = nullptr;
  uint8_t* del_status = nullptr;
  const void* vecs = nullptr;
  uint32_t* ids_out = nullptr;
  const void* q = nullptr;
  uint32_t k = 0, L = 0;
  uint32_t* q_ids = nullptr;
  uint32_t* q_d = nullptr;
  bool reclaim = false;
  int32_t* status = nullptr;
  int boot = -1;                     // 0 / 1 when the host knows it; -1: both variants, gated on the device
  uint64_t n_ids_max = 0;            // id bound of the reclaim scans
};

etale_status enqueue_reclaim(etale_index* ix, uint64_t n_ids_max, int32_t* status) {
  const Index& d = ix->dev;
  Dyn dn;
  dn.skip = G_FAIL;
  dn.n_ctr = C_NEXT_ID;
  HIP_TRY(launch_del_bitmap(d, n_ids_max, dn, ix->bitmap, ix->stream));
  HIP_TRY(launch_dirty(d, n_ids_max, dn, ix->bitmap, ix->dirty, ix->stream));
  HIP_TRY(launch_reclaim_gate(d, status, ix->stream));
  Dyn dc;
  dc.skip = G_FAIL | G_RFAIL;
  dc.n_ctr = C_DIRTY;
  HIP_TRY(launch_compact(d, ix->dirty, n_ids_max, dc, ix->bitmap, ix->stream));
  Dyn df;
  df.skip = G_FAIL | G_RFAIL;
  df.n_ctr = C_NEXT_ID;
  HIP_TRY(launch_free_tombstones(d, n_ids_max, df, ix->stream));
  if (!ix->concurrent) HIP_TRY(launch_recycle(d, ix->stream));
  return ETALE_OK;
}

etale_status enqueue_round(etale_index* ix, const RoundPlan& p) {
  const Index& d = ix->dev;
  const uint32_t R = ix->cfg.R;
  hipStream_t s = ix->stream;
  HIP_TRY(launch_round_begin(d, p.counts, p.counts ? 0 : p.max_d, p.counts ? 0 : p.max_i, p.counts ? 0 : p.max_q,
                             p.max_d, p.max_i, p.max_q, p.status, s));
  // P0: classify the deletes (sorted by id, first occurrence wins), then the gate
  if (p.max_d) {
    Dyn dd;
    dd.skip = G_FAIL;
    dd.n_ctr = C_R_NDEL;
    HIP_TRY(launch_del_keys(d, p.del_ids, p.max_d, dd, ix->pairs_a, s));
    uint64_t* sorted = nullptr;
    HIP_TRY(launch_sort(d, ix->pairs_a, ix->pairs_b, p.max_d, dd, 32, 32, ix->hist, s, &sorted));
    HIP_TRY(launch_del_classify(d, sorted, p.max_d, dd, p.del_status, ix->dlist, s));
  }
  HIP_TRY(launch_round_gate(d, ix->cfg.tombstone_only, BOOT_MAX, p.status, s));
  if (p.max_d) {
    Dyn dt;
    dt.skip = G_FAIL;
    dt.n_ctr = C_R_NDEL;  // dlist: the sorted deletes, NONE where not accepted
    HIP_TRY(launch_tombstone(d, ix->dlist, p.max_d, dt, s));
    Dyn dr;
    dr.skip = G_FAIL;
    dr.first_ctr = C_R_FIRST;  // this round's new ids are not live yet
    if (!ix->concurrent) HIP_TRY(launch_refresh_entries(d, 0, ix->cfg.n_entry, dr, s));
  }
  Dyn di;
  di.skip = G_FAIL;
  di.n_ctr = C_R_NINS;
  di.first_ctr = C_R_FIRST;
  const uint32_t vcap = ix->vcap_build;
  if (p.max_i) {
    HIP_TRY(launch_store_rows(d, p.vecs, p.ids_out, 0, p.max_i, di, s));
    if (ix->cfg.metric == ETALE_METRIC_L2_U8 && ix->cfg.dim <= 256) HIP_TRY(launch_row_norms(d, 0, p.max_i, di, s));
    if (ix->cfg.metric == ETALE_METRIC_IP_F32) HIP_TRY(launch_encode(d, 0, p.max_i, di, ix->xs, ix->xb, ix->x8, s));
    // P1: the insert searches on the state the tombstones left, or the bootstrap
    if (p.boot != 0) {
      Dyn db = di;
      db.skip = G_FAIL | G_NOBOOT;
      if (etale_status st = run_bootstrap(ix, p.max_i, vcap, db)) return st;
    }
    if (p.boot != 1) {
      Dyn ds = di;
      ds.skip = G_FAIL | G_BOOT;
      if (etale_status st = run_searches(ix, MODE_INSERT, nullptr, p.max_i, 0, ix->cfg.L_build, vcap, nullptr,
                                         nullptr, nullptr, ds, p.counts != nullptr))
        return st;
    }
  }
  // P1: the round's queries, on the same state
  if (p.max_q) {
    Dyn dq;
    dq.skip = G_FAIL;
    dq.n_ctr = C_R_NQ;
    if (etale_status st = run_searches(ix, MODE_QUERY, reinterpret_cast<const uint8_t*>(p.q), p.max_q, p.k, p.L,
                                       ix->cfg.visit_mult * p.L, p.q_ids, p.q_d, nullptr, dq, p.counts != nullptr))
      return st;
  }
  // P2: forward neighbors and the new node's own slab
  if (p.max_i) {
    MaintArgs fa = maint_args(ix, vcap);
    fa.n = p.max_i;
    fa.vis_keys = ix->vis_keys;
    fa.vis_cnt = ix->vis_cnt;
    fa.F = ix->F;
    fa.d = di;
    use_mx_prune(ix, fa);
    HIP_TRY(launch_maint(MK_FORWARD, d, fa, p.max_i, maint_waves_per_block(fa), s));
  }
  // P3: repair of the live out-neighbors of the deleted nodes, (a, u) order
  if (p.max_d && !ix->cfg.tombstone_only) {
    MaintArgs pa = maint_args(ix, 2 * R);
    pa.n = p.max_d;
    pa.dlist = ix->dlist;
    pa.pairs = ix->pairs_a;
    pa.d.skip = G_FAIL;
    pa.d.n_ctr = C_R_NDEL;
    HIP_TRY(launch_repair_pairs(d, pa, s));
    Dyn dp;
    dp.skip = G_FAIL;
    dp.n_ctr = C_R_NDEL;
    dp.n_mult = R;
    uint64_t* sorted = nullptr;
    // pairs are written in ascending source order (dlist keeps the sorted
    // deletes): the target half alone gives (target, source) order
    HIP_TRY(launch_sort(d, ix->pairs_a, ix->pairs_b, p.max_d * R, dp, 32, (int)ix->pair_bits, ix->hist, s, &sorted));
    HIP_TRY(launch_segments(d, sorted, p.max_d * R, dp, ix->seg, s));
    pa.pairs = sorted;
    pa.npairs = p.max_d * R;
    if (ix->cfg.metric == ETALE_METRIC_L2_U8 && R <= 32 && !ix->no_chain &&
        pool_lds_per_wave(pa.vstride) <= 65536u) {
      pa.chain = 1;
      pa.lds_per_wave = pool_lds_per_wave(pa.vstride);  // the pool kernel carves only the pool
    }
    pa.np_ctr = C_R_NDEL;
    pa.np_mult = R;
    pa.seg = ix->seg;
    HIP_TRY(launch_maint(MK_REPAIR, d, pa, pa.npairs, maint_waves_per_block(pa), s));
  }
  // P4: reverse edges in (target, source) order, one publication per target
  if (p.max_i) {
    MaintArgs fa = maint_args(ix, vcap);
    fa.n = p.max_i;
    fa.F = ix->F;
    fa.pairs = ix->pairs_a;
    fa.d = di;
    HIP_TRY(launch_reverse_pairs(d, fa, s));
    if (ix->concurrent) {
      // concurrent mode: every offer applied on its own, racing by CAS
      MaintArgs ra = maint_args(ix, R + 1);
      ra.n = p.max_i;
      ra.pairs = ix->pairs_a;
      ra.d = di;
      HIP_TRY(launch_maint(MK_REVERSE_FAST, d, ra, p.max_i * R, maint_waves_per_block(ra), s));
    } else {
    Dyn dp;
    dp.skip = G_FAIL;
    dp.n_ctr = C_R_NINS;
    dp.n_mult = R;
    uint64_t* sorted = nullptr;
    // pairs are written in ascending source order: the target half alone
    HIP_TRY(launch_sort(d, ix->pairs_a, ix->pairs_b, p.max_i * R, dp, 32, (int)ix->pair_bits, ix->hist, s, &sorted));
    HIP_TRY(launch_segments(d, sorted, p.max_i * R, dp, ix->seg, s));
    MaintArgs ra = maint_args(ix, R + 1);
    if (ix->cfg.metric == ETALE_METRIC_L2_U8 && R <= 32 && !ix->no_chain) {
      ra.chain = 1;
      // the chain kernel carves only the chain state; up to 128-byte rows it
      // reads rows from memory and stages none
      if (ix->cfg.dim <= 128) ra.vstride = 0;
      ra.lds_per_wave = chain_lds_per_wave(R, ra.vstride);
    }
    ra.n = p.max_i;
    ra.pairs = sorted;
    ra.npairs = p.max_i * R;
    ra.np_ctr = C_R_NINS;
    ra.np_mult = R;
    ra.seg = ix->seg;
    ra.d = di;
    HIP_TRY(launch_maint(MK_REVERSE, d, ra, ra.npairs, maint_waves_per_block(ra), s));
    }
    // P5: refine (not after a bootstrap)
    if (ix->cfg.refine && p.boot != 1) {
      MaintArgs ga = maint_args(ix, R + R * R);
      ga.n = p.max_i;
      ga.vis_keys = ix->vis_keys;  // free after P2: holds the refined lists until they are published
      ga.vis_cnt = ix->vis_cnt;
      ga.vcap = std::max(ga.vcap, R);
      ga.d = di;
      ga.d.skip = G_FAIL | G_BOOT;
      use_mx_prune(ix, ga);
      HIP_TRY(launch_maint(MK_REFINE, d, ga, p.max_i, maint_waves_per_block(ga), s));
    }
    Dyn de;
    de.skip = G_FAIL;
    de.first_ctr = C_NEXT_ID;
    if (!ix->concurrent) HIP_TRY(launch_refresh_entries(d, 0, ix->cfg.n_entry, de, s));
  }
  // end of the epoch (Lemma 1); in the concurrent mode searches may still read
  // what this round retired, so the recycle waits for the mode's end
  if (!ix->concurrent) HIP_TRY(launch_recycle(d, s));
  if (p.reclaim) return enqueue_reclaim(ix, p.n_ids_max, p.status);
  return ETALE_OK;
}

// Graph key: every descriptor field that is baked into the captured launches,
// and the query-side traversal settings.
std::string graph_key(const etale_round_desc& r, int32_t qtrav, uint32_t qrerank) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%p/%p/%u/%p/%p/%u/%p/%p/%p/%u/%u/%u/%p/%p/%d/%d/%u", (const void*)r.del_ids,
                (const void*)r.del_status, r.max_del, r.ins_vecs, (const void*)r.ins_ids, r.max_ins, r.queries,
                (const void*)r.q_ids, r.q_dists, r.max_q, r.k, r.L, (const void*)r.counts, (const void*)r.status,
                r.reclaim, qtrav, qrerank);
  return std::string(buf);
}

#define CHECK_HANDLE()                                       \
  do {                                                       \
    if (!ix) return ETALE_EINVAL;                            \
    if (ix->poisoned) return fail(ix, ETALE_ESTATE, "index poisoned by an earlier device error: " + ix->err); \
  } while (0)

}  // namespace

extern "C" {

etale_status etale_create(const etale_config* cfg, etale_t* out) {
  if (!cfg || !out) return ETALE_EINVAL;
  const etale_config& c = *cfg;
  if (c.metric == ETALE_METRIC_L2_U8) {
    if (!pow2(c.dim) || c.dim < 16 || c.dim > 1024) return ETALE_EINVAL;
  } else if (c.metric == ETALE_METRIC_IP_F32) {
    if (c.dim != 96 && c.dim != 192 && c.dim != 384 && c.dim != 768) return ETALE_EINVAL;
    if (c.traversal < ETALE_TRAV_NATIVE || c.traversal > ETALE_TRAV_FP8E4M3) return ETALE_EINVAL;
    if (c.rerank_mult > 64 || c.copies > 3) return ETALE_EINVAL;
  } else {
    return ETALE_EINVAL;
  }
  if (c.R < 1 || c.R > 64 || c.L_build < 1 || c.L_build > 256) return ETALE_EINVAL;
  if (c.alpha_num == 0 || c.alpha_den == 0 || c.alpha_num > 1000 || c.alpha_den > 1000) return ETALE_EINVAL;
  if (c.visit_mult < 1 || c.visit_mult * c.L_build > 4096) return ETALE_EINVAL;
  if (c.prune_cap < c.R || c.prune_cap > 2048) return ETALE_EINVAL;
  if (c.n_entry < 1 || c.n_entry > 16384) return ETALE_EINVAL;  // a start set is scored in registers
  if (c.publish_attempts < 1 || c.max_batch < 1) return ETALE_EINVAL;
  if ((c.W != 1 && c.W != 2 && c.W != 4) || (c.W > 1 && 2 * c.R > 64)) return ETALE_EINVAL;
  if (!pow2(c.vt_slots) || c.vt_slots < 64 || c.vt_slots > 16384) return ETALE_EINVAL;
  if (c.waves_per_block != 1 && c.waves_per_block != 2 && c.waves_per_block != 4) return ETALE_EINVAL;
  if (c.id_capacity < 1 || c.id_capacity >= 0xFFFFFFFFull || c.slab_capacity < 1 || c.slab_capacity >= 0xFFFFFFFFull)
    return ETALE_EINVAL;
  if ((uint64_t)c.max_batch > c.id_capacity) return ETALE_EINVAL;
  {
    // every kernel's LDS must fit one 64 KiB workgroup allocation
    etale_index probe;
    probe.cfg = c;
    probe.vcap_build = c.visit_mult * c.L_build;
    const uint32_t worst_nmax[] = {probe.vcap_build, c.R + 1, 2 * c.R, c.R + c.R * c.R};
    for (uint32_t nm : worst_nmax)
      if (maint_args(&probe, nm).lds_per_wave > 65536u) return ETALE_EINVAL;
    if (search_lds_per_wave(SCAN_L_MAX, c.vt_slots, c.W) > 65536u) return ETALE_EINVAL;
    if (4 * scan_select_lds_per_wave(std::max(SCAN_L_MAX, probe.vcap_build)) > 65536u) return ETALE_EINVAL;
  }

  etale_index* ix = new etale_index();
  ix->cfg = c;
  ix->stream = reinterpret_cast<hipStream_t>(c.hip_stream);
  ix->vcap_build = c.visit_mult * c.L_build;
  const uint64_t C = c.id_capacity, P = c.slab_capacity, B = c.max_batch, R = c.R;
  auto cleanup = [&](etale_status st, const std::string& why) {
    for (void* p : ix->allocs) (void)hipFree(p);
    delete ix;
    (void)why;
    return st;
  };
#define ALLOC(ptr, bytes)                                          \
  if (dalloc(ix, &(ptr), (bytes)) != hipSuccess) return cleanup(ETALE_ENOMEM, "hipMalloc");
  if (c.metric == ETALE_METRIC_L2_U8) {
    ALLOC(ix->x, C * c.dim);
  } else {
    ALLOC(ix->xf, C * c.dim * 4);
    if (c.traversal == ETALE_TRAV_BF16 || (c.copies & 1)) ALLOC(ix->xb, C * c.dim * 2);
    if (c.traversal == ETALE_TRAV_FP8E4M3 || (c.copies & 2)) {
      ALLOC(ix->x8, C * c.dim);
      ALLOC(ix->xs, C * 4);
    }
  }
  ALLOC(ix->refs, C * 8);
  ALLOC(ix->slabs, P * 2 * R * 4);
  ALLOC(ix->free_stack, P * 4);
  ALLOC(ix->retired_stack, P * 4);
  ALLOC(ix->ctr, CTR_WORDS * 8);
  ALLOC(ix->entries, (uint64_t)c.n_entry * 4);
  if (c.metric == ETALE_METRIC_L2_U8) {
    ALLOC(ix->ent_x, ent_copy_bytes(c.n_entry, c.dim));
    ALLOC(ix->ent_norm, ((uint64_t)c.n_entry + 63) / 64 * 64 * 4);
  }
  ALLOC(ix->vis_keys, B * std::max<uint64_t>(ix->vcap_build, R) * 8);  // also the refined lists (R per node)
  ALLOC(ix->vis_cnt, B * 4);
  ALLOC(ix->F, B * R * 4);
  ALLOC(ix->pairs_a, B * R * 8);
  ALLOC(ix->pairs_b, B * R * 8);
  ALLOC(ix->dlist, B * 4);
  ALLOC(ix->dirty, C * 4);
  ALLOC(ix->bitmap, ((C + 63) / 64) * 8);
  ix->scan_chunk = 16384;
  ALLOC(ix->scan_keys, (uint64_t)ix->scan_chunk * SCAN_L_MAX * 8);
  ALLOC(ix->scan_n, (uint64_t)ix->scan_chunk * 4);
  ix->dist_cap = std::min<uint64_t>(1ull << 27, std::max<uint64_t>((uint64_t)ix->scan_chunk * c.n_entry, B * 4096));
  ALLOC(ix->scan_dist, ix->dist_cap * 4);
  // a chunk of n queries (a multiple of 64) over ns start rows has at most
  // n (ns / 32 + 8) group slots
  ix->gmin_cap = ix->dist_cap / 32 + 8ull * ix->scan_chunk;
  ALLOC(ix->scan_gmin, ix->gmin_cap * 4);
  ALLOC(ix->scan_bound, (uint64_t)ix->scan_chunk * 4);
  ALLOC(ix->scan_ncand, (uint64_t)ix->scan_chunk * 64 * 4);
  ALLOC(ix->scan_cand, (uint64_t)ix->scan_chunk * SCAN_KEYS_Q * 8);
  ALLOC(ix->seg, B * R * 4);
  ALLOC(ix->hist, (uint64_t)sort_hist_words((uint32_t)(B * R)) * 4);
  ALLOC(ix->status, 16);
#undef ALLOC
  Index& d = ix->dev;
  d.dim = c.dim;
  d.R = c.R;
  d.a2 = c.alpha_num * c.alpha_num;
  d.b2 = c.alpha_den * c.alpha_den;
  {
    const uint64_t dmax = (uint64_t)c.dim * 255u * 255u;  // largest uint8 squared distance
    d.cmp32 = c.metric == ETALE_METRIC_L2_U8 && dmax < (1ull << 24) && d.a2 < (1u << 24) && d.b2 < (1u << 24) &&
              (uint64_t)std::max(d.a2, d.b2) * dmax < (1ull << 32);
  }
  d.publish_attempts = c.publish_attempts;
  d.fence = 0;  // every call is a round-synchronous launch sequence
  d.concurrent = 0;
  d.prune_cap = c.prune_cap;
  d.metric = c.metric;
  d.trav = c.metric == ETALE_METRIC_IP_F32 ? c.traversal : 0;
  d.rerank = c.rerank_mult;
  ix->qtrav = d.trav;
  ix->qrerank = c.rerank_mult;
  d.cap = C;
  d.P = P;
  d.x = ix->x;
  d.xf = ix->xf;
  d.xb = ix->xb;
  d.x8 = ix->x8;
  d.xs = ix->xs;
  d.refs = ix->refs;
  d.slabs = ix->slabs;
  d.free_stack = ix->free_stack;
  d.retired_stack = ix->retired_stack;
  d.ctr = ix->ctr;
  d.entries = ix->entries;
  d.ent_x = ix->ent_x;
  d.ent_norm = ix->ent_norm;
  ix->pair_bits = 1;
  while ((1ull << ix->pair_bits) <= C) ++ix->pair_bits;  // every id < 2^bits - 1: a KEY_NONE target sorts last
  if (launch_init(d, ix->stream) != hipSuccess || hipStreamSynchronize(ix->stream) != hipSuccess)
    return cleanup(ETALE_EDEVICE, "init");
  if (noalloc_scratch_address(&ix->noalloc) != hipSuccess) return cleanup(ETALE_EDEVICE, "scratch symbol");
  *out = ix;
  return ETALE_OK;
}

etale_status etale_destroy(etale_t ix) {
  if (!ix) return ETALE_OK;
  (void)hipStreamSynchronize(ix->stream);
  for (auto& g : ix->graphs) (void)hipGraphExecDestroy(g.second);
  if (ix->cap_stream) (void)hipStreamDestroy(ix->cap_stream);
  for (auto& q : ix->ev_used)
    for (hipEvent_t e : q) (void)hipEventDestroy(e);
  for (hipEvent_t e : ix->ev_pool) (void)hipEventDestroy(e);
  for (void* p : ix->allocs) (void)hipFree(p);
  for (void* p : ix->conc_bufs) (void)hipFree(p);
  delete ix;
  return ETALE_OK;
}

etale_status etale_set_stream(etale_t ix, void* stream) {
  if (!ix) return ETALE_EINVAL;
  ix->stream = reinterpret_cast<hipStream_t>(stream);
  return ETALE_OK;
}

etale_status etale_insert_batch(etale_t ix, const void* vecs_dev, uint64_t n, uint32_t* ids_out_dev) {
  CHECK_HANDLE();
  if (n == 0) return ETALE_OK;
  if (!vecs_dev || n > ix->cfg.max_batch) return fail(ix, ETALE_EINVAL, "insert: null vectors or n > max_batch");
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  if (!ix->concurrent && h[C_N_ENTRIES] != std::min<uint64_t>(ix->cfg.n_entry, h[C_LIVE])) {  // frozen in that mode
    ix->poisoned = true;
    return fail(ix, ETALE_ESTATE, "entry-set size on the device disagrees with the live count");
  }
  if (h[C_NEXT_ID] + n > ix->cfg.id_capacity) return fail(ix, ETALE_ECAPACITY, "insert: id space exhausted");
  if (h[C_FREE_TOP] < n * (uint64_t)(ix->cfg.R + 2))
    return fail(ix, ETALE_EPOOL, "insert: slab pool cannot cover n*(R+2)");
  const bool bootstrap = h[C_LIVE] == 0;
  if (bootstrap && n > BOOT_MAX) return fail(ix, ETALE_EINVAL, "insert: a bootstrap batch holds at most 16384 vectors");
  RoundPlan p;
  p.max_i = (uint32_t)n;
  p.vecs = vecs_dev;
  p.ids_out = ids_out_dev;
  p.status = ix->status;
  p.boot = bootstrap ? 1 : 0;
  return enqueue_round(ix, p);
}

etale_status etale_delete_batch(etale_t ix, const uint32_t* ids_dev, uint64_t n, uint8_t* status_out_dev) {
  CHECK_HANDLE();
  if (n == 0) return ETALE_OK;
  if (!ids_dev || n > ix->cfg.max_batch) return fail(ix, ETALE_EINVAL, "delete: null ids or n > max_batch");
  RoundPlan p;
  p.max_d = (uint32_t)n;
  p.del_ids = ids_dev;
  p.del_status = status_out_dev;
  p.status = ix->status;
  if (etale_status st = enqueue_round(ix, p)) return st;
  return round_status(ix, "delete");  // the pool check ran on the device, before any change
}

etale_status etale_search_batch(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                                uint32_t* ids_out_dev, void* dists_out_dev, uint32_t* counts_out_dev) {
  CHECK_HANDLE();
  if (k < 1 || k > L || L > 256) return fail(ix, ETALE_EINVAL, "search: need 1 <= k <= L <= 256");
  if (nq == 0) return ETALE_OK;
  if (!q_dev || !ids_out_dev || !dists_out_dev || nq > 0xFFFFFFFFull)
    return fail(ix, ETALE_EINVAL, "search: null buffer");
  if (ix->cfg.metric == ETALE_METRIC_IP_F32 && ix->qtrav != ETALE_TRAV_NATIVE && (uint64_t)ix->qrerank * k > 64)
    return fail(ix, ETALE_EINVAL, "search: rerank_mult * k must not exceed 64");
  if (ix->concurrent) {  // alongside the rounds: own stream, own scratch, the live state
    ScanScratch cs;
    cs.keys = ix->cs.keys;
    cs.n = ix->cs.n;
    cs.dist = ix->cs.dist;
    cs.gmin = ix->cs.gmin;
    cs.bound = ix->cs.bound;
    cs.ncand = ix->cs.ncand;
    cs.cand = ix->cs.cand;
    cs.chunk = scan_chunk_for(ix, ix->cfg.n_entry);
    return run_searches(ix, MODE_QUERY, reinterpret_cast<const uint8_t*>(q_dev), nq, k, L, ix->cfg.visit_mult * L,
                        ids_out_dev, reinterpret_cast<uint32_t*>(dists_out_dev), counts_out_dev, Dyn{}, false, &cs,
                        &ix->dev, ix->search_stream);
  }
  return run_searches(ix, MODE_QUERY, reinterpret_cast<const uint8_t*>(q_dev), nq, k, L, ix->cfg.visit_mult * L,
                      ids_out_dev, reinterpret_cast<uint32_t*>(dists_out_dev), counts_out_dev, Dyn{});
}

etale_status etale_search_batch_noalloc(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                                        uint32_t* ids_out_dev, void* dists_out_dev, uint32_t* counts_out_dev) {
  CHECK_HANDLE();
  if (k < 1 || k > L || L > 256) return fail(ix, ETALE_EINVAL, "search_noalloc: need 1 <= k <= L <= 256");
  if (nq == 0) return ETALE_OK;
  if (!q_dev || !ids_out_dev || !dists_out_dev || nq > 0xFFFFFFFFull)
    return fail(ix, ETALE_EINVAL, "search_noalloc: null buffer");
  if (ix->cfg.metric == ETALE_METRIC_IP_F32 && ix->qtrav != ETALE_TRAV_NATIVE && (uint64_t)ix->qrerank * k > 64)
    return fail(ix, ETALE_EINVAL, "search_noalloc: rerank_mult * k must not exceed 64");
  if (!ix->noalloc) return fail(ix, ETALE_ESTATE, "search_noalloc: static scratch not resolved");
  const ScanScratch scr = noalloc_scratch(ix->noalloc, ix->cfg.n_entry, L);
  if (scr.chunk == 0)
    return fail(ix, ETALE_EINVAL, "search_noalloc: one query's start-set scratch (n_entry, L) exceeds the " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES >> 20) + " MiB static scratch");
  return run_searches(ix, MODE_QUERY, reinterpret_cast<const uint8_t*>(q_dev), nq, k, L, ix->cfg.visit_mult * L,
                      ids_out_dev, reinterpret_cast<uint32_t*>(dists_out_dev), counts_out_dev, Dyn{}, false, &scr);
}

etale_status etale_reclaim(etale_t ix) {
  CHECK_HANDLE();
  if (ix->cfg.tombstone_only) return ETALE_OK;
  if (etale_status st = refresh_mirror(ix)) return st;
  HIP_TRY(launch_round_begin(ix->dev, nullptr, 0, 0, 0, 0, 0, 0, ix->status, ix->stream));
  if (etale_status st = enqueue_reclaim(ix, ix->next_id, ix->status)) return st;
  return round_status(ix, "reclaim");
}

etale_status etale_round(etale_t ix, const etale_round_desc* r) {
  CHECK_HANDLE();
  if (!r || !r->status) return fail(ix, ETALE_EINVAL, "round: null descriptor or status");
  const etale_round_desc& d = *r;
  if (d.max_del > ix->cfg.max_batch || d.max_ins > ix->cfg.max_batch)
    return fail(ix, ETALE_EINVAL, "round: max_del / max_ins above max_batch");
  if ((d.max_del && !d.del_ids) || (d.max_ins && !d.ins_vecs) || (d.max_q && (!d.queries || !d.q_ids || !d.q_dists)))
    return fail(ix, ETALE_EINVAL, "round: null buffer");
  if (d.max_q && (d.k < 1 || d.k > d.L || d.L > 256)) return fail(ix, ETALE_EINVAL, "round: need 1 <= k <= L <= 256");
  if (d.max_q && ix->cfg.metric == ETALE_METRIC_IP_F32 && ix->qtrav != ETALE_TRAV_NATIVE &&
      (uint64_t)ix->qrerank * d.k > 64)
    return fail(ix, ETALE_EINVAL, "round: rerank_mult * k must not exceed 64");
  RoundPlan p;
  p.max_d = d.max_del;
  p.max_i = d.max_ins;
  p.max_q = d.max_q;
  p.counts = d.counts;
  p.del_ids = d.del_ids;
  p.del_status = d.del_status;
  p.vecs = d.ins_vecs;
  p.ids_out = d.ins_ids;
  p.q = d.queries;
  p.k = d.k;
  p.L = d.L;
  p.q_ids = d.q_ids;
  p.q_d = reinterpret_cast<uint32_t*>(d.q_dists);
  p.reclaim = d.reclaim != 0 && !ix->cfg.tombstone_only;
  p.status = d.status;
  p.n_ids_max = ix->cfg.id_capacity;  // the id count is only known on the device
  if (!d.graph) return enqueue_round(ix, p);
  // capture once per descriptor, replay afterwards
  const std::string key = graph_key(d, ix->qtrav, ix->qrerank) + "/" + std::to_string(ix->cfg.waves_per_block) +
                          "/" + std::to_string(ix->cfg.vt_slots) + "/" + std::to_string(ix->row_lanes);
  auto it = ix->graphs.find(key);
  if (it == ix->graphs.end()) {
    if (!ix->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ix->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = ix->stream;
    const bool timing = ix->timing;
    ix->timing = false;
    ix->stream = ix->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(ix->cap_stream, hipStreamCaptureModeThreadLocal);
    etale_status st = ETALE_OK;
    if (e == hipSuccess) st = enqueue_round(ix, p);
    const hipError_t e2 = hipStreamEndCapture(ix->cap_stream, &g);
    ix->stream = user;
    ix->timing = timing;
    if (st) return st;
    HIP_TRY(e);
    HIP_TRY(e2);
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e3);
    it = ix->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, ix->stream));
  return ETALE_OK;
}

etale_status etale_bruteforce(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t* ids_out_dev,
                              void* dists_out_dev) {
  CHECK_HANDLE();
  if (k < 1 || k > 16 || nq > 0xFFFFFFFFull) return fail(ix, ETALE_EINVAL, "bruteforce: need 1 <= k <= 16");
  if (nq == 0) return ETALE_OK;
  if (etale_status st = refresh_mirror(ix)) return st;
  if (!q_dev || !ids_out_dev || !dists_out_dev) return fail(ix, ETALE_EINVAL, "bruteforce: null buffer");
  const uint64_t sb = bruteforce_scratch_bytes(ix->dev, (uint32_t)nq, ix->next_id);
  unsigned char* scr = nullptr;
  if (sb && hipMallocAsync(reinterpret_cast<void**>(&scr), sb, ix->stream) != hipSuccess) {
    scr = nullptr;  // no scratch: the one-wave-per-query kernel
    (void)hipGetLastError();
  }
  const hipError_t e = launch_bruteforce(ix->dev, q_dev, (uint32_t)nq, ix->next_id, k, ids_out_dev,
                                         reinterpret_cast<uint32_t*>(dists_out_dev), ix->stream, scr);
  if (scr) (void)hipFreeAsync(scr, ix->stream);
  HIP_TRY(e);
  return ETALE_OK;
}

etale_status etale_get_stats(etale_t ix, etale_stats* out) {
  if (!ix || !out) return ETALE_EINVAL;
  unsigned long long h[C_NCOUNTERS];
  HIP_TRY(hipMemcpyAsync(h, ix->ctr, sizeof(h), hipMemcpyDeviceToHost, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  etale_stats s{};
  s.next_id = h[C_NEXT_ID];
  s.live = h[C_LIVE];
  s.tombstones = h[C_TOMBSTONED] - h[C_FREED];
  s.slab_capacity = ix->cfg.slab_capacity;
  s.free_slabs = h[C_FREE_TOP];
  s.resident_slabs = ix->cfg.slab_capacity - h[C_FREE_TOP] - h[C_RETIRED_TOP];
  s.n_entries = h[C_N_ENTRIES];
  s.pub_forward = h[C_PUB_FORWARD];
  s.pub_repair = h[C_PUB_REPAIR];
  s.pub_reverse = h[C_PUB_REVERSE];
  s.pub_refine = h[C_PUB_REFINE];
  s.pub_compact = h[C_PUB_COMPACT];
  s.freed = h[C_FREED];
  s.dirty_last = h[C_DIRTY];
  s.dead_edges_last = h[C_DEAD];
  s.search_expansions = h[C_SEARCH_EXP];
  s.search_distances = h[C_SEARCH_DIST];
  s.cas_failures = h[C_CAS_FAIL];
  s.publish_dropped = h[C_PUB_DROPPED];
  s.device_bytes = ix->bytes;
  s.error_bits = h[C_ERROR];
  *out = s;
  return ETALE_OK;
}

etale_status etale_export(etale_t ix, uint64_t n_ids, uint32_t* nbr_host, void* dist_host, uint8_t* deg_host,
                          uint8_t* del_host, uint8_t* has_slab_host) {
  CHECK_HANDLE();
  if (etale_status st = refresh_mirror(ix)) return st;
  if (n_ids > ix->next_id) return fail(ix, ETALE_EINVAL, "export: n_ids > next id");
  if (n_ids == 0) return ETALE_OK;
  const uint64_t R = ix->cfg.R;
  uint32_t *nbr = nullptr, *rho = nullptr;
  uint8_t* flags = nullptr;
  HIP_TRY(hipMalloc(&nbr, n_ids * R * 4));
  HIP_TRY(hipMalloc(&rho, n_ids * R * 4));
  HIP_TRY(hipMalloc(&flags, n_ids * 3));
  hipError_t e = launch_export(ix->dev, n_ids, nbr, rho, flags, flags + n_ids, flags + 2 * n_ids, ix->stream);
  if (e == hipSuccess && nbr_host) e = hipMemcpyAsync(nbr_host, nbr, n_ids * R * 4, hipMemcpyDeviceToHost, ix->stream);
  if (e == hipSuccess && dist_host) e = hipMemcpyAsync(dist_host, rho, n_ids * R * 4, hipMemcpyDeviceToHost, ix->stream);
  if (e == hipSuccess && deg_host) e = hipMemcpyAsync(deg_host, flags, n_ids, hipMemcpyDeviceToHost, ix->stream);
  if (e == hipSuccess && del_host) e = hipMemcpyAsync(del_host, flags + n_ids, n_ids, hipMemcpyDeviceToHost, ix->stream);
  if (e == hipSuccess && has_slab_host)
    e = hipMemcpyAsync(has_slab_host, flags + 2 * n_ids, n_ids, hipMemcpyDeviceToHost, ix->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ix->stream);
  (void)hipFree(nbr);
  (void)hipFree(rho);
  (void)hipFree(flags);
  HIP_TRY(e);
  return ETALE_OK;
}

etale_status etale_get_entries(etale_t ix, uint32_t* ids_host, uint64_t cap, uint64_t* n_out) {
  CHECK_HANDLE();
  if (!ids_host || !n_out) return ETALE_EINVAL;
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  const uint64_t n = std::min<uint64_t>(h[C_N_ENTRIES], cap);
  if (n) {
    HIP_TRY(hipMemcpyAsync(ids_host, ix->entries, n * 4, hipMemcpyDeviceToHost, ix->stream));
    HIP_TRY(hipStreamSynchronize(ix->stream));
  }
  *n_out = h[C_N_ENTRIES];
  return ETALE_OK;
}

etale_status etale_set_query_traversal(etale_t ix, int32_t traversal, uint32_t rerank_mult) {
  CHECK_HANDLE();
  if (ix->cfg.metric != ETALE_METRIC_IP_F32) return fail(ix, ETALE_EINVAL, "query traversal: float metric only");
  const bool kept = traversal == ETALE_TRAV_NATIVE || (traversal == ETALE_TRAV_BF16 && ix->xb) ||
                    (traversal == ETALE_TRAV_FP8E4M3 && ix->x8);
  if (!kept || rerank_mult > 64) return fail(ix, ETALE_EINVAL, "query traversal: copy not kept or bad multiplier");
  ix->qtrav = traversal;
  ix->qrerank = rerank_mult;
  return ETALE_OK;
}

etale_status etale_set_lists(etale_t ix, uint64_t n, const uint32_t* ids_host, const uint32_t* nbr_host,
                             const uint32_t* deg_host) {
  CHECK_HANDLE();
  if (n == 0) return ETALE_OK;
  if (!ids_host || !nbr_host || !deg_host) return fail(ix, ETALE_EINVAL, "set_lists: null buffer");
  if (etale_status st = refresh_mirror(ix)) return st;
  const uint32_t R = ix->cfg.R;
  std::vector<uint8_t> seen(ix->next_id, 0);
  for (uint64_t i = 0; i < n; ++i) {
    if (ids_host[i] >= ix->next_id || deg_host[i] > R || seen[ids_host[i]])
      return fail(ix, ETALE_EINVAL, "set_lists: bad id, repeated id or degree");
    seen[ids_host[i]] = 1;
    for (uint32_t j = 0; j < deg_host[i]; ++j) {
      const uint32_t v = nbr_host[i * R + j];
      if (v >= ix->next_id || v == ids_host[i]) return fail(ix, ETALE_EINVAL, "set_lists: bad neighbor");
      for (uint32_t t = 0; t < j; ++t)
        if (nbr_host[i * R + t] == v) return fail(ix, ETALE_EINVAL, "set_lists: repeated neighbor");
    }
  }
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  if (h[C_FREE_TOP] < n) return fail(ix, ETALE_EPOOL, "set_lists: slab pool cannot cover n publications");
  // every listed id must be live
  std::vector<unsigned long long> refs(ix->next_id);
  HIP_TRY(hipMemcpyAsync(refs.data(), ix->refs, ix->next_id * 8, hipMemcpyDeviceToHost, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  for (uint64_t i = 0; i < n; ++i)
    if (ref_del(refs[ids_host[i]])) return fail(ix, ETALE_EINVAL, "set_lists: id not live");
  uint32_t *d_ids = nullptr, *d_nbr = nullptr, *d_deg = nullptr;
  HIP_TRY(hipMalloc(&d_ids, n * 4));
  HIP_TRY(hipMalloc(&d_nbr, n * R * 4));
  HIP_TRY(hipMalloc(&d_deg, n * 4));
  hipError_t e = hipMemcpy(d_ids, ids_host, n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_nbr, nbr_host, n * R * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_deg, deg_host, n * 4, hipMemcpyHostToDevice);
  MaintArgs a = maint_args(ix, R + 1);
  a.n = (uint32_t)n;
  if (e == hipSuccess) e = launch_set_lists(ix->dev, a, d_ids, d_nbr, d_deg, ix->stream);
  if (e == hipSuccess) e = launch_recycle(ix->dev, ix->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ix->stream);
  (void)hipFree(d_ids);
  (void)hipFree(d_nbr);
  (void)hipFree(d_deg);
  HIP_TRY(e);
  return ETALE_OK;
}

etale_status etale_export_rows(etale_t ix, uint64_t first, uint64_t n, int32_t which, void* out_host) {
  CHECK_HANDLE();
  if (etale_status st = refresh_mirror(ix)) return st;
  if (!out_host || first + n > ix->next_id) return fail(ix, ETALE_EINVAL, "export_rows: range");
  const uint64_t dim = ix->cfg.dim;
  const void* src = nullptr;
  uint64_t row_bytes = 0;
  switch (which) {
    case 0:
      src = ix->cfg.metric == ETALE_METRIC_L2_U8 ? (const void*)ix->x : (const void*)ix->xf;
      row_bytes = ix->cfg.metric == ETALE_METRIC_L2_U8 ? dim : dim * 4;
      break;
    case 1: src = ix->xb; row_bytes = dim * 2; break;
    case 2: src = ix->x8; row_bytes = dim; break;
    case 3: src = ix->xs; row_bytes = 4; break;
    default: break;
  }
  if (!src) return fail(ix, ETALE_EINVAL, "export_rows: copy not kept");
  if (n == 0) return ETALE_OK;
  HIP_TRY(hipMemcpyAsync(out_host, (const uint8_t*)src + first * row_bytes, n * row_bytes, hipMemcpyDeviceToHost,
                         ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return ETALE_OK;
}

namespace {
uint32_t size_bucket(uint32_t n, uint32_t floor, uint32_t cap) {
  if (n == 0) return 0;
  uint32_t b = floor;
  while (b < n) b <<= 1;
  return b < cap ? b : cap;
}

// One of the two tick slots of the serving loop: device inputs and outputs,
// pinned host staging, the events that mark the tick's stages, and what the
// host needs to finish the tick when they have passed.
struct TickSlot {
  uint32_t *d_idx = nullptr, *d_qids = nullptr, *d_qd = nullptr, *d_counts = nullptr, *d_ids = nullptr;
  uint32_t* d_pos = nullptr;  // request index of each search of the tick
  uint8_t *d_vecs = nullptr, *d_q = nullptr, *d_dst = nullptr;
  int32_t* d_status = nullptr;
  uint32_t* h_idx = nullptr;  // [3T + 4]: delete ids, insert rows, query rows, counts
  uint32_t* h_pos = nullptr;  // [T]
  int32_t* h_status = nullptr;
  unsigned long long* h_ctr = nullptr;  // free and retired stack tops after the tick's round
  hipEvent_t e_snap = nullptr, e_srch = nullptr, e_upd = nullptr;
  bool busy = false;
  uint64_t tick = 0;
  uint64_t demand = 0;  // worst-case slabs the tick's round may take
  uint32_t nd = 0, ni = 0, nq = 0;
  bool reclaim = false;
  double t_enqueue = 0.0;  // wall seconds since the loop's start
  std::vector<uint64_t> members;
};
}  // namespace

etale_status etale_serve(etale_t ix, const etale_serve_config* cfg, const etale_request* reqs, uint64_t n,
                         const void* rows_dev, uint64_t n_rows, float* latency_ms, uint32_t* tick_host,
                         uint32_t* res_ids_dev, void* res_dists_dev, etale_serve_stats* out) {
  CHECK_HANDLE();
  if (!cfg || !out || (n && !reqs)) return fail(ix, ETALE_EINVAL, "serve: null argument");
  const etale_serve_config c = *cfg;
  if (c.max_tick < 1 || c.max_tick > ix->cfg.max_batch || c.k < 1 || c.k > c.L || c.L > 256)
    return fail(ix, ETALE_EINVAL, "serve: need 1 <= max_tick <= max_batch and 1 <= k <= L <= 256");
  if ((res_ids_dev == nullptr) != (res_dists_dev == nullptr))
    return fail(ix, ETALE_EINVAL, "serve: result ids and distances go together");
  if (ix->cfg.metric == ETALE_METRIC_IP_F32 && ix->qtrav != ETALE_TRAV_NATIVE && (uint64_t)ix->qrerank * c.k > 64)
    return fail(ix, ETALE_EINVAL, "serve: rerank_mult * k must not exceed 64");
  for (uint64_t i = 0; i < n; ++i) {
    if (reqs[i].kind > ETALE_REQ_DELETE || (i && reqs[i].t_arrive < reqs[i - 1].t_arrive))
      return fail(ix, ETALE_EINVAL, "serve: bad kind or arrival order");
    if (reqs[i].kind != ETALE_REQ_DELETE && (!rows_dev || reqs[i].arg >= n_rows))
      return fail(ix, ETALE_EINVAL, "serve: row out of range");
  }
  unsigned long long h0[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h0)) return st;
  const uint32_t T = c.max_tick, k = c.k, R = ix->cfg.R;
  const uint32_t ns = ix->cfg.n_entry, dim = ix->cfg.dim;
  const uint64_t row_bytes = (uint64_t)dim * (ix->cfg.metric == ETALE_METRIC_L2_U8 ? 1 : 4);
  const uint64_t slab_bytes = 8ull * R;
  const uint64_t fixed = ix->bytes - ix->cfg.id_capacity * row_bytes - ix->cfg.slab_capacity * slab_bytes;

  // ---- resources: the update stream, the snapshot, the search scratch, two tick slots
  std::vector<void*> dev_bufs, host_bufs;
  std::vector<hipEvent_t> events;
  hipStream_t U = nullptr;
  auto release = [&]() {
    if (U) (void)hipStreamSynchronize(U);
    (void)hipStreamSynchronize(ix->stream);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (U) (void)hipStreamDestroy(U);
    for (void* p : dev_bufs) (void)hipFree(p);
    for (void* p : host_bufs) (void)hipHostFree(p);
  };
  hipError_t e = hipStreamCreateWithFlags(&U, hipStreamNonBlocking);  // default priority
  auto dev = [&](auto** p, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc((void**)p, bytes ? bytes : 16);
    if (e == hipSuccess) dev_bufs.push_back(*p);
  };
  auto host = [&](auto** p, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipHostMalloc((void**)p, bytes ? bytes : 16, hipHostMallocDefault);
    if (e == hipSuccess) host_bufs.push_back(*p);
  };
  auto event = [&](hipEvent_t* ev) {
    if (e != hipSuccess) return;
    e = hipEventCreate(ev);
    if (e == hipSuccess) events.push_back(*ev);
  };
  // the snapshot a tick's searches read: reference words, counters, entry set and its rows
  unsigned long long* snap_refs = nullptr;
  unsigned long long* snap_ctr = nullptr;
  uint32_t* snap_entries = nullptr;
  uint8_t* snap_ent_x = nullptr;
  int32_t* snap_ent_norm = nullptr;
  const uint64_t norm_words = ((uint64_t)ns + 63) / 64 * 64;
  dev(&snap_refs, ix->cfg.id_capacity * 8);
  dev(&snap_ctr, C_NCOUNTERS * 8);
  dev(&snap_entries, (uint64_t)ns * 4);
  if (ix->ent_x) {
    dev(&snap_ent_x, ent_copy_bytes(ns, dim));
    dev(&snap_ent_norm, norm_words * 4);
  }
  // start-set scratch of the searches, apart from the library's own (which the
  // concurrent round's insert searches use)
  ScanScratch ss;
  ss.chunk = T;
  dev(&ss.keys, (uint64_t)T * c.L * 8);
  dev(&ss.n, (uint64_t)T * 4);
  dev(&ss.dist, (uint64_t)T * ns * 4);
  dev(&ss.gmin, gmin_slots(T, ns) * 4);
  dev(&ss.bound, (uint64_t)T * 4);
  dev(&ss.ncand, (uint64_t)T * 64 * 4);
  dev(&ss.cand, (uint64_t)T * SCAN_KEYS_Q * 8);
  TickSlot slot[2];
  for (TickSlot& t : slot) {
    dev(&t.d_idx, (size_t)3 * T * 4);
    dev(&t.d_vecs, (size_t)T * row_bytes);
    dev(&t.d_q, (size_t)T * row_bytes);
    dev(&t.d_qids, (size_t)T * k * 4);
    dev(&t.d_qd, (size_t)T * k * 4);
    dev(&t.d_counts, 16);
    dev(&t.d_ids, (size_t)T * 4);
    dev(&t.d_pos, (size_t)T * 4);
    dev(&t.d_dst, (size_t)T);
    dev(&t.d_status, 16);
    host(&t.h_idx, (size_t)(3 * T + 4) * 4);
    host(&t.h_pos, (size_t)T * 4);
    host(&t.h_status, 16);
    host(&t.h_ctr, 16);
    event(&t.e_snap);
    event(&t.e_srch);
    event(&t.e_upd);
    t.members.reserve(T);
  }
  hipEvent_t e_ref = nullptr;
  event(&e_ref);
  if (e != hipSuccess) {
    release();
    return fail(ix, ETALE_ENOMEM, std::string("serve: resources: ") + hipGetErrorString(e));
  }
  Index view = ix->dev;  // the searches' state: the snapshot, and its own counters
  view.refs = snap_refs;
  view.ctr = snap_ctr;
  view.entries = snap_entries;
  view.ent_x = snap_ent_x;
  view.ent_norm = snap_ent_norm;

  // ---- the loop
  using clk = std::chrono::steady_clock;
  const hipStream_t S = ix->stream;
  const hipStream_t user_stream = ix->stream;
  const bool user_timing = ix->timing;
  ix->timing = false;
  e = hipStreamSynchronize(S);
  if (e == hipSuccess) e = hipEventRecord(e_ref, S);
  if (e == hipSuccess) e = hipEventSynchronize(e_ref);
  const auto t0 = clk::now();  // the wall time of e_ref
  auto wall = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  const double origin = n ? reqs[0].t_arrive : 0.0;  // the trace's clock at the loop's start
  std::vector<std::string> keys_before;  // rounds captured here name this call's buffers
  for (auto& g : ix->graphs) keys_before.push_back(g.first);
  etale_serve_stats Sx{};
  uint64_t next_id = h0[C_NEXT_ID];
  uint64_t free_known = h0[C_FREE_TOP];
  uint64_t resident = ix->cfg.slab_capacity - h0[C_FREE_TOP] - h0[C_RETIRED_TOP];
  Sx.peak_resident_slabs = resident;
  std::vector<uint64_t> pending;  // arrived, not yet admitted, in arrival order
  pending.reserve(4 * (size_t)T);
  uint64_t arrived = 0, tick_no = 0, done_reqs = 0;
  int oldest = 0;  // slot of the oldest tick in flight
  double last_done = 0.0;
  etale_status result = ETALE_OK;
  if (latency_ms)
    for (uint64_t i = 0; i < n; ++i) latency_ms[i] = -1.0f;
  if (tick_host)
    for (uint64_t i = 0; i < n; ++i) tick_host[i] = 0xFFFFFFFFu;

  // the tick in slot t has passed its events: finish it on the host
  auto finish = [&](TickSlot& t) -> etale_status {
    if (!t.busy) return ETALE_OK;
    hipError_t er = hipEventSynchronize(t.e_upd);
    if (er == hipSuccess) er = hipEventSynchronize(t.e_srch);
    float ms_s = 0.f, ms_u = 0.f, ms_0 = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms_s, e_ref, t.e_srch);
    if (er == hipSuccess) er = hipEventElapsedTime(&ms_u, e_ref, t.e_upd);
    if (er == hipSuccess) er = hipEventElapsedTime(&ms_0, e_ref, t.e_snap);
    if (er != hipSuccess) return fail(ix, ETALE_EDEVICE, std::string("serve: ") + hipGetErrorString(er));
    const bool ok = t.h_status[0] == 0;
    const double done_s = ms_s * 1e-3, done_u = ms_u * 1e-3;
    for (uint64_t m : t.members) {
      const double done = reqs[m].kind == ETALE_REQ_SEARCH ? done_s : done_u;
      const double start = c.realtime ? reqs[m].t_arrive - origin : t.t_enqueue;
      if (latency_ms) latency_ms[m] = ok ? (float)((done - start) * 1e3) : -1.0f;
    }
    if (ok) {
      Sx.searches += t.nq;
      Sx.inserts += t.ni;
      Sx.deletes += t.nd;
      if (t.reclaim) Sx.reclaims += t.h_status[1] == 0;
    } else {
      ++Sx.failed_ticks;
    }
    free_known = t.h_ctr[0];
    resident = ix->cfg.slab_capacity - t.h_ctr[0] - t.h_ctr[1];
    if (resident > Sx.peak_resident_slabs) Sx.peak_resident_slabs = resident;
    Sx.device_busy_seconds += std::max(done_s, done_u) - ms_0 * 1e-3;
    last_done = std::max(last_done, std::max(done_s, done_u));
    done_reqs += t.members.size();
    t.busy = false;
    return ETALE_OK;
  };

  while (result == ETALE_OK) {
    // arrivals
    if (c.realtime) {
      const double now = wall() + origin;
      while (arrived < n && reqs[arrived].t_arrive <= now) pending.push_back(arrived++);
    } else {
      while (arrived < n && pending.size() < 4 * (size_t)T) pending.push_back(arrived++);
    }
    TickSlot& free_slot = slot[oldest].busy ? slot[oldest ^ 1] : slot[oldest];
    const bool have_slot = !free_slot.busy;
    if (!have_slot || pending.empty()) {
      const bool any_busy = slot[0].busy || slot[1].busy;
      if (!have_slot || (pending.empty() && arrived == n && any_busy)) {
        // wait for the oldest tick in flight
        if (etale_status st = finish(slot[oldest])) {
          result = st;
          break;
        }
        oldest ^= 1;
        continue;
      }
      if (arrived == n && !any_busy) break;  // drained
      if (c.realtime && arrived < n) {
        // nothing pending: wait for the next arrival or a finished tick
        const double dt = reqs[arrived].t_arrive - origin - wall();
        if (any_busy && hipEventQuery(slot[oldest].e_upd) == hipSuccess && hipEventQuery(slot[oldest].e_srch) == hipSuccess) {
          if (etale_status st = finish(slot[oldest])) {
            result = st;
            break;
          }
          oldest ^= 1;
        } else if (dt > 2e-4) {
          std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
      }
      continue;
    }
    // ---- form a tick from the pending requests, in arrival order
    TickSlot& t = free_slot;
    t.members.clear();
    uint32_t nd = 0, ni = 0, nq = 0;
    uint64_t inflight = 0;
    for (const TickSlot& o : slot)
      if (o.busy) inflight += o.demand;
    const uint64_t avail = free_known > inflight ? free_known - inflight : 0;
    uint64_t used = next_id * row_bytes + (resident + inflight) * slab_bytes + fixed;
    size_t keep = 0;
    for (size_t pi = 0; pi < pending.size(); ++pi) {
      const uint64_t j = pending[pi];
      bool admit = t.members.size() < T, reject = false;
      if (admit && reqs[j].kind == ETALE_REQ_INSERT) {
        // ids are never reused and rows never freed: past the id space or the
        // budget an insert can never be admitted
        if ((c.hbm_budget_bytes && used + row_bytes + slab_bytes > c.hbm_budget_bytes) ||
            next_id + ni + 1 > ix->cfg.id_capacity)
          reject = true;
        else
          admit = (uint64_t)(ni + 1) * (R + 2) + (uint64_t)nd * R <= avail;
      } else if (admit && reqs[j].kind == ETALE_REQ_DELETE) {
        admit = ix->cfg.tombstone_only || (uint64_t)ni * (R + 2) + (uint64_t)(nd + 1) * R <= avail;
      }
      if (reject) {
        ++Sx.rejected_inserts;
        ++done_reqs;
        continue;
      }
      if (!admit) {
        if (t.members.size() < T && reqs[j].kind != ETALE_REQ_SEARCH) ++Sx.deferred;
        pending[keep++] = j;
        continue;
      }
      if (reqs[j].kind == ETALE_REQ_DELETE) {
        t.h_idx[nd++] = reqs[j].arg;
      } else if (reqs[j].kind == ETALE_REQ_INSERT) {
        t.h_idx[T + ni++] = reqs[j].arg;
        used += row_bytes + slab_bytes;
      } else {
        t.h_pos[nq] = (uint32_t)j;
        t.h_idx[2 * T + nq++] = reqs[j].arg;
      }
      t.members.push_back(j);
      if (tick_host) tick_host[j] = (uint32_t)tick_no;
    }
    pending.resize(keep);
    if (t.members.empty() && pending.empty()) continue;  // every pending request was rejected
    if (t.members.empty()) {
      // everything pending waits for slabs: let the oldest tick finish first
      if (slot[oldest].busy) {
        if (etale_status st = finish(slot[oldest])) {
          result = st;
          break;
        }
        oldest ^= 1;
        continue;
      }
      result = fail(ix, ETALE_EPOOL, "serve: pending updates cannot be covered by the free slab pool");
      break;
    }
    t.nd = nd;
    t.ni = ni;
    t.nq = nq;
    t.h_idx[3 * T] = nd;  // the round's counts: its deletes and inserts, no queries
    t.h_idx[3 * T + 1] = ni;
    t.h_idx[3 * T + 2] = 0;
    t.demand = ix->cfg.tombstone_only ? (uint64_t)ni * (R + 2) : (uint64_t)ni * (R + 2) + (uint64_t)nd * R;
    t.reclaim = c.reclaim_every && (tick_no + 1) % c.reclaim_every == 0 && !ix->cfg.tombstone_only;
    t.tick = tick_no++;
    t.t_enqueue = wall();
    t.busy = true;
    // search stream: inputs, then (after the previous tick's round) the snapshot, then the searches
    const TickSlot& prev = slot[&t == &slot[0] ? 1 : 0];
    e = hipMemcpyAsync(t.d_idx, t.h_idx, (size_t)3 * T * 4, hipMemcpyHostToDevice, S);
    if (e == hipSuccess) e = hipMemcpyAsync(t.d_counts, t.h_idx + 3 * T, 12, hipMemcpyHostToDevice, S);
    if (e == hipSuccess && nq) e = hipMemcpyAsync(t.d_pos, t.h_pos, (size_t)nq * 4, hipMemcpyHostToDevice, S);
    if (e == hipSuccess) e = launch_gather_rows(rows_dev, t.d_idx + T, ni, (uint32_t)row_bytes, t.d_vecs, S);
    if (e == hipSuccess) e = launch_gather_rows(rows_dev, t.d_idx + 2 * T, nq, (uint32_t)row_bytes, t.d_q, S);
    if (e == hipSuccess && prev.busy) e = hipStreamWaitEvent(S, prev.e_upd, 0);
    if (e == hipSuccess && next_id) e = hipMemcpyAsync(snap_refs, ix->refs, next_id * 8, hipMemcpyDeviceToDevice, S);
    if (e == hipSuccess) e = hipMemcpyAsync(snap_ctr, ix->ctr, C_NCOUNTERS * 8, hipMemcpyDeviceToDevice, S);
    if (e == hipSuccess) e = hipMemcpyAsync(snap_entries, ix->entries, (size_t)ns * 4, hipMemcpyDeviceToDevice, S);
    if (e == hipSuccess && snap_ent_x)
      e = hipMemcpyAsync(snap_ent_x, ix->ent_x, ent_copy_bytes(ns, dim), hipMemcpyDeviceToDevice, S);
    if (e == hipSuccess && snap_ent_x)
      e = hipMemcpyAsync(snap_ent_norm, ix->ent_norm, norm_words * 4, hipMemcpyDeviceToDevice, S);
    if (e == hipSuccess) e = hipEventRecord(t.e_snap, S);
    if (e != hipSuccess) {
      result = fail(ix, ETALE_EDEVICE, std::string("serve: ") + hipGetErrorString(e));
      break;
    }
    if (nq) {
      if (etale_status st = run_searches(ix, MODE_QUERY, t.d_q, nq, k, c.L, ix->cfg.visit_mult * c.L, t.d_qids,
                                         t.d_qd, nullptr, Dyn{}, false, &ss, &view, S)) {
        result = st;
        break;
      }
      if (res_ids_dev)
        e = launch_scatter_results(t.d_qids, t.d_qd, t.d_pos, nq, k, res_ids_dev,
                                   reinterpret_cast<uint32_t*>(res_dists_dev), S);
    }
    if (e == hipSuccess) e = hipEventRecord(t.e_srch, S);
    // update stream: after the snapshot, the tick's deletes and inserts as one round
    if (e == hipSuccess) e = hipStreamWaitEvent(U, t.e_snap, 0);
    if (e != hipSuccess) {
      result = fail(ix, ETALE_EDEVICE, std::string("serve: ") + hipGetErrorString(e));
      break;
    }
    if (nd || ni || t.reclaim) {
      etale_round_desc d{};
      d.del_ids = t.d_idx;
      d.del_status = t.d_dst;
      d.ins_vecs = t.d_vecs;
      d.ins_ids = t.d_ids;
      d.status = t.d_status;
      d.reclaim = t.reclaim ? 1 : 0;
      d.graph = c.graph;
      d.counts = c.graph ? t.d_counts : nullptr;
      d.max_del = c.graph ? size_bucket(nd, 256, T) : nd;
      d.max_ins = c.graph ? size_bucket(ni, 256, T) : ni;
      ix->stream = U;
      const etale_status st = etale_round(ix, &d);
      ix->stream = user_stream;
      if (st) {
        result = st;
        break;
      }
    } else {
      t.h_status[0] = t.h_status[1] = 0;
      e = hipMemsetAsync(t.d_status, 0, 8, U);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(t.h_status, t.d_status, 8, hipMemcpyDeviceToHost, U);
    if (e == hipSuccess) e = hipMemcpyAsync(t.h_ctr, ix->ctr + C_FREE_TOP, 16, hipMemcpyDeviceToHost, U);
    if (e == hipSuccess) e = hipEventRecord(t.e_upd, U);
    if (e != hipSuccess) {
      result = fail(ix, ETALE_EDEVICE, std::string("serve: ") + hipGetErrorString(e));
      break;
    }
    next_id += ni;
    ++Sx.ticks;
  }
  // finish whatever is still in flight (also after an error, so no buffer is freed under a kernel)
  for (int r = 0; r < 2; ++r) {
    TickSlot& t = slot[oldest];
    if (t.busy) {
      const etale_status st = finish(t);
      if (!result) result = st;
    }
    oldest ^= 1;
  }
  ix->timing = user_timing;
  ix->stream = user_stream;
  Sx.final_resident_slabs = resident;
  Sx.ids_handed_out = next_id;
  Sx.wall_seconds = last_done;
  release();
  for (auto it = ix->graphs.begin(); it != ix->graphs.end();) {
    if (std::find(keys_before.begin(), keys_before.end(), it->first) == keys_before.end()) {
      ++Sx.graphs;
      (void)hipGraphExecDestroy(it->second);
      it = ix->graphs.erase(it);
    } else {
      ++it;
    }
  }
  if (result) return result;
  if (etale_status st = refresh_mirror(ix)) return st;
  *out = Sx;
  return ETALE_OK;
}

etale_status etale_set_search_knobs(etale_t ix, uint32_t waves_per_block, uint32_t vt_slots) {
  CHECK_HANDLE();
  if ((waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4) || !pow2(vt_slots) || vt_slots < 64 ||
      vt_slots > 16384)
    return fail(ix, ETALE_EINVAL, "search knobs: waves 1/2/4, slots a power of two in 64..16384");
  if (search_lds_per_wave(SCAN_L_MAX, vt_slots, ix->cfg.W) > 65536u) return fail(ix, ETALE_EINVAL, "search knobs: LDS");
  ix->cfg.waves_per_block = waves_per_block;
  ix->cfg.vt_slots = vt_slots;
  return ETALE_OK;
}

etale_status etale_set_search_lanes(etale_t ix, uint32_t lanes_per_row) {
  CHECK_HANDLE();
  const bool ok = lanes_per_row == 0 ||
                  (ix->cfg.metric == ETALE_METRIC_L2_U8 && (lanes_per_row * 16u == ix->cfg.dim ||
                                                           (lanes_per_row * 32u == ix->cfg.dim &&
                                                            (ix->cfg.dim == 128 || ix->cfg.dim == 256))));
  if (!ok) return fail(ix, ETALE_EINVAL, "search lanes: 0, dim/16, or dim/32 for 128- and 256-byte rows");
  ix->row_lanes = lanes_per_row * 16u == ix->cfg.dim ? 0u : lanes_per_row;
  return ETALE_OK;
}

etale_status etale_autotune(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                            etale_tune_result* out) {
  CHECK_HANDLE();
  if (!q_dev || !out || nq == 0 || nq > 0xFFFFFFFFull || k < 1 || k > L || L > 256)
    return fail(ix, ETALE_EINVAL, "autotune: bad batch");
  uint32_t* ids = nullptr;
  uint32_t* d = nullptr;
  HIP_TRY(hipMalloc(&ids, nq * k * 4));
  HIP_TRY(hipMalloc(&d, nq * k * 4));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const uint32_t wpb0 = ix->cfg.waves_per_block, vt0 = ix->cfg.vt_slots, rl0 = ix->row_lanes;
  const bool timing = ix->timing;
  ix->timing = false;
  auto time_one = [&](uint32_t wpb, uint32_t vt, uint32_t rl, float* ms) -> etale_status {
    ix->cfg.waves_per_block = wpb;
    ix->cfg.vt_slots = vt;
    ix->row_lanes = rl;
    const uint32_t vcap = ix->cfg.visit_mult * L;
    if (etale_status st = run_searches(ix, MODE_QUERY, (const uint8_t*)q_dev, nq, k, L, vcap, ids, d, nullptr, Dyn{}))
      return st;  // warm-up
    HIP_TRY(hipEventRecord(e0, ix->stream));
    for (int rep = 0; rep < 3; ++rep)
      if (etale_status st = run_searches(ix, MODE_QUERY, (const uint8_t*)q_dev, nq, k, L, vcap, ids, d, nullptr,
                                         Dyn{}))
        return st;
    HIP_TRY(hipEventRecord(e1, ix->stream));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    *ms /= 3.0f;
    return ETALE_OK;
  };
  etale_status st = ETALE_OK;
  float best = 0.f, base = 0.f;
  uint32_t bw = wpb0, bv = vt0, br = rl0;
  st = time_one(wpb0, vt0, rl0, &base);
  best = base;
  const uint32_t waves[] = {1, 2, 4};
  const uint32_t slots[] = {256, 512, 1024, 2048, 4096};
  std::vector<uint32_t> lanes = {0};
  if (ix->cfg.metric == ETALE_METRIC_L2_U8 && (ix->cfg.dim == 128 || ix->cfg.dim == 256)) lanes.push_back(ix->cfg.dim / 32);
  for (uint32_t rl : lanes)
    for (uint32_t w : waves)
      for (uint32_t v : slots) {
        if (st) break;
        if (search_lds_per_wave(L, v, ix->cfg.W) > 65536u) continue;
        float ms = 0.f;
        st = time_one(w, v, rl, &ms);
        if (!st && ms < best) {
          best = ms;
          bw = w;
          bv = v;
          br = rl;
        }
      }
  ix->cfg.waves_per_block = st ? wpb0 : bw;
  ix->cfg.vt_slots = st ? vt0 : bv;
  ix->row_lanes = st ? rl0 : br;
  ix->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(ids);
  (void)hipFree(d);
  if (st) return st;
  out->waves_per_block = bw;
  out->vt_slots = bv;
  out->row_lanes = br ? br : (ix->cfg.metric == ETALE_METRIC_L2_U8 ? ix->cfg.dim / 16 : 0);
  out->ms = best;
  out->ms_default = base;
  return ETALE_OK;
}

etale_status etale_set_search_timing(etale_t ix, int32_t enable) {
  CHECK_HANDLE();
  ix->timing = enable != 0;
  return ETALE_OK;
}

etale_status etale_get_search_timing(etale_t ix, float* ms_host, uint64_t cap, uint64_t* launches) {
  CHECK_HANDLE();
  if ((!ms_host && cap) || !launches) return ETALE_EINVAL;
  HIP_TRY(hipStreamSynchronize(ix->stream));
  uint64_t n = 0;
  for (auto& q : ix->ev_used) {
    for (int i = 0; i < 3 && n < cap; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, q[i], q[i + 1]));
      ms_host[n * 3 + i] = ms;
    }
    ++n;
    for (hipEvent_t e : q) ix->ev_pool.push_back(e);
  }
  *launches = ix->ev_used.size();
  ix->ev_used.clear();
  return ETALE_OK;
}

etale_status etale_set_concurrent(etale_t ix, int32_t enable, void* search_stream) {
  CHECK_HANDLE();
  const bool on = enable != 0;
  if (on == ix->concurrent) {
    if (on) ix->search_stream = reinterpret_cast<hipStream_t>(search_stream);
    return ETALE_OK;
  }
  if (ix->cfg.tombstone_only) return fail(ix, ETALE_EINVAL, "concurrent mode: not with tombstone_only");
  if (on) {
    if (!search_stream || search_stream == (void*)ix->stream)
      return fail(ix, ETALE_EINVAL, "concurrent mode: searches need a stream of their own");
    HIP_TRY(hipStreamSynchronize(ix->stream));
    if (ix->conc_bufs.empty()) {
      const uint64_t C = ix->scan_chunk;
      auto al = [&](auto** p, uint64_t bytes) -> hipError_t {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
        if (e == hipSuccess) {
          ix->conc_bufs.push_back(q);
          *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(q);
        }
        return e;
      };
      HIP_TRY(al(&ix->cs.keys, C * SCAN_L_MAX * 8));
      HIP_TRY(al(&ix->cs.n, C * 4));
      HIP_TRY(al(&ix->cs.dist, ix->dist_cap * 4));
      HIP_TRY(al(&ix->cs.gmin, ix->gmin_cap * 4));
      HIP_TRY(al(&ix->cs.bound, C * 4));
      HIP_TRY(al(&ix->cs.ncand, C * 64 * 4));
      HIP_TRY(al(&ix->cs.cand, C * SCAN_KEYS_Q * 8));
    }
    ix->search_stream = reinterpret_cast<hipStream_t>(search_stream);
    ix->dev.fence = 1;
    ix->dev.concurrent = 1;
    ix->concurrent = true;
    return ETALE_OK;
  }
  // leaving: both streams drain, then the slabs retired meanwhile rejoin the
  // free pool and the entry set catches up with the deletes and inserts
  HIP_TRY(hipStreamSynchronize(ix->search_stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  ix->concurrent = false;
  ix->dev.fence = 0;
  ix->dev.concurrent = 0;
  ix->search_stream = nullptr;
  HIP_TRY(launch_recycle(ix->dev, ix->stream));
  Dyn de;
  de.first_ctr = C_NEXT_ID;
  HIP_TRY(launch_refresh_entries(ix->dev, 0, ix->cfg.n_entry, de, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return refresh_mirror(ix);
}

etale_status etale_sync(etale_t ix) {
  if (!ix) return ETALE_EINVAL;
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return ETALE_OK;
}

const char* etale_last_error(etale_t ix) { return ix ? ix->err.c_str() : "null handle"; }

}  // extern "C"
