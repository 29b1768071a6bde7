// C-ABI of the ETALE index: argument checks, device memory, and the order of
// the phase launches of each call. Every numeric step runs in the kernels of
// etale_kernels.hip; this file only moves sizes, pointers and counters.
#include <rocprim/device/device_radix_sort.hpp>

#include <array>
#include <string>
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
  // call scratch
  uint64_t* vis_keys = nullptr;
  uint32_t* vis_cnt = nullptr;
  uint32_t* F = nullptr;
  uint64_t* pairs_a = nullptr;
  uint64_t* pairs_b = nullptr;
  uint32_t* dlist = nullptr;
  uint32_t* dirty = nullptr;
  uint64_t* bitmap = nullptr;
  uint64_t* scan_keys = nullptr;  // [scan_chunk x 256] initial lists
  uint32_t* scan_n = nullptr;
  uint32_t* scan_dist = nullptr;  // [dist_cap] query x start-set distances
  uint64_t dist_cap = 0;
  uint32_t scan_chunk = 0;
  uint64_t live = 0;              // ids with deletion flag 0 (host mirror)
  int32_t qtrav = 0;              // query-side traversal copy
  uint32_t qrerank = 0;
  // opt-in stage timing of search calls: event quadruples per launch
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::array<hipEvent_t, 4>> ev_used;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  uint64_t next_id = 0;
  uint32_t vcap_build = 0;
  uint64_t bytes = 0;
  bool poisoned = false;
  std::string err;
  std::vector<void*> allocs;
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
  return ETALE_OK;
}

etale_status set_counter(etale_index* ix, Counter c, unsigned long long v) {
  HIP_TRY(hipMemcpyAsync(ix->ctr + c, &v, sizeof(v), hipMemcpyHostToDevice, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return ETALE_OK;
}

etale_status sort_keys(etale_index* ix, uint64_t* in, uint64_t* out, size_t n) {
  if (n == 0) return ETALE_OK;
  size_t bytes = 0;
  HIP_TRY(rocprim::radix_sort_keys(nullptr, bytes, in, out, n, 0, 64, ix->stream));
  if (bytes > ix->sort_tmp_bytes) return fail(ix, ETALE_EDEVICE, "sort scratch too small");
  bytes = ix->sort_tmp_bytes;
  HIP_TRY(rocprim::radix_sort_keys(ix->sort_tmp, bytes, in, out, n, 0, 64, ix->stream));
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

uint32_t n_entries(const etale_index* ix) { return (uint32_t)std::min<uint64_t>(ix->cfg.n_entry, ix->live); }

// queries per launch so that the distance matrix fits its scratch
uint32_t scan_chunk_for(const etale_index* ix, uint32_t ns) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ix->scan_chunk, ix->dist_cap / std::max(1u, ns)));
}

// start-set scoring, then the beam search, over queries [0, nq) in chunks
etale_status run_searches(etale_index* ix, int mode, const uint8_t* q, uint32_t first, uint64_t nq, uint32_t k,
                          uint32_t L, uint32_t vcap, uint32_t* out_ids, uint32_t* out_d, uint32_t* counts) {
  const uint32_t ns = n_entries(ix);
  const uint32_t chunk = scan_chunk_for(ix, ns);
  for (uint64_t c = 0; c < nq; c += chunk) {
    const uint32_t cn = (uint32_t)std::min<uint64_t>(chunk, nq - c);
    ScanArgs sc{};
    sc.mode = mode;
    sc.q = mode == MODE_QUERY ? q + c * ix->cfg.dim * (ix->cfg.metric == ETALE_METRIC_L2_U8 ? 1 : 4) : nullptr;
    sc.first = first + (uint32_t)c;
    sc.nq = cn;
    sc.L = L;
    sc.ns = ns;
    sc.dist = ix->scan_dist;
    sc.out_keys = ix->scan_keys;
    sc.out_n = ix->scan_n;
    sc.out_stride = L;
    sc.trav = mode == MODE_QUERY ? ix->qtrav : ix->dev.trav;
    std::array<hipEvent_t, 4> ev{};
    const bool timed = ix->timing && mode == MODE_QUERY;
    if (timed) {
      for (auto& e : ev) {
        if (ix->ev_pool.empty()) {
          hipEvent_t ne;
          HIP_TRY(hipEventCreate(&ne));
          ix->ev_pool.push_back(ne);
        }
        e = ix->ev_pool.back();
        ix->ev_pool.pop_back();
      }
      ix->ev_used.push_back(ev);
      HIP_TRY(hipEventRecord(ev[0], ix->stream));
    }
    if (ns == 0) {
      HIP_TRY(hipMemsetAsync(ix->scan_n, 0, (size_t)cn * 4, ix->stream));
      if (timed) {
        HIP_TRY(hipEventRecord(ev[1], ix->stream));
        HIP_TRY(hipEventRecord(ev[2], ix->stream));
      }
    } else {
      HIP_TRY(launch_scan(ix->dev, sc, ix->stream, timed ? ev[1] : nullptr));
      if (timed) HIP_TRY(hipEventRecord(ev[2], ix->stream));
    }
    SearchArgs sa{};
    sa.mode = mode;
    sa.q = sc.q;
    sa.first = sc.first;
    sa.nq = cn;
    sa.L = L;
    sa.k = k;
    sa.vcap = vcap;
    sa.vt_mask = ix->cfg.vt_slots - 1;
    sa.W = ix->cfg.W;
    sa.lds_per_wave = search_lds_per_wave(L, ix->cfg.vt_slots);
    sa.init_keys = ix->scan_keys;
    sa.init_n = ix->scan_n;
    sa.init_stride = L;
    sa.trav = sc.trav;
    sa.rerank = mode == MODE_QUERY ? ix->qrerank : 0;
    if (mode == MODE_QUERY) {
      sa.out_ids = out_ids + c * k;
      sa.out_d = out_d + c * k;
      sa.counts = counts ? counts + 2 * c : nullptr;
    } else {
      sa.vis_keys = ix->vis_keys + c * vcap;
      sa.vis_cnt = ix->vis_cnt + c;
    }
    HIP_TRY(launch_search(ix->dev, sa, search_waves_per_block(ix, sa.lds_per_wave), ix->stream));
    if (timed) HIP_TRY(hipEventRecord(ev[3], ix->stream));
  }
  return ETALE_OK;
}

// bootstrap: each new node's candidates are the vcap nearest other members
etale_status run_bootstrap(etale_index* ix, uint32_t first, uint32_t n, uint32_t vcap) {
  const uint32_t chunk = scan_chunk_for(ix, n);
  for (uint32_t c = 0; c < n; c += chunk) {
    ScanArgs sc{};
    sc.mode = MODE_BOOT;
    sc.first = first;  // the start set is the whole batch
    sc.nq = std::min(chunk, n - c);
    sc.L = vcap;
    sc.ns = n;
    sc.dist = ix->scan_dist;
    sc.out_keys = ix->vis_keys + (size_t)c * vcap;
    sc.out_n = ix->vis_cnt + c;
    sc.out_stride = vcap;
    sc.qoff = c;
    HIP_TRY(launch_scan(ix->dev, sc, ix->stream));
  }
  return ETALE_OK;
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
  if (c.W < 1 || c.W > 2 || c.W * c.R > 64) return ETALE_EINVAL;
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
    if (search_lds_per_wave(SCAN_L_MAX, c.vt_slots) > 65536u) return ETALE_EINVAL;
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
  ALLOC(ix->ctr, C_NCOUNTERS * 8);
  ALLOC(ix->entries, (uint64_t)c.n_entry * 4);
  ALLOC(ix->vis_keys, B * ix->vcap_build * 8);
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
  {
    size_t bytes = 0;
    if (rocprim::radix_sort_keys(nullptr, bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (size_t)(B * R), 0, 64,
                                 ix->stream) != hipSuccess)
      return cleanup(ETALE_EDEVICE, "sort size");
    ix->sort_tmp_bytes = bytes;
    ALLOC(ix->sort_tmp, bytes);
  }
#undef ALLOC
  Index& d = ix->dev;
  d.dim = c.dim;
  d.R = c.R;
  d.a2 = c.alpha_num * c.alpha_num;
  d.b2 = c.alpha_den * c.alpha_den;
  d.publish_attempts = c.publish_attempts;
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
  if (launch_init(d, ix->stream) != hipSuccess || hipStreamSynchronize(ix->stream) != hipSuccess)
    return cleanup(ETALE_EDEVICE, "init");
  *out = ix;
  return ETALE_OK;
}

etale_status etale_destroy(etale_t ix) {
  if (!ix) return ETALE_OK;
  (void)hipStreamSynchronize(ix->stream);
  for (auto& q : ix->ev_used)
    for (hipEvent_t e : q) (void)hipEventDestroy(e);
  for (hipEvent_t e : ix->ev_pool) (void)hipEventDestroy(e);
  for (void* p : ix->allocs) (void)hipFree(p);
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
  if (ix->next_id + n > ix->cfg.id_capacity) return fail(ix, ETALE_ECAPACITY, "insert: id space exhausted");
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  const uint32_t R = ix->cfg.R;
  if (h[C_N_ENTRIES] != n_entries(ix)) {
    ix->poisoned = true;
    return fail(ix, ETALE_ESTATE, "entry-set size on the device disagrees with the live count");
  }
  if (h[C_FREE_TOP] < n * (uint64_t)(R + 2)) return fail(ix, ETALE_EPOOL, "insert: slab pool cannot cover n*(R+2)");
  const uint32_t first = (uint32_t)ix->next_id;
  const Index& d = ix->dev;
  if (ix->cfg.metric == ETALE_METRIC_L2_U8) {
    HIP_TRY(hipMemcpyAsync(ix->x + (size_t)first * ix->cfg.dim, vecs_dev, n * ix->cfg.dim, hipMemcpyDeviceToDevice,
                           ix->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(ix->xf + (size_t)first * ix->cfg.dim, vecs_dev, n * ix->cfg.dim * 4,
                           hipMemcpyDeviceToDevice, ix->stream));
    HIP_TRY(launch_encode(d, first, (uint32_t)n, ix->xs, ix->xb, ix->x8, ix->stream));
  }
  if (ids_out_dev) HIP_TRY(launch_write_ids(ids_out_dev, first, n, ix->stream));
  const bool bootstrap = ix->live == 0;
  const uint32_t vcap = ix->vcap_build;

  // searches on the graph as it was at the call's start, or the bootstrap:
  // the visit_cap nearest other members of the batch
  if (bootstrap) {
    if (n > 16384) return fail(ix, ETALE_EINVAL, "insert: a bootstrap batch holds at most 16384 vectors");
    if (etale_status st = run_bootstrap(ix, first, (uint32_t)n, vcap)) return st;
  } else if (etale_status st = run_searches(ix, MODE_INSERT, nullptr, first, n, 0, ix->cfg.L_build, vcap, nullptr,
                                            nullptr, nullptr)) {
    return st;
  }

  // forward neighbors and the node's own slab
  MaintArgs fa = maint_args(ix, vcap);
  fa.first = first;
  fa.n = (uint32_t)n;
  fa.vis_keys = ix->vis_keys;
  fa.vis_cnt = ix->vis_cnt;
  fa.F = ix->F;
  HIP_TRY(launch_maint(MK_FORWARD, d, fa, (uint32_t)n, maint_waves_per_block(fa), ix->stream));

  // reverse edges, grouped by target in (target, source) order
  {
    fa.pairs = ix->pairs_a;
    HIP_TRY(launch_reverse_pairs(d, fa, ix->stream));
    if (etale_status st = sort_keys(ix, ix->pairs_a, ix->pairs_b, n * R)) return st;
    MaintArgs ra = maint_args(ix, R + 1);
    ra.first = first;
    ra.n = (uint32_t)n;
    ra.pairs = ix->pairs_b;
    ra.npairs = (uint32_t)(n * R);
    HIP_TRY(launch_maint(MK_REVERSE, d, ra, ra.npairs, maint_waves_per_block(ra), ix->stream));
  }
  if (ix->cfg.refine && !bootstrap) {
    MaintArgs ga = maint_args(ix, R + R * R);
    ga.first = first;
    ga.n = (uint32_t)n;
    HIP_TRY(launch_maint(MK_REFINE, d, ga, (uint32_t)n, maint_waves_per_block(ga), ix->stream));
  }
  HIP_TRY(launch_refresh_entries(d, first + (uint32_t)n, ix->cfg.n_entry, ix->stream));
  HIP_TRY(launch_recycle(d, ix->stream));
  ix->next_id += n;
  ix->live += n;
  return ETALE_OK;
}

etale_status etale_delete_batch(etale_t ix, const uint32_t* ids_dev, uint64_t n, uint8_t* status_out_dev) {
  CHECK_HANDLE();
  if (n == 0) return ETALE_OK;
  if (!ids_dev || n > ix->cfg.max_batch) return fail(ix, ETALE_EINVAL, "delete: null ids or n > max_batch");
  const Index& d = ix->dev;
  const uint32_t R = ix->cfg.R;
  if (etale_status st = set_counter(ix, C_DEL_OK, 0)) return st;
  HIP_TRY(launch_del_keys(ids_dev, n, ix->pairs_a, ix->stream));
  if (etale_status st = sort_keys(ix, ix->pairs_a, ix->pairs_b, n)) return st;
  HIP_TRY(launch_del_classify(d, ix->pairs_b, n, ix->next_id, status_out_dev, ix->dlist, ix->stream));
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  const uint64_t dok = h[C_DEL_OK];
  if (!ix->cfg.tombstone_only && h[C_FREE_TOP] < dok * R)
    return fail(ix, ETALE_EPOOL, "delete: slab pool cannot cover the repairs");
  HIP_TRY(launch_tombstone(d, ix->dlist, dok, ix->stream));
  ix->live -= dok;
  HIP_TRY(launch_refresh_entries(d, (uint32_t)ix->next_id, ix->cfg.n_entry, ix->stream));
  if (!ix->cfg.tombstone_only && dok) {
    MaintArgs pa = maint_args(ix, 2 * R);
    pa.n = (uint32_t)dok;
    pa.dlist = ix->dlist;
    pa.pairs = ix->pairs_a;
    HIP_TRY(launch_repair_pairs(d, pa, ix->stream));
    if (etale_status st = sort_keys(ix, ix->pairs_a, ix->pairs_b, dok * R)) return st;
    pa.pairs = ix->pairs_b;
    pa.npairs = (uint32_t)(dok * R);
    HIP_TRY(launch_maint(MK_REPAIR, d, pa, pa.npairs, maint_waves_per_block(pa), ix->stream));
  }
  HIP_TRY(launch_recycle(d, ix->stream));
  return ETALE_OK;
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
  if (etale_status st = run_searches(ix, MODE_QUERY, reinterpret_cast<const uint8_t*>(q_dev), 0, nq, k, L,
                                     ix->cfg.visit_mult * L, ids_out_dev, reinterpret_cast<uint32_t*>(dists_out_dev),
                                     counts_out_dev))
    return st;
  return ETALE_OK;
}

etale_status etale_reclaim(etale_t ix) {
  CHECK_HANDLE();
  if (ix->cfg.tombstone_only) return ETALE_OK;
  const Index& d = ix->dev;
  const uint64_t n_ids = ix->next_id;
  if (etale_status st = set_counter(ix, C_DIRTY, 0)) return st;
  if (etale_status st = set_counter(ix, C_DEAD, 0)) return st;
  HIP_TRY(launch_del_bitmap(d, n_ids, ix->bitmap, ix->stream));
  HIP_TRY(launch_dirty(d, n_ids, ix->bitmap, ix->dirty, ix->stream));
  unsigned long long h[C_NCOUNTERS];
  if (etale_status st = read_counters(ix, h)) return st;
  const uint64_t nd = h[C_DIRTY];
  if (h[C_FREE_TOP] < nd) return fail(ix, ETALE_EPOOL, "reclaim: slab pool cannot cover compaction");
  HIP_TRY(launch_compact(d, ix->dirty, nd, ix->bitmap, ix->stream));
  HIP_TRY(launch_free_tombstones(d, n_ids, ix->stream));
  HIP_TRY(launch_recycle(d, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return ETALE_OK;
}

etale_status etale_bruteforce(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t* ids_out_dev,
                              void* dists_out_dev) {
  CHECK_HANDLE();
  if (k < 1 || k > 16 || nq > 0xFFFFFFFFull) return fail(ix, ETALE_EINVAL, "bruteforce: need 1 <= k <= 16");
  if (nq == 0) return ETALE_OK;
  if (!q_dev || !ids_out_dev || !dists_out_dev) return fail(ix, ETALE_EINVAL, "bruteforce: null buffer");
  HIP_TRY(launch_bruteforce(ix->dev, q_dev, (uint32_t)nq, ix->next_id, k, ids_out_dev,
                            reinterpret_cast<uint32_t*>(dists_out_dev), ix->stream));
  return ETALE_OK;
}

etale_status etale_get_stats(etale_t ix, etale_stats* out) {
  if (!ix || !out) return ETALE_EINVAL;
  unsigned long long h[C_NCOUNTERS];
  HIP_TRY(hipMemcpyAsync(h, ix->ctr, sizeof(h), hipMemcpyDeviceToHost, ix->stream));
  HIP_TRY(hipStreamSynchronize(ix->stream));
  etale_stats s{};
  s.next_id = ix->next_id;
  s.live = ix->next_id - h[C_TOMBSTONED];
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

etale_status etale_sync(etale_t ix) {
  if (!ix) return ETALE_EINVAL;
  HIP_TRY(hipStreamSynchronize(ix->stream));
  return ETALE_OK;
}

const char* etale_last_error(etale_t ix) { return ix ? ix->err.c_str() : "null handle"; }

}  // extern "C"
