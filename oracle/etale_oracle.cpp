// CPU oracle for the ETALE dynamic graph index -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded implementation of what the GPU path computes.
// It exists to check the GPU path; nothing in the product links it, imports it
// or calls it. Only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark load it. It shares no code with the HIP sources.
//
// Paper: "ETALE" (arxiv 2607.02543). What each part follows:
//   * Definition 1 (ETALE graph): per id a deletion flag, a degree and a slab;
//     here the slab is modelled as the neighbor list itself, and slabs are
//     counted, not numbered (slab ids are not part of the result).
//   * Algorithm 1 (Publish): copy-on-write install; one publication allocates
//     one slab and retires the displaced one; the deletion flag is carried.
//   * Section 3.3 pool paragraph + Lemma 1: retired slabs only rejoin the free
//     count at the end of a launch (one API call here).
//   * Section 3.4.1 + Algorithm 2 (Insert): beam search, RobustPrune, own
//     publish, reverse edges (append below R, re-prune at R), refine pass.
//   * Section 3.4.2 + Algorithm 3 (Delete): tombstone, then repair every live
//     out-neighbor with two prunes and one publication.
//   * Section 3.4.3 + Algorithm 4 (Reclaim): compaction, then free tombstones.
//   * RobustPrune is the slack-alpha rule of DiskANN that Section 3.4.1 cites.
//
// Readings where the paper is silent (each listed in the design notes):
//   * Round-synchronous: one call = one launch; its phases run in a fixed
//     order, each reading the state the previous phase left. Searches of an
//     insert call all run on the state at the call's start.
//   * Writes to one target inside a phase are applied in ascending source id
//     order and published once.
//   * Order is lexicographic on (distance, id) everywhere.
//   * alpha = a/b is applied to squared distances as a^2*D1 <= b^2*D2.
//   * Every prune drops candidates whose deletion flag is set.
//   * BeamSearch returns the expanded set, capped at visit_cap.
//   * The fixed set of entry points: the n_entry smallest live ids.
//   * An insert call into an index without live nodes bootstraps: each new
//     node's candidates are the visit_cap nearest other members of its batch.
//   * Refine: 2-hop same-batch candidates, pruned; skipped on bootstrap calls.
//   * Float metric: d(a,b) = 1 - <a,b>, in fp64 from the fp32 values.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

enum { M_L2_U8 = 0, M_IP_F32 = 1 };
enum { T_NATIVE = 0, T_BF16 = 1, T_FP8 = 2 };
enum { OK = 0, EINVAL = -1, EPOOL = -3, ECAPACITY = -4 };
enum { DEL_OK = 0, DEL_NOT_LIVE = 1, DEL_OUT_OF_RANGE = 2, DEL_DUPLICATE = 3 };
const uint32_t NONE = 0xFFFFFFFFu;

struct Entry {
  double d;
  uint32_t id;
};

bool key_less(const Entry& a, const Entry& b) {
  return a.d < b.d || (a.d == b.d && a.id < b.id);
}

// ---- number formats, written from their definitions --------------------

// bfloat16: the upper 16 bits of an IEEE binary32, rounded to nearest even.
uint16_t bf16_encode(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
double bf16_decode(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// Round-half-to-even of a non-negative double to an integer.
double rne(double v) {
  double fl = std::floor(v);
  double fr = v - fl;
  if (fr > 0.5) return fl + 1.0;
  if (fr < 0.5) return fl;
  return std::fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
}

// OCP FP8 E4M3FN: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits, no
// infinities, S.1111.111 is NaN, largest finite 448, subnormal step 2^-9.
// Round to nearest even; magnitudes beyond 448 saturate to 448.
uint8_t fp8_encode(float y) {
  uint8_t sign = std::signbit(y) ? 0x80 : 0x00;
  double a = std::fabs((double)y);
  if (std::isnan(y)) return 0x7F;
  if (a >= 448.0) return sign | 0x7E;
  if (a < std::ldexp(1.0, -6)) {  // subnormal range: multiples of 2^-9
    double m = rne(a * 512.0);    // exact scaling by a power of two
    return sign | (uint8_t)m;     // m == 8 is the smallest normal, code 0x08
  }
  int e;
  double f = std::frexp(a, &e);  // a = f * 2^e, f in [0.5, 1)
  f *= 2.0;
  e -= 1;  // a = f * 2^e, f in [1, 2)
  double mant = rne((f - 1.0) * 8.0);
  if (mant == 8.0) {
    mant = 0.0;
    e += 1;
  }
  int biased = e + 7;
  if (biased > 15 || (biased == 15 && mant == 7.0)) return sign | 0x7E;
  return sign | (uint8_t)((biased << 3) | (int)mant);
}
double fp8_decode(uint8_t c) {
  int s = c >> 7, ex = (c >> 3) & 15, m = c & 7;
  if (ex == 15 && m == 7) return std::nan("");
  double v = ex == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, ex - 7);
  return s ? -v : v;
}

// ---- the index ------------------------------------------------------------

struct Oracle {
  int metric = M_L2_U8, trav = T_NATIVE;
  uint32_t dim = 0, R = 32, L_build = 64, W = 1, visit_mult = 4, prune_cap = 256;
  uint32_t alpha_num = 6, alpha_den = 5, rerank_mult = 4, n_entry = 1;
  uint64_t cap = 0, P = 0;
  int refine = 1, tombstone_only = 0;

  std::vector<uint8_t> xu8;
  std::vector<float> xf;
  std::vector<uint16_t> xbf;
  std::vector<uint8_t> xq8;
  std::vector<float> xscale;

  std::vector<uint8_t> del, has_slab;
  std::vector<std::vector<Entry>> adj;
  uint64_t next_id = 0;
  std::vector<uint32_t> entries;  // the entry set: the n_entry smallest live ids

  // pool counts (Section 3.3): free, resident, retired in the current launch
  uint64_t free_cnt = 0, resident = 0, retired = 0;

  // counters
  uint64_t pub_forward = 0, pub_repair = 0, pub_reverse = 0, pub_refine = 0, pub_compact = 0;
  uint64_t freed = 0, dirty_last = 0, dead_edges_last = 0;
  uint64_t search_expansions = 0, search_distances = 0;

  std::vector<uint32_t> stamp;
  uint32_t cur = 0;

  // ---- near-tie log (float metric) ------------------------------------------
  // The GPU decides float comparisons in FP32, this model in FP64. Where two
  // compared quantities lie within TIE_RTOL of each other (relative to the
  // larger of them, and at least to `scale`, the magnitude of the terms the
  // dot products sum), the two can decide the comparison differently. Each
  // such comparison is logged with the node whose list it decides: the node
  // being inserted (its search and its forward prune), or the owner of a
  // repair, reverse or refine prune. Searches for queries log nothing (their
  // results are checked against exact distances instead).
  static constexpr double TIE_RTOL = 1e-5;
  uint32_t tie_owner = NONE;
  struct Tie {
    uint32_t owner;
    double margin;  // the smallest relative margin logged for it in a row
  };
  mutable std::vector<Tie> ties;  // logging does not change the index
  // relative margin of a comparison between a and b (terms of magnitude scale)
  double margin(double a, double b, double scale = 1.0) const {
    const double m = std::max(std::max(std::fabs(a), std::fabs(b)), scale);
    return std::fabs(a - b) / m;
  }
  void tie_log(double a, double b, double scale = 1.0) const {
    if (metric != M_IP_F32 || tie_owner == NONE) return;
    const double r = margin(a, b, scale);
    if (r > TIE_RTOL) return;
    if (!ties.empty() && ties.back().owner == tie_owner)
      ties.back().margin = std::min(ties.back().margin, r);
    else
      ties.push_back({tie_owner, r});
  }
  // adjacent pairs among the first `upto` (+1) entries of a sorted list
  template <class V, class F>
  void tie_scan(const V& v, size_t upto, F dist) const {
    if (metric != M_IP_F32 || tie_owner == NONE) return;
    for (size_t i = 1; i < v.size() && i <= upto; ++i) tie_log(dist(v[i - 1]), dist(v[i]));
  }

  uint32_t visit_cap(uint32_t L) const { return visit_mult * L; }

  // exact distance between a query vector and a stored id (fp64 for floats)
  double dq(const void* q, uint32_t id) const {
    if (metric == M_L2_U8) {
      const uint8_t* a = (const uint8_t*)q;
      const uint8_t* b = &xu8[(size_t)id * dim];
      int64_t s = 0;
      for (uint32_t i = 0; i < dim; ++i) {
        int64_t t = (int64_t)a[i] - (int64_t)b[i];
        s += t * t;
      }
      return (double)s;
    }
    const float* a = (const float*)q;
    const float* b = &xf[(size_t)id * dim];
    double s = 0.0;
    for (uint32_t i = 0; i < dim; ++i) s += (double)a[i] * (double)b[i];
    return 1.0 - s;
  }
  // the distance traversal uses: exact, or against the bf16 / fp8 copy
  double dtrav(const void* q, uint32_t id) const {
    if (metric == M_L2_U8 || trav == T_NATIVE) return dq(q, id);
    const float* a = (const float*)q;
    double s = 0.0;
    if (trav == T_BF16) {
      const uint16_t* b = &xbf[(size_t)id * dim];
      for (uint32_t i = 0; i < dim; ++i) s += (double)a[i] * bf16_decode(b[i]);
      return 1.0 - s;
    }
    const uint8_t* b = &xq8[(size_t)id * dim];
    for (uint32_t i = 0; i < dim; ++i) s += (double)a[i] * fp8_decode(b[i]);
    return 1.0 - (double)xscale[id] * s;
  }
  const void* vec(uint32_t id) const {
    return metric == M_L2_U8 ? (const void*)&xu8[(size_t)id * dim] : (const void*)&xf[(size_t)id * dim];
  }
  double D(uint32_t a, uint32_t b) const { return dq(vec(a), b); }

  bool live(uint32_t u) const { return u < next_id && !del[u]; }

  void new_stamp() {
    if (++cur == 0) {
      std::fill(stamp.begin(), stamp.end(), 0u);
      cur = 1;
    }
  }

  // ---- Publish (Algorithm 1), as counts: one fresh slab, old one retired ----
  int publish(uint32_t u, const std::vector<Entry>& N) {
    if (free_cnt == 0) return EPOOL;
    free_cnt -= 1;
    resident += 1;
    if (has_slab[u]) {
      resident -= 1;
      retired += 1;
    }
    has_slab[u] = 1;
    adj[u] = N;
    return OK;
  }
  // end of a launch: the retired stack rejoins the free stack (Lemma 1)
  void recycle() {
    free_cnt += retired;
    retired = 0;
  }

  // ---- RobustPrune with slack alpha --------------------------------------
  // Candidates: drop the owner, tombstones and duplicates; order by (D, id);
  // keep at most prune_cap; then scan in order, keeping a candidate unless an
  // already-kept neighbor dominates it, i.e. alpha^2 * D(kept, c) <= D(p, c).
  std::vector<Entry> robust_prune(uint32_t p, const std::vector<uint32_t>& cand) const {
    std::vector<Entry> c;
    c.reserve(cand.size());
    for (uint32_t id : cand)
      if (id != p && !del[id]) c.push_back({D(p, id), id});
    std::sort(c.begin(), c.end(), key_less);
    std::vector<Entry> u;
    for (const Entry& e : c)
      if (u.empty() || u.back().id != e.id) u.push_back(e);
    tie_scan(u, prune_cap, [](const Entry& e) { return e.d; });  // order and the cap
    if (u.size() > prune_cap) u.resize(prune_cap);
    const double a2 = (double)alpha_num * alpha_num, b2 = (double)alpha_den * alpha_den;
    std::vector<char> alive(u.size(), 1);
    std::vector<Entry> out;
    for (size_t i = 0; i < u.size() && out.size() < R; ++i) {
      if (!alive[i]) continue;
      out.push_back(u[i]);
      for (size_t j = i + 1; j < u.size(); ++j) {
        if (!alive[j]) continue;
        const double lhs = a2 * D(u[i].id, u[j].id), rhs = b2 * u[j].d;
        tie_log(lhs, rhs, b2);
        if (lhs <= rhs) alive[j] = 0;
      }
    }
    return out;
  }

  // ---- greedy beam search -------------------------------------------------
  struct Slot {
    Entry e;
    bool expanded;
  };
  struct Search {
    std::vector<Slot> list;      // the candidate list, sorted by (d, id)
    std::vector<Entry> visited;  // expanded entries in expansion order
    uint64_t distances = 0;
  };

  Search beam_search(const void* q, uint32_t L, uint32_t vcap) {
    Search s;
    if (entries.empty() || L == 0) return s;
    new_stamp();
    // start: the L best of the entry set
    for (uint32_t e : entries) {
      stamp[e] = cur;
      s.list.push_back({{dtrav(q, e), e}, false});
    }
    s.distances = entries.size();
    std::sort(s.list.begin(), s.list.end(), [](const Slot& a, const Slot& b) { return key_less(a.e, b.e); });
    tie_scan(s.list, L, [](const Slot& x) { return x.e.d; });
    if (s.list.size() > L) s.list.resize(L);
    while (s.visited.size() < vcap) {
      std::vector<uint32_t> pick;  // up to W best unexpanded
      for (size_t i = 0; i < s.list.size() && pick.size() < W && s.visited.size() + pick.size() < vcap; ++i)
        if (!s.list[i].expanded) pick.push_back((uint32_t)i);
      if (pick.empty()) break;
      std::vector<uint32_t> nodes;
      for (uint32_t i : pick) {
        s.list[i].expanded = true;
        s.visited.push_back(s.list[i].e);
        nodes.push_back(s.list[i].e.id);
      }
      for (uint32_t p : nodes) {
        if (!has_slab[p]) continue;
        for (const Entry& nb : adj[p]) {
          uint32_t n = nb.id;
          if (stamp[n] == cur) continue;
          stamp[n] = cur;
          Entry c{dtrav(q, n), n};
          ++s.distances;
          if (s.list.size() == L && !key_less(c, s.list.back().e)) {
            tie_log(c.d, s.list.back().e.d);  // rejected at the worst entry
            continue;
          }
          auto it = std::upper_bound(s.list.begin(), s.list.end(), c,
                                     [](const Entry& a, const Slot& b) { return key_less(a, b.e); });
          if (it != s.list.begin()) tie_log(c.d, (it - 1)->e.d);  // its rank
          if (it != s.list.end()) tie_log(c.d, it->e.d);
          s.list.insert(it, Slot{c, false});
          if (s.list.size() > L) s.list.pop_back();
        }
      }
    }
    return s;
  }

  // The entry set: the n_entry smallest live ids (ids are handed out in
  // arrival order, so this is a sample of the live set that changes only
  // where a member is deleted).
  void refresh_entries() {
    entries.clear();
    for (uint64_t u = 0; u < next_id && entries.size() < n_entry; ++u)
      if (!del[u]) entries.push_back((uint32_t)u);
  }

  // ---- phases of one launch epoch (Definition 2) ---------------------------
  // Each phase reads the state the previous one left. An insert call runs
  // P0 (ids) P1 P2 P4 P5, a delete call P0 (tombstones) P3, and a round runs
  // all of them: P0, P1 (insert and query searches on the same state), P2,
  // P3, P4, P5, then the recycle that ends the epoch.

  // P0, deletes: per-position status; the accepted ids, ascending.
  std::vector<uint32_t> classify_deletes(const uint32_t* ids, uint64_t n, uint8_t* status) const {
    std::vector<uint32_t> Dl;
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t u = ids[i];
      bool dup = false;
      for (uint64_t j = 0; j < i && !dup; ++j) dup = ids[j] == u;
      uint8_t st;
      if (dup)
        st = DEL_DUPLICATE;
      else if (u >= next_id)
        st = DEL_OUT_OF_RANGE;
      else if (del[u])
        st = DEL_NOT_LIVE;
      else {
        st = DEL_OK;
        Dl.push_back(u);
      }
      if (status) status[i] = st;
    }
    std::sort(Dl.begin(), Dl.end());
    return Dl;
  }
  // P0, tombstones: the flag is set, degree and slab kept
  void tombstone(const std::vector<uint32_t>& Dl) {
    for (uint32_t u : Dl) del[u] = 1;
  }
  // P0, inserts: ids in input order, vectors (and their bf16 / fp8 copies)
  uint32_t store_rows(const void* vecs, uint64_t n, uint32_t* ids_out) {
    const uint32_t first = (uint32_t)next_id;
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t v = first + (uint32_t)i;
      if (ids_out) ids_out[i] = v;
      if (metric == M_L2_U8) {
        std::memcpy(&xu8[(size_t)v * dim], (const uint8_t*)vecs + i * dim, dim);
      } else {
        const float* src = (const float*)vecs + i * dim;
        std::memcpy(&xf[(size_t)v * dim], src, dim * sizeof(float));
        float amax = 0.f;
        for (uint32_t j = 0; j < dim; ++j) {
          xbf[(size_t)v * dim + j] = bf16_encode(src[j]);
          amax = std::max(amax, std::fabs(src[j]));
        }
        float sc = amax > 0.f ? amax / 448.0f : 1.0f;
        xscale[v] = sc;
        for (uint32_t j = 0; j < dim; ++j) xq8[(size_t)v * dim + j] = fp8_encode(src[j] / sc);
      }
    }
    next_id += n;
    return first;
  }
  // P1: candidate sets of the new nodes, from the state at the epoch's start;
  // bootstrap (no live node): the visit_cap nearest other batch members
  std::vector<std::vector<uint32_t>> candidates(uint32_t first, uint64_t n, bool bootstrap) {
    const uint32_t vcap = visit_cap(L_build);
    std::vector<std::vector<uint32_t>> cand(n);
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t v = first + (uint32_t)i;
      tie_owner = v;
      if (!bootstrap) {
        Search s = beam_search(vec(v), L_build, vcap);
        for (const Entry& e : s.visited) cand[i].push_back(e.id);
      } else {
        std::vector<Entry> all;
        for (uint64_t j = 0; j < n; ++j)
          if (j != i) all.push_back({D(v, first + (uint32_t)j), first + (uint32_t)j});
        std::sort(all.begin(), all.end(), key_less);
        tie_scan(all, vcap, [](const Entry& e) { return e.d; });
        if (all.size() > vcap) all.resize(vcap);
        for (const Entry& e : all) cand[i].push_back(e.id);
      }
    }
    tie_owner = NONE;
    return cand;
  }
  // P2: forward neighbors, own slab (uncontended)
  std::vector<std::vector<Entry>> forward(uint32_t first, uint64_t n, const std::vector<std::vector<uint32_t>>& cand) {
    std::vector<std::vector<Entry>> F(n);
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t v = first + (uint32_t)i;
      tie_owner = v;
      F[i] = robust_prune(v, cand[i]);
      publish(v, F[i]);
      ++pub_forward;
    }
    tie_owner = NONE;
    return F;
  }
  // P3: repair every live out-neighbor a of each deleted u, pairs sorted by
  // (a, u), one publication per a (Algorithm 3)
  void repair(const std::vector<uint32_t>& Dl) {
    std::vector<std::pair<uint32_t, uint32_t>> pairs;
    for (uint32_t u : Dl)
      for (const Entry& a : adj[u])
        if (!del[a.id]) pairs.push_back({a.id, u});
    std::sort(pairs.begin(), pairs.end());
    for (size_t i = 0; i < pairs.size();) {
      uint32_t a = pairs[i].first;
      tie_owner = a;
      std::vector<Entry> N = adj[a];
      size_t j = i;
      for (; j < pairs.size() && pairs[j].first == a; ++j) {
        uint32_t u = pairs[j].second;
        std::vector<uint32_t> B;
        for (const Entry& b : adj[u])
          if (b.id != a) B.push_back(b.id);
        std::vector<Entry> K = robust_prune(a, B);
        std::vector<uint32_t> c;
        for (const Entry& x : N)
          if (x.id != u) c.push_back(x.id);
        for (const Entry& x : K) c.push_back(x.id);
        N = robust_prune(a, c);
      }
      publish(a, N);
      ++pub_repair;
      i = j;
    }
    tie_owner = NONE;
  }
  // P4: reverse edges, sorted by (target, source), one publish per target
  void reverse(uint32_t first, uint64_t n, const std::vector<std::vector<Entry>>& F) {
    std::vector<std::pair<uint32_t, uint32_t>> pairs;
    for (uint64_t i = 0; i < n; ++i)
      for (const Entry& w : F[i])
        if (!del[w.id]) pairs.push_back({w.id, first + (uint32_t)i});
    std::sort(pairs.begin(), pairs.end());
    for (size_t a = 0; a < pairs.size();) {
      size_t b = a;
      uint32_t w = pairs[a].first;
      tie_owner = w;
      std::vector<Entry> N = adj[w];
      for (; b < pairs.size() && pairs[b].first == w; ++b) {
        uint32_t v = pairs[b].second;
        bool present = false;  // the offer is a set union: a listed v changes nothing
        for (const Entry& x : N) present = present || x.id == v;
        if (present) continue;
        if (N.size() < R) {
          Entry e{D(w, v), v};
          N.insert(std::upper_bound(N.begin(), N.end(), e, key_less), e);
        } else {
          std::vector<uint32_t> c;
          for (const Entry& x : N) c.push_back(x.id);
          c.push_back(v);
          N = robust_prune(w, c);
        }
      }
      publish(w, N);
      ++pub_reverse;
      a = b;
    }
    tie_owner = NONE;
  }
  // P5: refine -- offer each new node the same-batch nodes two hops away.
  // Every new node reads the lists as they stand when the pass starts; the
  // changed lists are published after all are computed.
  void refine_pass(uint32_t first, uint64_t n) {
    const uint32_t end = first + (uint32_t)n;
    std::vector<std::vector<Entry>> out(n);
    std::vector<char> changed(n, 0);
    for (uint64_t i = 0; i < n; ++i) {
      uint32_t v = first + (uint32_t)i;
      std::vector<uint32_t> c;
      for (const Entry& x : adj[v]) c.push_back(x.id);
      const size_t own = c.size();
      for (const Entry& w : adj[v])
        for (const Entry& b : adj[w.id])
          if (b.id >= first && b.id < end && b.id != v) c.push_back(b.id);
      bool extra = false;
      for (size_t j = own; j < c.size() && !extra; ++j) {
        bool in = false;
        for (size_t t = 0; t < own; ++t) in = in || c[t] == c[j];
        extra = !in;
      }
      if (!extra) continue;
      tie_owner = v;
      out[i] = robust_prune(v, c);
      tie_owner = NONE;
      bool same = out[i].size() == adj[v].size();
      for (size_t t = 0; same && t < out[i].size(); ++t) same = out[i][t].id == adj[v][t].id;
      changed[i] = !same;
    }
    for (uint64_t i = 0; i < n; ++i)
      if (changed[i]) {
        publish(first + (uint32_t)i, out[i]);
        ++pub_refine;
      }
  }

  // ---- insert call (Algorithm 2 over a batch; one launch) -------------------
  int insert(const void* vecs, uint64_t n, uint32_t* ids_out) {
    if (n == 0) return OK;
    if (next_id + n > cap) return ECAPACITY;
    if (free_cnt < n * (uint64_t)(R + 2)) return EPOOL;
    const uint32_t first = store_rows(vecs, n, ids_out);
    const bool bootstrap = entries.empty();
    auto cand = candidates(first, n, bootstrap);
    auto F = forward(first, n, cand);
    reverse(first, n, F);
    if (refine && !bootstrap) refine_pass(first, n);
    refresh_entries();
    recycle();
    return OK;
  }

  // ---- delete call (Algorithm 3 over a batch; one launch) -------------------
  int remove(const uint32_t* ids, uint64_t n, uint8_t* status) {
    std::vector<uint32_t> Dl = classify_deletes(ids, n, status);
    if (!tombstone_only && free_cnt < Dl.size() * (uint64_t)R) return EPOOL;
    tombstone(Dl);
    refresh_entries();
    if (!tombstone_only) repair(Dl);
    recycle();
    return OK;
  }

  // ---- round: deletes, inserts and queries in one launch epoch ---------------
  // The queries and the insert searches see the same state: the one left by
  // the tombstones (and the entry-set update) of this round, before any
  // repair or publication. Both checks run before any mutation.
  int round(const uint32_t* dids, uint64_t nd, uint8_t* status, const void* vecs, uint64_t ni, uint32_t* ids_out,
            const void* q, uint64_t nq, uint32_t k, uint32_t L, uint32_t* qids, void* qd) {
    std::vector<uint32_t> Dl = classify_deletes(dids, nd, status);
    if (next_id + ni > cap) return ECAPACITY;
    const uint64_t need = ni * (uint64_t)(R + 2) + (tombstone_only ? 0 : Dl.size() * (uint64_t)R);
    if (free_cnt < need) return EPOOL;
    tombstone(Dl);
    refresh_entries();
    const uint32_t first = store_rows(vecs, ni, ids_out);
    const bool bootstrap = entries.empty();
    auto cand = candidates(first, ni, bootstrap);
    const size_t qb = metric == M_L2_U8 ? dim : dim * sizeof(float);
    const size_t db = metric == M_L2_U8 ? sizeof(int32_t) : sizeof(double);
    for (uint64_t i = 0; i < nq; ++i)
      search((const uint8_t*)q + i * qb, k, L, qids + i * k, (uint8_t*)qd + i * k * db, nullptr, nullptr);
    auto F = forward(first, ni, cand);
    if (!tombstone_only) repair(Dl);
    reverse(first, ni, F);
    if (refine && !bootstrap) refine_pass(first, ni);
    refresh_entries();
    recycle();
    return OK;
  }

  // ---- reclaim call (Algorithm 4: compaction, then free) ---------------------
  int reclaim() {
    if (tombstone_only) return OK;
    std::vector<uint32_t> dirty;
    uint64_t dead = 0;
    for (uint64_t u = 0; u < next_id; ++u) {
      if (del[u]) continue;
      uint64_t k = 0;
      for (const Entry& e : adj[u]) k += del[e.id];
      if (k) dirty.push_back((uint32_t)u);
      dead += k;
    }
    if (free_cnt < dirty.size()) return EPOOL;
    dirty_last = dirty.size();
    dead_edges_last = dead;
    for (uint32_t u : dirty) {
      std::vector<Entry> N;
      for (const Entry& e : adj[u])
        if (!del[e.id]) N.push_back(e);
      publish(u, N);
      ++pub_compact;
    }
    for (uint64_t u = 0; u < next_id; ++u) {
      if (del[u] && has_slab[u]) {
        has_slab[u] = 0;
        adj[u].clear();
        resident -= 1;
        retired += 1;
        ++freed;
      }
    }
    recycle();
    return OK;
  }

  // ---- query call: top-k of the candidate list among live nodes -------------
  void search(const void* q, uint32_t k, uint32_t L, uint32_t* ids, void* dists, uint32_t* exp_out,
              uint32_t* dist_out) {
    Search s = beam_search(q, L, visit_cap(L));
    search_expansions += s.visited.size();
    search_distances += s.distances;
    if (exp_out) *exp_out = (uint32_t)s.visited.size();
    if (dist_out) *dist_out = (uint32_t)s.distances;
    std::vector<Entry> res;
    const bool rr = metric == M_IP_F32 && trav != T_NATIVE && rerank_mult > 0;  // 0: no re-rank
    const size_t want = rr ? (size_t)rerank_mult * k : k;
    for (const Slot& sl : s.list)
      if (res.size() < want && !del[sl.e.id]) res.push_back(sl.e);
    if (rr) {  // exact re-rank of the first rerank_mult*k live candidates
      for (Entry& e : res) e.d = dq(q, e.id);
      std::sort(res.begin(), res.end(), key_less);
      if (res.size() > k) res.resize(k);
    }
    for (uint32_t i = 0; i < k; ++i) {
      bool has = i < res.size();
      ids[i] = has ? res[i].id : NONE;
      if (metric == M_L2_U8)
        ((int32_t*)dists)[i] = has ? (int32_t)res[i].d : INT32_MAX;
      else
        ((double*)dists)[i] = has ? res[i].d : INFINITY;
    }
  }
};

}  // namespace

extern "C" {

void* oracle_create(int metric, int traversal, uint32_t dim, uint32_t R, uint32_t L_build, uint32_t W,
                    uint32_t visit_mult, uint32_t prune_cap, uint32_t alpha_num, uint32_t alpha_den,
                    uint32_t rerank_mult, uint32_t n_entry, uint64_t id_capacity, uint64_t slab_capacity,
                    int refine, int tombstone_only) {
  if (dim == 0 || R == 0 || R > 127 || W == 0 || alpha_den == 0 || id_capacity == 0 || n_entry == 0 ||
      id_capacity >= 0xFFFFFFFFull)
    return nullptr;
  if (metric != M_L2_U8 && metric != M_IP_F32) return nullptr;
  Oracle* o = new Oracle();
  o->metric = metric;
  o->trav = metric == M_L2_U8 ? T_NATIVE : traversal;
  o->dim = dim;
  o->R = R;
  o->L_build = L_build;
  o->W = W;
  o->visit_mult = visit_mult;
  o->prune_cap = prune_cap;
  o->alpha_num = alpha_num;
  o->alpha_den = alpha_den;
  o->rerank_mult = rerank_mult;
  o->n_entry = n_entry;
  o->cap = id_capacity;
  o->P = slab_capacity;
  o->free_cnt = slab_capacity;
  o->refine = refine;
  o->tombstone_only = tombstone_only;
  if (metric == M_L2_U8) {
    o->xu8.assign(id_capacity * dim, 0);
  } else {
    o->xf.assign(id_capacity * dim, 0.f);
    o->xbf.assign(id_capacity * dim, 0);
    o->xq8.assign(id_capacity * dim, 0);
    o->xscale.assign(id_capacity, 1.f);
  }
  o->del.assign(id_capacity, 0);
  o->has_slab.assign(id_capacity, 0);
  o->adj.assign(id_capacity, {});
  o->stamp.assign(id_capacity, 0);
  return o;
}

void oracle_destroy(void* h) { delete (Oracle*)h; }

int oracle_insert(void* h, const void* vecs, uint64_t n, uint32_t* ids_out) {
  return ((Oracle*)h)->insert(vecs, n, ids_out);
}

int oracle_delete(void* h, const uint32_t* ids, uint64_t n, uint8_t* status_out) {
  return ((Oracle*)h)->remove(ids, n, status_out);
}

int oracle_reclaim(void* h) { return ((Oracle*)h)->reclaim(); }

// One round: deletes, inserts and queries in one epoch, then (reclaim != 0)
// the reclaim call. Query results as for oracle_search.
int oracle_round(void* h, const uint32_t* del_ids, uint64_t nd, uint8_t* status_out, const void* vecs, uint64_t ni,
                 uint32_t* ids_out, const void* q, uint64_t nq, uint32_t k, uint32_t L, uint32_t* qids, void* qdists,
                 int reclaim) {
  Oracle* o = (Oracle*)h;
  if (nq && (k == 0 || k > L)) return EINVAL;
  int rc = o->round(del_ids, nd, status_out, vecs, ni, ids_out, q, nq, k, L, qids, qdists);
  if (rc == OK && reclaim) rc = o->reclaim();
  return rc;
}

// dists: int32 per result for the u8 metric, double for the float metric.
// expansions / distances (optional): per-query counts of expanded nodes and
// distance evaluations.
int oracle_search(void* h, const void* q, uint64_t nq, uint32_t k, uint32_t L, uint32_t* ids, void* dists,
                  uint32_t* expansions, uint32_t* distances) {
  Oracle* o = (Oracle*)h;
  if (k == 0 || k > L) return EINVAL;
  const size_t qb = o->metric == M_L2_U8 ? o->dim : o->dim * sizeof(float);
  const size_t db = o->metric == M_L2_U8 ? sizeof(int32_t) : sizeof(double);
  for (uint64_t i = 0; i < nq; ++i)
    o->search((const uint8_t*)q + i * qb, k, L, ids + i * k, (uint8_t*)dists + i * k * db,
              expansions ? expansions + i : nullptr, distances ? distances + i : nullptr);
  return OK;
}

// One beam search, returning the final candidate list (ids, distances,
// expanded flags) and the expanded set in expansion order.
int oracle_beam_search(void* h, const void* q, uint32_t L, uint32_t visit_cap, uint32_t* list_ids,
                       double* list_d, uint8_t* list_exp, uint32_t* list_n, uint32_t* vis_ids, double* vis_d,
                       uint32_t* vis_n, uint64_t* n_dist) {
  Oracle* o = (Oracle*)h;
  Oracle::Search s = o->beam_search(q, L, visit_cap);
  *list_n = (uint32_t)s.list.size();
  for (size_t i = 0; i < s.list.size(); ++i) {
    list_ids[i] = s.list[i].e.id;
    list_d[i] = s.list[i].e.d;
    list_exp[i] = s.list[i].expanded;
  }
  *vis_n = (uint32_t)s.visited.size();
  for (size_t i = 0; i < s.visited.size(); ++i) {
    vis_ids[i] = s.visited[i].id;
    vis_d[i] = s.visited[i].d;
  }
  if (n_dist) *n_dist = s.distances;
  return OK;
}

// RobustPrune of candidate ids for owner p, against the current state.
int oracle_robust_prune(void* h, uint32_t p, const uint32_t* cand, uint64_t n, uint32_t* out_ids, double* out_d,
                        uint32_t* out_n) {
  Oracle* o = (Oracle*)h;
  std::vector<uint32_t> c(cand, cand + n);
  for (uint32_t id : c)
    if (id >= o->next_id) return EINVAL;
  if (p >= o->next_id) return EINVAL;
  std::vector<Entry> r = o->robust_prune(p, c);
  *out_n = (uint32_t)r.size();
  for (size_t i = 0; i < r.size(); ++i) {
    out_ids[i] = r[i].id;
    out_d[i] = r[i].d;
  }
  return OK;
}

// Exact k nearest live nodes by (distance, id): the plain definition.
int oracle_bruteforce(void* h, const void* q, uint64_t nq, uint32_t k, uint32_t* ids, double* dists) {
  Oracle* o = (Oracle*)h;
  const size_t qb = o->metric == M_L2_U8 ? o->dim : o->dim * sizeof(float);
  for (uint64_t i = 0; i < nq; ++i) {
    const void* qi = (const uint8_t*)q + i * qb;
    std::vector<Entry> all;
    for (uint64_t u = 0; u < o->next_id; ++u)
      if (!o->del[u]) all.push_back({o->dq(qi, (uint32_t)u), (uint32_t)u});
    size_t kk = std::min<size_t>(k, all.size());
    std::partial_sort(all.begin(), all.begin() + kk, all.end(), key_less);
    for (uint32_t j = 0; j < k; ++j) {
      ids[i * k + j] = j < kk ? all[j].id : NONE;
      dists[i * k + j] = j < kk ? all[j].d : INFINITY;
    }
  }
  return OK;
}

// Install a neighbor list directly (test hook for hand-built graphs). The list
// is stored in (distance, id) order, with distances computed here.
int oracle_set_list(void* h, uint32_t u, const uint32_t* ids, uint32_t n) {
  Oracle* o = (Oracle*)h;
  if (u >= o->next_id || n > o->R) return EINVAL;
  std::vector<Entry> N;
  for (uint32_t i = 0; i < n; ++i) {
    if (ids[i] >= o->next_id) return EINVAL;
    N.push_back({o->D(u, ids[i]), ids[i]});
  }
  std::sort(N.begin(), N.end(), key_less);
  int rc = o->publish(u, N);
  o->recycle();
  return rc;
}

// Replace the entry set (test hook for hand-built graphs).
int oracle_set_entries(void* h, const uint32_t* ids, uint32_t n) {
  Oracle* o = (Oracle*)h;
  for (uint32_t i = 0; i < n; ++i)
    if (ids[i] >= o->next_id) return EINVAL;
  o->entries.assign(ids, ids + n);
  return OK;
}

int oracle_get_entries(void* h, uint32_t* ids) {
  Oracle* o = (Oracle*)h;
  for (size_t i = 0; i < o->entries.size(); ++i) ids[i] = o->entries[i];
  return (int)o->entries.size();
}

// State dump for ids [0, next_id): neighbor ids (R per id, unused = NONE),
// distances (double), degree, deletion flag, slab presence.
// meta: next_id, entry-set size, P, free, resident, retired, pub_forward, pub_repair,
//       pub_reverse, pub_refine, pub_compact, freed, dirty_last, dead_last,
//       search_expansions, search_distances
int oracle_export(void* h, uint32_t* nbr, double* rho, uint8_t* deg, uint8_t* del, uint8_t* has_slab,
                  int64_t* meta) {
  Oracle* o = (Oracle*)h;
  for (uint64_t u = 0; u < o->next_id; ++u) {
    const auto& N = o->adj[u];
    if (nbr)
      for (uint32_t i = 0; i < o->R; ++i) {
        nbr[u * o->R + i] = i < N.size() ? N[i].id : NONE;
        if (rho) rho[u * o->R + i] = i < N.size() ? N[i].d : 0.0;
      }
    if (deg) deg[u] = (uint8_t)N.size();
    if (del) del[u] = o->del[u];
    if (has_slab) has_slab[u] = o->has_slab[u];
  }
  if (meta) {
    int64_t m[16] = {(int64_t)o->next_id,     (int64_t)o->entries.size(),
                     (int64_t)o->P,           (int64_t)o->free_cnt,
                     (int64_t)o->resident,    (int64_t)o->retired,
                     (int64_t)o->pub_forward, (int64_t)o->pub_repair,
                     (int64_t)o->pub_reverse, (int64_t)o->pub_refine,
                     (int64_t)o->pub_compact, (int64_t)o->freed,
                     (int64_t)o->dirty_last,  (int64_t)o->dead_edges_last,
                     (int64_t)o->search_expansions, (int64_t)o->search_distances};
    std::memcpy(meta, m, sizeof(m));
  }
  return OK;
}

// Near-tie log (float metric): the nodes whose lists a comparison within the
// tie margin decided, since the last clear, in logging order (consecutive
// entries of one node folded, keeping the smallest relative margin). Writes up
// to cap (node, margin) pairs; returns the count; clear != 0 empties the log.
int64_t oracle_near_ties(void* h, uint32_t* owners, double* margins, uint64_t cap, int clear) {
  Oracle* o = (Oracle*)h;
  const uint64_t n = o->ties.size();
  for (uint64_t i = 0; i < n && i < cap; ++i) {
    owners[i] = o->ties[i].owner;
    margins[i] = o->ties[i].margin;
  }
  if (clear) o->ties.clear();
  return (int64_t)n;
}

// Stored low-precision copies of one vector (float metric only).
int oracle_get_codes(void* h, uint32_t u, uint16_t* bf16_out, uint8_t* fp8_out, float* scale_out) {
  Oracle* o = (Oracle*)h;
  if (o->metric != M_IP_F32 || u >= o->next_id) return EINVAL;
  for (uint32_t i = 0; i < o->dim; ++i) {
    if (bf16_out) bf16_out[i] = o->xbf[(size_t)u * o->dim + i];
    if (fp8_out) fp8_out[i] = o->xq8[(size_t)u * o->dim + i];
  }
  if (scale_out) *scale_out = o->xscale[u];
  return OK;
}

// Codec entry points for the format tests.
void oracle_bf16_encode(const float* x, uint64_t n, uint16_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = bf16_encode(x[i]);
}
void oracle_fp8_encode(const float* x, uint64_t n, uint8_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = fp8_encode(x[i]);
}
void oracle_fp8_decode(const uint8_t* c, uint64_t n, double* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = fp8_decode(c[i]);
}

}  // extern "C"
