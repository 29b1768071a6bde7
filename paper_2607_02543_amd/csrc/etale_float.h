// Float embeddings (inner-product similarity) for the ETALE kernels on gfx950.
//
// Distance d(a, b) = 1 - <a, b>; for unit vectors this is half the squared L2
// distance, so RobustPrune's alpha^2 rule reads the same on either. The FP32
// master rows decide everything that is stored (neighbor order, slab
// distances, RobustPrune, the re-rank); traversal may read a bf16 copy or an
// FP8 e4m3 copy with one FP32 scale per vector, always accumulating in FP32
// against the FP32 query.
//
// Rows are split into 16-byte chunks; G lanes share a row, each lane taking 3
// chunks (t*G + lane%G, t = 0..2), so a dimension of 96 * 2^j (j <= 3) maps
// onto a power-of-two G for all three element widths.
#pragma once

#include "etale_dev.h"

namespace etale {

enum Trav { TRAV_NATIVE = 0, TRAV_BF16 = 1, TRAV_FP8 = 2 };

// Order-preserving map of an FP32 value onto uint32, so (distance, id) keys
// compare as integers.
__host__ __device__ inline uint32_t fkey(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float fkey_inv(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __builtin_bit_cast(float, u);
}

// ---- number formats -------------------------------------------------------------------

// bfloat16 by round-to-nearest-even of the dropped 16 bits (NaN stays NaN)
__device__ inline uint16_t to_bf16(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// OCP FP8 E4M3FN (bias 7, no infinities, largest finite 448): round to
// nearest even on the binary32 bit pattern, saturating to +-448.
__device__ inline uint8_t to_e4m3(float y) {
  const uint32_t u = __builtin_bit_cast(uint32_t, y);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7FFFFFFFu;
  if (a > 0x7F800000u) return 0x7F;                 // NaN
  if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);  // >= 448
  if (a < 0x3C800000u) {                            // below 2^-6: multiples of 2^-9
    const float m = __builtin_rintf(__builtin_bit_cast(float, a) * 512.0f);  // exact scaling, ties to even
    return (uint8_t)(sign | (uint32_t)m);           // m == 8 is the smallest normal
  }
  int e = (int)(a >> 23) - 127;                     // -6 .. 8
  uint32_t m3 = (a >> 20) & 7u;
  const uint32_t rem = a & 0xFFFFFu;
  if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) ++m3;
  if (m3 == 8u) {
    m3 = 0;
    ++e;
  }
  if (e > 8 || (e == 8 && m3 == 7u)) return (uint8_t)(sign | 0x7Eu);
  return (uint8_t)(sign | ((uint32_t)(e + 7) << 3) | m3);
}

// e4m3fn code -> value / 256, exact: the code's low 7 bits shifted into a
// binary16 exponent/mantissa pattern give the same value scaled by 2^-8
// (subnormals included).
__device__ inline float e4m3_div256(uint32_t c) {
  const uint16_t h = (uint16_t)(((c & 0x80u) << 8) | ((c & 0x7Fu) << 7));
  return (float)__builtin_bit_cast(_Float16, h);
}

// ---- traversal distance: G lanes per row, 3 chunks per lane --------------------------------
template <int G, int TRAV>
struct TravF {
  static constexpr int EPC = TRAV == TRAV_NATIVE ? 4 : (TRAV == TRAV_BF16 ? 8 : 16);  // elements per chunk
  static constexpr int CPL = 3;
  static constexpr int VPP = 64 / G;
  struct Q {
    float v[CPL][EPC];
  };

  __device__ static Q load_query(const float* q) {
    Q r;
    const int c = lane_id() % G;
#pragma unroll
    for (int t = 0; t < CPL; ++t)
#pragma unroll
      for (int e = 0; e < EPC; ++e) r.v[t][e] = q[(size_t)(t * G + c) * EPC + e];
    return r;
  }

  __device__ static const uint4* row(const Index& ix, uint32_t id) {
    if (TRAV == TRAV_NATIVE) return reinterpret_cast<const uint4*>(ix.xf + (size_t)id * ix.dim);
    if (TRAV == TRAV_BF16) return reinterpret_cast<const uint4*>(ix.xb + (size_t)id * ix.dim);
    return reinterpret_cast<const uint4*>(ix.x8 + (size_t)id * ix.dim);
  }

  // this lane's share of <q, row> (FP8: of <q, row/scale>/256)
  __device__ static float partial(const Q& q, const uint4 (&w)[CPL]) {
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const uint32_t wd[4] = {w[t].x, w[t].y, w[t].z, w[t].w};
      if (TRAV == TRAV_NATIVE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_fmaf(q.v[t][e], __builtin_bit_cast(float, wd[e]), acc);
      } else if (TRAV == TRAV_BF16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc = __builtin_fmaf(q.v[t][2 * e], __builtin_bit_cast(float, wd[e] << 16), acc);
          acc = __builtin_fmaf(q.v[t][2 * e + 1], __builtin_bit_cast(float, wd[e] & 0xFFFF0000u), acc);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc = __builtin_fmaf(q.v[t][4 * e + b], e4m3_div256((wd[e] >> (8 * b)) & 0xFFu), acc);
      }
    }
    return acc;
  }

  __device__ static float scale(const Index& ix, uint32_t id) {
    return TRAV == TRAV_FP8 ? ix.xs[id] * 256.0f : 1.0f;
  }

  // keys (d, id) of ids[0..cnt) and, if cr, their reference words
  __device__ static void dist_batch(const Index& ix, const Q& q, const uint32_t* ids, int cnt, uint64_t* ck,
                                    uint64_t* cr) {
    const int l = lane_id();
    const int c = l % G, grp = l / G;
    for (int base = 0; base < cnt; base += 2 * VPP) {
      uint4 w[2][CPL];
      uint32_t id[2];
      uint64_t r[2];
      float sc[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int vi = base + u * VPP + grp;
        id[u] = vi < cnt ? ids[vi] : NONE;
        r[u] = 0;
        sc[u] = 1.f;
#pragma unroll
        for (int t = 0; t < CPL; ++t) w[u][t] = make_uint4(0, 0, 0, 0);
        if (id[u] != NONE) {
          const uint4* rw = row(ix, id[u]);
#pragma unroll
          for (int t = 0; t < CPL; ++t) w[u][t] = rw[t * G + c];
          if (c == 0) {
            if (cr) r[u] = load_ref(ix, id[u]);
            sc[u] = scale(ix, id[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float dot = partial(q, w[u]);
        dot = group_sum_t<G, float>(dot);
        const int vi = base + u * VPP + grp;
        if (c == 0 && vi < cnt) {
          ck[vi] = make_key(fkey(1.0f - sc[u] * dot), id[u]);
          if (cr) cr[vi] = r[u];
        }
      }
    }
  }
};

// ---- exact FP32 rows (master copy): G lanes per row, 3 float4 chunks per lane --------------
template <int G>
struct RowF {
  static constexpr int CPL = 3;
  static constexpr int VPP = 64 / G;
  __device__ static void load(const Index& ix, uint32_t id, float4 (&f)[CPL]) {
    const float4* rw = reinterpret_cast<const float4*>(ix.xf + (size_t)id * ix.dim);
    const int c = lane_id() % G;
#pragma unroll
    for (int t = 0; t < CPL; ++t) f[t] = rw[t * G + c];
  }
  __device__ static float dotp(const float4 (&a)[CPL], const float4 (&b)[CPL]) {
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      acc = __builtin_fmaf(a[t].x, b[t].x, acc);
      acc = __builtin_fmaf(a[t].y, b[t].y, acc);
      acc = __builtin_fmaf(a[t].z, b[t].z, acc);
      acc = __builtin_fmaf(a[t].w, b[t].w, acc);
    }
    return group_sum_t<G, float>(acc);
  }
};

// RobustPrune on FP32 rows, same selection rule as the uint8 variant: drop
// p, tombstones and duplicates; order by (d(p,c), id); keep at most
// prune_cap; keep c unless an earlier kept c' has a^2 d(c',c) <= b^2 d(p,c).
// Distances between candidates are computed when needed: for each kept c',
// the still-alive later candidates are listed and scored VPP at a time.
template <int G>
__device__ inline int robust_prune_f32(const Index& ix, uint32_t p, const uint32_t* cand, int n, PruneLds& s) {
  using RF = RowF<G>;
  constexpr int VPP = RF::VPP;
  const int l = lane_id();
  const int grp = l / G, c = l % G;
  float4 pf[3];
  RF::load(ix, p, pf);
  const int np = next_pow2_ge64(n);
  for (int base = 0; base < np; base += VPP) {
    const int vi = base + grp;
    uint32_t id = vi < n ? cand[vi] : NONE;
    if (id == p) id = NONE;
    if (id != NONE && ref_del(load_ref(ix, id))) id = NONE;
    float4 xf[3] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
    if (id != NONE) RF::load(ix, id, xf);
    const float dot = RF::dotp(pf, xf);
    if (c == 0 && vi < np) s.keys[vi] = id == NONE ? KEY_NONE : make_key(fkey(1.0f - dot), id);
  }
  wave_sync();
  wave_bitonic_sort(s.keys, np);
  int m = 0;
  for (int base = 0; base < np; base += 64) {
    const int i = base + l;
    const uint64_t k = s.keys[i];
    const bool keep = k != KEY_NONE && (i == 0 || s.keys[i - 1] != k);
    const uint64_t bm = ballot(keep);
    const int at = m + (int)lanes_below(bm);
    if (keep && at < s.rows) s.keys2[at] = k;
    m += __popcll(bm);
  }
  wave_sync();
  if (m > (int)ix.prune_cap) m = (int)ix.prune_cap;
  if (m > s.rows) m = s.rows;
  const int T = (m + 63) >> 6;
  uint32_t alive = 0;
  for (int t = 0; t < T; ++t)
    if (t * 64 + l < m) alive |= 1u << t;
  const float a2 = (float)ix.a2, b2 = (float)ix.b2;
  int cnt = 0, from = 0;
  while (cnt < (int)ix.R) {
    int j = -1;
    for (int t = from >> 6; t < T && j < 0; ++t) {
      const uint64_t bm = ballot(((alive >> t) & 1u) && (t * 64 + l) >= from);
      if (bm) j = t * 64 + (int)__builtin_ctzll(bm);
    }
    if (j < 0) break;
    const uint64_t kj = s.keys2[j];
    if (l == 0) {
      s.out_ids[cnt] = key_id(kj);
      s.out_d[cnt] = __builtin_bit_cast(uint32_t, fkey_inv(key_dist(kj)));
    }
    ++cnt;
    from = j + 1;
    if (cnt == (int)ix.R) break;
    // list the alive candidates after j
    int na = 0;
    for (int t = from >> 6; t < T; ++t) {
      const int i = t * 64 + l;
      const bool a = ((alive >> t) & 1u) && i >= from;
      const uint64_t bm = ballot(a);
      if (a) s.idx[na + (int)lanes_below(bm)] = (uint32_t)i;
      na += __popcll(bm);
    }
    wave_sync();
    if (na == 0) continue;
    float4 jf[3];
    RF::load(ix, key_id(kj), jf);
    for (int base = 0; base < na; base += VPP) {
      const int slot = base + grp;
      const int i = slot < na ? (int)s.idx[slot] : -1;
      float4 xf[3] = {make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0), make_float4(0, 0, 0, 0)};
      if (i >= 0) RF::load(ix, key_id(s.keys2[i]), xf);
      const float dji = 1.0f - RF::dotp(jf, xf);
      if (c == 0 && i >= 0) s.kill[i] = a2 * dji <= b2 * fkey_inv(key_dist(s.keys2[i])) ? 1 : 0;
    }
    wave_sync();
    for (int t = from >> 6; t < T; ++t) {
      const int i = t * 64 + l;
      if (((alive >> t) & 1u) && i >= from && s.kill[i]) alive &= ~(1u << t);
    }
    wave_sync();
  }
  wave_sync();
  return cnt;
}

// exact FP32 d(w, v) between stored rows, as the bit pattern stored in a slab
template <int G>
__device__ inline uint32_t dist1_f32(const Index& ix, uint32_t w, uint32_t v) {
  float4 a[3], b[3];
  RowF<G>::load(ix, w, a);
  RowF<G>::load(ix, v, b);
  const float d = 1.0f - RowF<G>::dotp(a, b);
  return __builtin_bit_cast(uint32_t, d);
}

}  // namespace etale
