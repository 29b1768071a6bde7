// Kernel argument blocks and host launchers shared by the kernels and the
// C-ABI implementation (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "etale_dev.h"

namespace etale {

enum SearchMode { MODE_QUERY = 0, MODE_INSERT = 1, MODE_BOOT = 2 };
enum DelStatus { DEL_OK = 0, DEL_NOT_LIVE = 1, DEL_OUT_OF_RANGE = 2, DEL_DUPLICATE = 3 };

struct SearchArgs {
  int mode;            // MODE_QUERY or MODE_INSERT
  const void* q;       // MODE_QUERY: [nq x dim] query rows (uint8 or FP32)
  uint32_t first;      // MODE_INSERT: query i is stored vector first + i
  uint32_t nq, L, k, vcap, vt_mask;
  uint32_t W;          // expansions per step: 1, 2 (2R <= 64) or 4 (2R <= 64, two halves of 64 lanes)
  uint32_t lds_per_wave;
  int32_t trav;        // float rows: traversal copy of this launch
  uint32_t rerank;     // float rows, bf16 / FP8 copy: re-rank rerank*k candidates (0: none)
  const uint64_t* init_keys;  // [nq x init_stride] initial list from k_scan
  const uint32_t* init_n;     // [nq]
  uint32_t init_stride;
  uint32_t* out_ids;   // MODE_QUERY: [nq x k]
  uint32_t* out_d;     // MODE_QUERY: [nq x k] int32 (uint8 rows) or FP32 (float rows) bit patterns
  uint64_t* vis_keys;  // MODE_INSERT: [nq x vcap] expanded keys
  uint32_t* vis_cnt;   // [nq]
  uint32_t* counts;    // optional [nq x 2]: expansions, distance evaluations
  Dyn d;               // launch-time count (nq) and first id
  uint32_t persistent; // 1: waves take queries from a work queue (count known only on the device)
  uint32_t row_lanes;  // uint8 rows: lanes per row in distance batches (0: dim / 16); result-invariant
};

// k_scan: the L best start nodes (entry set, or the batch for a bootstrap,
// excluding the query itself) of every query, in (distance, id) order
// uint8 start-set selection: start rows per span (a start set holds at most
// 64 spans), key slots per query (split evenly over the spans), keys sorted
// per query before the dense fallback, and the longest list selected from
// those keys (longer lists write the distance matrix)
constexpr uint32_t SCAN_SPAN = 256, SCAN_KEYS_Q = 2048, SCAN_CAND_CAP = 1024, SCAN_FILTER_L_MAX = 128;
// bytes of the uint8 entry set's operand-ordered copy: n entries padded to a
// multiple of 32, rows padded to whole 64-byte slices
inline uint64_t ent_copy_bytes(uint64_t n, uint32_t dim) { return (n + 31) / 32 * 32 * ((dim + 63) / 64 * 64); }

struct ScanArgs {
  int mode;
  const void* q;       // MODE_QUERY rows; otherwise query i is stored vector first + qoff + i
  uint32_t first, qoff, nq, L;  // a bootstrap's start set is stored vectors [first, first + ns)
  int32_t trav;        // float rows: traversal copy the start rows are read from
  uint32_t ns;         // start-set size (entry count, or the batch size for a bootstrap)
  uint32_t* dist;      // [nq x ns] scratch distance matrix
  uint32_t* gmin;      // [nq x g_stride] smallest distance of each group of start rows
  uint32_t g_stride;   // group slots per query (upper bound over the launch-time ns)
  uint32_t g_rows;     // start rows per scoring tile; each tile has g_rows / 32 group slots
  uint32_t* bound;     // uint8 rows: [nq] bound on the L-th smallest distance
  uint32_t* ncand;     // uint8 rows: [nq x spans] rows at or below the bound in each span of start rows,
                       // one byte per scoring lane
  uint64_t* cand;      // uint8 rows: [nq x SCAN_KEYS_Q] their (distance, row) keys, by span
  uint64_t* out_keys;  // [nq x out_stride]
  uint32_t* out_n;     // [nq]
  uint32_t out_stride;
  uint32_t ns_ctr;     // counter with the start-set size (NO_CTR: ns as given)
  Dyn d;               // launch-time count (nq) and first id
};

struct MaintArgs {
  uint32_t first, n;       // new ids [first, first + n) / number of deleted ids
  uint32_t vcap;
  uint64_t* vis_keys;       // insert searches' expanded keys; refine's new lists
  uint32_t* vis_cnt;
  uint32_t* F;             // [n x R] forward lists
  uint64_t* pairs;         // (target, source) keys, sorted for the apply kernels
  uint32_t npairs;
  const uint32_t* dlist;   // deleted ids of the call
  uint32_t nmax;           // largest candidate count one prune sees
  uint32_t nsort;          // power of two >= nmax, >= 64
  uint32_t prune_cap;      // LDS staging rows
  uint32_t vstride;        // bytes per staged row
  uint32_t lds_per_wave;
  const uint32_t* seg;     // starts of the runs of one target in the sorted pairs
  uint32_t np_ctr = NO_CTR, np_mult = 1;  // launch-time pair count
  uint32_t chain = 0;      // reverse edges: cached candidate state (uint8 rows, R <= 32)
  uint32_t mx = 0;         // RobustPrune selection on the matrix cores (uint8 rows, dim <= 128, R <= 32)
  Dyn d;                   // launch-time count (n) and first id
};

enum MaintKernel { MK_FORWARD = 0, MK_REVERSE = 1, MK_REFINE = 2, MK_REPAIR = 3, MK_REVERSE_FAST = 4 };

hipError_t launch_init(const Index& ix, hipStream_t s);
hipError_t launch_recycle(const Index& ix, hipStream_t s);
// round control: counts (device array, or the host values when null), gate
hipError_t launch_round_begin(const Index& ix, const uint32_t* counts, uint32_t nd, uint32_t ni, uint32_t nq,
                              uint32_t max_d, uint32_t max_i, uint32_t max_q, int32_t* status, hipStream_t s);
hipError_t launch_round_gate(const Index& ix, uint32_t tombstone_only, uint32_t boot_max, int32_t* status,
                             hipStream_t s);
hipError_t launch_reclaim_gate(const Index& ix, int32_t* status, hipStream_t s);
hipError_t launch_store_rows(const Index& ix, const void* src, uint32_t* ids_out, uint32_t first, uint32_t n, Dyn d,
                             hipStream_t s);
// uint8 rows with dim <= 256: their squared norms into the new ids' reference words
hipError_t launch_row_norms(const Index& ix, uint32_t first, uint32_t n, Dyn d, hipStream_t s);
hipError_t launch_refresh_entries(const Index& ix, uint32_t bound, uint32_t S, Dyn d, hipStream_t s);
// serving: results (nq x k) to rows pos[i] of the caller's (n_requests x k) arrays
hipError_t launch_scatter_results(const uint32_t* ids, const uint32_t* d, const uint32_t* pos, uint32_t nq, uint32_t k,
                                  uint32_t* out_ids, uint32_t* out_d, hipStream_t s);
hipError_t launch_gather_rows(const void* rows, const uint32_t* idx, uint32_t n, uint32_t row_bytes, void* out,
                              hipStream_t s);
uint32_t search_lds_per_wave(uint32_t L, uint32_t vt_slots, uint32_t W);
uint32_t scan_select_lds_per_wave(uint32_t L);
hipError_t launch_scan(const Index& ix, const ScanArgs& a, hipStream_t s, hipEvent_t after_dist = nullptr);
hipError_t launch_search(const Index& ix, const SearchArgs& a, uint32_t waves_per_block, hipStream_t s);
uint32_t maint_lds_per_wave(const MaintArgs& a, uint32_t R);
uint32_t chain_lds_per_wave(uint32_t R, uint32_t vstride);
uint32_t pool_lds_per_wave(uint32_t vstride);
hipError_t launch_maint(MaintKernel which, const Index& ix, const MaintArgs& a, uint32_t nwaves,
                        uint32_t waves_per_block, hipStream_t s);
hipError_t launch_reverse_pairs(const Index& ix, const MaintArgs& a, hipStream_t s);
hipError_t launch_repair_pairs(const Index& ix, const MaintArgs& a, hipStream_t s);
hipError_t launch_segments(const Index& ix, const uint64_t* pairs, uint32_t nmax, Dyn d, uint32_t* seg,
                           hipStream_t s);
// stable LSD radix sort of 64-bit keys on bits [lo, lo + nbits), preceded by
// bits [0, low_bits) (so the order is by the high range, then the low one);
// count read at launch time; returns the buffer (a or b) holding the result
uint32_t sort_hist_words(uint32_t nmax);
hipError_t launch_sort(const Index& ix, uint64_t* a, uint64_t* b, uint32_t nmax, Dyn d, int lo, int nbits,
                       uint32_t* hist, hipStream_t s, uint64_t** result, int low_bits = 0);
hipError_t launch_del_keys(const Index& ix, const uint32_t* ids, uint32_t n, Dyn d, uint64_t* keys, hipStream_t s);
hipError_t launch_del_classify(const Index& ix, const uint64_t* sorted, uint32_t n, Dyn d, uint8_t* status,
                               uint32_t* dlist, hipStream_t s);
hipError_t launch_tombstone(const Index& ix, const uint32_t* dlist, uint32_t n, Dyn d, hipStream_t s);
hipError_t launch_del_bitmap(const Index& ix, uint64_t n_ids, Dyn d, uint64_t* bitmap, hipStream_t s);
hipError_t launch_dirty(const Index& ix, uint64_t n_ids, Dyn d, const uint64_t* bitmap, uint32_t* dirty,
                        hipStream_t s);
hipError_t launch_compact(const Index& ix, const uint32_t* dirty, uint64_t n, Dyn d, const uint64_t* bitmap,
                          hipStream_t s);
hipError_t launch_free_tombstones(const Index& ix, uint64_t n_ids, Dyn d, hipStream_t s);
hipError_t launch_export(const Index& ix, uint64_t n_ids, uint32_t* nbr, uint32_t* rho, uint8_t* deg, uint8_t* del,
                         uint8_t* has_slab, hipStream_t s);
// exact k nearest live rows; uint8 rows of 64..256 bytes run on the matrix
// cores with `scratch` of bruteforce_scratch_bytes() (0: no scratch needed)
uint64_t bruteforce_scratch_bytes(const Index& ix, uint32_t nq, uint64_t n_ids);
hipError_t launch_bruteforce(const Index& ix, const void* q, uint32_t nq, uint64_t n_ids, uint32_t k,
                             uint32_t* out_ids, uint32_t* out_d, hipStream_t s, unsigned char* scratch = nullptr);
hipError_t launch_encode(const Index& ix, uint32_t first, uint32_t n, Dyn d, float* xs, uint16_t* xb, uint8_t* x8,
                         hipStream_t s);
hipError_t launch_set_lists(const Index& ix, const MaintArgs& a, const uint32_t* ids, const uint32_t* nbr,
                            const uint32_t* deg, hipStream_t s);

}  // namespace etale
