/* ETALE dynamic graph index on one AMD Instinct MI355X (gfx950): C ABI.
 *
 * The index is a degree-bounded directed proximity graph over a fixed id
 * space (paper Section 3.2, Definition 1). Each id owns one 64-bit reference
 * word <deletion flag, degree, slab id>; its neighbor list lives in an
 * immutable slab of R (neighbor id, distance) entries drawn from a pool, and
 * every list change is a copy-on-write publication that swaps the reference
 * with one 64-bit compare-and-swap (Section 3.3, Algorithm 1).
 *
 * Calls and what they follow in the paper:
 *   etale_insert_batch   Insert, Algorithm 2 (Section 3.4.1), over a batch
 *   etale_delete_batch   Delete with connectivity repair, Algorithm 3 (3.4.2)
 *   etale_reclaim        Reclaim, Algorithm 4 (3.4.3)
 *   etale_search_batch   the query side of the problem statement (3.1): a
 *                        greedy beam search whose output admits only nodes
 *                        whose reference has deletion flag 0 (3.4.2)
 *   etale_round          deletes, inserts and queries of one round in one
 *                        launch epoch (Definition 2), counts read on the
 *                        device, optionally replayed from a HIP graph
 *
 * Round semantics. Every mutating call is one round: its phases run in a
 * fixed order and each phase reads the state the previous one left. The
 * searches of an insert call all see the graph as it was when the call
 * started, so members of one batch do not see each other; writes aimed at the
 * same node within a phase are applied in ascending source-id order and
 * published once. Retired slabs return to the free pool only at the end of a
 * call (the epoch separation of Lemma 1). All orders are lexicographic on
 * (distance, id).
 *
 * Memory. The library owns every piece of index state (vectors, references,
 * slab pool, scratch) in device memory allocated by etale_create and freed by
 * etale_destroy. Arguments named *_dev are device pointers owned by the
 * caller, valid for the duration of the call's stream work; *_host arguments
 * are host pointers. Calls are ordered on the stream given in the config
 * (NULL = the default stream) and may return before the device work ends,
 * except create, destroy, get_stats, export and reclaim, which synchronize.
 * Calls that must check the slab pool (insert, delete, reclaim) synchronize
 * the stream once before mutating anything.
 *
 * Errors. No call aborts or throws. Argument errors return ETALE_EINVAL and
 * change nothing. A call that cannot be covered by the free slab pool returns
 * ETALE_EPOOL, or by the id space ETALE_ECAPACITY, before any change; the
 * caller may reclaim and retry. A HIP failure returns ETALE_EDEVICE and
 * poisons the handle: later calls return ETALE_ESTATE. etale_last_error
 * describes the last failure.
 *
 * Vectors: ETALE_METRIC_L2_U8 stores dim uint8 per vector (dim a power of two,
 * 16..1024) and uses the exact squared L2 distance in 32-bit integers; its
 * distances are int32. ETALE_METRIC_IP_F32 stores dim FP32 per vector (dim
 * 96, 192, 384 or 768), uses d = 1 - <a, b> (for unit vectors half the
 * squared L2 distance), and its distances are float. Neighbor lists, their
 * stored distances and RobustPrune always use the FP32 rows; only traversal
 * reads the bf16 / FP8 copy.
 */
#ifndef ETALE_H
#define ETALE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct etale_index* etale_t;
typedef int32_t etale_status;

enum {
  ETALE_OK = 0,
  ETALE_EINVAL = -1,
  ETALE_ENOMEM = -2,
  ETALE_EPOOL = -3,
  ETALE_ECAPACITY = -4,
  ETALE_EDEVICE = -5,
  ETALE_ESTATE = -6
};

enum { ETALE_METRIC_L2_U8 = 0, ETALE_METRIC_IP_F32 = 1 };

/* traversal copy of ETALE_METRIC_IP_F32 rows: FP32 itself, bf16, or FP8
 * e4m3 with one FP32 scale per row; accumulation is FP32 in every case */
enum { ETALE_TRAV_NATIVE = 0, ETALE_TRAV_BF16 = 1, ETALE_TRAV_FP8E4M3 = 2 };

/* per-id outcome of etale_delete_batch */
enum { ETALE_DEL_OK = 0, ETALE_DEL_NOT_LIVE = 1, ETALE_DEL_OUT_OF_RANGE = 2, ETALE_DEL_DUPLICATE = 3 };

typedef struct {
  uint32_t dim;              /* vector length */
  uint32_t R;                /* slab capacity = maximum out-degree, 1..64 */
  uint32_t L_build;          /* candidate-list length of insert searches */
  uint32_t alpha_num;        /* RobustPrune slack alpha = alpha_num / alpha_den, */
  uint32_t alpha_den;        /*   applied to squared distances as alpha^2 */
  uint32_t visit_mult;       /* a search expands at most visit_mult * L nodes */
  uint32_t prune_cap;        /* RobustPrune keeps at most this many nearest candidates */
  uint32_t n_entry;          /* entry set = the n_entry smallest live ids */
  uint32_t refine;           /* 1: run the same-batch refine pass of inserts */
  uint32_t tombstone_only;   /* 1: delete only flags; no repair, no reclaim */
  uint32_t publish_attempts; /* CAS attempt budget of one publication */
  uint32_t max_batch;        /* largest insert / delete batch of one call */
  uint32_t vt_slots;         /* visited-table slots per search (power of two) */
  uint32_t waves_per_block;  /* search wavefronts per workgroup */
  int32_t metric;            /* ETALE_METRIC_* */
  int32_t traversal;         /* ETALE_TRAV_* (float metric only) */
  uint32_t rerank_mult;      /* bf16 / FP8 traversal: re-rank rerank_mult*k results in FP32 (k*mult <= 64);
                                0 returns the traversal distances themselves */
  uint32_t copies;           /* extra traversal copies to keep (1: bf16, 2: FP8), for query-side switching */
  uint32_t W;                /* entries expanded per search step: 1, 2 or 4 (2 and 4 need 2R <= 64) */
  uint32_t reserved;
  uint64_t id_capacity;      /* size of the id space */
  uint64_t slab_capacity;    /* slabs in the pool */
  void* hip_stream;          /* hipStream_t, or NULL */
} etale_config;

typedef struct {
  uint64_t next_id;          /* ids handed out so far */
  uint64_t live;             /* ids with deletion flag 0 */
  uint64_t tombstones;       /* flagged ids that still hold a slab */
  uint64_t slab_capacity;
  uint64_t free_slabs;
  uint64_t resident_slabs;   /* slabs named by some reference */
  uint64_t n_entries;
  uint64_t pub_forward, pub_repair, pub_reverse, pub_refine, pub_compact;
  uint64_t freed;            /* tombstone slabs retired by reclaim */
  uint64_t dirty_last;       /* live nodes republished by the last compaction */
  uint64_t dead_edges_last;  /* edges into tombstones found by the last compaction */
  uint64_t search_expansions, search_distances; /* totals over search calls */
  uint64_t cas_failures, publish_dropped;
  uint64_t device_bytes;     /* device memory held by the index */
  uint64_t error_bits;
} etale_stats;

/* Create an index on the current HIP device. On success *out receives the
 * handle. Errors: EINVAL (bad config), ENOMEM, EDEVICE. */
etale_status etale_create(const etale_config* cfg, etale_t* out);

/* Release every device allocation of the index. NULL is accepted. */
etale_status etale_destroy(etale_t ix);

/* Make later calls run on stream (hipStream_t, NULL = default). */
etale_status etale_set_stream(etale_t ix, void* stream);

/* Insert n vectors (vecs_dev: n x dim elements, row-major). Ids are handed
 * out in input order, starting at the current next id, and written to
 * ids_out_dev (n uint32, may be NULL). Worst-case slab demand n * (R + 2)
 * must be free, else ETALE_EPOOL; next id + n must fit the id space, else
 * ETALE_ECAPACITY. n must not exceed max_batch. */
etale_status etale_insert_batch(etale_t ix, const void* vecs_dev, uint64_t n, uint32_t* ids_out_dev);

/* Delete the ids in ids_dev (n uint32). status_out_dev (n bytes, may be
 * NULL) receives ETALE_DEL_* per position: repeats of an id in one call are
 * DUPLICATE (the first occurrence wins), ids never handed out are
 * OUT_OF_RANGE, already deleted ids are NOT_LIVE. Worst-case slab demand
 * (OK count) * R must be free, else ETALE_EPOOL with nothing changed. */
etale_status etale_delete_batch(etale_t ix, const uint32_t* ids_dev, uint64_t n, uint8_t* status_out_dev);

/* Search nq query rows (q_dev: nq x dim) with candidate-list length L,
 * 1 <= k <= L <= 256. Writes the k best live results per query in (distance,
 * id) order: ids_out_dev (nq x k uint32) and dists_out_dev (nq x k int32 or
 * float), padded with id 0xFFFFFFFF and distance INT32_MAX / +inf. With a
 * bf16 / FP8 traversal the first rerank_mult*k live candidates are re-scored
 * from the FP32 rows and the best k returned. counts_out_dev (nq x 2 uint32,
 * may be NULL) receives the expansions and distance evaluations. */
etale_status etale_search_batch(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                                uint32_t* ids_out_dev, void* dists_out_dev, uint32_t* counts_out_dev);

/* etale_search_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that must not call hipMalloc,
 * harnesses that forbid it): the same search, same arguments, same results
 * bit for bit, but the start-set scan's scratch (initial lists, distance
 * rows, group minima, bounds and bounded keys) lives in one static device
 * array of 64 MiB per GPU, held from library load until the process ends,
 * instead of the buffers etale_create allocates. The call makes no
 * allocation of any kind; queries run in chunks of as many as fit that array
 * (about 1,500 at n_entry = 8,192). Every call on one GPU, from any index,
 * shares the array and leaves its contents behind (nothing in it needs to
 * start cleared: each chunk writes what it later reads), so calls that
 * overlap on one GPU (other streams, other threads) race: serialize them.
 * Errors: as etale_search_batch, plus EINVAL when the scratch of a single
 * query (n_entry and L) exceeds the array. */
etale_status etale_search_batch_noalloc(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                                        uint32_t* ids_out_dev, void* dists_out_dev, uint32_t* counts_out_dev);

/* Compaction, then release of every tombstone's slab (Algorithm 4). The
 * number of dirty nodes must be covered by free slabs, else ETALE_EPOOL with
 * nothing changed. A no-op in tombstone-only mode. */
etale_status etale_reclaim(etale_t ix);

/* One round (Definition 2 over a mixed batch): deletes, inserts and queries
 * in one launch epoch, phases in this order:
 *   P0  classify the deletes (as etale_delete_batch), check id space and the
 *       worst-case slab demand n_ins*(R+2) + n_del_accepted*R (n_ins*(R+2)
 *       with tombstone_only), then tombstone, update the entry set and hand
 *       out the new ids in input order;
 *   P1  the insert searches (or the bootstrap, when no live node is left) and
 *       the queries, all on the state P0 left;
 *   P2  forward prunes; P3 repairs (Algorithm 3); P4 reverse edges; P5 refine
 *       (as the separate calls); then the retired slabs are recycled;
 *   and, with reclaim != 0, the reclaim call (Algorithm 4).
 * A round without deletes and queries is etale_insert_batch, one with only
 * deletes is etale_delete_batch.
 *
 * Counts: `counts` (device, [3] = deletes, inserts, queries) is read by the
 * kernels when they run, so a round can be enqueued before its inputs are
 * known; NULL means the max_* values are the counts. The max_* values fix the
 * launch shapes and the buffer sizes: del_ids [max_del], del_status
 * [max_del] (optional), ins_vecs [max_ins x dim] (uint8 or FP32), ins_ids
 * [max_ins] (optional), queries [max_q x dim], q_ids / q_dists [max_q x k]
 * (int32 distances for the uint8 metric, FP32 for the float metric). All are
 * device pointers owned by the caller.
 *
 * Status: status (device, int32 [2]) receives the round status (ETALE_OK,
 * ETALE_EPOOL, ETALE_ECAPACITY, or ETALE_EINVAL for counts above their max or
 * a bootstrap batch above 16384) and the reclaim status (ETALE_OK or
 * ETALE_EPOOL). A failed round changes no index state (per-id delete statuses
 * are still written: they are the classification, not a change); a failed
 * reclaim changes nothing either. The call itself only checks its arguments
 * and returns before the device work ends; read status after etale_sync.
 *
 * graph != 0: the round's launches are captured into a HIP graph on first
 * use and replayed on later calls with the same descriptor (buffers, max_*,
 * k, L, reclaim) and query traversal; write the next round's inputs and
 * counts into the same buffers and call again. Returns before the device work
 * ends, like every stream-ordered call. */
typedef struct {
  const uint32_t* del_ids;
  uint8_t* del_status;
  uint32_t max_del;
  const void* ins_vecs;
  uint32_t* ins_ids;
  uint32_t max_ins;
  const void* queries;
  uint32_t* q_ids;
  void* q_dists;
  uint32_t max_q;
  uint32_t k, L;
  const uint32_t* counts;
  int32_t* status;
  int32_t reclaim;
  int32_t graph;
} etale_round_desc;

etale_status etale_round(etale_t ix, const etale_round_desc* desc);

/* Exact k nearest live nodes of each query by (distance, id), 1 <= k <= 16,
 * from the uint8 / FP32 rows: the plain definition used to measure recall. */
etale_status etale_bruteforce(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t* ids_out_dev,
                              void* dists_out_dev);

/* Counters and pool state (synchronizes). */
etale_status etale_get_stats(etale_t ix, etale_stats* out_host);

/* Dump ids [0, n_ids) (n_ids <= next id): R neighbor ids and R distances per
 * id (unused entries 0xFFFFFFFF / 0), degree, deletion flag and slab
 * presence, into host buffers (synchronizes). Any pointer may be NULL. */
etale_status etale_export(etale_t ix, uint64_t n_ids, uint32_t* nbr_host, void* dist_host, uint8_t* deg_host,
                          uint8_t* del_host, uint8_t* has_slab_host);

/* Entry-set members in ascending id order (up to cap ids); returns the
 * count through *n_out (synchronizes). */
etale_status etale_get_entries(etale_t ix, uint32_t* ids_host, uint64_t cap, uint64_t* n_out);

/* Queries from now on traverse the given copy (ETALE_TRAV_*; it must be the
 * configured one or kept through `copies`) with the given re-rank multiplier;
 * inserts keep using the configured traversal. */
etale_status etale_set_query_traversal(etale_t ix, int32_t traversal, uint32_t rerank_mult);

/* Install neighbor lists (import): for each of the n ids in ids_host, the
 * first deg_host[i] (<= R) entries of row i of nbr_host (n x R uint32) become
 * its list, with distances computed from the stored rows and ordered by
 * (distance, id); each install is one copy-on-write publication. Every id
 * must be live and every neighbor must be a handed-out id, else EINVAL with
 * nothing changed. Synchronizes. */
etale_status etale_set_lists(etale_t ix, uint64_t n, const uint32_t* ids_host, const uint32_t* nbr_host,
                             const uint32_t* deg_host);

/* Copy rows [first, first + n) of a stored copy into out_host: which = 0 the
 * vectors as inserted (uint8 or FP32), 1 the bf16 copy (uint16), 2 the FP8
 * e4m3 codes (uint8), 3 the FP8 scales (one float per row). EINVAL when that
 * copy is not kept. Synchronizes. */
etale_status etale_export_rows(etale_t ix, uint64_t first, uint64_t n, int32_t which, void* out_host);

/* Stage timing of search calls: when enabled, HIP events are recorded on the
 * index's stream around each start-set block kernel, start-set select kernel
 * and beam-search kernel of every search launch. etale_get_search_timing
 * synchronizes, writes up to cap launches as (scan, select, search)
 * millisecond triples in launch order into ms_host (cap x 3), the number of
 * recorded launches into *launches, and forgets them. */
/* ---- serving: continuous batching of a request stream ---------------------
 * The problem statement of Section 3.1 has readers (searches) and writers
 * (inserts, deletes) running against one graph at the same time. Here the
 * requests are admitted in ticks, and every tick's work runs on two streams:
 *   - its searches on the index's stream, against a snapshot taken when the
 *     tick starts (reference words, counters, entry set and its rows: the state
 *     the previous tick's updates left), and
 *   - its deletes and inserts as one round (etale_round without queries, plus
 *     the reclaim every reclaim_every ticks) on a second stream,
 * so a tick's searches and its updates overlap on the device. The next tick's
 * snapshot waits for both. Two sets of tick buffers alternate, so the host
 * admits and enqueues tick t+1 while tick t runs. A slab that tick t's round
 * retires is reused only by tick t+1's round, which starts after tick t's
 * searches end: the epoch separation of Lemma 1, kept across the two streams.
 * A search therefore returns exactly what the same query returns alone on the
 * tick's snapshot (etale_search_batch on the state after the previous tick).
 *
 * Admission: a tick takes pending requests in arrival order, up to max_tick.
 * A search is always admitted. An insert or delete is admitted only if the
 * free slab pool, less the worst-case demand of the tick still in flight,
 * covers the tick's worst-case demand n_ins*(R+2) + n_del*R; otherwise it
 * waits for a later tick while the requests behind it go ahead (counted in
 * `deferred`, once per skip). An insert that would take rows +
 * resident slabs + the library's fixed buffers past hbm_budget_bytes (if
 * nonzero), or the ids past the id space, is rejected (latency -1).
 *
 * Clock: realtime != 0 replays the arrival times on the wall clock from the
 * first request (a request is admitted no earlier than it arrives; latency =
 * completion - arrival, completions read from device events). realtime == 0
 * ignores the arrival times and admits the next max_tick requests per tick
 * (saturated throughput; the tick composition then depends only on the trace
 * and the pool); latency is then completion - the tick's start.
 * With graph != 0 each tick's round replays a captured round for the
 * power-of-two size bucket of its counts. */
enum { ETALE_REQ_SEARCH = 0, ETALE_REQ_INSERT = 1, ETALE_REQ_DELETE = 2 };

typedef struct {
  double t_arrive; /* seconds on the trace clock, nondecreasing */
  uint32_t kind;   /* ETALE_REQ_* */
  uint32_t arg;    /* search / insert: row of rows_dev; delete: the id */
} etale_request;

typedef struct {
  uint32_t k, L;             /* every search: top k from a list of L */
  uint32_t max_tick;         /* requests admitted per tick, at most max_batch */
  uint32_t reclaim_every;    /* ticks between reclaims (0: never) */
  uint64_t hbm_budget_bytes; /* 0, or the budget inserts are admitted against */
  int32_t graph;             /* replay size-bucketed captured rounds */
  int32_t realtime;          /* 1: arrivals on the wall clock; 0: saturated */
} etale_serve_config;

typedef struct {
  uint64_t ticks, searches, inserts, deletes, rejected_inserts, deferred, reclaims, failed_ticks;
  uint64_t peak_resident_slabs, final_resident_slabs, ids_handed_out, graphs;
  double wall_seconds;        /* from the loop's start to the last completion */
  double device_busy_seconds; /* sum over ticks of snapshot -> last of its two streams */
} etale_serve_stats;

/* Serve reqs_host[0..n) against the index. rows_dev holds n_rows vectors
 * (dim elements each, uint8 or FP32 as the index) that search and insert
 * requests name by row. Optional outputs (NULL to skip): latency_ms_host (n
 * floats; -1 for a rejected insert or a failed tick), tick_host (n uint32:
 * the tick that served each request, 0xFFFFFFFF if none), and res_ids_dev /
 * res_dists_dev (device, n x k each, row j for request j; written for search
 * requests only, padded as etale_search_batch). Synchronizes. Errors: EINVAL
 * (bad arguments, a row or kind out of range), ENOMEM (tick buffers), EPOOL
 * (pending updates that no slab pool state can cover), and those of
 * etale_round; a tick whose round fails on the device is counted in
 * failed_ticks and its requests get latency -1. */
etale_status etale_serve(etale_t ix, const etale_serve_config* cfg, const etale_request* reqs_host, uint64_t n,
                         const void* rows_dev, uint64_t n_rows, float* latency_ms_host, uint32_t* tick_host,
                         uint32_t* res_ids_dev, void* res_dists_dev, etale_serve_stats* out_host);

/* Result-invariant launch knobs of the beam search: waves per workgroup (1,
 * 2 or 4; halved further while a workgroup's LDS would exceed 64 KiB) and
 * visited-table slots (a power of two, 64..16384; the table may forget ids,
 * which only repeats distance evaluations). Rounds captured as graphs are
 * keyed by these values, so a change never alters a captured round. */
etale_status etale_set_search_knobs(etale_t ix, uint32_t waves_per_block, uint32_t vt_slots);

/* Result-invariant: lanes of a wave that share one uint8 row in a distance
 * batch, dim/16 (16 bytes each, the default; 0 means the same) or, for 128-
 * and 256-byte rows, dim/32 (32 bytes each: twice the rows per pass, shorter
 * group sums). EINVAL otherwise. */
etale_status etale_set_search_lanes(etale_t ix, uint32_t lanes_per_row);

typedef struct {
  uint32_t waves_per_block;
  uint32_t vt_slots;
  uint32_t row_lanes;  /* lanes per uint8 row (0 for float rows) */
  float ms;            /* mean search time of the chosen setting on the batch */
  float ms_default;    /* the same for the setting in force before the call */
} etale_tune_result;

/* Autotuner: times the query search on the caller's batch (q_dev [nq x dim],
 * k, L) for every setting of the result-invariant knobs above (waves 1/2/4 x
 * visited slots 256..4096 x lanes per row) and keeps the fastest; results do
 * not depend on the choice. Allocates its own output scratch; synchronizes. */
etale_status etale_autotune(etale_t ix, const void* q_dev, uint64_t nq, uint32_t k, uint32_t L,
                            etale_tune_result* out_host);

etale_status etale_set_search_timing(etale_t ix, int32_t enable);
etale_status etale_get_search_timing(etale_t ix, float* ms_host, uint64_t cap, uint64_t* launches);

/* Concurrent mode (the experiment of Section 5.6: readers and writers on two
 * streams that do not synchronize with each other). enable != 0: searches
 * (etale_search_batch) run on search_stream (a hipStream_t other than the
 * index's) with their own scratch, read the live reference words and slabs
 * while rounds on the index's stream publish, and return for each node the
 * list either before or after any publication that overlaps them (one
 * atomic reference load names an immutable slab). Meanwhile every publication
 * takes the release fence before its CAS; reverse edges are applied offer by
 * offer, racing by CAS with retries (Algorithm 1's loop; the list is rebuilt
 * from a fresh snapshot after a lost CAS; an offer whose attempt budget runs
 * out is counted in publish_dropped), so their order, and the lists, are not
 * deterministic; the entry set is frozen; and slabs retired by the rounds
 * are not recycled (a search may still hold them), so the pool must cover
 * every publication of the mode. enable == 0: both streams drain, the retired
 * slabs rejoin the free pool and the entry set is brought up to date
 * (synchronizes). Not with tombstone_only. The no-alloc search and serving
 * are not for this mode. */
etale_status etale_set_concurrent(etale_t ix, int32_t enable, void* search_stream);

/* Wait for the index's stream. */
etale_status etale_sync(etale_t ix);

/* Text of the last failure on this handle (owned by the library). */
const char* etale_last_error(etale_t ix);

#ifdef __cplusplus
}
#endif

#endif /* ETALE_H */
