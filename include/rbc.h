/*
 * rbc.h -- C ABI of the MI355X (gfx950) Random Ball Cover / brute-force
 * nearest-neighbour library (librbc.so).
 *
 * The library implements the brute-force primitive BF(Q, X) of Cayton,
 * "Accelerating Nearest Neighbor Search on Manycore Systems" (Sec. 3: for
 * every query, the distance to every database point followed by a
 * per-query comparison), and the Random Ball Cover built from it (Sec. 4:
 * representatives, ownership lists L_r, radii psi_r; Sec. 5.1 one-shot
 * search; Sec. 5.2 exact search with pruning rules (1) and (2)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are row-major float32 in DEVICE memory: row i of an m x d
 *    matrix A starts at A + i * lda, lda >= d.  Queries Q (m x d) and the
 *    database X (n x d) are owned by the caller.
 *  - Outputs are DEVICE arrays owned by the caller: out_idx (m x k, int64,
 *    row-major) and out_dist (m x k, float32).  For every query the k
 *    results are sorted ascending by (distance, database row id): a tie in
 *    distance is won by the lower row id.  out_dist holds rho itself:
 *    Euclidean distance for RBC_L2 (not squared), sum of absolute
 *    differences for RBC_L1.  out_idx holds the row of X.
 *  - Every call is asynchronous on the given HIP stream (NULL = the null
 *    stream).  The return value reports argument validation and kernel
 *    launch only; a device fault surfaces at the caller's next
 *    synchronisation.  No call synchronises the stream except rbc_build
 *    (which returns a finished index) and rbc_free.
 *  - No exception crosses the ABI.  A non-zero return is an rbc_status;
 *    rbc_last_error() then describes it (thread-local string).
 *  - m == 0 is a no-op returning RBC_OK.  Inputs must be finite.
 *  - Exactness: results equal exhaustive search in exact arithmetic on the
 *    float32 inputs (ranking by (distance, id)); distances are accurate to
 *    a few float32 ulps.  Candidates are ranked with a fast float32
 *    contraction, re-scored directly, near-ties re-ranked in float64, and a
 *    query whose shortlist cannot be certified is searched again
 *    exhaustively in float64.
 */
#ifndef RBC_H_
#define RBC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Metric rho (Sec. 4; the l1 form is the one written out in Sec. 6). */
typedef enum { RBC_L2 = 0, RBC_L1 = 1 } rbc_metric;

/* Arithmetic of the distance contraction (matrix cores, fp32 accumulate).
 * RBC_BF16 and RBC_FP8_E4M3 (OCP e4m3, per-row power-of-two scale) apply to
 * bf_search with RBC_L2 and d <= 128: candidates are ranked on quantised
 * rows, re-scored in fp32 from the original rows, certified with the
 * quantisation error added to the bound, near-ties re-ranked in float64;
 * results are as exact as with RBC_FP32. */
typedef enum { RBC_FP32 = 0, RBC_BF16 = 1, RBC_FP8_E4M3 = 2 } rbc_precision;

/* Ownership rule of the index (Sec. 4): RBC_EXACT -- each point is owned by
 * its nearest representative (lists partition X); RBC_ONESHOT -- each
 * representative owns its s nearest database points (lists overlap). */
typedef enum { RBC_EXACT = 0, RBC_ONESHOT = 1 } rbc_mode;

typedef enum {
    RBC_OK = 0,
    RBC_EINVAL = -1,        /* an argument is out of range or a pointer is NULL */
    RBC_ENOMEM = -2,        /* device allocation failed (rbc_build only) */
    RBC_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    RBC_EUNSUPPORTED = -4,  /* valid request outside what this build implements */
    RBC_EWORKSPACE = -5     /* workspace NULL or smaller than the size query says */
} rbc_status;

/* Largest k accepted by bf_search / rbc_search. */
#define RBC_MAX_K 1024
/* Largest dimension accepted. */
#define RBC_MAX_D 4096

/* Number of int64 counters written to rbc_search_opts.dev_stats. */
#define RBC_STATS_LEN 8
/* Counter slots (added to, never cleared by the library). */
#define RBC_STAT_FALLBACK   0  /* queries re-searched exhaustively in float64 */
#define RBC_STAT_NEARTIE    1  /* shortlist entries re-ranked in float64 */
#define RBC_STAT_PAIRS      2  /* (query, point) pairs scored by the main kernel */
#define RBC_STAT_LISTS      3  /* (query, list) pairs kept by the pruning rules */
#define RBC_STAT_CAND       4  /* (query, point) pairs inside kept lists */
#define RBC_STAT_CASCADE    5  /* low precision: queries whose certificate failed and that the
                                  float32 tile re-ranked over all rows */
#define RBC_STAT_ITEMS      6  /* stage-2 work items (list, query chunk) processed */
#define RBC_STAT_SLOTS      7  /* (query, point) slots the stage-2 kernel computed, padding
                                  included: per item its query-slot width times its rows
                                  rounded up to the kernel's row block */

/* rbc_search_opts.flags: search an exact index in one pass (every kept list
 * scanned in full, pruning by gamma_k) instead of the default two passes. */
#define RBC_FLAG_ONE_PASS 1

/* Per-call search options.  Pass NULL for the defaults. */
typedef struct rbc_search_opts {
    int32_t precision;  /* rbc_precision; default RBC_FP32 */
    int32_t shortlist;  /* per-query shortlist length c (0 = automatic: at least
                           k + 3; at least 8 for RBC_BF16, 32 for RBC_FP8_E4M3);
                           rounded up to one of 4, 8, 16, 32, 64, and >= k + 3 */
    int32_t splits;     /* database splits per query block (0 = automatic) */
    int32_t flags;      /* rbc_search: 0 or RBC_FLAG_ONE_PASS; bf_search: 0 */
    int64_t* dev_stats; /* optional DEVICE array of RBC_STATS_LEN int64 counters */
    float* dev_approx_dist; /* optional DEVICE m x k floats: the distance each result had in
                               the ranking tile, before re-scoring (not written for queries
                               re-ranked by the float32 cascade or the float64
                               fallback) */
    float prune_eps;    /* rbc_search, exact mode: 0 = exact.  eps > 0 prunes with the
                           bounds divided by (1 + eps) -- rule 1 at gamma_k / (1 + eps),
                           rule 2 at (2 gamma_k + gamma_1) / (1 + eps) -- the approximate
                           variant the paper mentions beside Sec. 5: the result is the exact
                           k-NN among the points of the lists kept, not necessarily the
                           exact k-NN of X.  Must be 0 for bf_search and one-shot indexes. */
    int32_t reserved;   /* must be 0 */
} rbc_search_opts;

/* Index construction parameters. */
typedef struct rbc_build_params {
    int32_t mode;            /* rbc_mode */
    int32_t metric;          /* rbc_metric */
    int64_t n_r;             /* number of representatives, 1 <= n_r <= n */
    int64_t s;               /* one-shot list length, 1 <= s <= n (ignored for RBC_EXACT) */
    uint64_t seed;           /* seed of the representative draw when rep_idx is NULL */
    const int64_t* rep_idx;  /* optional HOST array of n_r distinct row ids of X;
                                copied and sorted ascending by the library */
    int32_t precisions;      /* bit mask (1 << rbc_precision) of the low precisions that
                                rbc_search may use on this index (exact mode, RBC_L2,
                                d <= 128): their quantised copies of the rows are built
                                with the index; 0 = fp32 only */
    int32_t reserved;
} rbc_build_params;

typedef struct rbc_index rbc_index; /* opaque; owns its device memory */

/*
 * bf_search -- the brute-force primitive BF(Q, X) (Sec. 3), k-NN form: the
 * distance step (a query-by-database tile; for RBC_L2 the ranking value
 * ||x||^2 - 2 q.x is a dense contraction run on the matrix cores) followed
 * by the comparison step (a per-query top-k).
 *   Q: m x d (ldq), X: n x d (ldx) device float32; 1 <= k <= min(n, RBC_MAX_K).
 *   workspace: device memory of at least bf_search_workspace_size() bytes
 *   (same m, n, d, ldq, ldx, metric, k, opts), used only by the work the
 *   call queues on `stream`.  Q and X must be 16-byte aligned.
 * Errors: RBC_EINVAL for d < 1, n < 1, k < 1, k > n, ldq < d, ldx < d,
 * m < 0, NULL pointers with m > 0; RBC_EUNSUPPORTED for d > RBC_MAX_D,
 * k > RBC_MAX_K, n >= 2^31, or a low precision with RBC_L1 or d > 128;
 * RBC_EWORKSPACE when the workspace is too small.
 */
int bf_search_workspace_size(int64_t m, int64_t n, int32_t d, int64_t ldq, int64_t ldx,
                             int32_t metric, int32_t k, const rbc_search_opts* opts,
                             size_t* bytes);
int bf_search(const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n, int64_t ldx,
              int32_t d, int32_t metric, int32_t k, const rbc_search_opts* opts,
              int64_t* out_idx, float* out_dist, void* workspace, size_t ws_bytes,
              void* hip_stream);

/*
 * rbc_build -- build a Random Ball Cover over X (Sec. 4).
 *   RBC_EXACT: ownership by BF(X, R) with k = 1 (ties to the lower
 *   representative position), lists stored as contiguous row ranges of a
 *   permuted copy of X (ascending row id inside a list), psi_r = the largest
 *   distance from r to a point it owns.
 *   RBC_ONESHOT: each representative's s nearest database points (ties to
 *   the lower row id), psi_r = the s-th of those distances.
 * Representatives are the caller's rep_idx, or n_r distinct rows drawn
 * uniformly from `seed`.  The index copies what it needs: X may be freed
 * when the call returns.  The call synchronises `stream`.
 * Errors: RBC_EINVAL (bad sizes, duplicate or out-of-range rep ids, s > n,
 * NULL pointers); RBC_ENOMEM; RBC_EUNSUPPORTED as for bf_search.
 */
int rbc_build(const float* X, int64_t n, int64_t ldx, int32_t d,
              const rbc_build_params* params, void* hip_stream, rbc_index** out);

/*
 * rbc_search -- search an index (Sec. 5.2 for RBC_EXACT, Sec. 5.1 for
 * RBC_ONESHOT).  Exact mode returns exactly the k nearest neighbours; the
 * k-NN form of the pruning rules is: with gamma_1 <= ... <= gamma_k the k
 * smallest distances from q to the representatives, list L_r is skipped
 * when rho(q,r) - psi_r > gamma_k (rule 1) or rho(q,r) > 2 gamma_k +
 * gamma_1 (rule 2); bounds are widened by the float32 error of the
 * computed distances.  One-shot mode returns the k nearest points of q's
 * nearest representative's list (k <= s).
 *   Q: m x d (ldq) device float32; outputs as for bf_search; `workspace`
 *   of at least rbc_search_workspace_size() bytes.  Concurrent calls on
 *   different streams with different workspaces are safe (the index is
 *   read-only after rbc_build).
 *   Exact float32 searches (prune_eps 0, flags 0) take two passes: pass 1
 *   searches each query's nearest list in full, which bounds the k-th
 *   neighbour distance by tau_q <= gamma_k; pass 2 applies both rules with
 *   tau_q in place of gamma_k and, inside each kept list (rows ordered by
 *   their distance to the representative), scans only the rows x with
 *   abs(rho(x, r) - rho(q, r)) <= tau_q (triangle inequality); the nearest
 *   list is searched again over that range.  Low precision, prune_eps > 0 and
 *   RBC_FLAG_ONE_PASS search in one pass.
 *   opts->precision RBC_BF16 / RBC_FP8_E4M3 ranks the kept lists with the
 *   quantised rows built into an exact index (rbc_build_params.precisions);
 *   the answers stay exact (float32 re-score, certificate that includes the
 *   quantisation error, float64 fallback).  RBC_EUNSUPPORTED when the index
 *   holds no copy in that precision or is a one-shot index.
 */
int rbc_search_workspace_size(const rbc_index* index, int64_t m, int64_t ldq, int32_t k,
                              const rbc_search_opts* opts, size_t* bytes);
int rbc_search(const rbc_index* index, const float* Q, int64_t m, int64_t ldq, int32_t k,
               const rbc_search_opts* opts, int64_t* out_idx, float* out_dist,
               void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * Range search over an exact index (the eps-range extension named in the
 * introduction of Sec. 5): every database point x with rho(q, x) <= radius,
 * decided in float64 exactly as a direct float64 evaluation of rho decides
 * it (float32 distances settle only the points clearly inside or outside).
 * Same stage 1 as rbc_search; list L_r is skipped when rho(q, r) - psi_r >
 * radius (triangle inequality, the bound widened by the float32 error of
 * rho(q, r)); the kept lists are scanned with the vector tile.  The output
 * size depends on the data, so the search takes two calls on the same
 * index, Q and radius:
 *   rbc_range_count   writes offsets[m + 1] (device int64): offsets[0] = 0,
 *                     offsets[i + 1] - offsets[i] = the number of points
 *                     within radius of query i.  Asynchronous on the stream.
 *   rbc_range_search  given those offsets, writes the points of query i to
 *                     out_idx / out_dist[offsets[i] .. offsets[i + 1]) (device
 *                     int64 row ids of X and float32 roundings of the float64
 *                     distances) in ascending (float32 distance, id) order.
 *                     The call synchronises the stream: it checks that every
 *                     query found exactly as many points as its segment holds
 *                     (RBC_EINVAL when the offsets do not belong to this
 *                     index, Q and radius; points beyond a segment are then
 *                     dropped, never written outside it, and the segments
 *                     that do not match are left unsorted).
 * Q: m x d (ldq) device float32; radius finite and >= 0; `workspace` of at
 * least rbc_range_workspace_size() bytes, used by one call at a time.
 * Segments longer than 8192 points are sorted in global memory (slower).
 * Errors: RBC_EINVAL (bad sizes, NULL pointers, radius negative or not
 * finite, mismatched offsets); RBC_EUNSUPPORTED for one-shot indexes, d > 128
 * or m * n_r >= 2^31; RBC_EWORKSPACE.
 */
int rbc_range_workspace_size(const rbc_index* index, int64_t m, int64_t ldq, size_t* bytes);
int rbc_range_count(const rbc_index* index, const float* Q, int64_t m, int64_t ldq,
                    double radius, int64_t* offsets, void* workspace, size_t ws_bytes,
                    void* hip_stream);
int rbc_range_search(const rbc_index* index, const float* Q, int64_t m, int64_t ldq,
                     double radius, const int64_t* offsets, int64_t* out_idx, float* out_dist,
                     void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * rbc_index_info -- sizes of a built index (any output pointer may be NULL).
 */
int rbc_index_info(const rbc_index* index, int64_t* n, int32_t* d, int64_t* n_r,
                   int32_t* mode, int32_t* metric, size_t* device_bytes);

/*
 * rbc_index_export -- copy index arrays to HOST buffers (any may be NULL):
 *   rep_idx[n_r] (int64, ascending), psi[n_r] (float64),
 *   list_off[n_r + 1] (int64; exact mode: list r is entries
 *   list_off[r] .. list_off[r+1]-1 of list_ids; one-shot: r * s),
 *   list_ids[n (exact) or n_r * s (one-shot)] (int64 row ids of X).
 * Synchronises the device.
 */
int rbc_index_export(const rbc_index* index, int64_t* rep_idx, double* psi,
                     int64_t* list_off, int64_t* list_ids);

/*
 * rbc_index_export_order -- exact mode: the order of the rows inside each
 * list, to HOST buffers (either may be NULL).  own[n] (float32, in list_ids
 * order) is the distance of each row to its list's representative as the
 * build computed it (float32 re-score, float64 on near ties); every list r
 * with sorted[r] == 1 holds its rows in ascending (own, id) order, so the
 * rows of a list whose distance to the representative lies in a band form
 * one contiguous range (the triangle-inequality truncation of a list scan,
 * Sec. 5.2).  Lists longer than 8192 rows keep id order (sorted[r] == 0).
 * RBC_EUNSUPPORTED for one-shot indexes.  Synchronises the device.
 */
int rbc_index_export_order(const rbc_index* index, float* own, int32_t* sorted);

/* rbc_free -- release an index (NULL is a no-op).  Synchronises the device.
 * The index's main device block (everything but optional quantised copies)
 * is kept, one block per device, for the next rbc_build on that device that
 * needs at least half of it; a larger freed block replaces a cached one. */
void rbc_free(rbc_index* index);

/*
 * Kernel timing (instrumentation, off by default).  rbc_timer_enable(1)
 * clears the totals and makes every later call record a pair of HIP events
 * on its stream around each of its kernels; rbc_timer_read() waits for the
 * recorded events and returns the summed device time (ms) and launch count
 * of the kernels called `name`: "tile" (BF distance tile), "tile_items"
 * (RBC stage 2), "finalize", "fallback", "stage1", "prune", "worklist",
 * "quantize", "cascade" (the float32 re-ranking of low-precision queries
 * whose certificate failed), "oneshot_tile", "oneshot_select", "range_tile"
 * (both range passes), "range_sort".
 */
int rbc_timer_enable(int on);
int rbc_timer_read(const char* name, double* total_ms, int64_t* launches);

/*
 * Tile autotuner.  The distance step of BF(Q, X) (Sec. 3) runs on the fp32
 * matrix cores in one of two tile shapes -- 16x16x4 MFMAs with an LDS
 * transpose before the per-query comparison, or 32x32x2 MFMAs whose output
 * already holds one query per lane -- and the grouped stage-2 search of the
 * exact RBC (Sec. 5.2) is one persistent launch whose workgroup count is
 * free.  Which is fastest depends on d, the shortlist length and the list
 * sizes.  Untuned, the library uses the 16x16 shape, 64-query stage-2 items
 * and 1024 workgroups.
 *
 * rbc_autotune_search runs the given rbc_search once untimed and three times
 * timed (HIP events on hip_stream) under each candidate (16x16 with 64- or
 * 32-query stage-2 items, or 32x32; x 512 / 1024 / 2048 workgroups x pass-1
 * splits by the size rule or 4),
 * rbc_autotune_bf likewise for bf_search (2 shapes); the fastest is kept,
 * process-wide, for every later call with the
 * same launch kind, 16-feature slab count (ceil(d / 16)) and shortlist
 * length.  Arguments are those of rbc_search / bf_search (the outputs are
 * written by every run; results do not depend on the choice).  `out`
 * (optional, host) receives the choice and its time.  Both synchronise
 * hip_stream.  RBC_EUNSUPPORTED when the call runs no fp32 matrix-core
 * launch (L1, d < 12, low precision, one-shot indexes).  Concurrent tuning
 * calls are safe but time each other's work.
 */
typedef struct rbc_tune_result {
    int32_t shape;       /* 16 or 32 */
    int32_t blocks;      /* persistent workgroups (stage-2 launch; bf: unused) */
    int32_t splits;      /* row ranges per nearest list in pass 1 (0: size rule; bf: unused) */
    int32_t item_queries; /* queries per stage-2 item, 64 or 32 (bf: 64, unused) */
    float ms;            /* best time of the chosen candidate, whole call */
    float ms_before;     /* the same for the configuration used before tuning */
    int32_t candidates;  /* configurations timed */
} rbc_tune_result;

int rbc_autotune_search(const rbc_index* index, const float* Q, int64_t m, int64_t ldq,
                        int32_t k, const rbc_search_opts* opts, int64_t* out_idx,
                        float* out_dist, void* workspace, size_t ws_bytes, void* hip_stream,
                        rbc_tune_result* out);
int rbc_autotune_bf(const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n,
                    int64_t ldx, int32_t d, int32_t metric, int32_t k,
                    const rbc_search_opts* opts, int64_t* out_idx, float* out_dist,
                    void* workspace, size_t ws_bytes, void* hip_stream, rbc_tune_result* out);
/* Pin a choice by hand: kind 0 = bf_search (and the float32 cascade and
 * the exact-index fallback tile), 1 = rbc_search (stage 2 and pass 1); d and
 * shortlist (4, 8, 16, 32 or 64) select the entry as above; shape 16 or 32;
 * blocks the stage-2 workgroup count; splits 0 .. 8 the pass-1 row ranges per
 * nearest list (0: the size rule); item_queries 64, or 32 with shape 16 (the
 * queries of one stage-2 item of the two-pass search).  RBC_EINVAL on values
 * out of range. */
int rbc_autotune_set(int32_t kind, int32_t d, int32_t shortlist, int32_t shape, int32_t blocks,
                     int32_t splits, int32_t item_queries);
/* Forget every tuned choice (later calls use the fixed rule). */
void rbc_autotune_clear(void);

/* rbc_last_error -- message for the last non-OK return on this thread. */
const char* rbc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RBC_H_ */
