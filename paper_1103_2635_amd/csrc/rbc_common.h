// rbc_common.h -- types shared by the HIP kernels and the host side of librbc.
//
// Work decomposition of the brute-force primitive BF(Q, X) (Sec. 3 of the
// paper): the distance step is a query-by-database tile, the comparison step
// a per-query top-c shortlist kept in registers while the tile streams over
// the database.  A workgroup holds 256 query slots (4 wavefronts of 64) and
// scans one "split" of the database rows; each split leaves a sorted partial
// shortlist per query, merged and re-scored by the finalize kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbc {

constexpr int kWave = 64;
constexpr int kTileQ = 256;     // query slots per workgroup
constexpr int kRowsMfma = 32;   // database rows per MFMA step (two 16-row blocks)
constexpr int kRowsValu = 32;   // database rows per VALU tile
constexpr int kMaxKS = 8;       // 16-feature slabs held in registers: d <= 128
constexpr int kExactKCap = 1024;
constexpr int kItemRec = 8;        // int32 per stage-2 item record
constexpr int kCostBuckets = 2048; // cost classes of the longest-first item order
constexpr int kMaxHomeSplit = 8;   // row ranges per nearest list in pass 1 of the two-pass search

// tile launch forms
constexpr int kTileBF = 0;     // partial shortlists per (split, query)
constexpr int kTileItems = 1;  // persistent (representative, query chunk) items
constexpr int kTileAll = 2;    // every value written to pval[q * ldo + row]
constexpr int kTileRange = 3;  // range search items: count, or write, the rows within a radius
constexpr int kTileHome = 4;   // item mode for pass 1 of the two-pass search (a kernel of its
                               // own on the matrix path, so profiles tell the passes apart)

// shapes of the fp32 matrix-core tile (TileArgs.shape)
constexpr int kShape16 = 0;  // v_mfma_f32_16x16x4f32, LDS transpose for the comparison
constexpr int kShape32 = 1;  // v_mfma_f32_32x32x2f32, no transpose (BF and record items)

typedef float f4 __attribute__((ext_vector_type(4)));

// One tile launch.  BF mode: grid (query blocks of 256, database splits);
// split s scans database rows [s * rps, min(n, (s + 1) * rps)) and leaves a
// partial shortlist per query at pval[(s * m + q) * C].
// Item mode (exact RBC stage 2): a persistent grid takes items from a queue;
// item i belongs to the representative r with ioff[r] <= i < ioff[r + 1] and
// covers queries qlist[roff[r] + (i - ioff[r]) * 256 ...] (at most 256, all
// of which kept L_r); those queries scan the rows [list_off[r],
// list_off[r + 1]) of X, starting from the shortlist threshold tau[q], and
// leave their partial shortlist at pair qoff[q] + lrank[q * n_r + r] (exact
// mode) or at pair q when lrank is null (one-shot: one list per query); tau
// null means no seeded threshold.
struct TileArgs {
    const float* Q;
    int64_t ldq;
    int32_t m;
    const float* X;
    int64_t ldx;
    int32_t n;
    int32_t d;
    const float* xn;       // squared norms of X rows (MFMA path)
    int32_t rps;
    int32_t nsplit;
    const int32_t* item_total;
    int32_t* item_queue;
    const int32_t* irep;   // item -> representative (null: binary search over ioff)
    const int32_t* irows;  // item mode, optional: item i scans rows irows[2 i] .. irows[2 i + 1]
                           // (a run of its list) instead of the whole list
    const int32_t* irec;   // item mode, optional (exact pairs only): kItemRec int32 per queue
                           // position: representative, query range, row run, item (see
                           // item_rows_kernel); the queue hands the records out in this order
    int32_t isplit;        // item mode without lrank, > 1: each query chunk of a list is
                           // isplit items, item j scanning the j-th of isplit equal row
                           // ranges and leaving its shortlist at pair q * isplit + j
    const int32_t* ioff;
    const int32_t* roff;
    const int32_t* qlist;
    const int32_t* list_off;
    const int32_t* lrank;
    const int32_t* qoff;
    const float* tau;
    int32_t n_r;
    const uint8_t* qscale;  // fp8 tiles: per-row E8M0 scale bytes of Q and X
    const uint8_t* xscale;
    float* pval;           // partial shortlist values (kTileAll: the value matrix)
    int32_t* pidx;         // partial shortlist rows (-1 = no row)
    int64_t ldo;           // kTileAll: row stride of the value matrix
    int64_t* stats;        // optional device counters
    int32_t shape;         // fp32 matrix tile: kShape16 or kShape32
    int32_t qb;            // stage-2 items with records, 16x16 shape: 16-query blocks per
                           // item (4, or 2 for 32-query items; 0 means 4)
    // BF mode with a device-side query count (non-null m_dev): the first
    // *m_dev rows of Q are searched by a 1-D grid of dev_blocks workgroups
    // whose (query block, split) layout is derived from the count (dev_split)
    const int32_t* m_dev;
    int32_t dev_blocks;
    // Range mode (kTileRange, vector path): every row of an item's list within
    // range_radius of a query is counted (range_fill 0: range_cnt[q] += hits)
    // or written (range_fill 1: at range_off[q] + a cursor taken from
    // range_cnt[q], id ids[row], float64 distance rounded to float)
    int32_t range_fill;
    double range_radius;
    int32_t* range_cnt;
    const int64_t* range_off;
    int64_t* range_idx;
    float* range_dist;
    const int64_t* ids;
};

// Merge of the partial shortlists, direct re-score, float64 near-tie
// re-rank, certificate and output.
struct FinArgs {
    const float* Q;
    int64_t ldq;
    int32_t m;
    const float* X;
    int64_t ldx;
    int32_t d;
    int32_t metric;        // 0 = l2, 1 = l1
    int32_t approx_mode;   // 0: ||x||^2 - 2 q.x (MFMA); 1: direct d^2 (l2) or rho (l1);
                           // 2: ||x~||^2 - 2 q~.x~ on quantised rows
    const float* pval;
    const int32_t* pidx;
    int32_t nsplit;        // BF mode: lists of query q at (s * m + q) * C, s < nsplit
    const int32_t* qoff;   // pair mode (non-null): lists qoff[q] .. qoff[q] + npairs[q] - 1
    const int32_t* npairs;
    int32_t k;
    const float* qn;       // squared query norms (approx_mode 0)
    const uint32_t* xmax_bits;  // largest database row norm (float bits, approx_mode 0)
    const uint32_t* flags_q;    // value flags of Q and X (see tile_exact), may be null
    const uint32_t* flags_x;
    const float* qerr;          // approx_mode 2 (quantised tile): ||q - q~|| per query,
    const uint32_t* xerr_max_bits;  // and the largest ||x - x~|| (float bits)
    float* out_approx;          // optional [m][k]: tile distance of each result before re-scoring
    const int64_t* id_map; // row of X -> reported id (nullptr: identity)
    int64_t* out_idx;      // [rows of Q][k]
    float* out_dist;
    int32_t* fb_list;      // queries (rows of Q) whose shortlist is not certified
    int32_t* fb_count;
    int64_t* stats;
    int32_t fail_stat;     // stats slot counting the queries that are not certified
    // device-side query count (see TileArgs): rows i < *m_dev of Q are
    // finalized, the partial lists laid out by dev_split(*m_dev, dev_blocks, n);
    // qmap (optional) maps row i of Q to the output row / reported query
    const int32_t* m_dev;
    int32_t dev_blocks;
    int32_t n;
    const int32_t* qmap;
};

// Exhaustive float64 search for the rows of Q listed in list[0 .. *count).
struct ExactArgs {
    const float* Q;
    int64_t ldq;
    const float* X;
    int64_t ldx;
    int32_t n;
    int32_t d;
    int32_t metric;
    int32_t k;
    const int32_t* list;
    const int32_t* count;
    const int64_t* id_map;
    const int32_t* qrep;      // optional: search only rows list_off[qrep[q]] .. list_off[qrep[q] + 1]
    const int32_t* list_off;
    int64_t* out_idx;
    float* out_dist;
};

// ---- launchers (defined next to their kernels) ----
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t st);
hipError_t launch_iota_i32(int32_t* p, int32_t count, hipStream_t st);
hipError_t launch_set_count(int32_t* p, int32_t value, hipStream_t st);
hipError_t launch_repack(const float* A, int64_t rows, int64_t lda, int32_t d, float* out,
                         int64_t ldo, hipStream_t st);
hipError_t launch_row_norms(const float* A, int64_t rows, int64_t lda, int32_t d,
                            const int32_t* rowmap, float* out, uint32_t* maxbits,
                            hipStream_t st, uint32_t* flags = nullptr,
                            const int32_t* gate = nullptr);
// irep[i] = r for every item i of representative r (ioff[r] <= i < ioff[r + 1]).
hipError_t launch_item_reps(const int32_t* ioff, int32_t nr, int32_t* irep, hipStream_t st);
hipError_t launch_cascade_gather(const float* Q, int64_t ldq, int32_t d, int64_t m,
                                 const int32_t* list, const int32_t* count, float* Qc,
                                 int64_t ldc, float* qn, int32_t* qmap, int32_t* count_out,
                                 hipStream_t st);
hipError_t launch_tile_mfma(int ks, int c, int mode, dim3 grid, const TileArgs& a,
                            hipStream_t st);
hipError_t launch_tile_valu(int metric, int ks, int c, int mode, dim3 grid,
                            const TileArgs& a, hipStream_t st);

#define RBC_CAT_(a, b) a##b
#define RBC_CAT(a, b) RBC_CAT_(a, b)
#define RBC_DECL_KS(n)                                                                     \
    hipError_t launch_tile_mfma_ks##n(int c, int mode, dim3 grid, const TileArgs& a,       \
                                      hipStream_t st);                                     \
    hipError_t launch_tile_valu_ks##n(int metric, int c, int mode, dim3 grid,              \
                                      const TileArgs& a, hipStream_t st);
RBC_DECL_KS(1)
RBC_DECL_KS(2)
RBC_DECL_KS(3)
RBC_DECL_KS(4)
RBC_DECL_KS(5)
RBC_DECL_KS(6)
RBC_DECL_KS(7)
RBC_DECL_KS(8)
#define RBC_DECL_KB(n)                                                                     \
    hipError_t launch_tile_lowp_kb##n(int fmt, int c, int mode, dim3 grid,                 \
                                      const TileArgs& a, hipStream_t st);
RBC_DECL_KB(1)
RBC_DECL_KB(2)
RBC_DECL_KB(3)
RBC_DECL_KB(4)
// fmt 0: bf16 (kb = ceil(d / 32) feature blocks), 1: fp8 e4m3 (d <= 128)
hipError_t launch_tile_lowp(int fmt, int kb, int c, int mode, dim3 grid, const TileArgs& a,
                            hipStream_t st);
hipError_t launch_quantize(int fmt, const float* A, int64_t rows, int64_t lda, int32_t d,
                           float mult, void* out, int64_t ldo, int32_t dpad, float* norm2,
                           float* err, uint8_t* scale_out, uint32_t* stat, hipStream_t st);
hipError_t launch_finalize(int c, const FinArgs& a, hipStream_t st);
hipError_t launch_exact(const ExactArgs& a, int grid, hipStream_t st);

}  // namespace rbc
