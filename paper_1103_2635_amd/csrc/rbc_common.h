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

typedef float f4 __attribute__((ext_vector_type(4)));

// One tile launch.  BF mode (blk_reps == nullptr): split s scans database rows
// [s * rps, min(n, (s + 1) * rps)).  Grouped mode (exact RBC stage 2): the
// 256-slot query block b owns a list of representatives blk_reps[b * n_r + j],
// j < blk_cnt[b], whose lists L_r are the row ranges [list_off[r],
// list_off[r + 1]) of X; blk_pre[b * (n_r + 1) + j] is the number of rows
// before the j-th of them, and split s scans rows [s * U / S, (s + 1) * U / S)
// of that concatenation (U = blk_pre[b * (n_r + 1) + blk_cnt[b]]).  A query
// only scores lists it kept: keep[qrow * n_r + r] != 0.
struct TileArgs {
    const float* Q;
    int64_t ldq;
    int32_t m;             // query slots
    const int32_t* qmap;   // slot -> row of Q (nullptr: identity)
    const float* X;
    int64_t ldx;
    int32_t n;
    int32_t d;
    const float* xn;       // squared norms of X rows (MFMA path)
    int32_t rps;
    int32_t nsplit;
    const int32_t* blk_reps;
    const int32_t* blk_cnt;
    const int64_t* blk_pre;
    const int32_t* list_off;
    const uint8_t* keep;
    int32_t n_r;
    float* pval;           // [nsplit][m][C] partial shortlist values
    int32_t* pidx;         // [nsplit][m][C] partial shortlist rows (-1 = empty)
    int64_t* stats;        // optional device counters
};

// Merge of the partial shortlists, direct re-score, float64 near-tie
// re-rank, certificate and output.
struct FinArgs {
    const float* Q;
    int64_t ldq;
    int32_t m;
    const int32_t* qmap;
    const float* X;
    int64_t ldx;
    int32_t d;
    int32_t metric;        // 0 = l2, 1 = l1
    int32_t approx_mode;   // 0: values are ||x||^2 - 2 q.x (MFMA); 1: direct d^2 (l2) or rho (l1)
    const float* pval;
    const int32_t* pidx;
    int32_t nsplit;
    int32_t k;
    const float* qn;       // squared query norms by slot (approx_mode 0)
    const uint32_t* xmax_bits;  // largest database row norm (float bits, approx_mode 0)
    const int64_t* id_map; // row of X -> reported id (nullptr: identity)
    int64_t* out_idx;      // [rows of Q][k]
    float* out_dist;
    int32_t* fb_list;      // queries (rows of Q) whose shortlist is not certified
    int32_t* fb_count;
    int64_t* stats;
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
                            hipStream_t st);
hipError_t launch_tile_mfma(int ks, int c, bool grouped, dim3 grid, const TileArgs& a,
                            hipStream_t st);
hipError_t launch_tile_valu(int metric, int ks, int c, bool grouped, dim3 grid,
                            const TileArgs& a, hipStream_t st);

#define RBC_CAT_(a, b) a##b
#define RBC_CAT(a, b) RBC_CAT_(a, b)
#define RBC_DECL_KS(n)                                                                     \
    hipError_t launch_tile_mfma_ks##n(int c, bool grouped, dim3 grid, const TileArgs& a,   \
                                      hipStream_t st);                                     \
    hipError_t launch_tile_valu_ks##n(int metric, int c, bool grouped, dim3 grid,          \
                                      const TileArgs& a, hipStream_t st);
RBC_DECL_KS(1)
RBC_DECL_KS(2)
RBC_DECL_KS(3)
RBC_DECL_KS(4)
RBC_DECL_KS(5)
RBC_DECL_KS(6)
RBC_DECL_KS(7)
RBC_DECL_KS(8)
hipError_t launch_finalize(int c, const FinArgs& a, hipStream_t st);
hipError_t launch_exact(const ExactArgs& a, int grid, hipStream_t st);

}  // namespace rbc
