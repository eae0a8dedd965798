// rbc_kernels.h -- launchers of the RBC build / search kernels (k_rbc.hip).
#pragma once

#include "rbc_common.h"

namespace rbc {

constexpr int kSortBlock = 1024;   // items per block of the stable counting sort
constexpr int kMaxReps = 16384;    // LDS histogram of the counting sort
constexpr int kOsCap = 8192;       // one-shot build: candidates per representative (LDS sort)
constexpr int kSegCap = 8192;      // longest segment of the LDS segmented sort

// Scratch of the one-shot list selection for a chunk of representatives.
struct OneShotWork {
    uint32_t* hist = nullptr;    // reps x 4096
    uint32_t* prefix = nullptr;  // reps
    int32_t* need = nullptr;     // reps
    float* tval = nullptr;       // reps
    float* bound = nullptr;      // reps
    int32_t* cnt = nullptr;      // reps
    int32_t* cand = nullptr;     // reps x kOsCap
    int32_t* overflow = nullptr; // 1
};

int csort_blocks(int64_t n);
// int32 scratch entries launch_csort needs for n items and nk keys
int64_t csort_scratch(int64_t n, int32_t nk);
// in-place exclusive scan; sums needs ceil(n / 2048) + 1 entries; v[n] = total if with_total
hipError_t launch_scan(int32_t* v, int64_t n, int32_t* sums, bool with_total, hipStream_t st);
hipError_t launch_gather_rows(const float* A, int64_t lda, int32_t d, const int32_t* rows,
                              int64_t nrows, float* out, int64_t ldo, int64_t* ids_out,
                              hipStream_t st);
hipError_t launch_narrow(const int64_t* in, int64_t n, int32_t* out, hipStream_t st);
// keys -> perm (items ordered by (key, item)), offsets[nk + 1] (optional);
// cnt needs csort_scratch(n, nk) int32.
hipError_t launch_csort(const int32_t* keys, int64_t n, int32_t nk, int32_t* cnt, int32_t* perm,
                        int32_t* offsets, hipStream_t st);
hipError_t launch_dist_all(int metric, const float* Q, int64_t ldq, int32_t m, const float* R,
                           int64_t ldr, int32_t nr, int32_t d, float* DR, int64_t ldd,
                           hipStream_t st);
hipError_t launch_prune(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t k, int32_t c,
                        double delta, const double* psi, const int32_t* list_off, int32_t* lrank,
                        int32_t* nkept, float* gcup, int64_t* stats, hipStream_t st,
                        double shrink = 1.0, const float* taud = nullptr);
// Two-pass exact search: nearest representative per query, the k-th
// neighbour bound from the nearest list's shortlist, stage-2 item row ranges.
hipError_t launch_nearest_rep(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t* home,
                              hipStream_t st);
hipError_t launch_tau_home(const float* hval, int32_t c, int32_t nsplit, int32_t k, int32_t m,
                           int32_t mode, const float* qn, const uint32_t* xmax_bits, int32_t d,
                           double delta, float* taud, hipStream_t st);
hipError_t launch_item_rows(const int32_t* item_total, const int32_t* irep, const int32_t* ioff,
                            const int32_t* roff, const int32_t* qlist, int32_t isize,
                            const int32_t* list_off, const int32_t* lsorted, const float* own,
                            const float* DR, int64_t ldd, const float* taud, double tconst,
                            double rel, int32_t* irows, hipStream_t st, int32_t* rec = nullptr);
// Longest-first order of the stage-2 items: the records rec[0 .. *item_total)
// written by item_rows_kernel, copied to srec in descending cost class
// (queries x 32-row blocks / 8).
hipError_t launch_item_order(const int32_t* item_total, const int32_t* rec, int32_t* srec,
                             hipStream_t st);
// Items grouped by key without a fixed order inside a group: offsets
// [nk + 1] (total at offsets[nk]), perm [n]; cursor is nk int32 of scratch.
hipError_t launch_group(const int32_t* keys, int64_t n, int32_t nk, int32_t* cursor,
                        int32_t* perm, int32_t* offsets, hipStream_t st);
// launch_quantize that also writes the fp32 squared norm of every input row
// (norm32[rows]) and its value flags (flags32[3], zeroed by the caller; see
// launch_row_norms), reading each row once.
hipError_t launch_quantize_norms(int fmt, const float* A, int64_t rows, int64_t lda, int32_t d,
                                 float mult, void* out, int64_t ldo, int32_t dpad, float* norm2,
                                 float* err, uint8_t* scale_out, uint32_t* stat, float* norm32,
                                 uint32_t* flags32, hipStream_t st);
// a[i] = min(a[i], b[i]) for i < n.
hipError_t launch_min_f32(float* a, const float* b, int64_t n, hipStream_t st);
hipError_t launch_keep_transpose(const int32_t* lrank, int32_t m, int32_t nr, uint8_t* keep_rq,
                                 hipStream_t st);
// roff and ioff need nr + 1 entries; roff[nr] / ioff[nr] receive the totals.
hipError_t launch_worklist(const uint8_t* keep_rq, int32_t m, int32_t nr, int32_t isize,
                           int32_t* roff, int32_t* ioff, int32_t* qlist, hipStream_t st);
// exclusive scan of v[0 .. n), total to v[n]
hipError_t launch_scan_total(int32_t* v, int64_t n, hipStream_t st);
hipError_t launch_tau(const float* gcup, const float* qn, const uint32_t* xmax_bits,
                      const uint32_t* flags_q, const uint32_t* flags_x, int32_t m, int32_t d,
                      int32_t mode, double delta, float* tau, hipStream_t st,
                      const float* qerr = nullptr, const uint32_t* xerr_bits = nullptr);

// One-shot build, per chunk of `reps` representatives whose values (tile
// value space given by mode) are V[rep][0 .. n): candidate rows of each list.
hipError_t launch_oneshot_select(const float* V, int64_t ldv, int32_t n, int32_t reps, int32_t s,
                                 int32_t mode, double delta, int32_t d, const float* rnorm2,
                                 const uint32_t* xmax_bits, const uint32_t* flags, OneShotWork& w,
                                 hipStream_t st);
// float64 re-score and sort of the candidates: lists[rep0 + rep][0 .. s), psi.
hipError_t launch_oneshot_sort(const float* X, int64_t ldx, int32_t d, int32_t metric,
                               const float* R, int64_t ldr, int32_t reps, int32_t s, int32_t rep0,
                               OneShotWork& w, int32_t* lists, double* psi, hipStream_t st);
// ioff[r] = items of representative r from query offsets roff, scanned; ioff[nr] = total.
hipError_t launch_items_from_offsets(const int32_t* roff, int32_t nr, int32_t isize,
                                     int32_t* ioff, hipStream_t st, int32_t mult = 1);
hipError_t launch_list_offsets(int32_t* off, int32_t nr, int32_t s, hipStream_t st);
// psi_r from the own-sorted lists (float64 re-score of the screened rows).
hipError_t launch_psi_own(const float* Xp, int64_t ld, int32_t d, int32_t metric, const float* own,
                          const int32_t* list_off, const int32_t* lsorted, const float* R,
                          int64_t ldr, int32_t nr, double* psi, hipStream_t st);
// xn[i] = qn[perm[i]], largest norm (float bits, atomic max), 3 flag words copied.
hipError_t launch_gather_norms(const float* qn, const int32_t* perm, int64_t n, float* xn,
                               uint32_t* maxbits, const uint32_t* flags_in, uint32_t* flags_out,
                               hipStream_t st);
// Range search: pruning (keep r when rho(q,r) - psi_r <= radius), int64
// offsets from int32 counts, per-query sort of (dist, idx) pairs.
hipError_t launch_prune_range(const float* DR, int64_t ldd, int32_t m, int32_t nr, double delta,
                              const double* psi, double radius, int32_t* lrank, int32_t* nkept,
                              int64_t* stats, hipStream_t st);
hipError_t launch_offsets64(const int32_t* cnt, int64_t m, int64_t* off, hipStream_t st);
hipError_t launch_seg_sort_pairs(const int64_t* off, int64_t nseg, int64_t* idx, float* dist,
                                 const int32_t* cnt, int32_t* bad, hipStream_t st);
// Stable sort of each segment of vals by a float key (see k_rbc.hip).
hipError_t launch_seg_sort(const int32_t* off, int32_t nseg, int32_t* vals, const float* keys,
                           int64_t ldk, int32_t* sorted, hipStream_t st);

}  // namespace rbc
