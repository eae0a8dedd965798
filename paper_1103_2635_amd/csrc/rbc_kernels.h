// rbc_kernels.h -- launchers of the RBC build / search kernels (k_rbc.hip).
#pragma once

#include "rbc_common.h"

namespace rbc {

constexpr int kSortBlock = 4096;   // items per block of the stable counting sort
constexpr int kMaxReps = 16384;    // LDS histogram of the counting sort

int csort_blocks(int64_t n);
hipError_t launch_gather_rows(const float* A, int64_t lda, int32_t d, const int32_t* rows,
                              int64_t nrows, float* out, int64_t ldo, int64_t* ids_out,
                              hipStream_t st);
hipError_t launch_narrow(const int64_t* in, int64_t n, int32_t* out, hipStream_t st);
// keys -> perm (items ordered by (key, item)), offsets[nk + 1] (optional);
// cnt needs nk * csort_blocks(n) int32.
hipError_t launch_csort(const int32_t* keys, int64_t n, int32_t nk, int32_t* cnt, int32_t* perm,
                        int32_t* offsets, hipStream_t st);
hipError_t launch_psi(const float* X, int64_t ldx, int32_t d, int32_t metric, int64_t n,
                      const int32_t* owner, const float* R, int64_t ldr, double* psi,
                      hipStream_t st);
hipError_t launch_dist_all(int metric, const float* Q, int64_t ldq, int32_t m, const float* R,
                           int64_t ldr, int32_t nr, int32_t d, float* DR, int64_t ldd,
                           hipStream_t st);
hipError_t launch_prune(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t k, int32_t c,
                        double delta, const double* psi, const int32_t* list_off, int32_t* lrank,
                        uint8_t* keep_rq, int32_t* nkept, float* gcup, int64_t* stats,
                        hipStream_t st);
// roff and ioff need nr + 1 entries; roff[nr] / ioff[nr] receive the totals.
hipError_t launch_worklist(const uint8_t* keep_rq, int32_t m, int32_t nr, int32_t* roff,
                           int32_t* ioff, int32_t* qlist, hipStream_t st);
// exclusive scan of v[0 .. n), total to v[n]
hipError_t launch_scan_total(int32_t* v, int64_t n, hipStream_t st);
hipError_t launch_tau(const float* gcup, const float* qn, const uint32_t* xmax_bits, int32_t m,
                      int32_t d, int32_t mode, double delta, float* tau, hipStream_t st);

}  // namespace rbc
