// rbc_host.h -- host-side plan and workspace types of librbc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rbc.h"
#include "rbc_common.h"

namespace rbc {

constexpr int kPathMfma = 0;   // L2 tile on the matrix cores
constexpr int kPathValu = 1;   // l1 / small-d l2 tile on the vector ALUs
constexpr int kPathExact = 2;  // exhaustive float64 (k or d beyond the tiles)
constexpr int kPathLowp = 3;   // L2 tile on quantised rows (bf16 / fp8)
constexpr int kConcurrentBlocks = 512;  // 256 CUs x 2 resident tile workgroups
constexpr int kMaxSplits = 64;          // one partial list per lane in finalize
constexpr int kFallbackBlocks = 256;
constexpr int kItemBlocks = 1024;       // persistent grid of the stage-2 item kernels
constexpr int kCounters = 16;
// A matrix "xstat" block: [0] largest row norm (float bits), [1..3] value
// flags of tile_exact; 4 words, zeroed before the norms kernel fills it.

int set_err(int status, const char* fmt, ...);
const char* last_error();
int hip_status(hipError_t e, const char* what);
int shortlist_len(int k, int requested);

// Bump allocator over a caller-provided workspace (base == nullptr: size only).
class Carver {
public:
    explicit Carver(char* base) : base_(base), off_(0) {}
    template <class T>
    T* take(int64_t count) {
        off_ = (off_ + 255) / 256 * 256;
        T* p = base_ ? (T*)(base_ + off_) : nullptr;
        off_ += (size_t)(count > 0 ? count : 0) * sizeof(T);
        return p;
    }
    size_t size() const { return (off_ + 255) / 256 * 256; }

private:
    char* base_;
    size_t off_;
};

struct BfPlan {
    int path;
    int metric;
    int k;
    int d;
    int64_t ldp;       // leading dimension of repacked copies (d rounded up to 4)
    bool repack_q, repack_x;
    int c;             // shortlist length
    int ks;            // 16-feature slabs
    int32_t nqblk;     // 256-query blocks
    int32_t nsplit;    // database splits
    int32_t rps;       // rows per split (BF mode)
    int prec;          // rbc_precision
    int kb;            // low precision: 32-feature blocks (bf16) / 1 (fp8)
    int dq;            // low precision: padded row length of the quantised copies
    // low precision: queries whose certificate fails are re-ranked by the
    // fp32 matrix tile over all rows (a device-sized launch) before any
    // float64 fallback
    bool casc;
    int c32;           // shortlist length of that fp32 pass
    int ks32;          // its 16-feature slabs
    int64_t ldc;       // row length of the compacted query copies (d rounded up to 4)
    int32_t casc_blocks;  // its workgroups
    double prune_eps;     // exact RBC search: pruning bounds divided by (1 + eps)
    bool one_pass;        // RBC_FLAG_ONE_PASS given
    bool two_pass;        // exact RBC search in two passes (set by the index's planner)
    int shape;            // fp32 matrix tile shape of the BF launch (kShape16 / kShape32)
    bool lowp_seed;       // low-precision exact search: an fp32 pass over each query's
                          // nearest list tightens the stage-2 shortlist seeds
};

struct BfWork {
    int32_t* fb_list = nullptr;
    // [0] fallback count, [2] work queue, [4..7] query stats (see xstat),
    // [8..11] database stats: [8] max row norm bits, [9..11] value flags,
    // [12..13] quantised database: max ||x~||, max ||x - x~||; [14..15] the
    // same for the queries
    int32_t* counters = nullptr;
    float* Qp = nullptr;
    float* Xp = nullptr;
    float* qn = nullptr;
    float* xn = nullptr;
    float* pval = nullptr;
    int32_t* pidx = nullptr;
    void* Qq = nullptr;        // quantised rows (low precision)
    void* Xq = nullptr;
    uint8_t* qscale = nullptr;
    uint8_t* xscale = nullptr;
    float* qerr = nullptr;
    // fp32 cascade (low precision): compacted queries, their norms and
    // original rows, fp32 norms of X (bf_search only), partial lists
    float* Qc = nullptr;
    float* qnc = nullptr;
    int32_t* qmap = nullptr;
    float* xn32 = nullptr;
    // optional (set by the exact build): fp32 squared norms and value flags
    // of the rows of Q, written by the low-precision path's quantiser
    float* qn32 = nullptr;
    uint32_t* qflags32 = nullptr;
    float* pval_c = nullptr;
    int32_t* pidx_c = nullptr;
};

// Records a pair of HIP events around a launch when timing is enabled
// (rbc_timer_enable); the scope is the launch.
class KernelTimer {
public:
    KernelTimer(const char* name, hipStream_t st);
    ~KernelTimer();

private:
    const char* name_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool active_ = false;
};

// Tile configuration of one fp32 matrix-core launch (rbc_tune.cpp): the
// tuned choice for (kind, slabs, shortlist length), else the fixed rule.
constexpr int kTuneBF = 0;     // BF tile (bf_search, cascade, exact-index fallback)
constexpr int kTuneItems = 1;  // stage 2 of the exact RBC search
struct TileChoice {
    int shape = kShape16;
    int blocks = kItemBlocks;
    int splits = 0;  // row ranges per nearest list in pass 1 (0: the size rule)
    int qb = 4;      // stage 2, 16x16 shape: 16-query blocks per item (4 or 2)
};
TileChoice tile_choice(int kind, int ks, int c);

int make_bf_plan(int64_t m, int64_t n, int32_t d, int64_t ldq, int64_t ldx, int32_t metric,
                 int32_t k, const rbc_search_opts* opts, BfPlan* p);
void carve_bf(const BfPlan& p, int64_t m, int64_t n, Carver& cv, BfWork* w);
// xstat: precomputed stats of X (with xn), or null to compute them.
int run_bf(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n,
           int64_t ldx, const float* xn, const uint32_t* xstat, const int64_t* id_map,
           int64_t* out_idx, float* out_dist, BfWork& w, int64_t* stats, hipStream_t st,
           float* out_approx = nullptr);
FinArgs fin_args(const BfPlan& p, const float* Qk, int64_t m, int64_t ldqk, const float* Xk,
                 int64_t ldxk, const uint32_t* xstat, const int64_t* id_map,
                 int64_t* out_idx, float* out_dist, BfWork& w, int64_t* stats,
                 float* out_approx = nullptr);
int run_finalize(const BfPlan& p, const FinArgs& f, hipStream_t st);
int run_fallback(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X,
                 int64_t n, int64_t ldx, const int64_t* id_map, int64_t* out_idx,
                 float* out_dist, BfWork& w, hipStream_t st);
int validate_common(int64_t m, int64_t n, int32_t d, int32_t k, int32_t metric);
void carve_cascade(const BfPlan& p, int64_t m, int64_t n, bool xnorms, Carver& cv, BfWork* w);
// The fp32 cascade after a low-precision finalize: the queries in w.fb_list
// (count w.counters[0]) are compacted, searched by the fp32 tile over X and
// finalized; those still uncertified are left in w.fb_list for run_fallback.
// xn / xstat: fp32 norms and stats of X, or null to compute them (gated on a
// non-empty list).
int run_cascade(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X,
                int64_t n, int64_t ldx, const float* xn, const uint32_t* xstat,
                const int64_t* id_map, int64_t* out_idx, float* out_dist, BfWork& w,
                int64_t* stats, hipStream_t st);

}  // namespace rbc
