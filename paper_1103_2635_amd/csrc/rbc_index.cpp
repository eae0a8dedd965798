// rbc_index.cpp -- Random Ball Cover build and search (Sec. 4 and Sec. 5).
//
// Exact mode (Sec. 5.2):
//   build   R = the representatives, BF(X, R) with k = 1 gives every point its
//           owner; a stable counting sort by owner turns the lists L_r into
//           contiguous row ranges of a permuted copy Xp of X (ascending id
//           inside a list); psi_r is the largest owner distance (float64).
//   search  stage 1: rho(q, r) for every representative (fp32, direct);
//           pruning rules (1) and (2) in their k-NN form with error margins;
//           queries grouped by nearest representative into 256-query blocks;
//           stage 2: one grouped launch of the distance tile over the union of
//           the block's kept lists, each query scoring only its own kept
//           lists; then the shortlist finalize / float64 fallback of bf_search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/rbc.h"
#include "rbc_host.h"
#include "rbc_kernels.h"

using namespace rbc;

struct rbc_index {
    int32_t mode = 0, metric = 0, d = 0;
    int64_t n = 0, n_r = 0, s = 0, ld = 0;
    int64_t rows = 0;            // rows of Xp
    float* Xp = nullptr;         // list rows (exact: a permutation of X)
    float* xn = nullptr;         // squared norms of Xp rows
    int64_t* ids = nullptr;      // Xp row -> row of the original X
    int32_t* list_off = nullptr; // n_r + 1 row offsets of the lists in Xp
    float* R = nullptr;          // representatives, n_r x ld
    double* psi = nullptr;       // list radii
    uint32_t* norms_max = nullptr;  // xstat of Xp: [0] max row norm bits, [1..3] value flags
    float* own = nullptr;           // exact mode: rho(x, owner) of each row of Xp
    int32_t* lsorted = nullptr;     // exact mode: list r sorted by own (1) or not (0)
    // quantised copies of Xp for low-precision searches, indexed by rbc_precision
    struct Quant {
        void* X = nullptr;        // rows x dq elements (bf16) or bytes (fp8 e4m3)
        float* xn = nullptr;      // ||x~||^2
        uint8_t* scale = nullptr; // fp8: E8M0 row scales
        uint32_t* stat = nullptr; // [0] max ||x~||, [1] max ||x - x~|| (float bits)
        int dq = 0;
    } quant[3];
    std::vector<int64_t> rep_host;
    std::vector<void*> allocs;
    size_t bytes = 0;
    void* block = nullptr;       // the main allocation (Layout), returned to the block cache
    size_t block_bytes = 0;
    int block_dev = 0;
};

namespace {

template <class T>
int dev_alloc(rbc_index* ix, T** p, int64_t count) {
    const size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    void* q = nullptr;
    if (hipMalloc(&q, b) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(RBC_ENOMEM, "device allocation of %zu bytes failed", b);
    }
    ix->allocs.push_back(q);
    ix->bytes += b;
    *p = (T*)q;
    return RBC_OK;
}

// The main device block of the last freed index, one per device, handed to
// the next build that fits in it: a rebuild (a new batch of points) then
// neither frees nor maps a few hundred MB, which costs about 0.4 ms.
std::mutex g_block_mu;
std::map<int, std::pair<void*, size_t>> g_block_cache;

int take_block(size_t bytes, void** out, int* dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_err(RBC_EHIP, "hipGetDevice failed");
    *dev_out = dev;
    {
        std::lock_guard<std::mutex> lk(g_block_mu);
        auto it = g_block_cache.find(dev);
        // reuse a cached block no more than twice the size needed (plus 64 MB)
        if (it != g_block_cache.end() && it->second.second >= bytes &&
            it->second.second <= 2 * bytes + ((size_t)64 << 20)) {
            *out = it->second.first;
            g_block_cache.erase(it);
            return RBC_OK;
        }
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(RBC_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    return RBC_OK;
}

void give_block(void* p, size_t bytes, int dev) {
    void* drop = p;
    {
        std::lock_guard<std::mutex> lk(g_block_mu);
        auto it = g_block_cache.find(dev);
        if (it == g_block_cache.end()) {
            g_block_cache[dev] = {p, bytes};
            drop = nullptr;
        } else if (it->second.second < bytes) {
            drop = it->second.first;
            it->second = {p, bytes};
        }
    }
    if (drop) (void)hipFree(drop);
}

void free_index(rbc_index* ix) {
    if (!ix) return;
    (void)hipDeviceSynchronize();
    for (void* p : ix->allocs) (void)hipFree(p);
    if (ix->block) give_block(ix->block, ix->block_bytes, ix->block_dev);
    delete ix;
}

// Temporary device buffers of one build, released on every return path.
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    int take(T** p, int64_t count) {
        void* q = nullptr;
        const size_t b = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        if (hipMalloc(&q, b) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(RBC_ENOMEM, "device allocation of %zu bytes failed", b);
        }
        ptrs.push_back(q);
        *p = (T*)q;
        return RBC_OK;
    }
};

// Device memory of an index as one allocation: add() records the arrays,
// commit() allocates their sum (256-byte aligned pieces) and hands them out.
struct Layout {
    std::vector<std::pair<void**, size_t>> items;
    template <class T>
    void add(T** p, int64_t count) {
        items.push_back({(void**)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)});
    }
    int commit(rbc_index* ix) {
        size_t total = 0;
        for (auto& it : items) total += (it.second + 255) & ~(size_t)255;
        void* base = nullptr;
        int dev = 0;
        if (int rc = take_block(total, &base, &dev)) return rc;
        ix->block = base;
        ix->block_bytes = total;
        ix->block_dev = dev;
        ix->bytes += total;
        char* c = (char*)base;
        for (auto& it : items) {
            *it.first = c;
            c += (it.second + 255) & ~(size_t)255;
        }
        items.clear();
        return RBC_OK;
    }
};

// Scratch of exact builds, kept per device between builds (grown when a
// larger build needs more) so that a build allocates only its index.
// Builds hold g_build_mu from the first use of the scratch to their final
// synchronisation; searches never touch it.
std::mutex g_build_mu;
std::map<int, std::pair<void*, size_t>> g_build_scratch;

int build_scratch(size_t bytes, char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_err(RBC_EHIP, "hipGetDevice failed");
    auto& e = g_build_scratch[dev];
    if (e.second < bytes) {
        if (e.first) (void)hipFree(e.first);
        e.first = nullptr;
        e.second = 0;
        if (hipMalloc(&e.first, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(RBC_ENOMEM, "device allocation of %zu bytes failed", bytes);
        }
        e.second = bytes;
    }
    *out = (char*)e.first;
    return RBC_OK;
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// n_r distinct ids drawn uniformly from [0, n) (Floyd's sampling), sorted.
std::vector<int64_t> sample_reps(int64_t n, int64_t n_r, uint64_t seed) {
    std::unordered_set<int64_t> chosen;
    chosen.reserve((size_t)n_r * 2);
    uint64_t st = seed;
    for (int64_t j = n - n_r; j < n; ++j) {
        const uint64_t r = splitmix64(st);
        const int64_t t = (int64_t)(((unsigned __int128)r * (uint64_t)(j + 1)) >> 64);
        if (!chosen.insert(t).second) chosen.insert(j);
    }
    std::vector<int64_t> out(chosen.begin(), chosen.end());
    std::sort(out.begin(), out.end());
    return out;
}

int check(hipError_t e, const char* what) { return hip_status(e, what); }

// Exhaustive float64 search of the listed queries, each restricted to the
// list of its representative qrep[q] (one-shot).
int run_fallback_lists(const BfPlan& p, const float* Q, int64_t m, int64_t ldq,
                       const rbc_index* ix, const int32_t* qrep, int64_t* out_idx,
                       float* out_dist, BfWork& w, hipStream_t st) {
    ExactArgs e;
    std::memset(&e, 0, sizeof(e));
    e.Q = Q;
    e.ldq = ldq;
    e.X = ix->Xp;
    e.ldx = ix->ld;
    e.n = (int32_t)ix->rows;
    e.d = ix->d;
    e.metric = ix->metric;
    e.k = p.k;
    e.list = w.fb_list;
    e.count = w.counters;
    e.id_map = ix->ids;
    e.qrep = qrep;
    e.list_off = ix->list_off;
    e.out_idx = out_idx;
    e.out_dist = out_dist;
    const int grid = p.path == kPathExact ? (int)std::min<int64_t>(m, 2048) : kFallbackBlocks;
    KernelTimer kt("fallback", st);
    return check(launch_exact(e, grid, st), "exact fallback");
}

int build_exact(rbc_index* ix, const float* X, int64_t ldx, hipStream_t st) {
    const int64_t n = ix->n, n_r = ix->n_r, ld = ix->ld;
    const int32_t d = ix->d;
    int rc;
    Layout lay;
    lay.add(&ix->R, n_r * ld);
    lay.add(&ix->psi, n_r);
    lay.add(&ix->list_off, n_r + 1);
    lay.add(&ix->Xp, n * ld);
    lay.add(&ix->xn, n);
    lay.add(&ix->ids, n);
    lay.add(&ix->norms_max, 4);
    lay.add(&ix->own, n);
    lay.add(&ix->lsorted, n_r);
    if ((rc = lay.commit(ix))) return rc;
    ix->rows = n;

    // ownership: BF(X, R) with k = 1 (ties to the lower representative
    // position).  For l2 the ranking runs on bf16 copies (the matrix cores'
    // bf16 rate); the shortlist is re-scored in float32 and certified with the
    // quantisation error included, uncertified points are ranked again in
    // float32 and float64, so the owners are those of the exact search.
    BfPlan p;
    rbc_search_opts own_opts;
    std::memset(&own_opts, 0, sizeof(own_opts));
    own_opts.precision = RBC_BF16;
    own_opts.shortlist = 4;  // k = 1: the nearest owner is rarely within the bf16 error of a 5th
    const bool own_bf16 = ix->metric == RBC_L2 && d <= 128;
    if ((rc = make_bf_plan(n, n_r, d, ldx, ld, ix->metric, 1, own_bf16 ? &own_opts : nullptr, &p)))
        return rc;
    int32_t *reps = nullptr, *owner = nullptr, *perm = nullptr, *cnt = nullptr;
    int64_t* own64 = nullptr;
    float* ownd = nullptr;
    float* xn32 = nullptr;        // bf16 ownership: fp32 norms of X from the quantiser
    uint32_t* xflags = nullptr;   // and the value flags (3 words)
    BfWork w;
    auto carve = [&](Carver& cv) {
        xn32 = cv.take<float>(n);
        xflags = cv.take<uint32_t>(4);
        reps = cv.take<int32_t>(n_r);
        owner = cv.take<int32_t>(n);
        perm = cv.take<int32_t>(n);
        cnt = cv.take<int32_t>(csort_scratch(n, (int32_t)n_r));
        own64 = cv.take<int64_t>(n);
        ownd = cv.take<float>(n);
        carve_bf(p, n, n_r, cv, &w);
    };
    Carver probe(nullptr);
    carve(probe);
    std::lock_guard<std::mutex> lock(g_build_mu);
    char* ws = nullptr;
    if ((rc = build_scratch(probe.size(), &ws))) return rc;
    Carver cv(ws);
    carve(cv);
    std::vector<int32_t> reps32(ix->rep_host.begin(), ix->rep_host.end());
    if ((rc = check(hipMemcpyAsync(reps, reps32.data(), n_r * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st), "copy representatives")))
        return rc;
    if ((rc = check(launch_gather_rows(X, ldx, d, reps, n_r, ix->R, ld, nullptr, st), "gather R")))
        return rc;
    if (p.path == kPathLowp) {
        w.qn32 = xn32;
        w.qflags32 = xflags;
        if ((rc = check(launch_fill_i32((int32_t*)xflags, 4, 0, st), "clear flags"))) return rc;
    }
    if ((rc = run_bf(p, X, n, ldx, ix->R, n_r, ld, nullptr, nullptr, nullptr, own64, ownd, w,
                     nullptr, st)))
        return rc;
    if ((rc = check(launch_narrow(own64, n, owner, st), "owners"))) return rc;

    // lists: stable counting sort of the points by owner, then each list by
    // the distance to its owner (ties in id order), kept with the index
    if ((rc = check(launch_csort(owner, n, (int32_t)n_r, cnt, perm, ix->list_off, st), "sort")))
        return rc;
    if ((rc = check(launch_seg_sort(ix->list_off, (int32_t)n_r, perm, ownd, 0, ix->lsorted, st),
                    "sort lists")))
        return rc;
    if ((rc = check(launch_gather_rows(X, ldx, d, perm, n, ix->Xp, ld, ix->ids, st), "gather Xp")))
        return rc;
    if ((rc = check(launch_gather_rows(ownd, 1, 1, perm, n, ix->own, 1, nullptr, st), "gather own")))
        return rc;
    if ((rc = check(launch_fill_i32((int32_t*)ix->norms_max, 4, 0, st), "clear"))) return rc;
    if (p.path == kPathMfma) {
        // the ownership search already has ||x||^2 and the value flags of X
        if ((rc = check(launch_gather_norms(w.qn, perm, n, ix->xn, ix->norms_max,
                                            (const uint32_t*)w.counters + 5, ix->norms_max + 1,
                                            st), "norms")))
            return rc;
    } else if (p.path == kPathLowp) {
        // the bf16 quantiser read X once for the copies, the norms and the flags
        if ((rc = check(launch_gather_norms(xn32, perm, n, ix->xn, ix->norms_max, xflags,
                                            ix->norms_max + 1, st), "norms")))
            return rc;
    } else if ((rc = check(launch_row_norms(ix->Xp, n, ld, d, nullptr, ix->xn, ix->norms_max, st,
                                            ix->norms_max + 1), "norms"))) {
        return rc;
    }
    if ((rc = check(launch_psi_own(ix->Xp, ld, d, ix->metric, ix->own, ix->list_off, ix->lsorted,
                                   ix->R, ld, (int32_t)n_r, ix->psi, st), "psi")))
        return rc;
    return check(hipStreamSynchronize(st), "build");
}

// One-shot build (Sec. 4, Sec. 5.1): BF(R, X) keeping every value, chunk by
// chunk of representatives; each list is the s nearest points of its
// representative in (float64 distance, id) order, psi_r the s-th distance.
int build_oneshot(rbc_index* ix, const float* X, int64_t ldx, hipStream_t st) {
    const int64_t n = ix->n, n_r = ix->n_r, s = ix->s, ld = ix->ld;
    const int32_t d = ix->d;
    if (s > kOsCap)
        return set_err(RBC_EUNSUPPORTED, "one-shot list length s > %d", kOsCap);
    if (n_r * s >= ((int64_t)1 << 31))
        return set_err(RBC_EUNSUPPORTED, "n_r * s >= 2^31");
    const int ks = (d + 15) / 16;
    if (ks > kMaxKS) return set_err(RBC_EUNSUPPORTED, "one-shot build with d > %d", 16 * kMaxKS);
    const bool mfma = ix->metric == RBC_L2 && d >= 12;
    int rc;
    ix->rows = n_r * s;
    if ((rc = dev_alloc(ix, &ix->R, n_r * ld))) return rc;
    if ((rc = dev_alloc(ix, &ix->psi, n_r))) return rc;
    if ((rc = dev_alloc(ix, &ix->list_off, n_r + 1))) return rc;
    if ((rc = dev_alloc(ix, &ix->Xp, ix->rows * ld))) return rc;
    if ((rc = dev_alloc(ix, &ix->xn, ix->rows))) return rc;
    if ((rc = dev_alloc(ix, &ix->ids, ix->rows))) return rc;
    if ((rc = dev_alloc(ix, &ix->norms_max, 4))) return rc;

    Scratch sc;
    int32_t *reps = nullptr, *lists = nullptr, *ctr = nullptr;
    float *rn2 = nullptr, *xnf = nullptr;
    if ((rc = sc.take(&reps, n_r)) || (rc = sc.take(&lists, ix->rows)) || (rc = sc.take(&ctr, 8)) ||
        (rc = sc.take(&rn2, n_r)) || (rc = sc.take(&xnf, n)))
        return rc;
    std::vector<int32_t> reps32(ix->rep_host.begin(), ix->rep_host.end());
    if ((rc = check(hipMemcpyAsync(reps, reps32.data(), n_r * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st), "copy representatives")))
        return rc;
    if ((rc = check(launch_gather_rows(X, ldx, d, reps, n_r, ix->R, ld, nullptr, st), "gather R")))
        return rc;
    // the tile reads float4 rows: repack X when its layout does not allow it
    const float* Xk = X;
    int64_t ldxk = ldx;
    if ((ldx % 4) || (d % 4)) {
        float* xr = nullptr;
        if ((rc = sc.take(&xr, n * ld))) return rc;
        if ((rc = check(launch_repack(X, n, ldx, d, xr, ld, st), "repack X"))) return rc;
        Xk = xr;
        ldxk = ld;
    }
    if ((rc = check(launch_fill_i32(ctr, 8, 0, st), "clear"))) return rc;
    uint32_t* xmax = (uint32_t*)ctr;  // xstat of X
    if ((rc = check(launch_row_norms(Xk, n, ldxk, d, nullptr, xnf, xmax, st, xmax + 1), "norms X")))
        return rc;
    if ((rc = check(launch_row_norms(ix->R, n_r, ld, d, nullptr, rn2, nullptr, st), "norms R")))
        return rc;
    // value matrix of one chunk of representatives: at most 2 GiB
    const int64_t ldv = (n + 3) / 4 * 4;
    int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 31) / (ldv * 4));
    chunk = std::min<int64_t>(chunk, n_r);
    float* V = nullptr;
    OneShotWork w;
    if ((rc = sc.take(&V, chunk * ldv)) || (rc = sc.take(&w.hist, chunk * 4096)) ||
        (rc = sc.take(&w.prefix, chunk)) || (rc = sc.take(&w.need, chunk)) ||
        (rc = sc.take(&w.tval, chunk)) || (rc = sc.take(&w.bound, chunk)) ||
        (rc = sc.take(&w.cnt, chunk)) || (rc = sc.take(&w.cand, chunk * kOsCap)))
        return rc;
    w.overflow = ctr + 4;
    const double delta = 2.0 * (d + 2) * 5.9604644775390625e-8;
    const int mode = mfma ? 0 : (ix->metric == RBC_L2 ? 1 : 2);
    for (int64_t c0 = 0; c0 < n_r; c0 += chunk) {
        const int32_t rcnt = (int32_t)std::min<int64_t>(chunk, n_r - c0);
        TileArgs a;
        std::memset(&a, 0, sizeof(a));
        a.Q = ix->R + c0 * ld;
        a.ldq = ld;
        a.m = rcnt;
        a.X = Xk;
        a.ldx = ldxk;
        a.n = (int32_t)n;
        a.d = d;
        a.xn = xnf;
        const int64_t nqb = (rcnt + kTileQ - 1) / kTileQ;
        int64_t splits = std::max<int64_t>(1, (4 * kConcurrentBlocks) / nqb);
        int64_t rps = (n + splits - 1) / splits;
        rps = (rps + kRowsMfma - 1) / kRowsMfma * kRowsMfma;
        a.rps = (int32_t)rps;
        a.nsplit = (int32_t)((n + rps - 1) / rps);
        a.pval = V;
        a.ldo = ldv;
        const dim3 grid((unsigned)nqb, (unsigned)a.nsplit);
        {
            KernelTimer kt("oneshot_tile", st);
            rc = mfma ? check(launch_tile_mfma(ks, 4, kTileAll, grid, a, st), "one-shot tile")
                      : check(launch_tile_valu(ix->metric, ks, 4, kTileAll, grid, a, st),
                              "one-shot tile");
        }
        if (rc) return rc;
        {
            KernelTimer kt("oneshot_select", st);
            if ((rc = check(launch_oneshot_select(V, ldv, (int32_t)n, rcnt, (int32_t)s, mode, delta,
                                                  d, rn2 + c0, xmax, xmax + 1, w, st),
                            "one-shot select")))
                return rc;
            if ((rc = check(launch_oneshot_sort(X, ldx, d, ix->metric, ix->R, ld, rcnt, (int32_t)s,
                                                (int32_t)c0, w, lists, ix->psi, st),
                            "one-shot sort")))
                return rc;
        }
    }
    int32_t overflow = 0;
    if ((rc = check(hipMemcpyAsync(&overflow, w.overflow, sizeof(int32_t), hipMemcpyDeviceToHost,
                                   st), "read overflow")) ||
        (rc = check(hipStreamSynchronize(st), "one-shot lists")))
        return rc;
    if (overflow)
        return set_err(RBC_EUNSUPPORTED,
                       "%d representatives have more than %d points within the rounding margin "
                       "of their s-th neighbour", overflow, kOsCap);
    if ((rc = check(launch_gather_rows(X, ldx, d, lists, ix->rows, ix->Xp, ld, ix->ids, st),
                    "gather lists")))
        return rc;
    if ((rc = check(launch_list_offsets(ix->list_off, (int32_t)n_r, (int32_t)s, st), "offsets")))
        return rc;
    if ((rc = check(launch_fill_i32((int32_t*)ix->norms_max, 4, 0, st), "clear"))) return rc;
    if ((rc = check(launch_row_norms(ix->Xp, ix->rows, ld, d, nullptr, ix->xn, ix->norms_max, st,
                                     ix->norms_max + 1), "norms")))
        return rc;
    return check(hipStreamSynchronize(st), "build");
}

// Quantised copies of the index rows for the requested low precisions.
int build_quant(rbc_index* ix, int32_t precisions, hipStream_t st) {
    if (precisions & ~((1 << RBC_BF16) | (1 << RBC_FP8_E4M3)))
        return set_err(RBC_EINVAL, "unknown bits in precisions");
    if (ix->mode != RBC_EXACT || ix->metric != RBC_L2 || ix->d > 128)
        return set_err(RBC_EUNSUPPORTED, "low precision needs an exact L2 index with d <= 128");
    int rc;
    for (int prec : {RBC_BF16, RBC_FP8_E4M3}) {
        if (!(precisions & (1 << prec))) continue;
        rbc_index::Quant& q = ix->quant[prec];
        const int fmt = prec == RBC_BF16 ? 0 : 1;
        q.dq = prec == RBC_BF16 ? (ix->d + 31) / 32 * 32 : 128;
        uint8_t* xq = nullptr;
        if ((rc = dev_alloc(ix, &xq, ix->rows * q.dq * (prec == RBC_BF16 ? 2 : 1)))) return rc;
        q.X = xq;
        if ((rc = dev_alloc(ix, &q.xn, ix->rows))) return rc;
        if ((rc = dev_alloc(ix, &q.stat, 4))) return rc;
        if (prec == RBC_FP8_E4M3 && (rc = dev_alloc(ix, &q.scale, ix->rows))) return rc;
        if ((rc = check(launch_fill_i32((int32_t*)q.stat, 4, 0, st), "clear"))) return rc;
        if ((rc = check(launch_quantize(fmt, ix->Xp, ix->rows, ix->ld, ix->d, 1.0f, q.X, q.dq, q.dq,
                                        q.xn, nullptr, q.scale, q.stat, st), "quantize")))
            return rc;
    }
    return check(hipStreamSynchronize(st), "quantize");
}

struct SearchWork {
    BfWork bf;
    float* DR = nullptr;       // stage-1 distances, m x ldd
    int32_t* lrank = nullptr;  // m x n_r
    uint8_t* keep_rq = nullptr;  // n_r x m
    int32_t* npairs = nullptr;   // m
    int32_t* qoff = nullptr;     // m + 1
    float* gcup = nullptr;       // m
    float* tau = nullptr;        // m
    int32_t* roff = nullptr;     // n_r + 1
    int32_t* ioff = nullptr;     // n_r + 1
    int32_t* qlist = nullptr;    // up to m * n_r
    int32_t* irep = nullptr;     // item -> representative
    // two-pass search: pass 1 over each query's nearest list
    int32_t* home = nullptr;     // m: nearest representative
    int32_t* qa = nullptr;       // m: queries grouped by home
    int32_t* roffa = nullptr;    // n_r + 1
    int32_t* ioffa = nullptr;    // n_r + 1
    int32_t* irepa = nullptr;    // pass-1 item -> representative
    int32_t* csa = nullptr;      // counting-sort scratch
    float* hval = nullptr;       // m x c: pass-1 shortlists
    int32_t* hidx = nullptr;
    float* taud = nullptr;       // m: bound on the k-th neighbour distance
    float* tauc = nullptr;       // m: bound on the c-th neighbour distance (two passes)
    int32_t* irows = nullptr;    // 2 per pass-2 item: its row run
    int32_t* rec = nullptr;      // matrix path: kItemRec per pass-2 item, in item order
    int32_t* srec = nullptr;     // the same records, longest item first
    float* qn32 = nullptr;       // low-precision seeds: fp32 squared query norms
};

int64_t stage1_ld(int64_t nr) { return (nr + 3) / 4 * 4; }

// One-shot search scratch: the nearest-representative BF (its own plan) and
// the one-list-per-query stage 2.
struct OneShotSearchWork {
    BfPlan p1;
    BfWork w1;            // BF(Q, R), k = 1
    int64_t* near64 = nullptr;
    float* neard = nullptr;
    int32_t* nearest = nullptr;
    int32_t* cnt = nullptr;
    int32_t* qlist = nullptr;
    int32_t* roff = nullptr;
    int32_t* ioff = nullptr;
    int32_t* irep = nullptr;
};

int carve_oneshot(const rbc_index* ix, const BfPlan& p, int64_t m, int64_t ldq, Carver& cv,
                  SearchWork* w, OneShotSearchWork* o) {
    int rc = make_bf_plan(m, ix->n_r, ix->d, ldq, ix->ld, ix->metric, 1, nullptr, &o->p1);
    if (rc) return rc;
    carve_bf(o->p1, m, ix->n_r, cv, &o->w1);
    o->near64 = cv.take<int64_t>(m);
    o->neard = cv.take<float>(m);
    o->nearest = cv.take<int32_t>(m);
    o->cnt = cv.take<int32_t>(csort_scratch(m, (int32_t)ix->n_r));
    o->qlist = cv.take<int32_t>(m);
    o->roff = cv.take<int32_t>(ix->n_r + 1);
    o->ioff = cv.take<int32_t>(ix->n_r + 1);
    o->irep = cv.take<int32_t>(m / kWave + ix->n_r + 1);
    if (p.path == kPathExact) {
        carve_bf(p, m, ix->rows, cv, &w->bf);
        return RBC_OK;
    }
    w->bf.fb_list = cv.take<int32_t>(m);
    w->bf.counters = cv.take<int32_t>(kCounters);
    if (p.repack_q) w->bf.Qp = cv.take<float>(m * p.ldp);
    if (p.path == kPathMfma) w->bf.qn = cv.take<float>(m);
    w->bf.pval = cv.take<float>(m * p.c);
    w->bf.pidx = cv.take<int32_t>(m * p.c);
    return RBC_OK;
}

// One-shot search, Sec. 5.1: r_q = the nearest representative (certified
// BF(Q, R), ties to the lower position), then BF(q, L_{r_q}) for every query,
// run as one grouped launch over (representative, query chunk) items.
int search_oneshot(const rbc_index* ix, const BfPlan& p, const float* Q, int64_t m, int64_t ldq,
                   int64_t* out_idx, float* out_dist, SearchWork& w, OneShotSearchWork& o,
                   int64_t* stats, hipStream_t st) {
    const int32_t nr = (int32_t)ix->n_r;
    int rc;
    {
        KernelTimer kt("stage1", st);
        if ((rc = run_bf(o.p1, Q, m, ldq, ix->R, nr, ix->ld, nullptr, nullptr, nullptr, o.near64,
                         o.neard, o.w1, nullptr, st)))
            return rc;
    }
    {
        KernelTimer kt("worklist", st);
        if ((rc = check(launch_narrow(o.near64, m, o.nearest, st), "nearest"))) return rc;
        if ((rc = check(launch_csort(o.nearest, m, nr, o.cnt, o.qlist, o.roff, st), "group")))
            return rc;
        const int32_t isize = p.path == kPathMfma ? kWave : kTileQ;
        if ((rc = check(launch_items_from_offsets(o.roff, nr, isize, o.ioff, st), "items")))
            return rc;
        if ((rc = check(launch_item_reps(o.ioff, nr, o.irep, st), "item reps"))) return rc;
    }
    if (p.path == kPathExact) {
        // k beyond the register shortlist: exhaustive float64 inside each list
        if ((rc = check(launch_iota_i32(w.bf.fb_list, (int32_t)m, st), "iota"))) return rc;
        if ((rc = check(launch_set_count(w.bf.counters, (int32_t)m, st), "count"))) return rc;
        return run_fallback_lists(p, Q, m, ldq, ix, o.nearest, out_idx, out_dist, w.bf, st);
    }
    const float* Qk = Q;
    int64_t ldqk = ldq;
    if (p.repack_q) {
        if ((rc = check(launch_repack(Q, m, ldq, p.d, w.bf.Qp, p.ldp, st), "repack Q"))) return rc;
        Qk = w.bf.Qp;
        ldqk = p.ldp;
    }
    if ((rc = check(launch_fill_i32(w.bf.counters, kCounters, 0, st), "clear counters"))) return rc;
    if (p.path == kPathMfma &&
        (rc = check(launch_row_norms(Qk, m, ldqk, p.d, nullptr, w.bf.qn, nullptr, st,
                                     (uint32_t*)w.bf.counters + 5), "norms Q")))
        return rc;
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = Qk;
    a.ldq = ldqk;
    a.m = (int32_t)m;
    a.X = ix->Xp;
    a.ldx = ix->ld;
    a.n = (int32_t)ix->rows;
    a.d = ix->d;
    a.xn = ix->xn;
    a.item_total = o.ioff + nr;
    a.item_queue = w.bf.counters + 2;
    a.irep = o.irep;
    a.ioff = o.ioff;
    a.roff = o.roff;
    a.qlist = o.qlist;
    a.list_off = ix->list_off;
    a.n_r = nr;
    a.pval = w.bf.pval;
    a.pidx = w.bf.pidx;
    a.stats = stats;
    {
        KernelTimer kt("tile_items", st);
        const dim3 grid(kItemBlocks);
        rc = p.path == kPathMfma
                 ? check(launch_tile_mfma(p.ks, p.c, kTileItems, grid, a, st), "stage 2 (mfma)")
                 : check(launch_tile_valu(p.metric, p.ks, p.c, kTileItems, grid, a, st),
                         "stage 2 (valu)");
        if (rc) return rc;
    }
    FinArgs f = fin_args(p, Qk, m, ldqk, ix->Xp, ix->ld, ix->norms_max, ix->ids, out_idx,
                         out_dist, w.bf, stats);
    f.nsplit = 1;
    if ((rc = run_finalize(p, f, st))) return rc;
    return run_fallback_lists(p, Q, m, ldq, ix, o.nearest, out_idx, out_dist, w.bf, st);
}

// Pass 1 of the two-pass search splits each nearest list into this many row
// ranges (one work item each, about 128 rows or more), so that the few
// queries of a list are served by several wavefronts.
// 16-query blocks per stage-2 item: 2 only for the two-pass search on the
// 16x16 fp32 tile when the tuned choice says so (the item records exist on
// that path alone), else 4 (64-query items).
int stage2_qb(const BfPlan& p) {
    if (p.path != kPathMfma || !p.two_pass) return 4;
    const TileChoice tc = tile_choice(kTuneItems, p.ks, p.c);
    return (tc.shape == kShape16 && tc.qb == 2) ? 2 : 4;
}

int home_splits(const rbc_index* ix, const BfPlan& p) {
    // tuned choices belong to the fp32 matrix path; the vector path keeps the rule
    const TileChoice tc = p.path == kPathMfma ? tile_choice(kTuneItems, p.ks, p.c) : TileChoice();
    if (tc.splits > 0) return std::min(tc.splits, kMaxHomeSplit);
    // untuned: about 400 rows per range on the matrix path (two ranges for
    // lists of 1,000 rows measured fastest among 1 .. 8), 128 on the vector
    // path, whose rows cost more
    const int64_t per_list = ix->rows / std::max<int64_t>(ix->n_r, 1);
    const int64_t per_range = p.path == kPathMfma ? 400 : 128;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxHomeSplit, per_list / per_range));
}

void carve_search(const rbc_index* ix, const BfPlan& p, int64_t m, Carver& cv, SearchWork* w) {
    if (p.path == kPathExact) {
        carve_bf(p, m, ix->rows, cv, &w->bf);
        return;
    }
    const int64_t nr = ix->n_r;
    w->bf.fb_list = cv.take<int32_t>(m);
    w->bf.counters = cv.take<int32_t>(kCounters);
    if (p.repack_q) w->bf.Qp = cv.take<float>(m * p.ldp);
    if (p.path == kPathMfma || p.path == kPathLowp) w->bf.qn = cv.take<float>(m);
    if (p.path == kPathLowp) {
        w->bf.Qq = cv.take<uint8_t>(m * p.dq * (p.prec == RBC_BF16 ? 2 : 1));
        w->bf.qerr = cv.take<float>(m);
        if (p.prec == RBC_FP8_E4M3) w->bf.qscale = cv.take<uint8_t>(m);
        carve_cascade(p, m, ix->rows, false, cv, &w->bf);
    }
    w->bf.pval = cv.take<float>(m * nr * p.c);
    w->bf.pidx = cv.take<int32_t>(m * nr * p.c);
    w->DR = cv.take<float>(m * stage1_ld(nr));
    w->lrank = cv.take<int32_t>(m * nr);
    w->keep_rq = cv.take<uint8_t>(m * nr);
    w->npairs = cv.take<int32_t>(m);
    w->qoff = cv.take<int32_t>(m + 1);
    w->gcup = cv.take<float>(m);
    w->tau = cv.take<float>(m);
    w->roff = cv.take<int32_t>(nr + 1);
    w->ioff = cv.take<int32_t>(nr + 1);
    w->qlist = cv.take<int32_t>(m * nr);
    // stage-2 items hold 64 or 32 queries (matrix path), 256 (vector path)
    const int64_t max_items = m * nr / 32 + nr + 1;
    w->irep = cv.take<int32_t>(max_items);
    if (p.lowp_seed) w->qn32 = cv.take<float>(m);
    if (p.two_pass || p.lowp_seed) {
        w->home = cv.take<int32_t>(m);
        w->qa = cv.take<int32_t>(m);
        w->roffa = cv.take<int32_t>(nr + 1);
        w->ioffa = cv.take<int32_t>(nr + 1);
        // pass-1 items hold 16 queries (matrix path) or 256 (vector path)
        w->irepa = cv.take<int32_t>((m / 16 + nr + 1) * kMaxHomeSplit);
        w->csa = cv.take<int32_t>(nr);  // grouping cursors
        w->hval = cv.take<float>(m * kMaxHomeSplit * p.c);
        w->hidx = cv.take<int32_t>(m * kMaxHomeSplit * p.c);
        w->taud = cv.take<float>(m);
        if (p.two_pass) w->tauc = cv.take<float>(m);
        w->irows = cv.take<int32_t>(2 * max_items);
        if (p.path == kPathMfma) {
            w->rec = cv.take<int32_t>(kItemRec * max_items);
            w->srec = cv.take<int32_t>(kItemRec * max_items);
        }
    }
}

int search_plan(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k,
                const rbc_search_opts* opts, BfPlan* p) {
    if (opts && opts->precision != RBC_FP32) {
        const int pr = opts->precision;
        if (ix->mode != RBC_EXACT || pr < 0 || pr > 2 || ix->quant[pr].X == nullptr)
            return set_err(RBC_EUNSUPPORTED,
                           "rbc_search precision %d needs an exact index built with it", pr);
    }
    if (ix->mode == RBC_ONESHOT && k > ix->s)
        return set_err(RBC_EINVAL, "one-shot search needs k <= s (%lld)", (long long)ix->s);
    if (ix->mode == RBC_ONESHOT && opts && (opts->prune_eps != 0.0f || opts->flags != 0))
        return set_err(RBC_EINVAL, "prune_eps and flags apply to exact indexes");
    if (ix->mode == RBC_EXACT && (int64_t)m * ix->n_r >= ((int64_t)1 << 31))
        return set_err(RBC_EUNSUPPORTED, "m * n_r >= 2^31: split the query batch");
    int rc = make_bf_plan(m > 0 ? m : 1, ix->rows, ix->d, ldq, ix->ld, ix->metric, k, opts, p);
    if (rc) return rc;
    if (p->path == kPathLowp) {  // the index rows are zero-padded to float4 runs
        p->casc = true;
        p->ldc = ((int64_t)ix->d + 3) / 4 * 4;
    }
    p->two_pass = ix->mode == RBC_EXACT && (p->path == kPathMfma || p->path == kPathValu) &&
                  p->prune_eps == 0.0 && !p->one_pass;
    // low precision (one pass): the fp32 matrix tile scans each query's
    // nearest list first; rows of Q as whole float4 runs
    p->lowp_seed = ix->mode == RBC_EXACT && p->path == kPathLowp && ix->metric == RBC_L2 &&
                   (ix->d % 4) == 0 && (ldq % 4) == 0;
    return RBC_OK;
}

int validate_search(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k) {
    if (!ix) return set_err(RBC_EINVAL, "index is NULL");
    int rc = validate_common(m, ix->n, ix->d, k, ix->metric);
    if (rc) return rc;
    if (ldq < ix->d) return set_err(RBC_EINVAL, "ldq smaller than d");
    return RBC_OK;
}

// Stage 2 and finalize of the exact search on the quantised index rows.
int search_exact_lowp(const rbc_index* ix, const BfPlan& p, const float* Q, int64_t m,
                      int64_t ldq, int64_t* out_idx, float* out_dist, SearchWork& w,
                      int64_t* stats, hipStream_t st) {
    const rbc_index::Quant& qc = ix->quant[p.prec];
    const int32_t nr = (int32_t)ix->n_r;
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = (const float*)w.bf.Qq;
    a.ldq = p.dq;
    a.m = (int32_t)m;
    a.X = (const float*)qc.X;
    a.ldx = qc.dq;
    a.n = (int32_t)ix->rows;
    a.d = ix->d;
    a.xn = qc.xn;
    a.qscale = w.bf.qscale;
    a.xscale = qc.scale;
    a.item_total = w.ioff + nr;
    a.item_queue = w.bf.counters + 2;
    a.irep = w.irep;
    a.ioff = w.ioff;
    a.roff = w.roff;
    a.qlist = w.qlist;
    a.list_off = ix->list_off;
    a.lrank = w.lrank;
    a.qoff = w.qoff;
    a.tau = w.tau;
    a.n_r = nr;
    a.pval = w.bf.pval;
    a.pidx = w.bf.pidx;
    a.stats = stats;
    int rc;
    {
        KernelTimer kt("tile_items", st);
        if ((rc = check(launch_tile_lowp(p.prec == RBC_BF16 ? 0 : 1, p.kb, p.c, kTileItems,
                                         dim3(kItemBlocks), a, st), "stage 2 (low precision)")))
            return rc;
    }
    FinArgs f = fin_args(p, Q, m, ldq, ix->Xp, ix->ld, qc.stat, ix->ids, out_idx, out_dist, w.bf,
                         stats);
    f.qoff = w.qoff;
    f.npairs = w.npairs;
    f.qerr = w.bf.qerr;
    f.xerr_max_bits = qc.stat + 1;
    f.flags_q = nullptr;
    f.flags_x = nullptr;
    if (p.casc) f.fail_stat = RBC_STAT_CASCADE;
    if ((rc = run_finalize(p, f, st))) return rc;
    if (p.casc && (rc = run_cascade(p, Q, m, ldq, ix->Xp, ix->rows, ix->ld, ix->xn,
                                    ix->norms_max, ix->ids, out_idx, out_dist, w.bf, stats, st)))
        return rc;
    return run_fallback(p, Q, m, ldq, ix->Xp, ix->rows, ix->ld, ix->ids, out_idx, out_dist, w.bf,
                        st);
}

// Pass 1 of the two-pass exact search: every query searches the list of its
// nearest representative in full (queries grouped by that representative, one
// persistent launch, one shortlist per query), and the k-th value of that
// shortlist becomes taud[q], an upper bound on the distance of q's k-th
// nearest point (k points of X lie within it).
int search_pass1(const rbc_index* ix, const BfPlan& p, const float* Qk, int64_t ldqk, int64_t m,
                 int32_t k, SearchWork& w, double delta, int64_t ldd, hipStream_t st,
                 const float* qn = nullptr, float* tauc = nullptr) {
    const int32_t nr = (int32_t)ix->n_r;
    // items of 16 queries on the matrix path (tile_l2_mfma_home), 256 on the
    // vector path
    const int32_t isize = p.path == kPathValu ? kTileQ : 16;
    KernelTimer kt("pass1", st);
    int rc;
    if ((rc = check(launch_nearest_rep(w.DR, ldd, (int32_t)m, nr, w.home, st), "nearest rep")))
        return rc;
    // queries grouped by nearest representative; the order inside a group
    // changes which queries share a pass-1 item, never a query's bound
    if ((rc = check(launch_group(w.home, m, nr, w.csa, w.qa, w.roffa, st), "group by home")))
        return rc;
    const int ns = home_splits(ix, p);
    if ((rc = check(launch_items_from_offsets(w.roffa, nr, isize, w.ioffa, st, ns),
                    "pass-1 items")))
        return rc;
    if ((rc = check(launch_item_reps(w.ioffa, nr, w.irepa, st), "pass-1 item reps"))) return rc;
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = Qk;
    a.ldq = ldqk;
    a.m = (int32_t)m;
    a.X = ix->Xp;
    a.ldx = ix->ld;
    a.n = (int32_t)ix->rows;
    a.d = ix->d;
    a.xn = ix->xn;
    a.item_total = w.ioffa + nr;
    a.item_queue = w.bf.counters + 3;
    a.irep = w.irepa;
    a.ioff = w.ioffa;
    a.roff = w.roffa;
    a.qlist = w.qa;
    a.list_off = ix->list_off;
    a.n_r = nr;
    a.pval = w.hval;
    a.pidx = w.hidx;
    a.isplit = ns;
    const dim3 grid(kItemBlocks);
    rc = p.path == kPathMfma
             ? check(launch_tile_mfma(p.ks, p.c, kTileHome, grid, a, st), "pass 1 (mfma)")
             : check(launch_tile_valu(p.metric, p.ks, p.c, kTileHome, grid, a, st),
                     "pass 1 (valu)");
    if (rc) return rc;
    const int mode = p.path == kPathMfma ? 0 : (ix->metric == RBC_L2 ? 1 : 2);
    if ((rc = check(launch_tau_home(w.hval, p.c, ns, k, (int32_t)m, mode, qn ? qn : w.bf.qn,
                                    ix->norms_max, ix->d, delta, w.taud, st),
                    "k-th neighbour bound")))
        return rc;
    // the same shortlists bound the c-th neighbour distance too (c rows lie
    // within their c-th value): the stage-2 shortlists start from it
    if (tauc && (rc = check(launch_tau_home(w.hval, p.c, ns, p.c, (int32_t)m, mode,
                                            qn ? qn : w.bf.qn, ix->norms_max, ix->d, delta,
                                            tauc, st), "c-th neighbour bound")))
        return rc;
    return RBC_OK;
}

// Exact search, Sec. 5.2: stage 1 (all representative distances), [pass 1
// over the nearest lists], pruning, work list, grouped persistent stage-2
// tile, finalize, fallback.
int search_exact(const rbc_index* ix, const BfPlan& p, const float* Q, int64_t m, int64_t ldq,
                 int32_t k, int64_t* out_idx, float* out_dist, SearchWork& w, int64_t* stats,
                 hipStream_t st) {
    const int32_t nr = (int32_t)ix->n_r;
    const double delta = 2.0 * (ix->d + 2) * 5.9604644775390625e-8;
    const int64_t ldd = stage1_ld(nr);
    int rc;
    const float* Qk = Q;
    int64_t ldqk = ldq;
    if (p.repack_q) {
        if ((rc = check(launch_repack(Q, m, ldq, p.d, w.bf.Qp, p.ldp, st), "repack Q"))) return rc;
        Qk = w.bf.Qp;
        ldqk = p.ldp;
    }
    if ((rc = check(launch_fill_i32(w.bf.counters, kCounters, 0, st), "clear counters"))) return rc;
    {
        KernelTimer kt("stage1", st);
        if ((rc = check(launch_dist_all(ix->metric, Q, ldq, (int32_t)m, ix->R, ix->ld, nr, ix->d,
                                        w.DR, ldd, st), "stage 1")))
            return rc;
    }
    if (p.path == kPathMfma &&
        (rc = check(launch_row_norms(Qk, m, ldqk, p.d, nullptr, w.bf.qn, nullptr, st,
                                     (uint32_t*)w.bf.counters + 5), "norms Q")))
        return rc;
    if (p.two_pass &&
        (rc = search_pass1(ix, p, Qk, ldqk, m, k, w, delta, ldd, st, nullptr, w.tauc)))
        return rc;
    {
        KernelTimer kt("prune", st);
        if ((rc = check(launch_prune(w.DR, ldd, (int32_t)m, nr, k, p.c, delta, ix->psi,
                                     ix->list_off, w.lrank, w.npairs, w.gcup, stats, st,
                                     1.0 / (1.0 + p.prune_eps), p.two_pass ? w.taud : nullptr),
                        "prune")))
            return rc;
        if ((rc = check(launch_keep_transpose(w.lrank, (int32_t)m, nr, w.keep_rq, st), "keep")))
            return rc;
        // stage-2 shortlists start from the smaller of gamma_c and the pass-1
        // bound on the c-th neighbour distance
        if (p.two_pass && (rc = check(launch_min_f32(w.gcup, w.tauc, m, st), "seed bound")))
            return rc;
    }
    if (p.lowp_seed) {
        // low precision: an fp32 matrix-tile pass over each query's nearest
        // list bounds the distance of its c-th nearest point (c rows lie
        // within it); the smaller of that and gamma_c seeds the stage-2
        // shortlists, so far fewer values are inserted into them
        BfPlan p1 = p;
        p1.path = kPathMfma;
        if ((rc = check(launch_row_norms(Q, m, ldq, ix->d, nullptr, w.qn32, nullptr, st),
                        "norms Q (fp32)")))
            return rc;
        if ((rc = search_pass1(ix, p1, Q, ldq, m, p.c, w, delta, ldd, st, w.qn32))) return rc;
        if ((rc = check(launch_min_f32(w.gcup, w.taud, m, st), "seed bound"))) return rc;
    }
    {
        KernelTimer kt("worklist", st);
        if ((rc = check(hipMemcpyAsync(w.qoff, w.npairs, m * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, st), "copy counts")))
            return rc;
        if ((rc = check(launch_scan_total(w.qoff, m, st), "pair offsets"))) return rc;
        const int32_t isize = p.path == kPathValu ? kTileQ : 16 * stage2_qb(p);
        if ((rc = check(launch_worklist(w.keep_rq, (int32_t)m, nr, isize, w.roff, w.ioff, w.qlist,
                                        st), "work list")))
            return rc;
        // two-pass: the queries of each list in order of rho(q, r), so the
        // row runs of one item's queries overlap
        if (p.two_pass &&
            (rc = check(launch_seg_sort(w.roff, nr, w.qlist, w.DR, ldd, nullptr, st),
                        "order queries")))
            return rc;
        if ((rc = check(launch_item_reps(w.ioff, nr, w.irep, st), "item reps"))) return rc;
        if (p.two_pass &&
            (rc = check(launch_item_rows(w.ioff + nr, w.irep, w.ioff, w.roff, w.qlist, isize,
                                         ix->list_off, ix->lsorted, ix->own, w.DR, ldd, w.taud,
                                         0.0, 2.0 * delta, w.irows, st, w.rec),
                        "item rows")))
            return rc;
        // longest items first, so the persistent launch ends without a tail
        if (w.rec && (rc = check(launch_item_order(w.ioff + nr, w.rec, w.srec, st),
                                 "item order")))
            return rc;
        if (p.path == kPathLowp) {
            const rbc_index::Quant& qc = ix->quant[p.prec];
            uint32_t* ctr = (uint32_t*)w.bf.counters;
            if ((rc = check(launch_quantize(p.prec == RBC_BF16 ? 0 : 1, Q, m, ldq, p.d, -2.0f,
                                            w.bf.Qq, p.dq, p.dq, w.bf.qn, w.bf.qerr, w.bf.qscale,
                                            ctr + 14, st), "quantize Q")))
                return rc;
            if ((rc = check(launch_tau(w.gcup, w.bf.qn, qc.stat, nullptr, nullptr, (int32_t)m,
                                       ix->d, 3, delta, w.tau, st, w.bf.qerr, qc.stat + 1),
                            "thresholds")))
                return rc;
        }
        const int mode = p.path == kPathMfma ? 0 : (ix->metric == RBC_L2 ? 1 : 2);
        if (p.path != kPathLowp &&
            (rc = check(launch_tau(w.gcup, w.bf.qn, ix->norms_max,
                                   (const uint32_t*)w.bf.counters + 5, ix->norms_max + 1,
                                   (int32_t)m, ix->d, mode, delta, w.tau, st), "thresholds")))
            return rc;
    }
    if (p.path == kPathLowp) return search_exact_lowp(ix, p, Q, m, ldq, out_idx, out_dist, w, stats, st);
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = Qk;
    a.ldq = ldqk;
    a.m = (int32_t)m;
    a.X = ix->Xp;
    a.ldx = ix->ld;
    a.n = (int32_t)ix->rows;
    a.d = ix->d;
    a.xn = ix->xn;
    a.item_total = w.ioff + nr;
    a.item_queue = w.bf.counters + 2;
    a.irep = w.irep;
    a.ioff = w.ioff;
    a.roff = w.roff;
    a.qlist = w.qlist;
    a.list_off = ix->list_off;
    a.lrank = w.lrank;
    a.qoff = w.qoff;
    a.tau = w.tau;
    a.n_r = nr;
    a.pval = w.bf.pval;
    a.pidx = w.bf.pidx;
    a.stats = stats;
    a.irows = p.two_pass ? w.irows : nullptr;
    a.irec = w.srec;
    const TileChoice tc = p.path == kPathMfma ? tile_choice(kTuneItems, p.ks, p.c) : TileChoice();
    a.shape = tc.shape;
    a.qb = stage2_qb(p);
    {
        KernelTimer kt("tile_items", st);
        const dim3 grid(tc.blocks);
        rc = p.path == kPathMfma
                 ? check(launch_tile_mfma(p.ks, p.c, kTileItems, grid, a, st), "stage 2 (mfma)")
                 : check(launch_tile_valu(p.metric, p.ks, p.c, kTileItems, grid, a, st),
                         "stage 2 (valu)");
        if (rc) return rc;
    }
    FinArgs f = fin_args(p, Qk, m, ldqk, ix->Xp, ix->ld, ix->norms_max, ix->ids, out_idx,
                         out_dist, w.bf, stats);
    f.qoff = w.qoff;
    f.npairs = w.npairs;
    if ((rc = run_finalize(p, f, st))) return rc;
    return run_fallback(p, Q, m, ldq, ix->Xp, ix->rows, ix->ld, ix->ids, out_idx, out_dist, w.bf,
                        st);
}

// ---------------------------------------------------------------- range search
// Scratch of one range call: stage 1, pruning and the work list as for the
// k-NN search, plus the per-query hit counters (and an overflow counter).
struct RangeWork {
    float* Qp = nullptr;
    int32_t* counters = nullptr;
    float* DR = nullptr;
    int32_t* lrank = nullptr;
    uint8_t* keep_rq = nullptr;
    int32_t* npairs = nullptr;
    int32_t* roff = nullptr;
    int32_t* ioff = nullptr;
    int32_t* qlist = nullptr;
    int32_t* irep = nullptr;
    int32_t* irows = nullptr;  // 2 per item: the run of its list within the radius
    int32_t* cnt = nullptr;    // m + 1
};

struct RangePlan {
    int ks;
    bool repack;
    int64_t ldp;
};

int range_plan(const rbc_index* ix, int64_t m, int64_t ldq, RangePlan* rp) {
    if (!ix) return set_err(RBC_EINVAL, "index is NULL");
    if (m < 0) return set_err(RBC_EINVAL, "m < 0");
    if (ldq < ix->d) return set_err(RBC_EINVAL, "ldq smaller than d");
    if (ix->mode != RBC_EXACT) return set_err(RBC_EUNSUPPORTED, "range search needs an exact index");
    rp->ks = (ix->d + 15) / 16;
    if (rp->ks > kMaxKS) return set_err(RBC_EUNSUPPORTED, "range search supports d <= 128");
    if ((int64_t)m * ix->n_r >= ((int64_t)1 << 31))
        return set_err(RBC_EUNSUPPORTED, "m * n_r >= 2^31: split the query batch");
    rp->ldp = ((int64_t)ix->d + 3) / 4 * 4;
    rp->repack = (ix->d % 4) != 0 || (ldq % 4) != 0;
    return RBC_OK;
}

void carve_range(const rbc_index* ix, const RangePlan& rp, int64_t m, Carver& cv, RangeWork* w) {
    const int64_t nr = ix->n_r;
    if (rp.repack) w->Qp = cv.take<float>(m * rp.ldp);
    w->counters = cv.take<int32_t>(kCounters);
    w->DR = cv.take<float>(m * stage1_ld(nr));
    w->lrank = cv.take<int32_t>(m * nr);
    w->keep_rq = cv.take<uint8_t>(m * nr);
    w->npairs = cv.take<int32_t>(m);
    w->roff = cv.take<int32_t>(nr + 1);
    w->ioff = cv.take<int32_t>(nr + 1);
    w->qlist = cv.take<int32_t>(m * nr);
    w->irep = cv.take<int32_t>(m * nr / kTileQ + nr + 1);
    w->irows = cv.take<int32_t>(2 * (m * nr / kTileQ + nr + 1));
    w->cnt = cv.take<int32_t>(m + 1);
}

int range_args(const rbc_index* ix, const RangePlan& rp, const float* Q, int64_t m, int64_t ldq,
               double radius, void* workspace, size_t ws_bytes, RangeWork* w) {
    if (!std::isfinite(radius) || radius < 0.0)
        return set_err(RBC_EINVAL, "radius must be finite and >= 0");
    if (m > 0 && !Q) return set_err(RBC_EINVAL, "Q is NULL");
    if ((uintptr_t)Q & 15) return set_err(RBC_EINVAL, "Q must be 16-byte aligned");
    Carver cv((char*)workspace);
    carve_range(ix, rp, m, cv, w);
    if (!workspace || ws_bytes < cv.size())
        return set_err(RBC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed",
                       ws_bytes, cv.size());
    return RBC_OK;
}

// Stage 1, pruning for the radius, work list, then one pass of the range tile
// (fill = 0: count into w.cnt; fill = 1: write at offsets).
int range_pass(const rbc_index* ix, const RangePlan& rp, const float* Q, int64_t m, int64_t ldq,
               double radius, int fill, const int64_t* offsets, int64_t* out_idx,
               float* out_dist, RangeWork& w, hipStream_t st) {
    const int32_t nr = (int32_t)ix->n_r;
    const double delta = 2.0 * (ix->d + 2) * 5.9604644775390625e-8;
    const int64_t ldd = stage1_ld(nr);
    int rc;
    const float* Qk = Q;
    int64_t ldqk = ldq;
    if (rp.repack) {
        if ((rc = check(launch_repack(Q, m, ldq, ix->d, w.Qp, rp.ldp, st), "repack Q"))) return rc;
        Qk = w.Qp;
        ldqk = rp.ldp;
    }
    if ((rc = check(launch_fill_i32(w.counters, kCounters, 0, st), "clear counters"))) return rc;
    if ((rc = check(launch_fill_i32(w.cnt, m + 1, 0, st), "clear hit counts"))) return rc;
    {
        KernelTimer kt("stage1", st);
        if ((rc = check(launch_dist_all(ix->metric, Q, ldq, (int32_t)m, ix->R, ix->ld, nr, ix->d,
                                        w.DR, ldd, st), "stage 1")))
            return rc;
    }
    {
        KernelTimer kt("prune", st);
        if ((rc = check(launch_prune_range(w.DR, ldd, (int32_t)m, nr, delta, ix->psi, radius,
                                           w.lrank, w.npairs, nullptr, st), "range prune")))
            return rc;
        if ((rc = check(launch_keep_transpose(w.lrank, (int32_t)m, nr, w.keep_rq, st), "keep")))
            return rc;
    }
    {
        KernelTimer kt("worklist", st);
        if ((rc = check(launch_worklist(w.keep_rq, (int32_t)m, nr, kTileQ, w.roff, w.ioff,
                                        w.qlist, st), "work list")))
            return rc;
        // queries of a list in order of rho(q, r); each item then scans the run
        // of its list (sorted by the distance to r) where abs(rho(x, r) -
        // rho(q, r)) <= radius for one of its queries (triangle inequality)
        if ((rc = check(launch_seg_sort(w.roff, nr, w.qlist, w.DR, ldd, nullptr, st),
                        "order queries")))
            return rc;
        if ((rc = check(launch_item_reps(w.ioff, nr, w.irep, st), "item reps"))) return rc;
        if ((rc = check(launch_item_rows(w.ioff + nr, w.irep, w.ioff, w.roff, w.qlist, kTileQ,
                                         ix->list_off, ix->lsorted, ix->own, w.DR, ldd, nullptr,
                                         radius, 2.0 * delta, w.irows, st), "item rows")))
            return rc;
    }
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = Qk;
    a.ldq = ldqk;
    a.m = (int32_t)m;
    a.X = ix->Xp;
    a.ldx = ix->ld;
    a.n = (int32_t)ix->rows;
    a.d = ix->d;
    a.item_total = w.ioff + nr;
    a.item_queue = w.counters + 2;
    a.irep = w.irep;
    a.ioff = w.ioff;
    a.roff = w.roff;
    a.qlist = w.qlist;
    a.list_off = ix->list_off;
    a.n_r = nr;
    a.irows = w.irows;
    a.range_fill = fill;
    a.range_radius = radius;
    a.range_cnt = w.cnt;
    a.range_off = offsets;
    a.range_idx = out_idx;
    a.range_dist = out_dist;
    a.ids = ix->ids;
    KernelTimer kt("range_tile", st);
    return check(launch_tile_valu(ix->metric, rp.ks, 0, kTileRange, dim3(kItemBlocks), a, st),
                 "range tile");
}

}  // namespace

extern "C" {

int rbc_build(const float* X, int64_t n, int64_t ldx, int32_t d, const rbc_build_params* prm,
              void* hip_stream, rbc_index** out) {
    try {
        if (!out) return set_err(RBC_EINVAL, "out is NULL");
        *out = nullptr;
        if (!prm) return set_err(RBC_EINVAL, "params is NULL");
        int rc = validate_common(1, n, d, 1, prm->metric);
        if (rc) return rc;
        if (!X) return set_err(RBC_EINVAL, "X is NULL");
        if (ldx < d) return set_err(RBC_EINVAL, "ldx smaller than d");
        if ((uintptr_t)X & 15) return set_err(RBC_EINVAL, "X must be 16-byte aligned");
        if (prm->mode != RBC_EXACT && prm->mode != RBC_ONESHOT)
            return set_err(RBC_EINVAL, "unknown mode %d", prm->mode);
        if (prm->n_r < 1 || prm->n_r > n)
            return set_err(RBC_EINVAL, "n_r must be in [1, n] (got %lld)", (long long)prm->n_r);
        if (prm->n_r > kMaxReps)
            return set_err(RBC_EUNSUPPORTED, "n_r > %d", kMaxReps);
        if (prm->mode == RBC_ONESHOT && (prm->s < 1 || prm->s > n))
            return set_err(RBC_EINVAL, "s must be in [1, n]");
        std::vector<int64_t> reps;
        if (prm->rep_idx) {
            reps.assign(prm->rep_idx, prm->rep_idx + prm->n_r);
            std::sort(reps.begin(), reps.end());
            for (int64_t i = 0; i < prm->n_r; ++i) {
                if (reps[i] < 0 || reps[i] >= n)
                    return set_err(RBC_EINVAL, "representative id %lld out of range",
                                   (long long)reps[i]);
                if (i > 0 && reps[i] == reps[i - 1])
                    return set_err(RBC_EINVAL, "duplicate representative id %lld",
                                   (long long)reps[i]);
            }
        } else {
            reps = sample_reps(n, prm->n_r, prm->seed);
        }
        rbc_index* ix = new (std::nothrow) rbc_index();
        if (!ix) return set_err(RBC_ENOMEM, "host allocation failed");
        ix->mode = prm->mode;
        ix->metric = prm->metric;
        ix->d = d;
        ix->n = n;
        ix->n_r = prm->n_r;
        ix->s = prm->s;
        ix->ld = ((int64_t)d + 3) / 4 * 4;
        ix->rep_host = std::move(reps);
        rc = ix->mode == RBC_EXACT ? build_exact(ix, X, ldx, (hipStream_t)hip_stream)
                                   : build_oneshot(ix, X, ldx, (hipStream_t)hip_stream);
        if (!rc && prm->precisions) rc = build_quant(ix, prm->precisions, (hipStream_t)hip_stream);
        if (rc) {
            free_index(ix);
            return rc;
        }
        *out = ix;
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_search_workspace_size(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k,
                              const rbc_search_opts* opts, size_t* bytes) {
    try {
        if (!bytes) return set_err(RBC_EINVAL, "bytes is NULL");
        int rc = validate_search(ix, m, ldq, k);
        if (rc) return rc;
        BfPlan p;
        if ((rc = search_plan(ix, m, ldq, k, opts, &p))) return rc;
        Carver cv(nullptr);
        SearchWork w;
        if (ix->mode == RBC_ONESHOT) {
            OneShotSearchWork o;
            if ((rc = carve_oneshot(ix, p, m > 0 ? m : 1, ldq, cv, &w, &o))) return rc;
        } else {
            carve_search(ix, p, m, cv, &w);
        }
        *bytes = cv.size();
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_search(const rbc_index* ix, const float* Q, int64_t m, int64_t ldq, int32_t k,
               const rbc_search_opts* opts, int64_t* out_idx, float* out_dist, void* workspace,
               size_t ws_bytes, void* hip_stream) {
    try {
        int rc = validate_search(ix, m, ldq, k);
        if (rc) return rc;
        if (m == 0) return RBC_OK;
        if (!Q || !out_idx || !out_dist) return set_err(RBC_EINVAL, "NULL pointer");
        if ((uintptr_t)Q & 15) return set_err(RBC_EINVAL, "Q must be 16-byte aligned");
        BfPlan p;
        if ((rc = search_plan(ix, m, ldq, k, opts, &p))) return rc;
        Carver cv((char*)workspace);
        SearchWork w;
        OneShotSearchWork o;
        if (ix->mode == RBC_ONESHOT) {
            if ((rc = carve_oneshot(ix, p, m, ldq, cv, &w, &o))) return rc;
        } else {
            carve_search(ix, p, m, cv, &w);
        }
        if (!workspace || ws_bytes < cv.size())
            return set_err(RBC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed",
                           ws_bytes, cv.size());
        hipStream_t st = (hipStream_t)hip_stream;
        int64_t* stats = opts ? opts->dev_stats : nullptr;
        if (ix->mode == RBC_ONESHOT)
            return search_oneshot(ix, p, Q, m, ldq, out_idx, out_dist, w, o, stats, st);
        if (p.path == kPathExact)
            return run_bf(p, Q, m, ldq, ix->Xp, ix->rows, ix->ld, nullptr, nullptr, ix->ids,
                          out_idx, out_dist, w.bf, stats, st);
        return search_exact(ix, p, Q, m, ldq, k, out_idx, out_dist, w, stats, st);
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

}  // extern "C"

// Tuning key of an rbc_search call (rbc_tune.cpp): kind kTuneItems when the
// exact search runs its stage 2 on the fp32 matrix tile, -1 otherwise.
int search_tune_key(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k,
                    const rbc_search_opts* opts, int32_t* kind, int32_t* ks, int32_t* c) {
    int rc = validate_search(ix, m, ldq, k);
    if (rc) return rc;
    BfPlan p;
    if ((rc = search_plan(ix, m > 0 ? m : 1, ldq, k, opts, &p))) return rc;
    *kind = (ix->mode == RBC_EXACT && p.path == kPathMfma) ? kTuneItems : -1;
    *ks = p.ks;
    *c = p.c;
    return RBC_OK;
}

extern "C" {

int rbc_range_workspace_size(const rbc_index* ix, int64_t m, int64_t ldq, size_t* bytes) {
    try {
        if (!bytes) return set_err(RBC_EINVAL, "bytes is NULL");
        RangePlan rp;
        int rc = range_plan(ix, m, ldq, &rp);
        if (rc) return rc;
        Carver cv(nullptr);
        RangeWork w;
        carve_range(ix, rp, m, cv, &w);
        *bytes = cv.size();
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_range_count(const rbc_index* ix, const float* Q, int64_t m, int64_t ldq, double radius,
                    int64_t* offsets, void* workspace, size_t ws_bytes, void* hip_stream) {
    try {
        RangePlan rp;
        int rc = range_plan(ix, m, ldq, &rp);
        if (rc) return rc;
        if (!offsets) return set_err(RBC_EINVAL, "offsets is NULL");
        RangeWork w;
        if ((rc = range_args(ix, rp, Q, m, ldq, radius, workspace, ws_bytes, &w))) return rc;
        hipStream_t st = (hipStream_t)hip_stream;
        if (m > 0 && (rc = range_pass(ix, rp, Q, m, ldq, radius, 0, nullptr, nullptr, nullptr, w,
                                      st)))
            return rc;
        return check(launch_offsets64(w.cnt, m, offsets, st), "range offsets");
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_range_search(const rbc_index* ix, const float* Q, int64_t m, int64_t ldq, double radius,
                     const int64_t* offsets, int64_t* out_idx, float* out_dist, void* workspace,
                     size_t ws_bytes, void* hip_stream) {
    try {
        RangePlan rp;
        int rc = range_plan(ix, m, ldq, &rp);
        if (rc) return rc;
        if (m == 0) return RBC_OK;
        if (!offsets || !out_idx || !out_dist) return set_err(RBC_EINVAL, "NULL pointer");
        RangeWork w;
        if ((rc = range_args(ix, rp, Q, m, ldq, radius, workspace, ws_bytes, &w))) return rc;
        hipStream_t st = (hipStream_t)hip_stream;
        if ((rc = range_pass(ix, rp, Q, m, ldq, radius, 1, offsets, out_idx, out_dist, w, st)))
            return rc;
        {
            KernelTimer kt("range_sort", st);
            if ((rc = check(launch_seg_sort_pairs(offsets, m, out_idx, out_dist, w.cnt, w.cnt + m,
                                                  st), "range sort")))
                return rc;
        }
        int32_t over = 0;
        if ((rc = check(hipMemcpyAsync(&over, w.cnt + m, sizeof(int32_t), hipMemcpyDeviceToHost,
                                       st), "read overflow")))
            return rc;
        if ((rc = check(hipStreamSynchronize(st), "range search"))) return rc;
        if (over)
            return set_err(RBC_EINVAL, "%d points or segments do not match the offsets (offsets "
                           "from another index, query set or radius)", over);
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_index_info(const rbc_index* ix, int64_t* n, int32_t* d, int64_t* n_r, int32_t* mode,
                   int32_t* metric, size_t* device_bytes) {
    if (!ix) return set_err(RBC_EINVAL, "index is NULL");
    if (n) *n = ix->n;
    if (d) *d = ix->d;
    if (n_r) *n_r = ix->n_r;
    if (mode) *mode = ix->mode;
    if (metric) *metric = ix->metric;
    if (device_bytes) *device_bytes = ix->bytes;
    return RBC_OK;
}

int rbc_index_export(const rbc_index* ix, int64_t* rep_idx, double* psi, int64_t* list_off,
                     int64_t* list_ids) {
    try {
        if (!ix) return set_err(RBC_EINVAL, "index is NULL");
        int rc;
        if ((rc = check(hipDeviceSynchronize(), "sync"))) return rc;
        if (rep_idx) std::copy(ix->rep_host.begin(), ix->rep_host.end(), rep_idx);
        if (psi &&
            (rc = check(hipMemcpy(psi, ix->psi, ix->n_r * sizeof(double), hipMemcpyDeviceToHost),
                        "copy psi")))
            return rc;
        if (list_off) {
            std::vector<int32_t> off(ix->n_r + 1);
            if ((rc = check(hipMemcpy(off.data(), ix->list_off, off.size() * sizeof(int32_t),
                                      hipMemcpyDeviceToHost), "copy offsets")))
                return rc;
            std::copy(off.begin(), off.end(), list_off);
        }
        if (list_ids &&
            (rc = check(hipMemcpy(list_ids, ix->ids, ix->rows * sizeof(int64_t),
                                  hipMemcpyDeviceToHost), "copy ids")))
            return rc;
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_index_export_order(const rbc_index* ix, float* own, int32_t* sorted) {
    try {
        if (!ix) return set_err(RBC_EINVAL, "index is NULL");
        if (ix->mode != RBC_EXACT) return set_err(RBC_EUNSUPPORTED, "exact-mode indexes only");
        int rc;
        if ((rc = check(hipDeviceSynchronize(), "sync"))) return rc;
        if (own && (rc = check(hipMemcpy(own, ix->own, ix->rows * sizeof(float),
                                         hipMemcpyDeviceToHost), "copy distances")))
            return rc;
        if (sorted && (rc = check(hipMemcpy(sorted, ix->lsorted, ix->n_r * sizeof(int32_t),
                                            hipMemcpyDeviceToHost), "copy flags")))
            return rc;
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

void rbc_free(rbc_index* ix) { free_index(ix); }

}  // extern "C"
