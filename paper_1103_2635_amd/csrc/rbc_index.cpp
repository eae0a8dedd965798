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
#include <cstring>
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
    uint32_t* norms_max = nullptr;  // [0] max row norm of Xp (float bits)
    std::vector<int64_t> rep_host;
    std::vector<void*> allocs;
    size_t bytes = 0;
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

void free_index(rbc_index* ix) {
    if (!ix) return;
    (void)hipDeviceSynchronize();
    for (void* p : ix->allocs) (void)hipFree(p);
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

int build_exact(rbc_index* ix, const float* X, int64_t ldx, hipStream_t st) {
    const int64_t n = ix->n, n_r = ix->n_r, ld = ix->ld;
    const int32_t d = ix->d;
    int rc;
    if ((rc = dev_alloc(ix, &ix->R, n_r * ld))) return rc;
    if ((rc = dev_alloc(ix, &ix->psi, n_r))) return rc;
    if ((rc = dev_alloc(ix, &ix->list_off, n_r + 1))) return rc;
    if ((rc = dev_alloc(ix, &ix->Xp, n * ld))) return rc;
    if ((rc = dev_alloc(ix, &ix->xn, n))) return rc;
    if ((rc = dev_alloc(ix, &ix->ids, n))) return rc;
    if ((rc = dev_alloc(ix, &ix->norms_max, 4))) return rc;
    ix->rows = n;

    Scratch s;
    int32_t *reps = nullptr, *owner = nullptr, *perm = nullptr, *cnt = nullptr;
    int64_t* own64 = nullptr;
    float* ownd = nullptr;
    if ((rc = s.take(&reps, n_r)) || (rc = s.take(&owner, n)) || (rc = s.take(&perm, n)) ||
        (rc = s.take(&cnt, n_r * csort_blocks(n))) || (rc = s.take(&own64, n)) ||
        (rc = s.take(&ownd, n)))
        return rc;
    std::vector<int32_t> reps32(ix->rep_host.begin(), ix->rep_host.end());
    if ((rc = check(hipMemcpyAsync(reps, reps32.data(), n_r * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st), "copy representatives")))
        return rc;
    if ((rc = check(launch_gather_rows(X, ldx, d, reps, n_r, ix->R, ld, nullptr, st), "gather R")))
        return rc;

    // ownership: BF(X, R) with k = 1 (ties to the lower representative position)
    BfPlan p;
    if ((rc = make_bf_plan(n, n_r, d, ldx, ld, ix->metric, 1, nullptr, &p))) return rc;
    Carver probe(nullptr);
    BfWork w;
    carve_bf(p, n, n_r, probe, &w);
    char* ws = nullptr;
    if ((rc = s.take(&ws, (int64_t)probe.size()))) return rc;
    Carver cv(ws);
    carve_bf(p, n, n_r, cv, &w);
    if ((rc = run_bf(p, X, n, ldx, ix->R, n_r, ld, nullptr, nullptr, nullptr, own64, ownd, w,
                     nullptr, st)))
        return rc;
    if ((rc = check(launch_narrow(own64, n, owner, st), "owners"))) return rc;

    // lists: stable counting sort of the points by owner
    if ((rc = check(launch_csort(owner, n, (int32_t)n_r, cnt, perm, ix->list_off, st), "sort")))
        return rc;
    if ((rc = check(launch_gather_rows(X, ldx, d, perm, n, ix->Xp, ld, ix->ids, st), "gather Xp")))
        return rc;
    if ((rc = check(launch_fill_i32((int32_t*)ix->norms_max, 4, 0, st), "clear"))) return rc;
    if ((rc = check(launch_row_norms(ix->Xp, n, ld, d, nullptr, ix->xn, ix->norms_max, st),
                    "norms")))
        return rc;
    if ((rc = check(launch_fill_i32((int32_t*)ix->psi, 2 * n_r, 0, st), "clear psi"))) return rc;
    if ((rc = check(launch_psi(X, ldx, d, ix->metric, n, owner, ix->R, ld, ix->psi, st), "psi")))
        return rc;
    return check(hipStreamSynchronize(st), "build");
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
};

int64_t stage1_ld(int64_t nr) { return (nr + 3) / 4 * 4; }

void carve_search(const rbc_index* ix, const BfPlan& p, int64_t m, Carver& cv, SearchWork* w) {
    if (p.path == kPathExact) {
        carve_bf(p, m, ix->rows, cv, &w->bf);
        return;
    }
    const int64_t nr = ix->n_r;
    w->bf.fb_list = cv.take<int32_t>(m);
    w->bf.counters = cv.take<int32_t>(4);
    if (p.repack_q) w->bf.Qp = cv.take<float>(m * p.ldp);
    if (p.path == kPathMfma) w->bf.qn = cv.take<float>(m);
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
}

int search_plan(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k,
                const rbc_search_opts* opts, BfPlan* p) {
    if (ix->mode != RBC_EXACT) return set_err(RBC_EUNSUPPORTED, "one-shot search is not built yet");
    if ((int64_t)m * ix->n_r >= ((int64_t)1 << 31))
        return set_err(RBC_EUNSUPPORTED, "m * n_r >= 2^31: split the query batch");
    return make_bf_plan(m > 0 ? m : 1, ix->rows, ix->d, ldq, ix->ld, ix->metric, k, opts, p);
}

int validate_search(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k) {
    if (!ix) return set_err(RBC_EINVAL, "index is NULL");
    int rc = validate_common(m, ix->n, ix->d, k, ix->metric);
    if (rc) return rc;
    if (ldq < ix->d) return set_err(RBC_EINVAL, "ldq smaller than d");
    return RBC_OK;
}

// Exact search, Sec. 5.2: stage 1 (all representative distances), pruning,
// work list, grouped persistent stage-2 tile, finalize, fallback.
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
    if ((rc = check(launch_fill_i32(w.bf.counters, 4, 0, st), "clear counters"))) return rc;
    {
        KernelTimer kt("stage1", st);
        if ((rc = check(launch_dist_all(ix->metric, Q, ldq, (int32_t)m, ix->R, ix->ld, nr, ix->d,
                                        w.DR, ldd, st), "stage 1")))
            return rc;
    }
    {
        KernelTimer kt("prune", st);
        if ((rc = check(launch_prune(w.DR, ldd, (int32_t)m, nr, k, p.c, delta, ix->psi,
                                     ix->list_off, w.lrank, w.keep_rq, w.npairs, w.gcup, stats,
                                     st), "prune")))
            return rc;
    }
    {
        KernelTimer kt("worklist", st);
        if ((rc = check(hipMemcpyAsync(w.qoff, w.npairs, m * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, st), "copy counts")))
            return rc;
        if ((rc = check(launch_scan_total(w.qoff, m, st), "pair offsets"))) return rc;
        if ((rc = check(launch_worklist(w.keep_rq, (int32_t)m, nr, w.roff, w.ioff, w.qlist, st),
                        "work list")))
            return rc;
        if (p.path == kPathMfma &&
            (rc = check(launch_row_norms(Qk, m, ldqk, p.d, nullptr, w.bf.qn, nullptr, st),
                        "norms Q")))
            return rc;
        const int mode = p.path == kPathMfma ? 0 : (ix->metric == RBC_L2 ? 1 : 2);
        if ((rc = check(launch_tau(w.gcup, w.bf.qn, ix->norms_max, (int32_t)m, ix->d, mode, delta,
                                   w.tau, st), "thresholds")))
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
    a.xn = ix->xn;
    a.item_total = w.ioff + nr;
    a.item_queue = w.bf.counters + 2;
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
    {
        KernelTimer kt("tile_items", st);
        const dim3 grid(kItemBlocks);
        rc = p.path == kPathMfma
                 ? check(launch_tile_mfma(p.ks, p.c, true, grid, a, st), "stage 2 (mfma)")
                 : check(launch_tile_valu(p.metric, p.ks, p.c, true, grid, a, st),
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
        if (prm->mode == RBC_ONESHOT) {
            if (prm->s < 1 || prm->s > n) return set_err(RBC_EINVAL, "s must be in [1, n]");
            return set_err(RBC_EUNSUPPORTED, "one-shot build is not built yet");
        }
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
        rc = build_exact(ix, X, ldx, (hipStream_t)hip_stream);
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
        carve_search(ix, p, m, cv, &w);
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
        carve_search(ix, p, m, cv, &w);
        if (!workspace || ws_bytes < cv.size())
            return set_err(RBC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed",
                           ws_bytes, cv.size());
        hipStream_t st = (hipStream_t)hip_stream;
        int64_t* stats = opts ? opts->dev_stats : nullptr;
        if (p.path == kPathExact)
            return run_bf(p, Q, m, ldq, ix->Xp, ix->rows, ix->ld, nullptr, nullptr, ix->ids,
                          out_idx, out_dist, w.bf, stats, st);
        return search_exact(ix, p, Q, m, ldq, k, out_idx, out_dist, w, stats, st);
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

void rbc_free(rbc_index* ix) { free_index(ix); }

}  // extern "C"
