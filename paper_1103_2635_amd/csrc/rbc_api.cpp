// rbc_api.cpp -- the C ABI of librbc (declared in include/rbc.h): argument
// validation, plans (path, shortlist length, database splits), workspace
// carving and the launch sequence of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/rbc.h"
#include "rbc_common.h"
#include "rbc_host.h"
#include "rbc_kernels.h"

namespace rbc {

static thread_local char g_err[512] = "";

int set_err(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

const char* last_error() { return g_err; }

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return RBC_OK;
    return set_err(RBC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int shortlist_len(int k, int requested) {
    int want = k + 3;
    if (requested > want) want = requested;
    for (int c : {4, 8, 16, 32, 64})
        if (c >= want) return c;
    return 0;  // beyond the register shortlist: exhaustive float64 path
}

// ---------------------------------------------------------------- BF plan

int make_bf_plan(int64_t m, int64_t n, int32_t d, int64_t ldq, int64_t ldx, int32_t metric,
                 int32_t k, const rbc_search_opts* opts, BfPlan* p) {
    std::memset(p, 0, sizeof(*p));
    const int prec = opts ? opts->precision : RBC_FP32;
    if (prec != RBC_FP32 && prec != RBC_BF16 && prec != RBC_FP8_E4M3)
        return set_err(RBC_EINVAL, "unknown precision %d", prec);
    if (prec != RBC_FP32 && (metric != RBC_L2 || d > 128))
        return set_err(RBC_EUNSUPPORTED, "low precision needs the L2 metric and d <= 128");
    if (opts && ((opts->flags & ~RBC_FLAG_ONE_PASS) != 0 || opts->reserved != 0))
        return set_err(RBC_EINVAL, "opts->flags must be 0 or RBC_FLAG_ONE_PASS, opts->reserved 0");
    p->one_pass = opts && (opts->flags & RBC_FLAG_ONE_PASS);
    if (opts && !(opts->prune_eps >= 0.0f && opts->prune_eps < 1e30f))
        return set_err(RBC_EINVAL, "opts->prune_eps must be finite and >= 0");
    p->prune_eps = opts ? (double)opts->prune_eps : 0.0;
    p->metric = metric;
    p->k = k;
    p->d = d;
    p->ldp = ((int64_t)d + 3) / 4 * 4;
    p->repack_q = (d % 4) != 0 || (ldq % 4) != 0;
    p->repack_x = (d % 4) != 0 || (ldx % 4) != 0;
    p->prec = prec;
    // Default shortlist: fp32 the shortest with c >= k + 3; bf16 at least 8
    // (its ranking error is ~0.3 %, so a short list still certifies, and the
    // insert cost grows with c); fp8 32 (an error of several percent needs the
    // wider margin, or most queries go to the fp32 cascade).
    const int cdef = prec == RBC_FP8_E4M3 ? 32 : (prec == RBC_BF16 ? 8 : 0);
    p->c = shortlist_len(k, opts && opts->shortlist ? opts->shortlist : cdef);
    p->ks = (d + 15) / 16;
    if (p->c == 0 || p->ks > kMaxKS) {
        p->path = kPathExact;
        p->c = 0;
        p->ks = 0;
        p->repack_q = p->repack_x = false;
    } else if (prec != RBC_FP32) {
        p->path = kPathLowp;
        p->repack_q = p->repack_x = false;  // the quantiser reads any stride
        p->kb = prec == RBC_BF16 ? (d + 31) / 32 : 1;
        p->dq = prec == RBC_BF16 ? 32 * p->kb : 128;
        // the fp32 pass reads X in place: rows of whole float4 runs
        p->casc = (d % 4) == 0 && (ldx % 4) == 0;
        p->c32 = shortlist_len(k, 0);
        p->ks32 = (d + 15) / 16;
        p->ldc = ((int64_t)d + 3) / 4 * 4;
    } else if (metric == RBC_L2 && d >= 12) {
        p->path = kPathMfma;
        p->shape = tile_choice(kTuneBF, p->ks, p->c).shape;
    } else {
        p->path = kPathValu;
    }
    p->nqblk = (int32_t)((m + kTileQ - 1) / kTileQ);
    if (p->path != kPathExact) {
        int64_t s = opts && opts->splits > 0 ? opts->splits : (4 * kConcurrentBlocks) / p->nqblk;
        s = std::max<int64_t>(1, std::min<int64_t>(s, kMaxSplits));
        s = std::min<int64_t>(s, (n + 255) / 256);
        s = std::max<int64_t>(s, 1);
        int64_t rps = (n + s - 1) / s;
        rps = (rps + kRowsMfma - 1) / kRowsMfma * kRowsMfma;
        p->rps = (int32_t)rps;
        p->nsplit = (int32_t)((n + rps - 1) / rps);
    }
    if (p->path == kPathLowp) {
        const int64_t s = std::max<int64_t>(1, std::min<int64_t>(4 * kConcurrentBlocks / p->nqblk,
                                                                 kMaxSplits));
        p->casc_blocks = (int32_t)std::max<int64_t>(p->nqblk * s, 4 * kConcurrentBlocks);
    }
    return RBC_OK;
}

void carve_cascade(const BfPlan& p, int64_t m, int64_t n, bool xnorms, Carver& cv, BfWork* w) {
    if (p.path != kPathLowp || !p.casc) return;
    w->Qc = cv.take<float>(m * p.ldc);
    w->qnc = cv.take<float>(m);
    w->qmap = cv.take<int32_t>(m);
    if (xnorms) w->xn32 = cv.take<float>(n);
    w->pval_c = cv.take<float>((int64_t)p.casc_blocks * kTileQ * p.c32);
    w->pidx_c = cv.take<int32_t>((int64_t)p.casc_blocks * kTileQ * p.c32);
}

int run_cascade(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X,
                int64_t n, int64_t ldx, const float* xn, const uint32_t* xstat,
                const int64_t* id_map, int64_t* out_idx, float* out_dist, BfWork& w,
                int64_t* stats, hipStream_t st) {
    int32_t* ctr = w.counters;
    int rc;
    KernelTimer kt("cascade", st);
    if ((rc = hip_status(launch_cascade_gather(Q, ldq, p.d, m, w.fb_list, ctr, w.Qc, p.ldc, w.qnc,
                                               w.qmap, ctr + 1, st), "cascade gather")))
        return rc;
    if ((rc = hip_status(launch_fill_i32(ctr, 1, 0, st), "cascade reset"))) return rc;
    if (xn == nullptr) {
        if ((rc = hip_status(launch_row_norms(X, n, ldx, p.d, nullptr, w.xn32, (uint32_t*)ctr + 8,
                                              st, nullptr, ctr + 1), "cascade norms X")))
            return rc;
        xn = w.xn32;
        xstat = (const uint32_t*)ctr + 8;
    }
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = w.Qc;
    a.ldq = p.ldc;
    a.m = (int32_t)m;
    a.X = X;
    a.ldx = ldx;
    a.n = (int32_t)n;
    a.d = p.d;
    a.xn = xn;
    a.pval = w.pval_c;
    a.pidx = w.pidx_c;
    a.m_dev = ctr + 1;
    a.dev_blocks = p.casc_blocks;
    a.shape = tile_choice(kTuneBF, p.ks32, p.c32).shape;
    if ((rc = hip_status(launch_tile_mfma(p.ks32, p.c32, kTileBF, dim3(p.casc_blocks), a, st),
                         "cascade tile")))
        return rc;
    FinArgs f;
    std::memset(&f, 0, sizeof(f));
    f.Q = w.Qc;
    f.ldq = p.ldc;
    f.m = (int32_t)m;
    f.X = X;
    f.ldx = ldx;
    f.d = p.d;
    f.metric = RBC_L2;
    f.approx_mode = 0;
    f.pval = w.pval_c;
    f.pidx = w.pidx_c;
    f.k = p.k;
    f.qn = w.qnc;
    f.xmax_bits = xstat;
    f.id_map = id_map;
    f.out_idx = out_idx;
    f.out_dist = out_dist;
    f.fb_list = w.fb_list;
    f.fb_count = ctr;
    f.stats = stats;
    f.fail_stat = RBC_STAT_FALLBACK;
    f.m_dev = ctr + 1;
    f.dev_blocks = p.casc_blocks;
    f.n = (int32_t)n;
    f.qmap = w.qmap;
    return hip_status(launch_finalize(p.c32, f, st), "cascade finalize");
}

void carve_bf(const BfPlan& p, int64_t m, int64_t n, Carver& cv, BfWork* w) {
    w->fb_list = cv.take<int32_t>(m);
    w->counters = cv.take<int32_t>(kCounters);
    if (p.path == kPathExact) return;
    if (p.repack_q) w->Qp = cv.take<float>(m * p.ldp);
    if (p.repack_x) w->Xp = cv.take<float>(n * p.ldp);
    if (p.path == kPathMfma || p.path == kPathLowp) {
        w->qn = cv.take<float>(m);
        w->xn = cv.take<float>(n);
    }
    if (p.path == kPathLowp) {
        const int64_t esz = p.prec == RBC_BF16 ? 2 : 1;
        w->Qq = cv.take<uint8_t>(m * p.dq * esz);
        w->Xq = cv.take<uint8_t>(n * p.dq * esz);
        w->qerr = cv.take<float>(m);
        if (p.prec == RBC_FP8_E4M3) {
            w->qscale = cv.take<uint8_t>(m);
            w->xscale = cv.take<uint8_t>(n);
        }
    }
    w->pval = cv.take<float>((int64_t)p.nsplit * m * p.c);
    w->pidx = cv.take<int32_t>((int64_t)p.nsplit * m * p.c);
    carve_cascade(p, m, n, true, cv, w);
}

// BF(Q, X) with the contraction on quantised rows: quantise Q (times -2) and
// X, run the bf16 / fp8 tile, finalize (re-score from the fp32 rows; the
// certificate adds the quantisation errors), fallback.
int run_bf_lowp(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n,
                int64_t ldx, const int64_t* id_map, int64_t* out_idx, float* out_dist, BfWork& w,
                int64_t* stats, hipStream_t st, float* out_approx) {
    int rc;
    const int fmt = p.prec == RBC_BF16 ? 0 : 1;
    if ((rc = hip_status(launch_fill_i32(w.counters, kCounters, 0, st), "clear counters")))
        return rc;
    uint32_t* ctr = (uint32_t*)w.counters;
    {
        KernelTimer kt("quantize", st);
        if ((rc = hip_status(launch_quantize_norms(fmt, Q, m, ldq, p.d, -2.0f, w.Qq, p.dq, p.dq,
                                                   w.qn, w.qerr, w.qscale, ctr + 14, w.qn32,
                                                   w.qflags32, st), "quantize Q")))
            return rc;
        if ((rc = hip_status(launch_quantize(fmt, X, n, ldx, p.d, 1.0f, w.Xq, p.dq, p.dq, w.xn,
                                             nullptr, w.xscale, ctr + 12, st), "quantize X")))
            return rc;
    }
    // w.qn / w.xn now hold ||q~||^2 and ||x~||^2 of the quantised rows
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = (const float*)w.Qq;
    a.ldq = p.dq;
    a.m = (int32_t)m;
    a.X = (const float*)w.Xq;
    a.ldx = p.dq;
    a.n = (int32_t)n;
    a.d = p.d;
    a.xn = w.xn;
    a.rps = p.rps;
    a.nsplit = p.nsplit;
    a.qscale = w.qscale;
    a.xscale = w.xscale;
    a.pval = w.pval;
    a.pidx = w.pidx;
    a.stats = stats;
    {
        KernelTimer kt("tile", st);
        const dim3 grid(p.nqblk, p.nsplit);
        if ((rc = hip_status(launch_tile_lowp(fmt, p.kb, p.c, kTileBF, grid, a, st), "tile (low precision)")))
            return rc;
    }
    FinArgs f = fin_args(p, Q, m, ldq, X, ldx, ctr + 12, id_map, out_idx, out_dist, w, stats,
                         out_approx);
    f.nsplit = p.nsplit;
    f.qerr = w.qerr;
    f.xerr_max_bits = ctr + 13;
    f.flags_q = nullptr;
    f.flags_x = nullptr;
    if (p.casc) f.fail_stat = RBC_STAT_CASCADE;
    if ((rc = run_finalize(p, f, st))) return rc;
    if (p.casc && (rc = run_cascade(p, Q, m, ldq, X, n, ldx, nullptr, nullptr, id_map, out_idx,
                                    out_dist, w, stats, st)))
        return rc;
    return run_fallback(p, Q, m, ldq, X, n, ldx, id_map, out_idx, out_dist, w, st);
}

// The launch sequence of BF(Q, X) (bf_search and the RBC build): tile over
// the database rows, finalize, exhaustive fallback.  xn / xmax_bits may be
// given (precomputed norms of X), id_map maps rows of X to reported ids.
int run_bf(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n,
           int64_t ldx, const float* xn, const uint32_t* xstat, const int64_t* id_map,
           int64_t* out_idx, float* out_dist, BfWork& w, int64_t* stats, hipStream_t st,
           float* out_approx) {
    int32_t* fb_count = w.counters;
    int rc;
    if (p.path == kPathLowp)
        return run_bf_lowp(p, Q, m, ldq, X, n, ldx, id_map, out_idx, out_dist, w, stats, st,
                           out_approx);
    if (p.path == kPathExact) {
        if ((rc = hip_status(launch_iota_i32(w.fb_list, (int32_t)m, st), "iota"))) return rc;
        if ((rc = hip_status(launch_set_count(fb_count, (int32_t)m, st), "set_count"))) return rc;
        return run_fallback(p, Q, m, ldq, X, n, ldx, id_map, out_idx, out_dist, w, st);
    }
    const float* Qk = Q;
    int64_t ldqk = ldq;
    const float* Xk = X;
    int64_t ldxk = ldx;
    if (p.repack_q) {
        if ((rc = hip_status(launch_repack(Q, m, ldq, p.d, w.Qp, p.ldp, st), "repack Q"))) return rc;
        Qk = w.Qp;
        ldqk = p.ldp;
    }
    if (p.repack_x) {
        if ((rc = hip_status(launch_repack(X, n, ldx, p.d, w.Xp, p.ldp, st), "repack X"))) return rc;
        Xk = w.Xp;
        ldxk = p.ldp;
    }
    if ((rc = hip_status(launch_fill_i32(w.counters, kCounters, 0, st), "clear counters")))
        return rc;
    if (p.path == kPathMfma) {
        if ((rc = hip_status(launch_row_norms(Qk, m, ldqk, p.d, nullptr, w.qn, nullptr, st,
                                              (uint32_t*)w.counters + 5), "norms Q")))
            return rc;
        if (xn == nullptr) {
            uint32_t* xs = (uint32_t*)w.counters + 8;
            if ((rc = hip_status(launch_row_norms(Xk, n, ldxk, p.d, nullptr, w.xn, xs, st, xs + 1),
                                 "norms X")))
                return rc;
            xn = w.xn;
            xstat = xs;
        }
    }
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Q = Qk;
    a.ldq = ldqk;
    a.m = (int32_t)m;
    a.X = Xk;
    a.ldx = ldxk;
    a.n = (int32_t)n;
    a.d = p.d;
    a.xn = xn;
    a.rps = p.rps;
    a.nsplit = p.nsplit;
    a.pval = w.pval;
    a.pidx = w.pidx;
    a.stats = stats;
    a.shape = p.shape;
    {
        KernelTimer kt("tile", st);
        const dim3 grid(p.nqblk, p.nsplit);
        rc = p.path == kPathMfma
                 ? hip_status(launch_tile_mfma(p.ks, p.c, kTileBF, grid, a, st), "tile (mfma)")
                 : hip_status(launch_tile_valu(p.metric, p.ks, p.c, kTileBF, grid, a, st),
                              "tile (valu)");
    }
    if (rc) return rc;
    FinArgs f = fin_args(p, Qk, m, ldqk, Xk, ldxk, xstat, id_map, out_idx, out_dist, w, stats,
                         out_approx);
    f.nsplit = p.nsplit;
    if ((rc = run_finalize(p, f, st))) return rc;
    return run_fallback(p, Q, m, ldq, X, n, ldx, id_map, out_idx, out_dist, w, st);
}

FinArgs fin_args(const BfPlan& p, const float* Qk, int64_t m, int64_t ldqk, const float* Xk,
                 int64_t ldxk, const uint32_t* xstat, const int64_t* id_map,
                 int64_t* out_idx, float* out_dist, BfWork& w, int64_t* stats,
                 float* out_approx) {
    FinArgs f;
    std::memset(&f, 0, sizeof(f));
    f.Q = Qk;
    f.ldq = ldqk;
    f.m = (int32_t)m;
    f.X = Xk;
    f.ldx = ldxk;
    f.d = p.d;
    f.metric = p.metric;
    f.approx_mode = p.path == kPathMfma ? 0 : (p.path == kPathLowp ? 2 : 1);
    f.out_approx = out_approx;
    f.pval = w.pval;
    f.pidx = w.pidx;
    f.k = p.k;
    f.qn = w.qn;
    f.xmax_bits = xstat;
    f.flags_q = (const uint32_t*)w.counters + 5;
    f.flags_x = xstat ? xstat + 1 : nullptr;
    f.id_map = id_map;
    f.out_idx = out_idx;
    f.out_dist = out_dist;
    f.fb_list = w.fb_list;
    f.fb_count = w.counters;
    f.stats = stats;
    return f;
}

int run_finalize(const BfPlan& p, const FinArgs& f, hipStream_t st) {
    KernelTimer kt("finalize", st);
    return hip_status(launch_finalize(p.c, f, st), "finalize");
}

// Exhaustive float64 search of the queries listed in w.fb_list (count in
// w.counters[0]) over X, on the original (not repacked) inputs.
int run_fallback(const BfPlan& p, const float* Q, int64_t m, int64_t ldq, const float* X,
                 int64_t n, int64_t ldx, const int64_t* id_map, int64_t* out_idx,
                 float* out_dist, BfWork& w, hipStream_t st) {
    ExactArgs e;
    std::memset(&e, 0, sizeof(e));
    e.Q = Q;
    e.ldq = ldq;
    e.X = X;
    e.ldx = ldx;
    e.n = (int32_t)n;
    e.d = p.d;
    e.metric = p.metric;
    e.k = p.k;
    e.list = w.fb_list;
    e.count = w.counters;
    e.id_map = id_map;
    e.out_idx = out_idx;
    e.out_dist = out_dist;
    const int grid = p.path == kPathExact ? (int)std::min<int64_t>(m, 2048) : kFallbackBlocks;
    KernelTimer kt("fallback", st);
    return hip_status(launch_exact(e, grid, st), "exact fallback");
}

int validate_common(int64_t m, int64_t n, int32_t d, int32_t k, int32_t metric) {
    if (d < 1) return set_err(RBC_EINVAL, "d must be >= 1 (got %d)", d);
    if (n < 1) return set_err(RBC_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
    if (m < 0) return set_err(RBC_EINVAL, "m must be >= 0 (got %lld)", (long long)m);
    if (k < 1) return set_err(RBC_EINVAL, "k must be >= 1 (got %d)", k);
    if (k > n) return set_err(RBC_EINVAL, "k (%d) exceeds the database size (%lld)", k, (long long)n);
    if (metric != RBC_L2 && metric != RBC_L1) return set_err(RBC_EINVAL, "unknown metric %d", metric);
    if (d > RBC_MAX_D) return set_err(RBC_EUNSUPPORTED, "d > %d", RBC_MAX_D);
    if (k > RBC_MAX_K) return set_err(RBC_EUNSUPPORTED, "k > %d", RBC_MAX_K);
    if (n >= (int64_t)1 << 31) return set_err(RBC_EUNSUPPORTED, "n >= 2^31");
    if (m >= (int64_t)1 << 31) return set_err(RBC_EUNSUPPORTED, "m >= 2^31");
    return RBC_OK;
}

}  // namespace rbc

using namespace rbc;

extern "C" {

const char* rbc_last_error(void) { return last_error(); }

int bf_search_workspace_size(int64_t m, int64_t n, int32_t d, int64_t ldq, int64_t ldx,
                             int32_t metric, int32_t k, const rbc_search_opts* opts,
                             size_t* bytes) {
    try {
        if (!bytes) return set_err(RBC_EINVAL, "bytes is NULL");
        int rc = validate_common(m, n, d, k, metric);
        if (rc) return rc;
        if (ldq < d || ldx < d) return set_err(RBC_EINVAL, "leading dimension smaller than d");
        BfPlan p;
        rc = make_bf_plan(m > 0 ? m : 1, n, d, ldq, ldx, metric, k, opts, &p);
        if (rc) return rc;
        if (p.prune_eps != 0.0 || p.one_pass)
            return set_err(RBC_EINVAL, "prune_eps and flags apply to rbc_search only");
        Carver cv(nullptr);
        BfWork w;
        carve_bf(p, m, n, cv, &w);
        *bytes = cv.size();
        return RBC_OK;
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int bf_search(const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n, int64_t ldx,
              int32_t d, int32_t metric, int32_t k, const rbc_search_opts* opts, int64_t* out_idx,
              float* out_dist, void* workspace, size_t ws_bytes, void* hip_stream) {
    try {
        int rc = validate_common(m, n, d, k, metric);
        if (rc) return rc;
        if (ldq < d || ldx < d) return set_err(RBC_EINVAL, "leading dimension smaller than d");
        if (m == 0) return RBC_OK;
        if (!Q || !X || !out_idx || !out_dist) return set_err(RBC_EINVAL, "NULL pointer");
        if (((uintptr_t)Q | (uintptr_t)X) & 15)
            return set_err(RBC_EINVAL, "Q and X must be 16-byte aligned");
        BfPlan p;
        rc = make_bf_plan(m, n, d, ldq, ldx, metric, k, opts, &p);
        if (rc) return rc;
        if (p.prune_eps != 0.0 || p.one_pass)
            return set_err(RBC_EINVAL, "prune_eps and flags apply to rbc_search only");
        Carver cv((char*)workspace);
        BfWork w;
        carve_bf(p, m, n, cv, &w);
        if (!workspace || ws_bytes < cv.size())
            return set_err(RBC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu needed",
                           ws_bytes, cv.size());
        return run_bf(p, Q, m, ldq, X, n, ldx, nullptr, nullptr, nullptr, out_idx, out_dist, w,
                      opts ? opts->dev_stats : nullptr, (hipStream_t)hip_stream,
                      opts ? opts->dev_approx_dist : nullptr);
    } catch (...) {
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

}  // extern "C"
