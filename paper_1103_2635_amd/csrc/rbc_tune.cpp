// rbc_tune.cpp -- the tile autotuner: which fp32 matrix-core tile shape
// (16x16x4 with an LDS transpose, or 32x32x2 without) and, for the exact
// search, how many queries a stage-2 item holds (64, or 32 on the 16x16
// shape), how many workgroups the persistent stage-2 launch has and into how
// many row ranges pass 1 splits each nearest list, per (launch kind,
// 16-feature slab count, shortlist length).
//
// Until a configuration is tuned the library uses the 16x16 shape and
// kItemBlocks workgroups (on the 10^6 x 64 subspace workload the 16x16 shape
// measured 5 % faster than the 32x32 one in both the BF and the stage-2
// launch).
// rbc_autotune_search / rbc_autotune_bf run the caller's own call once per
// candidate on the caller's stream, time each with HIP events, and keep the
// fastest in a process-wide table that later calls consult.
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rbc.h"
#include "rbc_host.h"

namespace rbc {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int>, TileChoice> g_table;
thread_local bool t_forced = false;
thread_local TileChoice t_force;
}  // namespace

TileChoice tile_choice(int kind, int ks, int c) {
    if (t_forced) return t_force;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(std::make_tuple(kind, ks, c));
        if (it != g_table.end()) return it->second;
    }
    (void)ks;
    (void)c;
    return TileChoice();  // 16x16 shape, kItemBlocks workgroups
}

namespace {

struct Candidate {
    TileChoice t;
    float ms;
};

// Times fn() under each forced choice: one untimed run, then the best of
// `reps` timed runs, all on stream st.
template <class Fn>
int time_choices(const std::vector<TileChoice>& cands, hipStream_t st, int reps, Fn fn,
                 std::vector<Candidate>* out) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return set_err(RBC_EHIP, "hipEventCreate failed");
    int rc = RBC_OK;
    for (const TileChoice& c : cands) {
        t_forced = true;
        t_force = c;
        float best = -1.f;
        for (int r = 0; r <= reps && rc == RBC_OK; ++r) {
            if (hipEventRecord(a, st) != hipSuccess) rc = set_err(RBC_EHIP, "hipEventRecord");
            if (rc == RBC_OK) rc = fn();
            if (rc == RBC_OK && hipEventRecord(b, st) != hipSuccess)
                rc = set_err(RBC_EHIP, "hipEventRecord");
            if (rc == RBC_OK && hipEventSynchronize(b) != hipSuccess)
                rc = set_err(RBC_EHIP, "hipEventSynchronize");
            float ms = 0.f;
            if (rc == RBC_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess)
                rc = set_err(RBC_EHIP, "hipEventElapsedTime");
            if (rc == RBC_OK && r > 0 && (best < 0.f || ms < best)) best = ms;
        }
        t_forced = false;
        if (rc) break;
        out->push_back({c, best});
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return rc;
}

int pick(int kind, int ks, int c, const std::vector<Candidate>& res, rbc_tune_result* out) {
    const TileChoice def = tile_choice(kind, ks, c);
    const Candidate* best = nullptr;
    float def_ms = -1.f;
    for (const Candidate& r : res) {
        if (!best || r.ms < best->ms) best = &r;
        if (r.t.shape == def.shape && r.t.blocks == def.blocks && r.t.splits == def.splits &&
            r.t.qb == def.qb)
            def_ms = r.ms;
    }
    if (!best) return set_err(RBC_EINVAL, "no candidate configuration");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[std::make_tuple(kind, ks, c)] = best->t;
    }
    if (out) {
        out->shape = best->t.shape == kShape32 ? 32 : 16;
        out->blocks = best->t.blocks;
        out->splits = best->t.splits;
        out->item_queries = 16 * best->t.qb;
        out->ms = best->ms;
        out->ms_before = def_ms;
        out->candidates = (int32_t)res.size();
    }
    return RBC_OK;
}

std::vector<TileChoice> shapes_for(int ks, int c) {
    (void)ks;
    (void)c;
    std::vector<TileChoice> v;
    for (int sh : {kShape16, kShape32}) {
        TileChoice t;
        t.shape = sh;
        t.blocks = kItemBlocks;
        v.push_back(t);
    }
    return v;
}

}  // namespace

}  // namespace rbc

using namespace rbc;

int search_tune_key(const rbc_index* ix, int64_t m, int64_t ldq, int32_t k,
                    const rbc_search_opts* opts, int32_t* kind, int32_t* ks, int32_t* c);

extern "C" {

int rbc_autotune_search(const rbc_index* ix, const float* Q, int64_t m, int64_t ldq, int32_t k,
                        const rbc_search_opts* opts, int64_t* out_idx, float* out_dist,
                        void* workspace, size_t ws_bytes, void* hip_stream,
                        rbc_tune_result* out) {
    try {
        int32_t kind = 0, ks = 0, c = 0;
        int rc = search_tune_key(ix, m, ldq, k, opts, &kind, &ks, &c);
        if (rc) return rc;
        if (kind < 0) return set_err(RBC_EUNSUPPORTED,
                                     "this search runs no tunable matrix-core launch");
        // tile variants: 16x16 with 64- or 32-query items, 32x32 with 64
        std::vector<TileChoice> cands;
        for (int v = 0; v < 3; ++v)
            for (int blocks : {kItemBlocks / 2, kItemBlocks, 2 * kItemBlocks})
                for (int splits : {0, 4}) {
                    TileChoice t;
                    t.shape = v == 2 ? kShape32 : kShape16;
                    t.qb = v == 1 ? 2 : 4;
                    t.blocks = blocks;
                    t.splits = splits;
                    cands.push_back(t);
                }
        std::vector<Candidate> res;
        hipStream_t st = (hipStream_t)hip_stream;
        rc = time_choices(cands, st, 3, [&]() {
            return rbc_search(ix, Q, m, ldq, k, opts, out_idx, out_dist, workspace, ws_bytes,
                              hip_stream);
        }, &res);
        if (rc) return rc;
        return pick(kind, ks, c, res, out);
    } catch (...) {
        t_forced = false;
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_autotune_bf(const float* Q, int64_t m, int64_t ldq, const float* X, int64_t n,
                    int64_t ldx, int32_t d, int32_t metric, int32_t k,
                    const rbc_search_opts* opts, int64_t* out_idx, float* out_dist,
                    void* workspace, size_t ws_bytes, void* hip_stream, rbc_tune_result* out) {
    try {
        BfPlan p;
        int rc = make_bf_plan(m > 0 ? m : 1, n, d, ldq, ldx, metric, k, opts, &p);
        if (rc) return rc;
        if (p.path != kPathMfma)
            return set_err(RBC_EUNSUPPORTED, "this search runs no tunable matrix-core launch");
        std::vector<Candidate> res;
        rc = time_choices(shapes_for(p.ks, p.c), (hipStream_t)hip_stream, 3, [&]() {
            return bf_search(Q, m, ldq, X, n, ldx, d, metric, k, opts, out_idx, out_dist,
                             workspace, ws_bytes, hip_stream);
        }, &res);
        if (rc) return rc;
        return pick(kTuneBF, p.ks, p.c, res, out);
    } catch (...) {
        t_forced = false;
        return set_err(RBC_EHIP, "unexpected exception");
    }
}

int rbc_autotune_set(int32_t kind, int32_t d, int32_t shortlist, int32_t shape,
                     int32_t blocks, int32_t splits, int32_t item_queries) {
    if (kind != 0 && kind != 1) return set_err(RBC_EINVAL, "kind must be 0 (bf) or 1 (search)");
    if (d < 1 || d > 16 * kMaxKS) return set_err(RBC_EINVAL, "d must be in 1 .. %d", 16 * kMaxKS);
    if (shortlist != 4 && shortlist != 8 && shortlist != 16 && shortlist != 32 && shortlist != 64)
        return set_err(RBC_EINVAL, "shortlist must be 4, 8, 16, 32 or 64");
    if (shape != 16 && shape != 32) return set_err(RBC_EINVAL, "shape must be 16 or 32");
    if (blocks < 1 || blocks > 65536) return set_err(RBC_EINVAL, "blocks must be in 1 .. 65536");
    if (splits < 0 || splits > kMaxHomeSplit)
        return set_err(RBC_EINVAL, "splits must be in 0 .. %d", kMaxHomeSplit);
    if (item_queries != 64 && !(item_queries == 32 && shape == 16))
        return set_err(RBC_EINVAL, "item_queries must be 64, or 32 with shape 16");
    TileChoice t;
    t.shape = shape == 32 ? kShape32 : kShape16;
    t.blocks = blocks;
    t.splits = splits;
    t.qb = item_queries / 16;
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[std::make_tuple(kind == 0 ? kTuneBF : kTuneItems, (d + 15) / 16, shortlist)] = t;
    return RBC_OK;
}

void rbc_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

}  // extern "C"
