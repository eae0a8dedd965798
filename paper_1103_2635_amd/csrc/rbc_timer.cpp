// rbc_timer.cpp -- optional per-kernel timing with HIP events recorded on the
// launching stream around the library's kernels (instrumentation for the
// benchmark; off by default, no cost when off).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rbc.h"
#include "rbc_host.h"

namespace rbc {

namespace {
struct Pending {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::map<std::string, std::pair<double, int64_t>> g_totals;
}  // namespace

KernelTimer::KernelTimer(const char* name, hipStream_t st) : name_(name), st_(st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
    if (hipEventRecord(a_, st_) != hipSuccess) return;
    active_ = true;
}

KernelTimer::~KernelTimer() {
    if (!active_) return;
    if (hipEventRecord(b_, st_) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name_, a_, b_});
}

}  // namespace rbc

using namespace rbc;

extern "C" {

int rbc_timer_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    g_totals.clear();
    return RBC_OK;
}

int rbc_timer_read(const char* name, double* total_ms, int64_t* launches) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Pending& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& t = g_totals[p.name];
            t.first += ms;
            t.second += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    auto it = name ? g_totals.find(name) : g_totals.end();
    if (total_ms) *total_ms = it == g_totals.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == g_totals.end() ? 0 : it->second.second;
    return RBC_OK;
}

}  // extern "C"
