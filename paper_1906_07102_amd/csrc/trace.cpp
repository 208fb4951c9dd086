// Optional per-kernel timing with HIP events on the launch stream.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "trace.h"

namespace lmg {
namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;     // events for reuse (creating events costs more than recording them)
std::string g_only;                 // if set, only this kernel name is recorded
int g_on = -1;      // -1: not yet read from the environment

bool take(hipEvent_t* e) {
    if (!g_pool.empty()) {
        *e = g_pool.back();
        g_pool.pop_back();
        return true;
    }
    return hipEventCreate(e) == hipSuccess;
}

bool enabled() {
    if (g_on < 0) {
        const char* v = std::getenv("LMG_TRACE");
        g_on = (v && *v && *v != '0') ? 1 : 0;
    }
    return g_on == 1;
}
}  // namespace

TraceScope::TraceScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!enabled()) return;
    if (!g_only.empty() && g_only != name) return;
    if (!take(&a_)) return;
    if (!take(&b_)) { g_pool.push_back(a_); return; }
    if (hipEventRecord(a_, s_) != hipSuccess) { g_pool.push_back(a_); g_pool.push_back(b_); return; }
    active_ = true;
}

TraceScope::~TraceScope() {
    if (!active_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(b_, s_);
    g_recs.push_back({name_, a_, b_});
}

}  // namespace lmg

extern "C" {

lmg_status lmg_trace_enable(int on) {
    std::lock_guard<std::mutex> lk(lmg::g_mu);
    lmg::g_on = on ? 1 : 0;
    return LMG_OK;
}

lmg_status lmg_trace_only(const char* name) {
    std::lock_guard<std::mutex> lk(lmg::g_mu);
    lmg::g_only = name ? name : "";
    return LMG_OK;
}

lmg_status lmg_trace_report(char* buf, size_t len) {
    if (!buf || len == 0) return LMG_EINVAL;
    std::lock_guard<std::mutex> lk(lmg::g_mu);
    std::map<std::string, std::pair<int, double>> acc;
    std::vector<std::string> order;
    lmg_status st = LMG_OK;
    for (auto& r : lmg::g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) st = LMG_EHIP;
        if (!acc.count(r.name)) order.push_back(r.name);
        auto& e = acc[r.name];
        e.first += 1;
        e.second += ms;
        lmg::g_pool.push_back(r.a);
        lmg::g_pool.push_back(r.b);
    }
    lmg::g_recs.clear();
    std::string out;
    char line[256];
    for (auto& n : order) {
        std::snprintf(line, sizeof(line), "%s %d %.6f\n", n.c_str(), acc[n].first, acc[n].second);
        out += line;
    }
    std::strncpy(buf, out.c_str(), len - 1);
    buf[len - 1] = 0;
    return st;
}

}  // extern "C"
