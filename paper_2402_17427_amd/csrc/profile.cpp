// Stage timing with HIP events: when enabled, every kernel stage the C ABI
// enqueues is bracketed by a pair of events on the stream it runs on, so
// the elapsed times are the device-side durations of those stages.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.h"
#include "profile.h"

namespace gs {

namespace {

struct Pending {
    const char* name;
    hipEvent_t a, b;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::string only;   // ",a,b," : bracket only these stages; empty: all

    bool wanted(const char* name) const {
        if (only.empty()) return true;
        return only.find("," + std::string(name) + ",") != std::string::npos;
    }
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

Profiler& prof() {
    static Profiler* p = new Profiler();   // lives until the process ends
    return *p;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st), a_(nullptr) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (!p.on || !p.wanted(name)) return;
    a_ = p.get();
    if (a_ && hipEventRecord(static_cast<hipEvent_t>(a_), st) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
    if (!a_) return;
    Profiler& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    hipEvent_t b = p.get();
    if (!b) return;
    if (hipEventRecord(b, st_) != hipSuccess) return;
    p.pending.push_back({name_, static_cast<hipEvent_t>(a_), b});
}

}  // namespace gs

using namespace gs;

extern "C" {

gs_status gs_profile_enable(int on) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    for (auto& e : p.pending) {
        p.pool.push_back(e.a);
        p.pool.push_back(e.b);
    }
    p.pending.clear();
    p.on = on != 0;
    return GS_OK;
}

gs_status gs_profile_select(const char* stages) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    p.only.clear();
    if (stages && *stages) {
        p.only = ",";
        for (const char* c = stages; *c; ++c)
            if (*c != ' ') p.only += *c;
        p.only += ",";
    }
    return GS_OK;
}

gs_status gs_profile_report(char* buf, size_t len) {
    if (!buf || len == 0) return fail(GS_ERR_INVALID, "buffer is NULL");
    Profiler& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    std::map<std::string, std::pair<double, long>> agg;
    std::vector<std::string> order;
    for (auto& e : p.pending) {
        if (hipEventSynchronize(e.b) != hipSuccess) return check_hip("gs_profile_report");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return check_hip("gs_profile_report");
        auto it = agg.find(e.name);
        if (it == agg.end()) {
            order.push_back(e.name);
            agg[e.name] = {ms, 1};
        } else {
            it->second.first += ms;
            it->second.second += 1;
        }
        p.pool.push_back(e.a);
        p.pool.push_back(e.b);
    }
    p.pending.clear();
    std::string out = "{";
    for (size_t i = 0; i < order.size(); ++i) {
        char item[256];
        const auto& v = agg[order[i]];
        snprintf(item, sizeof item, "%s\"%s\": [%.6f, %ld]", i ? ", " : "", order[i].c_str(), v.first, v.second);
        out += item;
    }
    out += "}";
    if (out.size() + 1 > len) return fail(GS_ERR_INVALID, "buffer too small (%zu bytes needed)", out.size() + 1);
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return GS_OK;
}

}  // extern "C"
