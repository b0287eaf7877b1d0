// Optional per-launch timing with HIP events recorded on the launch stream
// (csdyn_profile_begin / csdyn_profile_end).  Off by default: then every
// ProfScope is a no-op.
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "profile.h"

namespace csd {

namespace {
struct Pair {
    const char *name;
    int64_t size;
    double bytes, flops;
    hipEvent_t a, b;
};
std::mutex g_mu;
std::atomic<bool> g_on{false};
std::vector<Pair> g_pool;
size_t g_next = 0;
int64_t g_dropped = 0;
std::vector<std::string> g_select;  // kernel names to time; empty: all
std::vector<int64_t> g_seen;         // launches of each selected name so far
int g_every = 1;                     // time one launch in g_every of each selected name
thread_local bool t_suspended = false;
}  // namespace

void prof_suspend(bool on) { t_suspended = on; }

ProfScope::ProfScope(const char *name, int64_t size, double bytes, hipStream_t s, double flops) : s_(s) {
    if (!g_on.load(std::memory_order_relaxed) || t_suspended) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_select.empty()) {
        size_t k = 0;
        while (k < g_select.size() && g_select[k] != name) ++k;
        if (k == g_select.size() || g_seen[k]++ % g_every != 0) return;
    }
    if (g_next >= g_pool.size()) { ++g_dropped; return; }
    slot_ = int64_t(g_next++);
    g_pool[slot_].name = name;
    g_pool[slot_].size = size;
    g_pool[slot_].bytes = bytes;
    g_pool[slot_].flops = flops;
    hipEventRecord(g_pool[slot_].a, s_);
}

ProfScope::~ProfScope() {
    if (slot_ < 0) return;
    hipEventRecord(g_pool[slot_].b, s_);
}

}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_profile_begin(int32_t max_launches) {
    clear_error();
    if (max_launches < 1) { set_error("profile: max_launches must be >= 1"); return CSDYN_EINVAL; }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_on) { set_error("profile: already active"); return CSDYN_EINVAL; }
    g_pool.resize(size_t(max_launches));
    for (auto &p : g_pool) {
        CSD_HIP(hipEventCreate(&p.a));
        CSD_HIP(hipEventCreate(&p.b));
        p.name = nullptr;
    }
    g_next = 0;
    g_dropped = 0;
    g_on = true;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_profile_select(const char *names, int32_t every) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_on) { set_error("profile: select before begin"); return CSDYN_EINVAL; }
    if (every < 1) { set_error("profile: every must be >= 1"); return CSDYN_EINVAL; }
    g_select.clear();
    g_every = every;
    if (!names) return CSDYN_OK;
    std::string cur;
    for (const char *c = names;; ++c) {
        if (*c == ',' || *c == 0) {
            if (!cur.empty()) g_select.push_back(cur);
            cur.clear();
            if (*c == 0) break;
        } else {
            cur += *c;
        }
    }
    g_seen.assign(g_select.size(), 0);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_profile_end(csdyn_profile_entry *out, int32_t max_entries, int32_t *n_entries) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) { set_error("profile: not active"); return CSDYN_EINVAL; }
    g_on = false;
    struct Acc { int64_t count = 0; double ms = 0, bytes = 0, flops = 0; };
    std::map<std::pair<std::string, int64_t>, Acc> agg;
    int32_t rc = CSDYN_OK;
    for (size_t i = 0; i < g_next; ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(g_pool[i].b) != hipSuccess ||
            hipEventElapsedTime(&ms, g_pool[i].a, g_pool[i].b) != hipSuccess) {
            set_error("profile: event timing failed");
            rc = CSDYN_EHIP;
            break;
        }
        auto &e = agg[{g_pool[i].name, g_pool[i].size}];
        e.count += 1;
        e.ms += ms;
        e.bytes += g_pool[i].bytes;
        e.flops += g_pool[i].flops;
    }
    for (auto &p : g_pool) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    g_pool.clear();
    int32_t k = 0;
    for (auto &kv : agg) {
        if (out && k < max_entries) {
            std::memset(&out[k], 0, sizeof(out[k]));
            std::strncpy(out[k].name, kv.first.first.c_str(), sizeof(out[k].name) - 1);
            out[k].size = kv.first.second;
            out[k].count = kv.second.count;
            out[k].total_ms = kv.second.ms;
            out[k].bytes = kv.second.bytes;
            out[k].flops = kv.second.flops;
        }
        ++k;
    }
    if (n_entries) *n_entries = k;
    if (g_dropped) set_error("profile: %lld launches not recorded (pool full)", (long long)g_dropped);
    return rc;
}
