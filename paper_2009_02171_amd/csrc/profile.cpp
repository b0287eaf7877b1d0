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
bool prof_active() { return g_on.load(std::memory_order_relaxed) && !t_suspended; }

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
    (void)hipEventRecord(g_pool[slot_].a, s_);  // a failed record fails the elapsed-time query that reads it
}

ProfScope::~ProfScope() {
    if (slot_ < 0) return;
    (void)hipEventRecord(g_pool[slot_].b, s_);
}

// ---------------------------------------------------------------- phases
namespace {
struct PhaseTimer {
    std::vector<hipEvent_t> ev;               // event pool, reused by later timed solves on this thread
    std::vector<std::pair<int, int>> recs;    // (phase, first event of its pair)
    size_t used = 0;
    int open = 0;                             // PhaseScopes currently open
};
thread_local PhaseTimer t_phase;
thread_local bool t_phase_on = false;

int take_events(PhaseTimer &T, int count) {
    while (T.ev.size() < T.used + count) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        T.ev.push_back(e);
    }
    const int k = int(T.used);
    T.used += count;
    return k;
}
}  // namespace

PhaseScope::PhaseScope(Phase ph, hipStream_t s) : s_(s) {
    if (!t_phase_on) return;
    counted_ = true;
    if (t_phase.open++ > 0) return;  // inside another phase
    slot_ = take_events(t_phase, 2);
    if (slot_ < 0) return;
    t_phase.recs.emplace_back(int(ph), slot_);
    (void)hipEventRecord(t_phase.ev[slot_], s_);  // a failed record fails the elapsed-time query that reads it
}

PhaseScope::~PhaseScope() {
    if (!counted_) return;
    --t_phase.open;
    if (slot_ >= 0) (void)hipEventRecord(t_phase.ev[slot_ + 1], s_);
}

int32_t phase_timer_begin(hipStream_t s) {
    t_phase.recs.clear();
    t_phase.used = 0;
    t_phase.open = 0;
    const int k = take_events(t_phase, 2);  // span start and end
    if (k != 0) { set_error("phase timer: event creation failed"); return CSDYN_EHIP; }
    CSD_HIP(hipEventRecord(t_phase.ev[0], s));
    t_phase_on = true;
    return CSDYN_OK;
}

void phase_timer_abort() { t_phase_on = false; }

int32_t phase_timer_end(hipStream_t s, double t_ms[PH_COUNT + 1], double *span_ms) {
    t_phase_on = false;
    CSD_HIP(hipEventRecord(t_phase.ev[1], s));
    CSD_HIP(hipEventSynchronize(t_phase.ev[1]));
    for (int q = 0; q <= PH_COUNT; ++q) t_ms[q] = 0.0;
    double sum = 0.0;
    for (const auto &r : t_phase.recs) {
        float ms = 0.f;
        CSD_HIP(hipEventElapsedTime(&ms, t_phase.ev[r.second], t_phase.ev[r.second + 1]));
        t_ms[r.first] += ms;
        sum += ms;
    }
    float span = 0.f;
    CSD_HIP(hipEventElapsedTime(&span, t_phase.ev[0], t_phase.ev[1]));
    t_ms[PH_COUNT] = double(span) - sum;
    *span_ms = span;
    return CSDYN_OK;
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
    for (auto &p : g_pool) {  // the pool is reset whatever the destroys return
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
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
