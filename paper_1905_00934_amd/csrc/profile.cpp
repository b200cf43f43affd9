// Event-based timing of the library's kernels on the streams they run on.
#include <cstring>
#include <mutex>

#include "common.h"
#include "profile.h"

namespace dect {

namespace {
struct Entry {
    const char* name;
    hipEvent_t start, stop;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Entry> g_entries;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool prof_enabled() { return g_on; }

int prof_begin(const char* name, hipStream_t s) {
    if (!g_on) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    Entry e{name, take_event(), take_event()};
    if (!e.start || !e.stop) return -1;
    if (hipEventRecord(e.start, s) != hipSuccess) return -1;
    g_entries.push_back(e);
    return (int)g_entries.size() - 1;
}

void prof_end(int token, hipStream_t s) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(g_entries[token].stop, s);
}

}  // namespace dect

using namespace dect;

extern "C" {

dect_status dect_profile_start(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& e : g_entries) {
        g_pool.push_back(e.start);
        g_pool.push_back(e.stop);
    }
    g_entries.clear();
    g_on = true;
    return DECT_OK;
}

dect_status dect_profile_stop(dect_kernel_time* out, int max, int* n_out) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = false;
    std::vector<dect_kernel_time> agg;
    for (auto& e : g_entries) {
        if (hipEventSynchronize(e.stop) != hipSuccess)
            return fail(DECT_E_DEVICE, "event synchronisation failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.start, e.stop) != hipSuccess)
            return fail(DECT_E_DEVICE, "event timing failed");
        dect_kernel_time* t = nullptr;
        for (auto& a : agg)
            if (std::strncmp(a.name, e.name, sizeof a.name) == 0) t = &a;
        if (!t) {
            agg.push_back(dect_kernel_time{});
            t = &agg.back();
            std::strncpy(t->name, e.name, sizeof t->name - 1);
        }
        t->total_ms += ms;
        t->launches += 1;
    }
    for (auto& e : g_entries) {
        g_pool.push_back(e.start);
        g_pool.push_back(e.stop);
    }
    g_entries.clear();
    if (n_out) *n_out = (int)agg.size();
    for (int k = 0; k < (int)agg.size() && k < max; ++k) out[k] = agg[k];
    return DECT_OK;
}

}  // extern "C"
