// Kernel-class timing with HIP events attached to the dispatches of sampled
// launches (see jfnk_internal.hpp).  A pair that no launch consumed is
// withdrawn when its scope ends.
#include "jfnk_internal.hpp"

namespace jfnk {

thread_local Profiler* g_prof = nullptr;
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void Profiler::begin(int c, double b) {
    if (used + 2 > pool.size()) {
        const size_t grow = pool.size() < 256 ? 256 : pool.size();
        for (size_t i = 0; i < grow; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            pool.push_back(e);
        }
    }
    const size_t token = used;
    used += 2;
    cls.push_back(c);
    pend.push_back(b);
    g_ev_start = pool[token];
    g_ev_stop = pool[token + 1];
}

void Profiler::withdraw() {
    if (cls.empty()) return;
    cls.pop_back();
    pend.pop_back();
    used -= 2;
}

void Profiler::drain() {
    for (size_t i = 0; i < cls.size(); ++i) {
        float t = 0.0f;
        if (cls[i] >= 0 && hipEventElapsedTime(&t, pool[2 * i], pool[2 * i + 1]) == hipSuccess) {
            ms[cls[i]] += t;
            count[cls[i]] += 1;
            bytes[cls[i]] += pend[i];
        }
    }
    cls.clear();
    pend.clear();
    used = 0;
}

void Profiler::release() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    cls.clear();
    pend.clear();
    used = 0;
}

}  // namespace jfnk
