// Kernel-class timing with HIP events (see jfnk_internal.hpp).
#include "jfnk_internal.hpp"

namespace jfnk {

thread_local Profiler* g_prof = nullptr;

int Profiler::begin(int c, hipStream_t s, double b) {
    if (used + 2 > pool.size()) {
        const size_t grow = pool.size() < 256 ? 256 : pool.size();
        for (size_t i = 0; i < grow; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            pool.push_back(e);
        }
    }
    const int token = (int)used;
    used += 2;
    cls.push_back(c);
    pend.push_back(b);
    (void)hipEventRecord(pool[token], s);
    return token;
}

void Profiler::end(int c, hipStream_t s, int token) {
    (void)c;
    (void)hipEventRecord(pool[token + 1], s);
}

void Profiler::drain() {
    for (size_t i = 0; i < cls.size(); ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, pool[2 * i], pool[2 * i + 1]) == hipSuccess) {
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
