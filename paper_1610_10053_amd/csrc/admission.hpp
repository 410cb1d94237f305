// Host-side admission logic of the serving runtime: a first-fit range
// allocator over the device arena and the choice of the next request to
// admit.  No HIP here, so the logic is tested on the host.
#pragma once
#include <cstddef>
#include <deque>
#include <iterator>
#include <map>

namespace jfnk {

// first-fit allocator over [0, size) with coalescing of freed ranges
class RangeAllocator {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    // lowest-addressed free range of at least `bytes`
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            return true;
        }
        return false;
    }
    // return [off, off + bytes), merging it with free neighbours
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto& kv : free_) s += kv.second;
        return s;
    }
    size_t free_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;  // offset -> size, disjoint and never adjacent
};

// Choose the request to admit from `waiting` (arrival order): the oldest one
// whose range fits; requests passed over count a skip, and a request with
// `max_skips` skips lets nothing pass it.  Q: pointer to a type with members
// `size_t bytes` and `int skips`.  On success the request leaves `waiting`
// and its range is allocated at *off.
template <typename Q>
bool pick_request(std::deque<Q>& waiting, RangeAllocator& ranges, int max_skips, Q* out, size_t* off) {
    for (size_t i = 0; i < waiting.size(); ++i) {
        Q q = waiting[i];
        if (ranges.alloc(q->bytes, off)) {
            for (size_t j = 0; j < i; ++j) waiting[j]->skips++;
            waiting.erase(waiting.begin() + (long)i);
            *out = q;
            return true;
        }
        if (q->skips >= max_skips) return false;
    }
    return false;
}

}  // namespace jfnk
