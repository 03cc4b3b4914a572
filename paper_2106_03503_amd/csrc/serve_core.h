// Host-side bookkeeping of the request server that needs no GPU: the arena
// allocator that carves workspaces out of the caller's device buffer, and the
// latency percentile.  Plain C++ (no HIP), so that it is also built and tested
// on its own.
#pragma once

#include <stddef.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace edt {

// First-fit allocator over the byte range [0, size), in multiples of 256
// bytes (every block it hands out is 256-byte aligned relative to 0).  Free
// blocks are kept by offset and merged with their neighbours on release.
class Arena {
public:
    static constexpr size_t kAlign = 256;

    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        size_ = size / kAlign * kAlign;
        free_.clear();
        if (size_ > 0) free_[0] = size_;
        used_ = high_ = 0;
    }

    static size_t round(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // Take `bytes` (rounded up); false when no free block is large enough.
    bool alloc(size_t bytes, size_t* off) {
        const size_t need = round(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need;
            const size_t at = it->first + need;
            free_.erase(it);
            if (rest > 0) free_[at] = rest;
            used_ += need;
            high_ = std::max(high_, used_);
            return true;
        }
        return false;
    }

    // Give back a block that alloc(bytes) returned at `off`.
    void release(size_t off, size_t bytes) {
        const size_t len = round(bytes == 0 ? 1 : bytes);
        used_ -= len;
        auto next = free_.lower_bound(off);
        size_t start = off, end = off + len;
        if (next != free_.end() && next->first == end) {
            end += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                free_.erase(prev);
            }
        }
        free_[start] = end - start;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return used_; }
    size_t high_water() const { return high_; }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length of each free block
    size_t size_ = 0, used_ = 0, high_ = 0;
};

// Nearest-rank percentile (q in (0, 1]) of the values; 0 for none.
inline double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::ceil(q * (double)v.size());
    if (k < 1) k = 1;
    if (k > v.size()) k = v.size();
    return v[k - 1];
}

}  // namespace edt
