// Host-side bookkeeping of the request server that needs no GPU: the arena
// allocator that carves workspaces out of the caller's device buffer, the
// ticket book (request status and latency record) and the latency
// percentile.  Plain C++ (no HIP), so that it is also built and tested on its
// own.
#pragma once

#include <stddef.h>

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <deque>
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

// Status of every ticket a server has issued (tickets 1, 2, ... in order) and
// the latencies of the completed requests, in memory bounded by the requests
// in flight rather than by the server's lifetime: a ticket's entry is dropped
// once it and every older ticket have completed (a failed one keeps its
// status in a side map, so any issued ticket can still be asked about), and
// latencies are kept for the last kWindow completions, with their count, sum
// and maximum over all completions.  Status codes: kPending while in flight,
// 0 for success, anything else is a failure.
class TicketBook {
public:
    static constexpr int32_t kPending = 1;
    static constexpr size_t kWindow = size_t(1) << 16;

    uint64_t issue() {
        st_.push_back(kPending);
        return base_ + st_.size() - 1;
    }
    bool known(uint64_t t) const { return t >= 1 && t < base_ + st_.size(); }
    // kPending or the final status of a known ticket.
    int32_t status(uint64_t t) const {
        if (t >= base_) return st_[t - base_];
        const auto it = failed_.find(t);
        return it == failed_.end() ? 0 : it->second;
    }
    // Record the completion of a known, pending ticket.
    void complete(uint64_t t, int32_t status, double latency) {
        st_[t - base_] = status;
        while (!st_.empty() && st_.front() != kPending) {
            if (st_.front() != 0) failed_[base_] = st_.front();
            st_.pop_front();
            ++base_;
        }
        if (win_.size() < kWindow)
            win_.push_back(latency);
        else
            win_[n_ % kWindow] = latency;
        ++n_;
        sum_ += latency;
        max_ = std::max(max_, latency);
    }
    const std::vector<double>& window() const { return win_; }  // unordered
    uint64_t completed() const { return n_; }
    double latency_sum() const { return sum_; }
    double latency_max() const { return max_; }
    size_t entries() const { return st_.size() + failed_.size(); }

private:
    std::deque<int32_t> st_;         // tickets base_, base_ + 1, ...
    uint64_t base_ = 1;
    std::map<uint64_t, int32_t> failed_;  // dropped tickets that failed
    std::vector<double> win_;
    uint64_t n_ = 0;
    double sum_ = 0.0, max_ = 0.0;
};

}  // namespace edt
