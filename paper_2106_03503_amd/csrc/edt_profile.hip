// Per-kernel timing for observability: while enabled, every kernel launch of
// the library is bracketed by two HIP events recorded on the launch stream,
// and edt_profile_end() sums the elapsed times per kernel name.
#include "../../include/edt.h"
#include "edt_internal.h"

#include <atomic>
#include <mutex>
#include <string.h>
#include <vector>

namespace edt {
namespace {

struct Rec {
    const char* name;
    hipEvent_t start, stop;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;

    hipEvent_t take() {
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
    static Profiler p;
    return p;
}

}  // namespace

// Launches until the armed failure (0: none armed), and whether this thread
// has a failure to report.
std::atomic<int64_t> g_fail_in{0};
thread_local bool t_failed = false;

bool skip_launch() {
    if (t_failed) return true;
    if (g_fail_in.load(std::memory_order_relaxed) <= 0) return false;
    if (g_fail_in.fetch_sub(1) == 1) {
        t_failed = true;
        return true;
    }
    return false;
}

hipError_t launch_status() {
    const hipError_t e = hipGetLastError();
    if (t_failed) {
        t_failed = false;
        return hipErrorLaunchFailure;
    }
    return e;
}

bool prof_enabled() {
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    return p.on;
}

int prof_begin(const char* name, hipStream_t stream) {
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on) return -1;
    Rec r{name, p.take(), p.take()};
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, stream) != hipSuccess) return -1;
    p.recs.push_back(r);
    return (int)p.recs.size() - 1;
}

void prof_end(int token, hipStream_t stream) {
    if (token < 0) return;
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (token < (int)p.recs.size()) (void)hipEventRecord(p.recs[token].stop, stream);
}

}  // namespace edt

extern "C" {

edt_status edt_profile_begin(void) {
    edt::Profiler& p = edt::prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto& r : p.recs) {
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.recs.clear();
    p.on = true;
    return EDT_OK;
}

edt_status edt_profile_end(edt_kernel_time* out, int32_t capacity, int32_t* count) {
    if (!count || capacity < 0 || (capacity > 0 && !out)) return EDT_ERR_INVALID_ARG;
    edt::Profiler& p = edt::prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = false;
    std::vector<edt_kernel_time> acc;
    edt_status st = EDT_OK;
    for (auto& r : p.recs) {
        if (hipEventSynchronize(r.stop) != hipSuccess) {
            st = EDT_ERR_DEVICE;
            continue;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            st = EDT_ERR_DEVICE;
            continue;
        }
        size_t q = 0;
        while (q < acc.size() && strncmp(acc[q].name, r.name, sizeof(acc[q].name)) != 0) ++q;
        if (q == acc.size()) {
            edt_kernel_time t;
            memset(&t, 0, sizeof(t));
            strncpy(t.name, r.name, sizeof(t.name) - 1);
            acc.push_back(t);
        }
        acc[q].launches += 1;
        acc[q].total_ms += ms;
    }
    for (auto& r : p.recs) {
        p.pool.push_back(r.start);
        p.pool.push_back(r.stop);
    }
    p.recs.clear();
    const int32_t n = (int32_t)acc.size();
    for (int32_t q = 0; q < n && q < capacity; ++q) out[q] = acc[q];
    *count = n;
    return st;
}

}  // extern "C"

extern "C" edt_status edt_debug_fail_launch(int32_t k) {
    if (k < 0) return EDT_ERR_INVALID_ARG;
    edt::g_fail_in.store(k);
    return EDT_OK;
}
