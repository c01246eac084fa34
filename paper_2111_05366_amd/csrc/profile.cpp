// Sampled per-launch timing with HIP events on the launch stream, for two
// kernel families: 0 = Sinkhorn row sweep, 1 = gradient product. Per calling
// thread; off unless goat_profile_enable() set a stride. The row sweep's
// events are taken by the launch itself (prof_sample / prof_commit with
// hipExtLaunchKernel: the kernel's own start and end); a gradient product
// (two launches) is bracketed by events recorded on the stream
// (prof_begin / prof_end).
#include <utility>
#include <vector>

#include "common.h"

namespace goat {
namespace {

constexpr size_t kMaxPairs = 8192;

struct Prof {
    int stride = 0;
    long long counter = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    bool open = false;
};
thread_local Prof g_prof[2];

}  // namespace

void prof_begin(int which, hipStream_t s) {
    Prof& P = g_prof[which];
    P.open = false;
    if (P.stride <= 0) return;
    if ((P.counter++ % P.stride) != 0 || P.used >= kMaxPairs) return;
    if (P.used == P.pool.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
        P.pool.emplace_back(a, b);
    }
    if (hipEventRecord(P.pool[P.used].first, s) == hipSuccess) P.open = true;
}

void prof_end(int which, hipStream_t s) {
    Prof& P = g_prof[which];
    if (!P.open) return;
    if (hipEventRecord(P.pool[P.used].second, s) == hipSuccess) P.used += 1;
    P.open = false;
}

bool prof_sample(int which, hipEvent_t* start, hipEvent_t* stop) {
    Prof& P = g_prof[which];
    *start = *stop = nullptr;
    P.open = false;
    if (P.stride <= 0) return false;
    if ((P.counter++ % P.stride) != 0 || P.used >= kMaxPairs) return false;
    if (P.used == P.pool.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess) return false;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return false;
        }
        P.pool.emplace_back(a, b);
    }
    *start = P.pool[P.used].first;
    *stop = P.pool[P.used].second;
    P.open = true;
    return true;
}

void prof_commit(int which) {
    Prof& P = g_prof[which];
    if (P.open) P.used += 1;
    P.open = false;
}

}  // namespace goat

using namespace goat;

extern "C" {

int goat_profile_enable(int which, int stride) {
    clear_error();
    GOAT_CHECK_ARG(which == 0 || which == 1, "unknown kernel family");
    Prof& P = g_prof[which];
    P.stride = stride > 0 ? stride : 0;
    P.counter = 0;
    P.used = 0;
    P.open = false;
    if (P.stride == 0) {
        for (auto& e : P.pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        P.pool.clear();
    }
    return GOAT_OK;
}

int goat_profile_read(int which, double* ms_total, long long* count) {
    clear_error();
    GOAT_CHECK_ARG(which == 0 || which == 1, "unknown kernel family");
    Prof& P = g_prof[which];
    double tot = 0.0;
    for (size_t i = 0; i < P.used; ++i) {
        GOAT_HIP(hipEventSynchronize(P.pool[i].second));
        float ms = 0.0f;
        GOAT_HIP(hipEventElapsedTime(&ms, P.pool[i].first, P.pool[i].second));
        tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (count) *count = (long long)P.used;
    P.used = 0;
    return GOAT_OK;
}

}  // extern "C"
