// Kernel timer: optional HIP-event brackets around the launches of selected
// kernels, for measuring one kernel's device time inside a larger call.
// Measurement only; it changes nothing that the kernels compute.
#include <mutex>
#include <vector>

#include "geo_internal.h"

namespace {

struct KernelTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs, reused across reads
    size_t used = 0;             // events recorded since the last read
};

std::mutex kt_mu;
KernelTimer kt[GEO_KT_COUNT];

}  // namespace

void kt_record(int kernel, hipStream_t s, bool stop) {
    std::lock_guard<std::mutex> g(kt_mu);
    KernelTimer& k = kt[kernel];
    if (!k.on) return;
    // a stop only follows a recorded start; a start needs room for its pair
    if (stop != ((k.used & 1) == 1)) return;
    if (!stop && k.used + 2 > 2 * (size_t)GEO_KT_MAX_LAUNCHES) return;
    if (k.used == k.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        k.ev.push_back(e);
    }
    if (hipEventRecord(k.ev[k.used], s) == hipSuccess) k.used++;
}

extern "C" {

int geo_kernel_timer(int32_t kernel, int32_t enable) {
    if (kernel < 0 || kernel >= GEO_KT_COUNT) return GEO_ERR_ARG;
    std::lock_guard<std::mutex> g(kt_mu);
    kt[kernel].on = enable != 0;
    kt[kernel].used = 0;
    return GEO_OK;
}

int geo_kernel_timer_read(int32_t kernel, double* total_ms, int64_t* launches) {
    if (kernel < 0 || kernel >= GEO_KT_COUNT || !total_ms || !launches) return GEO_ERR_ARG;
    std::lock_guard<std::mutex> g(kt_mu);
    KernelTimer& k = kt[kernel];
    double sum = 0.0;
    const size_t pairs = k.used / 2;
    for (size_t i = 0; i < pairs; i++) {
        if (hipEventSynchronize(k.ev[2 * i + 1]) != hipSuccess) return GEO_ERR_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, k.ev[2 * i], k.ev[2 * i + 1]) != hipSuccess) return GEO_ERR_DEVICE;
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)pairs;
    k.used = 0;
    return GEO_OK;
}

}  // extern "C"
