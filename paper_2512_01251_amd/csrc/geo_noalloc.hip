// geo_cutlinks with its scratch in a fixed device array instead of a caller
// workspace, for callers that cannot allocate device memory.
#include <mutex>

#include "geo_internal.h"

size_t geo_cutlinks_ws_bytes(int64_t nb, int64_t cap);

// The call's scratch.  In host code this name stands for the array but is not
// its device address: kernels and copies take the per-device address that
// hipGetSymbolAddress returns (each GPU holds its own copy of the array).
static __device__ __align__(256) unsigned char scratch[GEO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch, looked up once per device
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GEO_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GEO_ERR_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GEO_OK;
}
}  // namespace

extern "C" int geo_cutlinks_noalloc(const geo_mesh* mesh, const geo_level* lv, const geo_bins* rows,
                                    const geo_bins* links, int32_t lattice, int32_t precision, uint32_t* link_mask,
                                    int64_t cap, int64_t* d_nlinks, int32_t* link_cell, uint8_t* link_dir,
                                    float* link_q, int32_t* link_tri, uint64_t* d_stats, geo_stream_t stream) {
    if (!mesh || !lv || cap < 0 || lv->nblocks < 0) return GEO_ERR_ARG;
    // size check first: a request over the limit touches no device
    if (geo_cutlinks_ws_bytes(lv->nblocks, cap) > GEO_NOALLOC_SCRATCH_BYTES) return GEO_ERR_TOO_LARGE;
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != GEO_OK) return rc;
    return geo_cutlinks(mesh, lv, rows, links, lattice, precision, link_mask, cap, d_nlinks, link_cell, link_dir,
                        link_q, link_tri, d_stats, ws, GEO_NOALLOC_SCRATCH_BYTES, stream);
}
