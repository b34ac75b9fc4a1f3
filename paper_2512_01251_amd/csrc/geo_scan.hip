// Device-wide exclusive scan of int32 counts and small fill kernels.
#include "geo_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// exclusive scan across the block (every thread calls it; the wave scan is
// the shared data-parallel one); returns the block total in *total
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
    __shared__ int wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = wave_incl_scan(v);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / 64; i++) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const int32_t* in, int64_t n, int32_t* partials) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (k < n) s += in[k];
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of the tile sums, total at partials[ntiles]
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_partials(int32_t* partials, int64_t ntiles) {
    int carry = 0;
    for (int64_t c0 = 0; c0 < ntiles; c0 += SCAN_TILE) {
        int v[SCAN_ITEMS];
        int s = 0;
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; i++) {
            int64_t k = c0 + (int64_t)threadIdx.x * SCAN_ITEMS + i;
            v[i] = k < ntiles ? partials[k] : 0;
            s += v[i];
        }
        int tot;
        int ex = block_excl_scan(s, &tot) + carry;
#pragma unroll
        for (int i = 0; i < SCAN_ITEMS; i++) {
            int64_t k = c0 + (int64_t)threadIdx.x * SCAN_ITEMS + i;
            if (k < ntiles) partials[k] = ex;
            ex += v[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[ntiles] = carry;
}

// The tile passes through LDS so that global reads and writes are coalesced
// (lane-consecutive), while each thread scans SCAN_ITEMS consecutive values.
// The LDS rows are padded by one word per SCAN_ITEMS, so a thread's
// consecutive items fall in distinct banks.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(const int32_t* in, int32_t* out, int64_t n,
                                                            const int32_t* partials, int64_t ntiles) {
    __shared__ int tile[SCAN_TILE + SCAN_TILE / SCAN_ITEMS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const int t = threadIdx.x;
    auto slot = [](int j) { return j + j / SCAN_ITEMS; };
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int j = i * SCAN_THREADS + t;
        tile[slot(j)] = base + j < n ? in[base + j] : 0;
    }
    __syncthreads();
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        v[i] = tile[slot(t * SCAN_ITEMS + i)];
        s += v[i];
    }
    int tot;
    int ex = block_excl_scan(s, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        tile[slot(t * SCAN_ITEMS + i)] = ex;
        ex += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int j = i * SCAN_THREADS + t;
        if (base + j < n) out[base + j] = tile[slot(j)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partials[ntiles];
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// zero one 64-bit counter and n 32-bit counts in one launch
__global__ void k_zero_counts(uint64_t* one, int32_t* p, int64_t n) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) *one = 0ull;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// *out += sum of in[0..n-1] in 64-bit (one atomic per workgroup of 256)
__global__ void __launch_bounds__(256) k_sum_i32(const int32_t* in, int64_t n, unsigned long long* out) {
    __shared__ unsigned long long part[4];
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += (unsigned long long)(uint32_t)in[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(out, t);
    }
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

size_t geo_scan_partials_bytes(int64_t n) {
    int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return sizeof(int32_t) * (size_t)(ntiles + 1);
}

// out[0..n-1] = exclusive prefix sums of in, out[n] = total.  in and out must
// not overlap.  partials: geo_scan_partials_bytes(n) bytes.
int geo_scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* partials, hipStream_t s) {
    int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 0) {
        k_fill_i32<<<1, 64, 0, s>>>(out, 0, 1);
        GEO_LAUNCH_CHECK();
        return GEO_OK;
    }
    k_tile_sums<<<(unsigned)ntiles, SCAN_THREADS, 0, s>>>(in, n, partials);
    k_scan_partials<<<1, SCAN_THREADS, 0, s>>>(partials, ntiles);
    k_scan_tiles<<<(unsigned)ntiles, SCAN_THREADS, 0, s>>>(in, out, n, partials, ntiles);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return GEO_OK;
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo_zero_counts(uint64_t* one, int32_t* p, int64_t n, hipStream_t s) {
    k_zero_counts<<<grid_for(n > 0 ? n : 1, 256), 256, 0, s>>>(one, p, n);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return GEO_OK;
    k_fill_u64<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

// *out = sum of the non-negative in[0..n-1], exact in 64 bits
int geo_sum_i32(const int32_t* in, int64_t n, int64_t* out, hipStream_t s) {
    int rc = geo_fill_u64(reinterpret_cast<uint64_t*>(out), 0, 1, s);
    if (rc != GEO_OK || n <= 0) return rc;
    int64_t g = (n + 255) / 256;
    if (g > 256) g = 256;
    k_sum_i32<<<(unsigned)g, 256, 0, s>>>(in, n, reinterpret_cast<unsigned long long*>(out));
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
