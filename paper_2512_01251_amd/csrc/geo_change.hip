// Solid-flag changes between two classifications of the same blocks: with a
// moving geometry, the nodes that the geometry uncovers become fluid and
// need an initial state, and the nodes it newly covers leave the fluid
// (Limitations and Future Work).  HBM-bound: 16 bytes read and 16 written
// per block; one atomic per workgroup for the two counts.
#include "geo_internal.h"

namespace {

constexpr int CH_THREADS = 256;
constexpr int64_t CH_GRID_MAX = 2048;

__global__ void __launch_bounds__(CH_THREADS) k_solid_change(int64_t n, const uint64_t* __restrict__ prev,
                                                             const uint64_t* __restrict__ cur,
                                                             uint64_t* __restrict__ spawned,
                                                             uint64_t* __restrict__ covered,
                                                             unsigned long long* d_counts) {
    __shared__ unsigned long long part[2][CH_THREADS / 64];
    unsigned long long ns = 0, nc = 0;
    for (int64_t b = (int64_t)blockIdx.x * CH_THREADS + threadIdx.x; b < n; b += (int64_t)gridDim.x * CH_THREADS) {
        const uint64_t p = prev[b], c = cur[b];
        const uint64_t s = p & ~c, v = c & ~p;
        if (spawned) spawned[b] = s;
        if (covered) covered[b] = v;
        ns += __popcll(s);
        nc += __popcll(v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ns += __shfl_xor(ns, o, 64);
        nc += __shfl_xor(nc, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = ns;
        part[1][w] = nc;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (int i = 0; i < CH_THREADS / 64; i++) t += part[threadIdx.x][i];
        if (t) atomicAdd(d_counts + threadIdx.x, t);
    }
}

}  // namespace

int launch_solid_change(int64_t n, const uint64_t* prev, const uint64_t* cur, uint64_t* spawned, uint64_t* covered,
                        unsigned long long* d_counts, hipStream_t s) {
    if (n == 0) return GEO_OK;
    int64_t g = (n + CH_THREADS - 1) / CH_THREADS;
    if (g > CH_GRID_MAX) g = CH_GRID_MAX;
    k_solid_change<<<(unsigned)g, CH_THREADS, 0, s>>>(n, prev, cur, spawned, covered, d_counts);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
