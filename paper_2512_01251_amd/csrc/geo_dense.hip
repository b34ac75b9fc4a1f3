// Dense per-block layout of the cut-link table (Methodology, "Memory
// Allocations for Boundary Cells"): a map from every block of the level to
// its index among the boundary blocks (blocks with at least one link), and
// the link lengths and face ids of each boundary block as 64 x Q arrays,
// direction-major (structure of arrays: the 64 cells of one direction are
// contiguous), -1 where a (cell, direction) has no link.
//
//   k_dn_flag    one thread per link: marks the block of each run of links
//   scan         boundary-block index of every block
//   k_dn_map     block map (-1 for blocks without links) and the count
//   k_dn_starts  first link of every boundary block (the table is sorted by block)
//   k_dn_write   one workgroup per boundary block: entries built in LDS, written once
#include "geo_internal.h"

namespace {

// position of lattice direction k among the lattice's directions (-1 if not one)
__device__ __forceinline__ int dir_slot(int k, int lattice) {
    int slot = 0;
    for (int j = 0; j < k; j++) {
        const int cx = j % 3 - 1, cy = (j / 3) % 3 - 1, cz = j / 9 - 1;
        const int n2 = cx * cx + cy * cy + cz * cz;
        if (j != 13 && (lattice == 27 || n2 <= 2)) slot++;
    }
    const int cx = k % 3 - 1, cy = (k / 3) % 3 - 1, cz = k / 9 - 1;
    const int n2 = cx * cx + cy * cy + cz * cz;
    return (k != 13 && k >= 0 && k < 27 && (lattice == 27 || n2 <= 2)) ? slot : -1;
}

__global__ void k_dn_flag(int64_t n_links, const int32_t* link_cell, int64_t nb, int32_t* flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_links; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = link_cell[i] >> 6;
        if (b >= 0 && b < nb) flag[b] = 1;  // every writer stores the same value
    }
}

__global__ void k_dn_map(int64_t nb, const int32_t* flag, const int32_t* pre, int32_t* block_map, int64_t* d_nbnd) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x)
        block_map[b] = flag[b] ? pre[b] : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_nbnd = pre[nb];
}

// first link of each boundary block (the table is sorted by block), and
// start[nbnd] = n_links
__global__ void k_dn_starts(int64_t n_links, const int32_t* link_cell, int64_t nb, const int32_t* block_map,
                            const int64_t* d_nbnd, int32_t* start) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_links; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = link_cell[i] >> 6;
        if (i > 0 && (link_cell[i - 1] >> 6) == b) continue;
        if (b >= 0 && b < nb) {
            const int j = block_map[b];
            if (j >= 0) start[j] = (int32_t)i;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[*d_nbnd] = (int32_t)n_links;
}

// one workgroup per boundary block: its 64 x Q entries built in LDS (-1
// where no link), then written once with 16-byte stores
constexpr int DN_THREADS = 256;
__global__ void __launch_bounds__(DN_THREADS) k_dn_write(const int32_t* link_cell, const uint8_t* link_dir,
                                                         const float* link_q, const int32_t* link_tri,
                                                         const int32_t* start, const int64_t* d_nbnd, int64_t cap,
                                                         int64_t n_links, int lattice, int q_dirs, float* dense_q,
                                                         int32_t* dense_tri) {
    __shared__ __align__(16) float sq[26 * 64];
    __shared__ __align__(16) int32_t st[26 * 64];
    __shared__ int8_t slot_of[27];
    int64_t nbnd = *d_nbnd;
    if (nbnd > cap) nbnd = cap;
    const int n = q_dirs * 64;
    if (threadIdx.x < 27) slot_of[threadIdx.x] = (int8_t)dir_slot(threadIdx.x, lattice);
    for (int64_t j = blockIdx.x; j < nbnd; j += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += DN_THREADS) {
            sq[i] = -1.0f;
            st[i] = -1;
        }
        __syncthreads();
        int64_t s0 = start[j], s1 = start[j + 1];
        s0 = s0 < 0 ? 0 : s0;
        s1 = s1 > n_links ? n_links : s1;
        for (int64_t i = s0 + threadIdx.x; i < s1; i += DN_THREADS) {
            const int k = link_dir[i];
            const int sl = k < 27 ? slot_of[k] : -1;
            if (sl < 0) continue;
            const int e = sl * 64 + (link_cell[i] & 63);
            sq[e] = link_q[i];
            st[e] = link_tri[i];
        }
        __syncthreads();
        uint4* q4 = reinterpret_cast<uint4*>(dense_q + j * n);
        uint4* t4 = reinterpret_cast<uint4*>(dense_tri + j * n);
        const uint4* sq4 = reinterpret_cast<const uint4*>(sq);
        const uint4* st4 = reinterpret_cast<const uint4*>(st);
        for (int i = threadIdx.x; i < n / 4; i += DN_THREADS) {
            q4[i] = sq4[i];
            t4[i] = st4[i];
        }
        __syncthreads();
    }
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

size_t geo_dense_ws_bytes(int64_t nb) {
    return ((sizeof(int32_t) * (size_t)(nb + 1) + 255) & ~(size_t)255) * 3 + geo_scan_partials_bytes(nb);
}

int launch_links_dense(int64_t nb, int64_t n_links, const int32_t* link_cell, const uint8_t* link_dir,
                       const float* link_q, const int32_t* link_tri, int lattice, int64_t cap, int32_t* block_map,
                       float* dense_q, int32_t* dense_tri, int64_t* d_nbnd, void* ws, size_t ws_bytes, hipStream_t s) {
    if (ws_bytes < geo_dense_ws_bytes(nb)) return GEO_ERR_WORKSPACE;
    const int q_dirs = lattice == 27 ? 26 : 18;
    char* p = static_cast<char*>(ws);
    const size_t a = (sizeof(int32_t) * (size_t)(nb + 1) + 255) & ~(size_t)255;
    int32_t* flag = reinterpret_cast<int32_t*>(p);
    int32_t* pre = reinterpret_cast<int32_t*>(p + a);
    int32_t* start = reinterpret_cast<int32_t*>(p + 2 * a);
    int32_t* partials = reinterpret_cast<int32_t*>(p + 3 * a);
    int rc;
    if (nb == 0) return geo_fill_u64(reinterpret_cast<uint64_t*>(d_nbnd), 0, 1, s);
    if ((rc = geo_fill_i32(flag, 0, nb, s)) != GEO_OK) return rc;
    if ((rc = geo_fill_i32(start, 0, nb + 1, s)) != GEO_OK) return rc;
    if (n_links > 0) {
        k_dn_flag<<<grid_for(n_links, 256), 256, 0, s>>>(n_links, link_cell, nb, flag);
        GEO_LAUNCH_CHECK();
    }
    if ((rc = geo_scan_exclusive(flag, pre, nb, partials, s)) != GEO_OK) return rc;
    k_dn_map<<<grid_for(nb, 256), 256, 0, s>>>(nb, flag, pre, block_map, d_nbnd);
    GEO_LAUNCH_CHECK();
    // start[] has nb + 1 entries, enough for any count of boundary blocks
    k_dn_starts<<<grid_for(n_links > 0 ? n_links : 1, 256), 256, 0, s>>>(n_links, link_cell, nb, block_map, d_nbnd,
                                                                          start);
    GEO_LAUNCH_CHECK();
    if (cap > 0) {
        const int64_t g = cap < 16384 ? cap : 16384;
        k_dn_write<<<(unsigned)g, DN_THREADS, 0, s>>>(link_cell, link_dir, link_q, link_tri, start, d_nbnd, cap,
                                                       n_links, lattice, q_dirs, dense_q, dense_tri);
        GEO_LAUNCH_CHECK();
    }
    return GEO_OK;
}
