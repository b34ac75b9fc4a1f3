// Solid voxelization of one level (integer gather over the ROWS bins).
//
// The paper flags cells near the surface by local ray casts and fills the
// interior by scan-line propagation inside and across blocks (Algorithms 3-5).
// Here the exact surface events of every row line are already in the ROWS
// bins, so the solid flag of a cell is a local function of its own line:
// parity of the crossings ahead of it on its +x ray, or'ed with the
// on-surface intervals.  No propagation between blocks is needed, so holes in
// the block set of a level cannot leave cells unfilled.
//
// Layout: a wave handles 4 blocks, 16 lanes per block, one lane per row line
// (J, K) of the block; each lane produces the 4 flags of its line and an
// OR over the block's DPP row assembles the 64-bit block mask (bit
// t = I + 4 J + 16 K).
#include "geo_internal.h"

namespace {

// OR of v over the 16 lanes of the wave's row of 16 (DPP row shifts, an
// inclusive OR-scan): the result is whole in the row's last lane
__device__ __forceinline__ unsigned row_or16(unsigned v) {
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v |= (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    return v;
}

// flags of cells x0..x0+3 of one line from its entries
__device__ __forceinline__ unsigned line_nibble(const int32_t* off, const int32_t* val, int64_t cap,
                                                int64_t line, int x0) {
    int64_t e0 = off[line], e1 = off[line + 1];
    if (e1 > cap) e1 = cap;
    if (e0 < 0) e0 = 0;
    unsigned par = 0, surf = 0;
    for (int64_t e = e0; e < e1; e += 4) {
        // four independent loads in flight before the first use
        int32_t v4[4];
#pragma unroll
        for (int i = 0; i < 4; i++) v4[i] = e + i < e1 ? val[e + i] : 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (e + i >= e1) break;
            const int32_t v = v4[i];
            if (v >= 0) {
                // cells x < v see this crossing ahead: flip those of x0..x0+3
                int n = v - x0;
                n = n < 0 ? 0 : (n > 4 ? 4 : n);
                par ^= (1u << n) - 1u;
            } else {
                const int lo = v & 0x7fff, hi = (v >> 15) & 0x7fff;
                int a = lo - x0, b = hi - x0;
                a = a < 0 ? 0 : a;
                b = b > 3 ? 3 : b;
                if (a <= b) surf |= ((1u << (b + 1)) - 1u) & ~((1u << a) - 1u);
            }
        }
    }
    return (par | surf) & 0xfu;
}

__global__ void __launch_bounds__(256) k_voxelize(DevLevel d, const int32_t* off, const int32_t* val,
                                                  int64_t cap, uint64_t* solid) {
    const int L = d.level;
    const int ny = d.n0[1] << L;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t wb = wave * 4; wb < d.nblocks; wb += nwaves * 4) {
        const int64_t b = wb + (lane >> 4);
        const int l = lane & 15;
        unsigned nib = 0;
        if (b < d.nblocks) {
            const int bx = d.bcoord[3 * b], by = d.bcoord[3 * b + 1], bz = d.bcoord[3 * b + 2];
            const int64_t line = (int64_t)(4 * by + (l & 3)) + (int64_t)ny * (4 * bz + (l >> 2));
            nib = line_nibble(off, val, cap, line, 4 * bx);
        }
        // the block's 16 lanes are one DPP row: nibble l of the mask comes
        // from row lane l (bit t = I + 4 J + 16 K with l = J + 4 K)
        const unsigned lo = row_or16(l < 8 ? nib << (4 * l) : 0u);
        const unsigned hi = row_or16(l >= 8 ? nib << (4 * (l - 8)) : 0u);
        if (l == 15 && b < d.nblocks) solid[b] = ((unsigned long long)hi << 32) | lo;
    }
}

__global__ void k_level0(int nbx, int nby, int nbz, int32_t* bcoord) {
    const int64_t n = (int64_t)nbx * nby * nbz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bcoord[3 * i] = (int)(i % nbx);
        bcoord[3 * i + 1] = (int)((i / nbx) % nby);
        bcoord[3 * i + 2] = (int)(i / ((int64_t)nbx * nby));
    }
}

}  // namespace

int launch_voxelize(const DevLevel& d, const int32_t* off, const int32_t* val, int64_t cap, uint64_t* solid,
                    hipStream_t s) {
    if (d.nblocks == 0) return GEO_OK;
    int64_t waves = (d.nblocks + 3) / 4;
    int64_t g = (waves * 64 + 255) / 256;
    if (g > 65536) g = 65536;
    kt_record(GEO_KT_VOXELIZE, s, false);
    k_voxelize<<<(unsigned)g, 256, 0, s>>>(d, off, val, cap, solid);
    kt_record(GEO_KT_VOXELIZE, s, true);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_level0(const int32_t n0[3], int32_t* bcoord, hipStream_t s) {
    const int nbx = n0[0] / 4, nby = n0[1] / 4, nbz = n0[2] / 4;
    const int64_t n = (int64_t)nbx * nby * nbz;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    k_level0<<<(unsigned)g, 256, 0, s>>>(nbx, nby, nbz, bcoord);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
