// Interpolated bounce-back on the dense link layout: the boundary step of a
// lattice Boltzmann solver that consumes the cut-link lengths (Related Work:
// the linear interpolated bounce-back of Bouzidi et al., which needs one
// fluid node besides the boundary node; Methodology, "Memory Allocations for
// Boundary Cells", for the per-block layout it reads).
//
// For a link of fluid node x in direction p (x + c_p is solid) with length
// fraction q, the population that enters x in the opposite direction pb is
//   q <  1/2:  2q f*_p(x) + (1 - 2q) f*_p(x - c_p)
//   q >= 1/2:  f*_p(x) / (2q) + (1 - 1/(2q)) f*_pb(x)
// from the post-collision populations f*; plain bounce-back gives f*_p(x).
// The kernel evaluates them as fu + 2q (fp - fu) and fb + (fp - fb) / (2q).
// Where q < 1/2 and the upstream node x - c_p is solid or lies in no block of
// the level, the link takes simple bounce-back, and is counted: the q >= 1/2
// form would extrapolate with weight 1 - 1/(2q) -> -infinity as q -> 0.
//
// The 26 neighbour blocks come from the level's neighbour table when one is
// given (built by k_block_nbr, the indices a block-structured solver keeps),
// else from a walk down the forest.
#include "geo_internal.h"

namespace {

// Direction tables of a lattice (LAT = 19 or 27), evaluated at compile time:
// kdir[s] = direction k of the s-th link slot (rest direction left out),
// pslot[k] = slot of k among the population directions (rest included).
template <int LAT>
struct LatTab {
    int kdir[26];
    int pslot[27];
    constexpr LatTab() : kdir(), pslot() {
        int ns = 0, np = 0;
        for (int k = 0; k < 27; k++) {
            const int cx = k % 3 - 1, cy = (k / 3) % 3 - 1, cz = k / 9 - 1;
            const bool in = LAT == 27 || cx * cx + cy * cy + cz * cz <= 2;
            pslot[k] = in ? np++ : -1;
            if (in && k != 13) kdir[ns++] = k;
        }
        for (; ns < 26; ns++) kdir[ns] = -1;
    }
};

constexpr int IBB_GRID_MAX = 32768;

// Link slots [S0, S1) of one boundary block: load every population the links
// among them need, then compute and store.  q: the block's q of every slot.
template <typename T, int LAT, bool INTERP, int S0, int S1>
__device__ __forceinline__ void ibb_slots(const float* q, const T* __restrict__ f_post, const T* __restrict__ fx,
                                          T* __restrict__ out, const int* nbr, const uint64_t* nsolid,
                                          const uint16_t* upc, int lane, unsigned& fallback) {
    constexpr int QF = LAT == 27 ? 27 : 19;
    constexpr LatTab<LAT> tab{};
    T fp[S1 - S0], f2[S1 - S0];
    uint32_t up = 0;  // bit s - S0: the upstream node of slot s is a fluid node
#pragma unroll
    for (int s = S0; s < S1; s++) {
        const int k = tab.kdir[s];
        fp[s - S0] = T(0);
        f2[s - S0] = T(0);
        if (q[s] >= 0.0f) {
            fp[s - S0] = fx[tab.pslot[k] * 64];
            if (INTERP) {
                if (q[s] < 0.5f) {
                    // upstream node x - c_k: its block offset and its cell there
                    const int code = upc[k * 64 + lane];
                    const int bo = code & 31, ut = code >> 5;
                    if (!((nsolid[bo] >> ut) & 1)) {
                        up |= 1u << (s - S0);
                        f2[s - S0] = f_post[((int64_t)nbr[bo] * QF + tab.pslot[k]) * 64 + ut];
                    }
                } else {
                    f2[s - S0] = fx[tab.pslot[26 - k] * 64];
                }
            }
        }
    }
#pragma unroll
    for (int s = S0; s < S1; s++) {
        const int k = tab.kdir[s];
        if (q[s] >= 0.0f) {
            const T a = fp[s - S0], c = f2[s - S0];
            T v = a;
            if (INTERP) {
                const T qq = (T)q[s];
                if (q[s] >= 0.5f)
                    v = c + (a - c) / (T(2) * qq);
                else if ((up >> (s - S0)) & 1)
                    v = c + T(2) * qq * (a - c);
                else
                    fallback++;
            }
            out[tab.pslot[26 - k] * 64] = v;
        }
    }
}

// One wave per boundary block at a time: the wave scans 64 entries of the
// block map, then serves the boundary blocks among them; lanes are the cells.
// Per block, every q of the block is loaded first, then the populations of
// the link slots, all at once for bounce-back and a third of the slots at a
// time for the interpolated form (a bound on live registers), each group
// loaded in full before its results are stored.
// Populations of type T (float or double); the arithmetic is done in T.
template <typename T, int LAT, bool INTERP>
__global__ void __launch_bounds__(64) k_ibb(DevLevel d, const uint64_t* __restrict__ solid,
                                            const int32_t* __restrict__ block_map, const float* __restrict__ dense_q,
                                            int64_t nbnd, const int32_t* __restrict__ nbr_table,
                                            const T* __restrict__ f_post, T* __restrict__ f_new,
                                            unsigned long long* d_fallback) {
    constexpr int QD = LAT == 27 ? 26 : 18, QF = QD + 1, C3 = (QD + 2) / 3;
    __shared__ int nbr[27];          // neighbour block per offset (ox+1) + 3 (oy+1) + 9 (oz+1), < 0 if none
    __shared__ uint64_t nsolid[27];  // its solid bits (all set where there is no block)
    __shared__ uint16_t upc[INTERP ? 27 * 64 : 1];  // per direction and cell: upstream block offset | cell << 5
    const int lane = threadIdx.x;
    if (INTERP) {
        // kept in LDS rather than registers: 27 values per lane, read once per link
        const int I = lane & 3, J = (lane >> 2) & 3, K = lane >> 4;
        for (int k = 0; k < 27; k++) {
            const int ux = I - (k % 3 - 1), uy = J - ((k / 3) % 3 - 1), uz = K - (k / 9 - 1);
            const int bo = ((ux >> 2) + 1) + 3 * ((uy >> 2) + 1) + 9 * ((uz >> 2) + 1);
            const int ut = (ux & 3) + 4 * (uy & 3) + 16 * (uz & 3);
            upc[k * 64 + lane] = (uint16_t)(bo | ut << 5);
        }
    }
    unsigned fallback = 0;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < d.nblocks; base += (int64_t)gridDim.x * 64) {
        const int64_t mb = base + lane;
        const int32_t mj = mb < d.nblocks ? block_map[mb] : -1;
        uint64_t todo = __ballot(mj >= 0 && mj < nbnd);
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int64_t b = base + src;
            const int64_t j = __shfl(mj, src);
            const float* qrow = dense_q + j * (QD * 64) + lane;
            float q[QD];
#pragma unroll
            for (int s = 0; s < QD; s++) q[s] = qrow[s * 64];
            if (INTERP) {
                __syncthreads();
                if (lane < 27) {
                    int n = (int)b;
                    if (nbr_table)
                        n = nbr_table[b * 27 + lane];  // the level's neighbour table (one coalesced read)
                    else if (lane != 13)
                        n = forest_lookup(d, d.bcoord[3 * b] + lane % 3 - 1, d.bcoord[3 * b + 1] + (lane / 3) % 3 - 1,
                                          d.bcoord[3 * b + 2] + lane / 9 - 1);
                    nbr[lane] = n;
                    nsolid[lane] = n >= 0 ? solid[n] : ~0ull;
                }
                __syncthreads();
            }
            const T* fx = f_post + b * (QF * 64) + lane;
            T* out = f_new + b * (QF * 64) + lane;
            if constexpr (!INTERP) {
                ibb_slots<T, LAT, INTERP, 0, QD>(q, f_post, fx, out, nbr, nsolid, upc, lane, fallback);
            } else {
                ibb_slots<T, LAT, INTERP, 0, C3>(q, f_post, fx, out, nbr, nsolid, upc, lane, fallback);
                __builtin_amdgcn_sched_barrier(0);
                ibb_slots<T, LAT, INTERP, C3, 2 * C3>(q, f_post, fx, out, nbr, nsolid, upc, lane, fallback);
                __builtin_amdgcn_sched_barrier(0);
                ibb_slots<T, LAT, INTERP, 2 * C3, QD>(q, f_post, fx, out, nbr, nsolid, upc, lane, fallback);
            }
        }
    }
    if (d_fallback) wave_count(reinterpret_cast<uint64_t*>(d_fallback), fallback);
}

template <typename T, int LAT>
void launch_ibb_t(unsigned g, const DevLevel& d, const uint64_t* solid, const int32_t* block_map,
                  const float* dense_q, int64_t nbnd, const int32_t* nbr, int interpolate, const void* f_post,
                  void* f_new, unsigned long long* d_fallback, hipStream_t s) {
    const T* fi = static_cast<const T*>(f_post);
    T* fo = static_cast<T*>(f_new);
    if (interpolate)
        k_ibb<T, LAT, true><<<g, 64, 0, s>>>(d, solid, block_map, dense_q, nbnd, nbr, fi, fo, d_fallback);
    else
        k_ibb<T, LAT, false><<<g, 64, 0, s>>>(d, solid, block_map, dense_q, nbnd, nbr, fi, fo, d_fallback);
}

// the 27 same-level neighbours of every block (offset 13 is the block itself)
__global__ void k_block_nbr(DevLevel d, int32_t* nbr) {
    const int64_t n = (int64_t)d.nblocks * 27;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / 27;
        const int o = (int)(i - b * 27);
        nbr[i] = o == 13 ? (int32_t)b
                         : forest_lookup(d, d.bcoord[3 * b] + o % 3 - 1, d.bcoord[3 * b + 1] + (o / 3) % 3 - 1,
                                         d.bcoord[3 * b + 2] + o / 9 - 1);
    }
}

}  // namespace

int launch_block_nbr(const DevLevel& d, int32_t* nbr, hipStream_t s) {
    if (d.nblocks == 0) return GEO_OK;
    int64_t g = ((int64_t)d.nblocks * 27 + 255) / 256;
    if (g > 65536) g = 65536;
    k_block_nbr<<<(unsigned)g, 256, 0, s>>>(d, nbr);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_ibb(const DevLevel& d, const uint64_t* solid, const int32_t* block_map, const float* dense_q,
               int64_t nbnd, const int32_t* nbr, int lattice, int interpolate, int dtype, const void* f_post,
               void* f_new, unsigned long long* d_fallback, hipStream_t s) {
    if (d.nblocks == 0 || nbnd == 0) return GEO_OK;
    const int64_t chunks = ((int64_t)d.nblocks + 63) / 64;
    const int64_t g = chunks < IBB_GRID_MAX ? chunks : IBB_GRID_MAX;
    kt_record(GEO_KT_IBB, s, false);
    const unsigned gu = (unsigned)g;
    if (dtype == GEO_F64) {
        if (lattice == 27)
            launch_ibb_t<double, 27>(gu, d, solid, block_map, dense_q, nbnd, nbr, interpolate, f_post, f_new, d_fallback, s);
        else
            launch_ibb_t<double, 19>(gu, d, solid, block_map, dense_q, nbnd, nbr, interpolate, f_post, f_new, d_fallback, s);
    } else {
        if (lattice == 27)
            launch_ibb_t<float, 27>(gu, d, solid, block_map, dense_q, nbnd, nbr, interpolate, f_post, f_new, d_fallback, s);
        else
            launch_ibb_t<float, 19>(gu, d, solid, block_map, dense_q, nbnd, nbr, interpolate, f_post, f_new, d_fallback, s);
    }
    kt_record(GEO_KT_IBB, s, true);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
