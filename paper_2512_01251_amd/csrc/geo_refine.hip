// Refinement flagging of one level (Methodology, "Refinement Flagging and
// Propagation", Eq. 3), block-parallel (the paper's secondary access mode):
//   1-2. 26-neighbour indices through the forest child maps, and in the
//      same pass the class bits: solid, solid-boundary (solid with a fully
//      fluid neighbour) and eligibility (every in-domain neighbour exists:
//      refining keeps the 2:1 balance);
//   3. marks M1 = (solid-boundary and eligible) or next to a solid-boundary
//      block; solid-adjacent class for the fluid ones;
//   4. n_prop synchronous passes (double-buffered, as the paper avoids the
//      read/write race): fluid blocks, and solid blocks in the first pass,
//      join when a neighbour is marked;
//   5. refine = marked and eligible (written by the last pass of step 4);
//      children emitted in parent order via an exclusive scan, octant
//      o = ox + 2 oy + 4 oz.
#include "geo_internal.h"

namespace {

enum { F_S = 1, F_SB = 2, F_EL = 4 };

__device__ __forceinline__ void nbr_offset(int k, int& dx, int& dy, int& dz) {
    const int kk = k < 13 ? k : k + 1;  // skip the centre of the 3x3x3 cube
    dx = kk % 3 - 1;
    dy = (kk / 3) % 3 - 1;
    dz = kk / 9 - 1;
}

// 26-neighbour indices (forest_lookup values: index, -1 missing, -2 outside
// the domain).  On levels L >= 1 the 26 neighbours have at most 8 distinct
// parents, the 2x2x2 parents from (b-1) >> 1 to (b+1) >> 1 on each axis: the
// first-child indices of those 8 are found by 8 descents of the forest run
// side by side (their dependent loads overlap), and each neighbour is its
// parent's first child plus its octant, with no further load.
__global__ void k_ref_nbr(DevLevel d, const uint64_t* solid, int32_t* nbr, uint8_t* cls) {
    const int64_t nb = d.nblocks;
    const int L = d.level;
    const int nb0[3] = {d.n0[0] >> 2, d.n0[1] >> 2, d.n0[2] >> 2};
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int bc[3] = {d.bcoord[3 * b], d.bcoord[3 * b + 1], d.bcoord[3 * b + 2]};
        // class bits from the neighbours' solid words: solid-boundary (solid
        // with a fully fluid neighbour) and eligible (every in-domain
        // neighbour exists)
        bool fluid_nbr = false, elig = true;
        auto note = [&](int n) {
            if (n == -1) elig = false;
            if (n >= 0 && solid[n] == 0ull) fluid_nbr = true;
        };
        if (L == 0) {  // the dense root grid: no loads
            for (int k = 0; k < 26; k++) {
                int dx, dy, dz;
                nbr_offset(k, dx, dy, dz);
                const int n = forest_lookup(d, bc[0] + dx, bc[1] + dy, bc[2] + dz);
                nbr[(int64_t)k * nb + b] = n;
                note(n);
            }
        } else {
            int p0[3];  // lowest parent coordinate per axis (level L-1)
            for (int a = 0; a < 3; a++) p0[a] = (bc[a] - 1) >> 1;
            int idx[8];
            bool inside[8];
#pragma unroll
            for (int s = 0; s < 8; s++) {
                const int p[3] = {p0[0] + (s & 1), p0[1] + ((s >> 1) & 1), p0[2] + (s >> 2)};
                inside[s] = true;
                for (int a = 0; a < 3; a++)
                    if (p[a] < 0 || p[a] >= (nb0[a] << (L - 1))) inside[s] = false;
                idx[s] = inside[s] ? (p[0] >> (L - 1)) + nb0[0] * ((p[1] >> (L - 1)) + nb0[1] * (p[2] >> (L - 1)))
                                   : -1;
            }
            // descend to level L-1, then the parent's first child on level L
            for (int l = 0; l < L; l++) {
                int c[8];
#pragma unroll
                for (int s = 0; s < 8; s++) c[s] = idx[s] >= 0 ? d.child[l][idx[s]] : -1;
                const int sh = L - 2 - l;
#pragma unroll
                for (int s = 0; s < 8; s++) {
                    if (l == L - 1 || c[s] < 0) {
                        idx[s] = c[s];
                    } else {
                        const int p[3] = {p0[0] + (s & 1), p0[1] + ((s >> 1) & 1), p0[2] + (s >> 2)};
                        idx[s] = c[s] + (((p[0] >> sh) & 1) | (((p[1] >> sh) & 1) << 1) | (((p[2] >> sh) & 1) << 2));
                    }
                }
            }
            for (int k = 0; k < 26; k++) {
                int dv[3];
                nbr_offset(k, dv[0], dv[1], dv[2]);
                int n[3], s = 0;
                bool out = false;
                for (int a = 0; a < 3; a++) {
                    n[a] = bc[a] + dv[a];
                    if (n[a] < 0 || n[a] >= (nb0[a] << L)) out = true;
                    s |= ((n[a] >> 1) - p0[a]) << a;
                }
                int r = -2;
                if (!out) {
                    const int fc = idx[s];
                    r = fc < 0 ? -1 : fc + ((n[0] & 1) | ((n[1] & 1) << 1) | ((n[2] & 1) << 2));
                }
                nbr[(int64_t)k * nb + b] = r;
                note(r);
            }
        }
        const bool is_solid = solid[b] != 0ull;
        uint8_t g = is_solid ? F_S : 0;
        if (is_solid && fluid_nbr) g |= F_SB;
        if (elig) g |= F_EL;
        cls[b] = g;
    }
}

__global__ void k_ref_m1(int64_t nb, const int32_t* nbr, const uint8_t* flags, uint8_t* M, uint8_t* bclass) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t f = flags[b];
        bool adj = false;
        for (int k = 0; k < 26; k++) {
            const int n = nbr[(int64_t)k * nb + b];
            if (n >= 0 && (flags[n] & F_SB)) adj = true;
        }
        const bool m0 = (f & F_SB) && (f & F_EL);
        const bool m = m0 || adj;
        M[b] = m ? 1 : 0;
        bclass[b] = (f & F_SB) ? 2 : ((f & F_S) ? 1 : ((m && !m0) ? 3 : 0));
    }
}

// one propagation pass; the last one (refine != null) also writes refine =
// marked and eligible, and its count for the children's scan
__global__ void k_ref_prop(int64_t nb, const int32_t* nbr, const uint8_t* flags, const uint8_t* Min,
                           uint8_t* Mout, int first, uint8_t* refine, int32_t* cnt) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        uint8_t m = Min[b];
        const uint8_t f = flags[b];
        if (!m && (!(f & F_S) || first)) {
            for (int k = 0; k < 26; k++) {
                const int n = nbr[(int64_t)k * nb + b];
                if (n >= 0 && Min[n]) { m = 1; break; }
            }
        }
        Mout[b] = m;
        if (refine) {
            const int r = (m && (f & F_EL)) ? 1 : 0;
            refine[b] = (uint8_t)r;
            cnt[b] = r;
        }
    }
}

__global__ void k_ref_final(int64_t nb, const uint8_t* flags, const uint8_t* M, uint8_t* refine, int32_t* cnt) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int r = (M[b] && (flags[b] & F_EL)) ? 1 : 0;
        refine[b] = (uint8_t)r;
        cnt[b] = r;
    }
}

__global__ void k_ref_emit(DevLevel d, const uint8_t* refine, const int32_t* offs, int32_t* child_map,
                           int32_t* child_bcoord, int64_t* d_nchild) {
    const int64_t nb = d.nblocks;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        if (!refine[b]) {
            child_map[b] = -1;
            continue;
        }
        const int64_t c0 = 8 * (int64_t)offs[b];
        child_map[b] = (int32_t)c0;
        const int bx = d.bcoord[3 * b], by = d.bcoord[3 * b + 1], bz = d.bcoord[3 * b + 2];
        for (int o = 0; o < 8; o++) {
            child_bcoord[3 * (c0 + o)] = 2 * bx + (o & 1);
            child_bcoord[3 * (c0 + o) + 1] = 2 * by + ((o >> 1) & 1);
            child_bcoord[3 * (c0 + o) + 2] = 2 * bz + ((o >> 2) & 1);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_nchild = 8 * (int64_t)offs[nb];
}

inline unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t geo_refine_ws_bytes(int64_t nb) {
    return al(sizeof(int32_t) * 26 * (size_t)nb) + 3 * al((size_t)nb) + al(sizeof(int32_t) * (size_t)nb) +
           al(sizeof(int32_t) * ((size_t)nb + 1)) + al(geo_scan_partials_bytes(nb));
}

int launch_refine(const DevLevel& d, const uint64_t* solid, int n_prop, uint8_t* bclass, uint8_t* refine,
                  int32_t* child_map, int32_t* child_bcoord, int64_t* d_nchild, void* ws, size_t ws_bytes,
                  hipStream_t s) {
    const int64_t nb = d.nblocks;
    if (ws_bytes < geo_refine_ws_bytes(nb)) return GEO_ERR_WORKSPACE;
    char* p = static_cast<char*>(ws);
    int32_t* nbr = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * 26 * (size_t)nb);
    uint8_t* cls = reinterpret_cast<uint8_t*>(p);
    p += al((size_t)nb);
    uint8_t* M = reinterpret_cast<uint8_t*>(p);
    p += al((size_t)nb);
    uint8_t* Mn = reinterpret_cast<uint8_t*>(p);
    p += al((size_t)nb);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)nb);
    int32_t* offs = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nb + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);

    if (nb == 0) {
        int rc = geo_fill_u64(reinterpret_cast<uint64_t*>(d_nchild), 0, 1, s);
        return rc;
    }
    const unsigned g = grid_for(nb);
    k_ref_nbr<<<g, 256, 0, s>>>(d, solid, nbr, cls);
    k_ref_m1<<<g, 256, 0, s>>>(nb, nbr, cls, M, bclass);
    for (int k = 1; k <= n_prop; k++) {
        const bool last = k == n_prop;
        k_ref_prop<<<g, 256, 0, s>>>(nb, nbr, cls, M, Mn, k == 1 ? 1 : 0, last ? refine : nullptr,
                                     last ? cnt : nullptr);
        uint8_t* t = M;
        M = Mn;
        Mn = t;
    }
    if (n_prop == 0) k_ref_final<<<g, 256, 0, s>>>(nb, cls, M, refine, cnt);
    GEO_LAUNCH_CHECK();
    int rc = geo_scan_exclusive(cnt, offs, nb, partials, s);
    if (rc != GEO_OK) return rc;
    k_ref_emit<<<g, 256, 0, s>>>(d, refine, offs, child_map, child_bcoord, d_nchild);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
