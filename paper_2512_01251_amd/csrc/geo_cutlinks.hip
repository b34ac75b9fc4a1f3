// Cut links of one level (Methodology, "Boundary Cell Identification",
// "Memory Allocations for Boundary Cells", "Link-Length Computation", Eq. 2).
//
//  k_cl_mask   one wave per block with link-bin candidates: the solid flags
//              of the block's one-cell halo (6^3 centres) come from the ROWS
//              bins of 36 row lines, so a neighbour centre is classified even
//              where its block does not exist; lane t forms the link mask of
//              cell t.  The masks are kept (the caller's link_mask, else the
//              workspace) and the block's link count is reduced.
//  scans       block counts -> table offsets, so the table is laid out in
//              the order (block, t, k) without atomics; tasks per block ->
//              task offsets.
//  k_cl_multi  blocks whose candidates span several chunks of 64: the 64-bit
//              nearest-hit keys of their links are set to "no hit" before
//              k_cl_q and turned into q and triangle after it.
//  k_cl_q      tasks of (64 links x 64 candidates) of a block: candidates
//              (LINKS bins) staged in LDS as certified plane and edge data,
//              box tests as bit masks, the (link, candidate) pairs flattened
//              over the wave and tested in the form's precision; each link
//              keeps its nearest hit (the minimum over binned faces).  A
//              block whose candidates fit one chunk writes its links' q and
//              triangle directly; the links of other blocks merge into their
//              keys.  A link with a pair the filters cannot decide is queued
//              once.
//  k_cl_fix    one wave per queued link: exact tests against all candidates
//              of its block; the link's q and triangle are overwritten.
//
// The pair test (both forms, precision R) in the frame centred on the block
// (cell centres at -1.5 .. 1.5):
//   plane  s(P) = n . (v0 - P) for the link ends X and Y = X + c, with a
//          bound on |s_R - orient3d(V0, V1, V2, P)| evaluated per pair;
//   edges  e_i = c . (E_i x X - M_i), E_i = V_i - V_j, M_i = V_i x V_j
//          (Pluecker form of orient3d(X, Y, V_i, V_j)), with a bound per
//          candidate that holds for every cell of the block and direction;
//   hit    all three e_i of one strict sign and s(X), s(Y) of opposite
//          strict signs; t = s(X) / (n . c) with its error bound.  The
//          float32 form keeps t when the bound leaves q within 1e-5;
//          otherwise t is recomputed in float64 from the same (exact) data.
#include <type_traits>

#include "geo_internal.h"

namespace {

constexpr int CL_CAND = 64;  // candidates staged per round
constexpr int CL_MAXC = 8;   // pairs per link and flattening round

__device__ __forceinline__ void dirvec(int k, int& cx, int& cy, int& cz) {
    cx = k % 3 - 1;
    cy = (k / 3) % 3 - 1;
    cz = k / 9 - 1;
}

__device__ __forceinline__ uint32_t lattice_dirs(int lattice) {
    uint32_t m = 0;
    for (int k = 0; k < 27; k++) {
        int cx, cy, cz;
        dirvec(k, cx, cy, cz);
        const int n2 = cx * cx + cy * cy + cz * cz;
        if (k != 13 && (lattice == 27 || n2 <= 2)) m |= 1u << k;
    }
    return m;
}

// 6-bit solid vectors of centres x0-1 .. x0+4 of row lines, from the ROWS
// bins: parity of the crossings ahead, or'ed with the on-surface intervals

// fold entries v[0..n-1] of a halo line (centres xm1 .. xm1+5) into par / surf
__device__ __forceinline__ void fold_halo(const int32_t* v4, int64_t n, int xm1, unsigned& par, unsigned& surf) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (i >= n) break;
        const int32_t v = v4[i];
        if (v >= 0) {
            int c = v - xm1;
            c = c < 0 ? 0 : (c > 6 ? 6 : c);
            par ^= (1u << c) - 1u;
        } else {
            int a = (v & 0x7fff) - xm1, b = ((v >> 15) & 0x7fff) - xm1;
            a = a < 0 ? 0 : a;
            b = b > 5 ? 5 : b;
            if (a <= b) surf |= ((1u << (b + 1)) - 1u) & ~((1u << a) - 1u);
        }
    }
}

// halo_bits of two lines (of two blocks) with their loads in flight together:
// both offset pairs, then the first four entries of both lines
__device__ __forceinline__ void halo_bits2(const int32_t* off, const int32_t* val, int64_t cap, bool ha, int64_t la,
                                           int xa, bool hb, int64_t lb, int xb, int nx, unsigned& ra, unsigned& rb) {
    int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (ha) { a0 = off[la]; a1 = off[la + 1]; }
    if (hb) { b0 = off[lb]; b1 = off[lb + 1]; }
    if (a1 > cap) a1 = cap;
    if (a0 < 0) a0 = 0;
    if (b1 > cap) b1 = cap;
    if (b0 < 0) b0 = 0;
    int32_t va[4], vb[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        va[i] = a0 + i < a1 ? val[a0 + i] : 0;
        vb[i] = b0 + i < b1 ? val[b0 + i] : 0;
    }
    unsigned pa = 0, sa = 0, pb = 0, sb = 0;
    fold_halo(va, a1 - a0, xa, pa, sa);
    fold_halo(vb, b1 - b0, xb, pb, sb);
    for (int64_t e = a0 + 4; e < a1; e += 4) {  // lines with more than four entries
#pragma unroll
        for (int i = 0; i < 4; i++) va[i] = e + i < a1 ? val[e + i] : 0;
        fold_halo(va, a1 - e, xa, pa, sa);
    }
    for (int64_t e = b0 + 4; e < b1; e += 4) {
#pragma unroll
        for (int i = 0; i < 4; i++) vb[i] = e + i < b1 ? val[e + i] : 0;
        fold_halo(vb, b1 - e, xb, pb, sb);
    }
    ra = (pa | sa) & 0x3fu;
    rb = (pb | sb) & 0x3fu;
    // centres outside the domain are fluid
    for (int p = 0; p < 6; p++) {
        if (xa + p < 0 || xa + p >= nx) ra &= ~(1u << p);
        if (xb + p < 0 || xb + p >= nx) rb &= ~(1u << p);
    }
}

// link masks of blocks ba and bb (bb < 0: none) together: lanes 0..35
// classify the 36 halo row lines of both into LDS, then lane t forms the
// masks of cell t of both
__device__ __forceinline__ void block_link_mask2(const DevLevel& d, const int32_t* off, const int32_t* val, int64_t cap,
                                                 uint32_t dirs, int64_t ba, int64_t bb, unsigned* halo, uint32_t& ma,
                                                 uint32_t& mb) {
    const int L = d.level;
    const int nx = d.n0[0] << L, ny = d.n0[1] << L, nz = d.n0[2] << L;
    const int lane = threadIdx.x;
    const bool two = bb >= 0;
    const int ax = d.bcoord[3 * ba], ay = d.bcoord[3 * ba + 1], az = d.bcoord[3 * ba + 2];
    int bx = 0, by = 0, bz = 0;
    if (two) {
        bx = d.bcoord[3 * bb];
        by = d.bcoord[3 * bb + 1];
        bz = d.bcoord[3 * bb + 2];
    }
    __syncthreads();
    if (lane < 36) {
        const int J = lane % 6 - 1, K = lane / 6 - 1;
        const int ja = 4 * ay + J, ka = 4 * az + K, jb = 4 * by + J, kb = 4 * bz + K;
        const bool ha = ja >= 0 && ja < ny && ka >= 0 && ka < nz;
        const bool hb = two && jb >= 0 && jb < ny && kb >= 0 && kb < nz;
        unsigned ra, rb;
        halo_bits2(off, val, cap, ha, (int64_t)ja + (int64_t)ny * ka, 4 * ax - 1, hb, (int64_t)jb + (int64_t)ny * kb,
                   4 * bx - 1, nx, ra, rb);
        halo[lane] = ha ? ra : 0u;
        halo[36 + lane] = hb ? rb : 0u;
    }
    __syncthreads();
    const int I = lane & 3, J = (lane >> 2) & 3, K = lane >> 4;
    // 27-bit neighbourhood words, bit (cx+1) + 3 (cy+1) + 9 (cz+1)
    uint32_t na = 0, nb = 0;
#pragma unroll
    for (int dz = 0; dz < 3; dz++)
#pragma unroll
        for (int dy = 0; dy < 3; dy++) {
            const int h = (J + dy) + 6 * (K + dz);
            na |= ((halo[h] >> I) & 7u) << (3 * dy + 9 * dz);
            nb |= ((halo[36 + h] >> I) & 7u) << (3 * dy + 9 * dz);
        }
    ma = ((na >> 13) & 1u) ? 0u : (na & dirs);
    mb = ((nb >> 13) & 1u) ? 0u : (nb & dirs);
}

__global__ void __launch_bounds__(64) k_cl_mask(DevLevel d, const int32_t* off, const int32_t* val, int64_t cap,
                                                const int32_t* loff, int lattice, uint32_t* wmask, int zero_fill,
                                                int32_t* blk_cnt, int32_t* fixn) {
    __shared__ unsigned halo[72];
    // the exact pass's queue counters start at zero (read from the next launch on)
    if (blockIdx.x == 0 && threadIdx.x < 3) fixn[threadIdx.x] = 0;
    const uint32_t dirs = lattice_dirs(lattice);
    const int lane = threadIdx.x;
    const int64_t nchunks = (d.nblocks + 63) / 64;
    // chunks of 64 blocks: one coalesced read of their candidate counts, then
    // only the blocks with candidates are classified, two per wave step
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t b0 = ch * 64;
        const int64_t bl = b0 + lane;
        const bool inb = bl < d.nblocks;
        // a cut link crosses the surface inside the block's reach, so a block
        // without candidate triangles has none
        const bool has = inb && loff[bl] != loff[bl + 1];
        if (inb && !has) blk_cnt[bl] = 0;
        unsigned long long todo = __ballot(has);
        while (todo) {  // uniform
            const int i = __ffsll(todo) - 1;
            todo &= todo - 1;
            int j = -1;
            if (todo) {
                j = __ffsll(todo) - 1;
                todo &= todo - 1;
            }
            const int64_t ba = b0 + i, bb = j >= 0 ? b0 + j : -1;
            uint32_t ma, mb;
            block_link_mask2(d, off, val, cap, dirs, ba, bb, halo, ma, mb);
            wmask[64 * ba + lane] = ma;
            if (bb >= 0) wmask[64 * bb + lane] = mb;
            int ca = __popc(ma), cb = __popc(mb);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                ca += __shfl_xor(ca, o, 64);
                cb += __shfl_xor(cb, o, 64);
            }
            if (lane == 0) {
                blk_cnt[ba] = ca;
                if (bb >= 0) blk_cnt[bb] = cb;
            }
        }
        if (zero_fill) {  // the caller's mask: every block is written
            unsigned long long empty = __ballot(inb && !has);
            while (empty) {  // uniform
                const int i = __ffsll(empty) - 1;
                empty &= empty - 1;
                wmask[64 * (b0 + i) + lane] = 0;
            }
        }
    }
}

// ------------------------------------------------------------------------
// candidate records
// ------------------------------------------------------------------------
enum { C_SLOW = 1, C_EXACT = 2 };
constexpr int TRI_MASK = (1 << 30) - 1;

// Staged candidate triangles, in the frame centred on the block (cell
// centres at -1.5 .. 1.5), V_i the vertices in that frame (exact in float64
// unless flagged slow).  Field-major in LDS: lanes reading one field of
// different candidates hit different banks.
enum {
    F_N = 0,       // normal (V1 - V0) x (V2 - V0), float64 rounded to R (3)
    F_V0 = 3,      // V0 rounded to R, |v0 - V0| <= delta per coordinate (3)
    F_E = 6,       // E_i = V_i - V_{i+1}, rounded (3 x 3)
    F_M = 15,      // M_i = V_i x V_{i+1}, rounded (3 x 3)
    F_BABS = 24,   // plane-value bound from the float64 error of n and the rounding of v0,
                   // for every cell of the block: nerr max|v0 - X|_1 + delta (|n|_1 + 3 nerr)
    F_BD = 25,     // |(n . c)_R - n_exact . c| <= bd for every lattice direction c
    F_BE = 26,     // |e_R - e_exact| <= be for every edge, cell of the block and direction
    F_COUNT = 27
};

template <typename R>
struct CandSoA {
    R f[F_COUNT][CL_CAND];
    int tri[CL_CAND];  // triangle id | C_EXACT << 30 (v0, E_0, E_2 hold V exactly)
};

// one candidate's view: field k of candidate c
template <typename R>
struct CandRef {
    CandSoA<R>& s;
    int c;
    __device__ __forceinline__ R& operator()(int k) const { return s.f[k][c]; }
};

// scaled vertex coordinate x 2^L (exact: a power-of-two scaling)
__device__ __forceinline__ double vert_scaled2(const DevMesh& m, int vid, int a, double s) {
    return load_coord(m, vid, a) * s;
}

__device__ __forceinline__ float down_f(double x) {
    float f = (float)x;
    return (double)f > x ? nextafterf(f, -1e30f) : f;
}
__device__ __forceinline__ float up_f(double x) {
    float f = (float)x;
    return (double)f < x ? nextafterf(f, 1e30f) : f;
}
template <typename R> __device__ __forceinline__ R up_r(double x);
template <> __device__ __forceinline__ float up_r<float>(double x) { return up_f(x); }
template <> __device__ __forceinline__ double up_r<double>(double x) { return x; }

// x - y exactly representable? (two-sum error term of x + (-y))
__device__ __forceinline__ bool diff_exact(double x, double y, double d) {
    const double bb = d - x;
    return (x - (d - bb)) + (-y - bb) == 0.0;
}

struct QStats {
    unsigned fb = 0, ex = 0, tq = 0, staged = 0, pairs = 0, tasks = 0, t64 = 0;
};

// Stage one candidate of the block whose cell centres are at b0 + (0..3)
// (scaled coordinates x 2^L - 1/2): local float64 coordinates, plane and
// edge data rounded to R with their error bounds, and a float box (rounded
// outward).  A triangle of exactly zero area is left inert (empty box): it
// is never hit (the oracle skips it too).
template <typename R>
__device__ void stage_cand(const DevMesh& m, int L, int tri, const int vid[3], const int b0[3], CandSoA<R>& CS, int ci,
                           float lo[3], float hi[3], QStats& st) {
    constexpr double uR = (double)Unit<R>::u;
    constexpr double u64 = 1.1102230246251565e-16;
    const double s = ldexp(1.0, L);
    double v[3][3];
    bool exact = true;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            // centre frame: x 2^L - 1/2 - (b0 + 3/2) = x 2^L - (b0 + 2)
            const double g = vert_scaled2(m, vid[i], a, s), o = (double)(b0[a] + 2);
            const double d = g - o;
            if (!diff_exact(g, o, d)) exact = false;
            v[i][a] = d;
        }
    int flags = exact ? 0 : C_SLOW;
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    double n[3], perm[3];
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    perm[0] = geo_fabs(e1[1] * e2[2]) + geo_fabs(e1[2] * e2[1]);
    perm[1] = geo_fabs(e1[2] * e2[0]) + geo_fabs(e1[0] * e2[2]);
    perm[2] = geo_fabs(e1[0] * e2[1]) + geo_fabs(e1[1] * e2[0]);
    bool inert = false;
    if (geo_fabs(n[0]) <= 5 * u64 * perm[0] && geo_fabs(n[1]) <= 5 * u64 * perm[1] &&
        geo_fabs(n[2]) <= 5 * u64 * perm[2]) {
        // possibly zero area: decided exactly where the coordinates are exact
        if (exact && orient2d_exact(v[0][1], v[0][2], v[1][1], v[1][2], v[2][1], v[2][2]) == 0 &&
            orient2d_exact(v[0][2], v[0][0], v[1][2], v[1][0], v[2][2], v[2][0]) == 0 &&
            orient2d_exact(v[0][0], v[0][1], v[1][0], v[1][1], v[2][0], v[2][1]) == 0)
            inert = true;
        else
            flags |= C_SLOW;
    }
    // float64 errors: the edge vectors carry u64 each, the products and the
    // difference of each normal component two more
    const double pmax = geo_max(perm[0], geo_max(perm[1], perm[2]));
    const double nerr = 5.01 * u64 * pmax;
    double n1 = 0, delta0 = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        CS.f[F_N + a][ci] = (R)n[a];
        CS.f[F_V0 + a][ci] = (R)v[0][a];
        n1 += geo_fabs((double)CS.f[F_N + a][ci]);
        delta0 = geo_max(delta0, geo_fabs((double)CS.f[F_V0 + a][ci] - v[0][a]));
    }
    // largest |v0 - X|_1 over the cells X of the block (coordinates -1.5 .. 1.5)
    double dmax = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) dmax += geo_fabs((double)CS.f[F_V0 + a][ci]) + 1.5;
    CS.f[F_BABS][ci] = up_r<R>((nerr * dmax + delta0 * (n1 * (1 + 2 * uR) + 3 * nerr)) * (1 + 8 * uR));
    CS.f[F_BD][ci] = up_r<R>((3.02 * uR * n1 + 3 * nerr) * (1 + 8 * uR));
    // edges and moments; exactness of v0, E_0, E_2 in R decides whether t can
    // be recomputed in float64 from the staged data
    bool rexact = exact && delta0 == 0.0;
    double be = 0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int j = (i + 1) % 3;
        double K = 0, PM = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double e = v[i][a] - v[j][a];
            if (i != 1 && !diff_exact(v[i][a], v[j][a], e)) rexact = false;
            CS.f[F_E + 3 * i + a][ci] = (R)e;
            if (i != 1 && (double)CS.f[F_E + 3 * i + a][ci] != e) rexact = false;
            K += 3 * geo_fabs(e);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const double p = v[i][b] * v[j][c], q = v[i][c] * v[j][b];
            CS.f[F_M + 3 * i + a][ci] = (R)(p - q);
            K += geo_fabs(p - q);
            PM += geo_fabs(p) + geo_fabs(q);
        }
        be = geo_max(be, (7.05 * uR * K + 4.01 * u64 * (K + PM)) * (1 + 8 * uR));
    }
    CS.f[F_BE][ci] = up_r<R>(be);
    if (rexact) flags |= C_EXACT;
    if (flags & C_SLOW) CS.f[F_BE][ci] = (R)INFINITY;  // every pair with it is left to the exact pass
    CS.tri[ci] = tri | ((flags & C_EXACT) ? (C_EXACT << 29) : 0);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = down_f(geo_min(v[0][a], geo_min(v[1][a], v[2][a])));
        hi[a] = up_f(geo_max(v[0][a], geo_max(v[1][a], v[2][a])));
    }
    // inexact local coordinates: no box rejection for this candidate
    if (!exact) {
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = -1e30f; hi[a] = 1e30f; }
    }
    if (inert) {
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = 1e30f; hi[a] = -1e30f; }
    }
    st.staged++;
}

// a d - b c with Kahan's algorithm: relative error at most 2u (Jeannerod,
// Louvet, Muller 2013); exactly zero iff a d = b c
__device__ __forceinline__ float kahan_det(float a, float d, float b, float c) {
    const float w = b * c;
    const float e = fmaf(-b, c, w);   // w - b c, exact
    const float f = fmaf(a, d, -w);
    return f + e;
}

// exact float sum check: the two-sum error of x + y is zero
__device__ __forceinline__ bool sum_exact_f(float x, float y, float s) {
    const float bb = s - x;
    return (x - (s - bb)) + (y - bb) == 0.0f;
}

// Staging of the float32 form for float32 vertices: float arithmetic only.
// Local coordinates v = x 2^L - (b0 + 2) and the edge vectors v1 - v0, v2 - v0
// are checked exact (otherwise the float64 staging runs); the normal then has
// a relative error of at most 2u per component, and a triangle of exactly
// zero area has n = 0 exactly.
__device__ void stage_cand_f32in(const DevMesh& m, int L, int tri, const int vid[3], const int b0[3],
                                 CandSoA<float>& CS, int ci, float lo[3], float hi[3], QStats& st) {
    constexpr float u = Unit<float>::u;
    const float sc = ldexpf(1.0f, L);
    const float* V = static_cast<const float*>(m.verts);
    float v[3][3];
    bool exact = true;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float g = V[3 * (int64_t)vid[i] + a] * sc;  // exact (power-of-two scaling)
            const float o = (float)(b0[a] + 2);
            const float d = g - o;
            exact &= sum_exact_f(g, -o, d);
            v[i][a] = d;
        }
    float e1[3], e2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        e1[a] = v[1][a] - v[0][a];
        e2[a] = v[2][a] - v[0][a];
        exact &= sum_exact_f(v[1][a], -v[0][a], e1[a]) && sum_exact_f(v[2][a], -v[0][a], e2[a]);
    }
    if (!exact) {  // rare: the float64 staging handles it
        stage_cand<float>(m, L, tri, vid, b0, CS, ci, lo, hi, st);
        return;
    }
    const float n[3] = {kahan_det(e1[1], e2[2], e1[2], e2[1]), kahan_det(e1[2], e2[0], e1[0], e2[2]),
                        kahan_det(e1[0], e2[1], e1[1], e2[0])};
    const bool inert = n[0] == 0.0f && n[1] == 0.0f && n[2] == 0.0f;
    float n1 = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        CS.f[F_N + a][ci] = n[a];
        CS.f[F_V0 + a][ci] = v[0][a];
        n1 += geo_fabs(n[a]);
    }
    CS.f[F_BABS][ci] = 1e-30f;  // every term is exact or relative (in the 6.1u A of the pair test)
    CS.f[F_BD][ci] = 4.1f * u * n1 * (1.0f + 16 * u) + 1e-30f;
    // E_0 = V0 - V1 = -e1 and E_2 = V2 - V0 = e2 are exact; E_1 is rounded
    const float E[3][3] = {{-e1[0], -e1[1], -e1[2]},
                           {v[1][0] - v[2][0], v[1][1] - v[2][1], v[1][2] - v[2][2]},
                           {e2[0], e2[1], e2[2]}};
    float be = 0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int j = (i + 1) % 3;
        float K = 0, PM = 0;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            CS.f[F_E + 3 * i + a][ci] = E[i][a];
            K += 3 * geo_fabs(E[i][a]);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const float q = v[i][c] * v[j][b];
            const float Mx = fmaf(v[i][b], v[j][c], -q);  // |Mx - M| <= u |q| + u |Mx|
            CS.f[F_M + 3 * i + a][ci] = Mx;
            K += geo_fabs(Mx);
            PM += geo_fabs(v[i][b] * v[j][c]) + geo_fabs(q);
        }
        be = geo_max(be, (7.05f * u * K + 1.05f * u * PM) * (1.0f + 16 * u));
    }
    CS.f[F_BE][ci] = be + 1e-30f;
    CS.tri[ci] = tri | (C_EXACT << 29);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = geo_min(v[0][a], geo_min(v[1][a], v[2][a]));
        hi[a] = geo_max(v[0][a], geo_max(v[1][a], v[2][a]));
    }
    if (inert) {  // zero area: never hit (the oracle skips it too)
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = 1e30f; hi[a] = -1e30f; }
    }
    st.staged++;
}

// packed nearest-hit key: t in [0,1] as 37-bit fixed point, then the
// triangle id (27 bits); the minimum key is the nearest hit, ties (equal t to
// 2^-37) going to the smallest triangle id
constexpr double Q37 = 137438953471.0;  // 2^37 - 1
constexpr unsigned long long KEY_MISS = ~0ull;
__device__ __forceinline__ unsigned long long hit_key(double t, int tri) {
    const double c = fmin(fmax(t, 0.0), 1.0);
    return ((unsigned long long)(c * Q37 + 0.5) << 27) | (unsigned long long)(unsigned)tri;
}
__device__ __forceinline__ float key_q(unsigned long long k) {
    return k == KEY_MISS ? -1.0f : (float)((double)(k >> 27) / Q37);
}
__device__ __forceinline__ int32_t key_tri(unsigned long long k) {
    return k == KEY_MISS ? -1 : (int32_t)(k & ((1ull << 27) - 1));
}

// largest hit-parameter error for which a float32 t is kept: q is then within
// 1e-5 of the exact value (t quantised to 2^-38, stored as float32)
constexpr double T_ERR_MAX = 9.5e-6;

// Pair test of the link from X (centre frame) along c against a staged
// candidate: 0 miss, 1 hit (t), -1 undecided (left to the exact pass).
template <typename R>
__device__ __forceinline__ int pair_test(const CandSoA<R>& CS, int ci, const R Xp[3], const R cv[3], double& t, QStats& st) {
#define CF(k) CS.f[(k)][ci]
    constexpr R u = Unit<R>::u;
    const R d0 = CF(F_V0) - Xp[0], d1 = CF(F_V0 + 1) - Xp[1], d2 = CF(F_V0 + 2) - Xp[2];
    const R sX = fma(CF(F_N), d0, fma(CF(F_N + 1), d1, CF(F_N + 2) * d2));
    const R A = fma(geo_fabs(CF(F_N)), geo_fabs(d0), fma(geo_fabs(CF(F_N + 1)), geo_fabs(d1), geo_fabs(CF(F_N + 2)) * geo_fabs(d2)));
    // rounding of n (2u: float64 rounded, or float32 by Kahan's determinant),
    // of v0 - X (u), of the product and the two fmas (3u)
    const R BX = fma(R(6.1) * u, A, CF(F_BABS));
    const R D = fma(cv[0], CF(F_N), fma(cv[1], CF(F_N + 1), cv[2] * CF(F_N + 2)));
    const R sY = sX - D;
    const R BY = fma(u, geo_fabs(sX) + geo_fabs(D), BX + CF(F_BD)) * (R(1) + R(8) * u);
    const bool cX = geo_fabs(sX) > BX, cY = geo_fabs(sY) > BY;
    if (cX && cY && ((sX > R(0)) == (sY > R(0)))) return 0;
    if (!cX || !cY) return -1;
    bool pos = false, neg = false, unc = false;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const R Wx = fma(CF(F_E + 3 * i + 1), Xp[2], fma(-CF(F_E + 3 * i + 2), Xp[1], -CF(F_M + 3 * i + 0)));
        const R Wy = fma(CF(F_E + 3 * i + 2), Xp[0], fma(-CF(F_E + 3 * i + 0), Xp[2], -CF(F_M + 3 * i + 1)));
        const R Wz = fma(CF(F_E + 3 * i + 0), Xp[1], fma(-CF(F_E + 3 * i + 1), Xp[0], -CF(F_M + 3 * i + 2)));
        const R e = fma(cv[0], Wx, fma(cv[1], Wy, cv[2] * Wz));
        pos |= e > CF(F_BE);
        neg |= e < -CF(F_BE);
        unc |= geo_fabs(e) <= CF(F_BE);
    }
    if (pos && neg) return 0;
    if (unc) return -1;
    if constexpr (std::is_same<R, float>::value) {
        const float r = __builtin_amdgcn_rcpf(D);
        const float tf = sX * r;
        // |t_R - t| <= (BX + bd) / |D| for the exact division, plus the
        // reciprocal (1 ulp) and the product (1/2 ulp)
        const float terr = fma((BX + CF(F_BD)) * geo_fabs(r), 1.0f + 16 * u, 4 * u);
        if (terr <= (float)T_ERR_MAX) {
            t = (double)tf;
            return 1;
        }
        if (!((CS.tri[ci] >> 29) & C_EXACT)) return -1;
        // t from the staged vertices in float64: V0 = v0, V1 - V0 = -E_0,
        // V2 - V0 = E_2, all exact
        st.t64++;
        const double a1[3] = {-(double)CF(F_E + 3 * 0 + 0), -(double)CF(F_E + 3 * 0 + 1), -(double)CF(F_E + 3 * 0 + 2)};
        const double a2[3] = {(double)CF(F_E + 3 * 2 + 0), (double)CF(F_E + 3 * 2 + 1), (double)CF(F_E + 3 * 2 + 2)};
        const double nn[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                              a1[0] * a2[1] - a1[1] * a2[0]};
        const double sx = nn[0] * ((double)CF(F_V0) - (double)Xp[0]) + nn[1] * ((double)CF(F_V0 + 1) - (double)Xp[1]) +
                          nn[2] * ((double)CF(F_V0 + 2) - (double)Xp[2]);
        const double dd = nn[0] * (double)cv[0] + nn[1] * (double)cv[1] + nn[2] * (double)cv[2];
        t = sx / dd;
        return 1;
    } else {
        t = sX / D;
        return 1;
    }
}
#undef CF

// select the r-th (0-based) set bit of m (r < popcount(m))
__device__ __forceinline__ int select_bit(uint32_t m, int r) {
    int lo = 0;
#pragma unroll
    for (int step = 16; step > 0; step >>= 1) {
        const int mid = lo + step;
        if (__popc(m & ((1u << mid) - 1u)) <= r) lo = mid;
    }
    return lo;
}

// sign of orient3d with float64 filter then exact arithmetic
__device__ __forceinline__ int o3_sign64(const double* a, const double* b, const double* c, const double* d,
                                         QStats& st) {
    int r = orient3d_filter<double>(a, b, c, d, 0.0);
    if (r != 0) return r;
    st.ex++;
    return orient3d_exact(a, b, c, d);
}

__device__ __forceinline__ int o2_sign64(double ax, double ay, double bx, double by, double cx, double cy,
                                         QStats& st) {
    int r = orient2d_filter<double>(ax, ay, bx, by, cx, cy, 0.0);
    if (r != 0) return r;
    st.ex++;
    return orient2d_exact(ax, ay, bx, by, cx, cy);
}

// axis dropped for in-plane 2D tests: one with a non-zero projected area
__device__ int drop_axis(const double* A, const double* B, const double* C, int& area, QStats& st) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int u = (k + 1) % 3, w = (k + 2) % 3;
        const int s = o2_sign64(A[u], A[w], B[u], B[w], C[u], C[w], st);
        if (s != 0) { area = s; return k; }
    }
    return -1;
}

template <int K>
__device__ __forceinline__ bool in_tri_axis(const double* A, const double* B, const double* C, const double* P, int area,
                                            QStats& st) {
    constexpr int u = (K + 1) % 3, w = (K + 2) % 3;
    if (o2_sign64(A[u], A[w], B[u], B[w], P[u], P[w], st) * area < 0) return false;
    if (o2_sign64(B[u], B[w], C[u], C[w], P[u], P[w], st) * area < 0) return false;
    if (o2_sign64(C[u], C[w], A[u], A[w], P[u], P[w], st) * area < 0) return false;
    return true;
}

__device__ bool in_closed_tri_coplanar(const double* A, const double* B, const double* C, const double* P,
                                       QStats& st) {
    int area;
    const int k = drop_axis(A, B, C, area, st);
    switch (k) {  // compile-time axes keep the arrays in registers
        case 0: return in_tri_axis<0>(A, B, C, P, area, st);
        case 1: return in_tri_axis<1>(A, B, C, P, area, st);
        case 2: return in_tri_axis<2>(A, B, C, P, area, st);
        default: return false;
    }
}

// float64 value of orient3d (for hit parameters)
__device__ __forceinline__ double o3_value(const double* a, const double* b, const double* c, const double* d) {
    const double adx = a[0] - d[0], bdx = b[0] - d[0], cdx = c[0] - d[0];
    const double ady = a[1] - d[1], bdy = b[1] - d[1], cdy = c[1] - d[1];
    const double adz = a[2] - d[2], bdz = b[2] - d[2], cdz = c[2] - d[2];
    return adz * (bdx * cdy - cdx * bdy) + bdz * (cdx * ady - adx * cdy) + cdz * (adx * bdy - bdx * ady);
}

// segment X->Y in the plane of T: entry parameter into the closed triangle
template <int K>
__device__ __forceinline__ int clip_axis(const double* A, const double* B, const double* C, const double* X,
                                         const double* Y, int area, double& t, QStats& st) {
    constexpr int u = (K + 1) % 3, w = (K + 2) % 3;
    const double* V[3] = {A, B, C};
    double lo = 0.0, hi = 1.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const double* p = V[i];
        const double* q = V[(i + 1) % 3];
        const int g0 = o2_sign64(p[u], p[w], q[u], q[w], X[u], X[w], st) * area;
        const int g1 = o2_sign64(p[u], p[w], q[u], q[w], Y[u], Y[w], st) * area;
        if (g0 < 0 && g1 < 0) ok = false;
        if (!ok || (g0 >= 0 && g1 >= 0)) continue;
        const double f0 = area * ((p[u] - X[u]) * (q[w] - X[w]) - (p[w] - X[w]) * (q[u] - X[u]));
        const double f1 = area * ((p[u] - Y[u]) * (q[w] - Y[w]) - (p[w] - Y[w]) * (q[u] - Y[u]));
        const double tt = f0 / (f0 - f1);
        if (g0 < 0) lo = fmax(lo, tt);
        else hi = fmin(hi, tt);
    }
    if (!ok || lo > hi) return 0;
    t = lo;
    return 1;
}

__device__ int coplanar_clip(const double* A, const double* B, const double* C, const double* X, const double* Y,
                             double& t, QStats& st) {
    int area;
    const int k = drop_axis(A, B, C, area, st);
    switch (k) {
        case 0: return clip_axis<0>(A, B, C, X, Y, area, t, st);
        case 1: return clip_axis<1>(A, B, C, X, Y, area, t, st);
        case 2: return clip_axis<2>(A, B, C, X, Y, area, t, st);
        default: return 0;
    }
}

// Exact closed segment / closed triangle test in scaled global coordinates.
// Returns 1 with the hit parameter t, or 0.
__device__ __noinline__ int exact_seg_hit(const double* A, const double* B, const double* C, const double* X,
                                          const double* Y, double& t, QStats& st) {
    const int sx = o3_sign64(A, B, C, X, st), sy = o3_sign64(A, B, C, Y, st);
    if (sx * sy > 0) return 0;
    if (sx == 0 && sy == 0) return coplanar_clip(A, B, C, X, Y, t, st);
    if (sx == 0) {
        if (in_closed_tri_coplanar(A, B, C, X, st)) { t = 0.0; return 1; }
        return 0;
    }
    if (sy == 0) {
        if (in_closed_tri_coplanar(A, B, C, Y, st)) { t = 1.0; return 1; }
        return 0;
    }
    const int v0 = o3_sign64(X, Y, A, B, st), v1 = o3_sign64(X, Y, B, C, st), v2 = o3_sign64(X, Y, C, A, st);
    const bool pos = v0 > 0 || v1 > 0 || v2 > 0, neg = v0 < 0 || v1 < 0 || v2 < 0;
    if (pos && neg) return 0;
    const double px = o3_value(A, B, C, X), py = o3_value(A, B, C, Y);
    t = px / (px - py);
    t = fmin(fmax(t, 0.0), 1.0);
    return 1;
}

// tasks per block: ceil(links / 64) x ceil(candidates / 64); blocks with
// links and more than one chunk of candidates are listed (in no particular
// order) for k_cl_multi
__global__ void __launch_bounds__(256) k_cl_ntask(int64_t nb, const int32_t* blk_off, const int32_t* loff,
                                                  int64_t lcap, int32_t* ntask, int32_t* mlist, int32_t* mcount) {
    __shared__ int wg_count, wg_base;
    const int lane = threadIdx.x & 63;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < nb; b0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = b0 + threadIdx.x;
        bool multi = false;
        if (b < nb) {
            const int n = blk_off[b + 1] - blk_off[b];
            int64_t c0 = loff[b], c1 = loff[b + 1];
            if (c1 > lcap) c1 = lcap;
            if (c0 < 0) c0 = 0;
            const int nc = c1 > c0 ? (int)(c1 - c0) : 0;
            ntask[b] = n > 0 ? ((n + 63) / 64) * (nc > 0 ? (nc + CL_CAND - 1) / CL_CAND : 1) : 0;
            multi = n > 0 && nc > CL_CAND;
        }
        // list slots: one LDS reservation per wave, one global one per
        // workgroup (same-address atomics serialise)
        if (threadIdx.x == 0) wg_count = 0;
        __syncthreads();
        const unsigned long long bal = __ballot(multi);
        int wofs = 0;
        if (bal && lane == 0) wofs = atomicAdd(&wg_count, __popcll(bal));
        wofs = __shfl(wofs, 0, 64);
        __syncthreads();
        if (threadIdx.x == 0) wg_base = wg_count ? atomicAdd(mcount, wg_count) : 0;
        __syncthreads();
        if (multi) mlist[wg_base + wofs + __popcll(bal & ((1ull << lane) - 1ull))] = (int32_t)b;
        __syncthreads();
    }
}

// Blocks whose candidates span several chunks (their tasks merge into keys),
// from the list of k_cl_ntask: mode 0 sets the keys of their links to "no
// hit" and clears the queue marks, mode 1 turns the keys into q and triangle.
// One wave per listed block, lanes over its links.
__global__ void k_cl_multi(const int32_t* mlist, const int32_t* mcount, const int32_t* blk_off, int64_t cap,
                           int mode, unsigned long long* keys, int32_t* mark, float* link_q, int32_t* link_tri) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nm = *mcount;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < nm; i += nw) {
        const int64_t b = mlist[i];
        int64_t p1 = blk_off[b + 1];
        if (p1 > cap) p1 = cap;
        for (int64_t p = blk_off[b] + lane; p < p1; p += 64) {
            if (mode == 0) {
                keys[p] = KEY_MISS;
                mark[p] = 0;
            } else {
                const unsigned long long k = keys[p];
                link_q[p] = key_q(k);
                link_tri[p] = key_tri(k);
            }
        }
    }
}

// block of a task: largest b with task_off[b] <= task (64-ary search by the wave)
__device__ __forceinline__ int64_t task_block(const int32_t* task_off, int64_t nb, int task) {
    int64_t lo = 0, hi = nb;  // task_off[lo] <= task < task_off[hi]
    const int lane = threadIdx.x;
    while (hi - lo > 1) {
        const int64_t span = hi - lo;
        const int64_t step = (span + 63) / 64;
        const int64_t pos = lo + (int64_t)lane * step;
        const bool le = pos < hi && task_off[pos] <= task;
        const unsigned long long m = __ballot(le);
        const int last = 63 - __clzll((long long)m);  // lane 0 always qualifies
        const int64_t nlo = lo + (int64_t)last * step;
        const int64_t nhi = (nlo + step < hi) ? nlo + step : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// block of `task` searching forward from block b (task_off[b] <= task): the
// wave tests 64 blocks per step, so runs of blocks without tasks cost one
// load each 64 blocks
__device__ __forceinline__ int64_t advance_block(const int32_t* task_off, int64_t nb, int64_t b, int task) {
    const int lane = threadIdx.x;
    for (;;) {
        const int64_t i = b + 1 + lane;  // block b + lane ends at task_off[i]
        const bool ends_after = i > nb || task < task_off[i];
        const unsigned long long m = __ballot(ends_after);
        if (m) return b + (__ffsll(m) - 1);
        b += 64;
    }
}

// link queue of the exact pass: pos, with bit 31 set when the link must be
// redone over all its candidates (an undecided pair did not fit the pair queue)
constexpr int32_t FIX_FULL = (int32_t)0x80000000u;
__device__ __forceinline__ void enqueue_fix(int32_t* fixq, int32_t* fixn, int64_t cap, int64_t pos, bool full) {
    const int qi = atomicAdd(fixn, 1);
    if (qi < cap) fixq[qi] = (int32_t)pos | (full ? FIX_FULL : 0);
}

#define CL_Q_PARAMS                                                                                            \
    DevMesh m, DevLevel d, const uint32_t *wmask, const int32_t *loff, const int32_t *lval, int64_t lcap,      \
        const int32_t *blk_off, const int32_t *task_off, int64_t cap, int32_t *link_cell, uint8_t *link_dir,   \
        float *link_q, int32_t *link_tri, unsigned long long *keys, int32_t *mark, int32_t *fixq, int32_t *fixn, \
        int2 *pairq, int32_t *pairn, int64_t pcap, uint64_t *stats
#define CL_Q_ARGS \
    m, d, wmask, loff, lval, lcap, blk_off, task_off, cap, link_cell, link_dir, link_q, link_tri, keys, mark, fixq, fixn, \
        pairq, pairn, pcap, stats

// the q kernel's body, one wave per workgroup (both forms)
template <typename R>
__device__ __forceinline__ void cl_q_body(CL_Q_PARAMS) {
    __shared__ CandSoA<R> cand;
    // box test as bit masks over the staged candidates: for axis a and lattice
    // position j in -1..4 (block-corner frame), bmask[12a + 1 + j] holds the
    // candidates with hi_a >= j and bmask[12a + 7 + j] those with lo_a <= j
    __shared__ unsigned long long bmask[36];
    __shared__ unsigned char cellat[64];       // cell whose links start at a chunk position
    __shared__ unsigned long long sstart;      // chunk positions where a cell's links start
    __shared__ uint16_t flat[64 * CL_MAXC];    // flattened pairs: owner lane | candidate slot << 6
    __shared__ float4 sxp[64];                 // each lane's link: centre-frame cell | direction (bytes)
    __shared__ unsigned long long lbest[64];   // nearest hit of each lane's link (packed key)
    __shared__ unsigned long long lunc;        // links with an undecided pair (bit = lane)
    __shared__ unsigned long long lfull;       // ... one of which did not fit the pair queue
    const int L = d.level;
    const int lane = threadIdx.x;
    const int ntasks = task_off[d.nblocks];
    // contiguous task range per workgroup, so that consecutive tasks share a block
    const int per = (ntasks + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t0 = (int)blockIdx.x * per;
    const int t1 = t0 + per < ntasks ? t0 + per : ntasks;
    QStats st;
    if (t0 >= t1) return;
    int64_t b = task_block(task_off, d.nblocks, t0);
    int64_t b_prev = -1;
    int64_t staged_b = -1;  // (block, candidate chunk) held in LDS
    int staged_c = -1;
    uint32_t my_mask = 0;
    int my_pre = 0;
    // prefetch of the next staging unit: candidate triangle (at staging) and
    // its vertex ids (at the end of the task), so staging waits for one load
    int pf_task = -1, pf_n = 0;
    bool pf_vid_ok = false;
    int pf_tri = 0, pf_v0 = 0, pf_v1 = 0, pf_v2 = 0;
    for (int task = t0; task < t1; task++) {
        if (task >= task_off[b + 1]) b = advance_block(task_off, d.nblocks, b + 1, task);  // uniform
        const int n = blk_off[b + 1] - blk_off[b];
        int64_t c0 = loff[b], c1 = loff[b + 1];
        if (c1 > lcap) c1 = lcap;
        if (c0 < 0) c0 = 0;
        if (c0 > c1) c0 = c1;
        const int nc = (int)(c1 - c0);
        const int ncc = nc > CL_CAND ? (nc + CL_CAND - 1) / CL_CAND : 1;
        // a block's tasks run candidate chunk by candidate chunk, so that
        // consecutive link chunks reuse the staged candidates
        const int nlc = (n + 63) / 64;
        const int local = task - task_off[b];
        const int cchunk = local / nlc, lchunk = local % nlc;
        const int b0[3] = {4 * d.bcoord[3 * b], 4 * d.bcoord[3 * b + 1], 4 * d.bcoord[3 * b + 2]};
        st.tasks++;
        if (b != b_prev) {  // uniform: the block's cell masks and their prefix
            my_mask = wmask[64 * b + lane];
            const int c = __popc(my_mask), incl = wave_incl_scan(c);
            my_pre = incl - c;
            b_prev = b;
        }
        const int cb = cchunk * CL_CAND;
        const int nstage = nc - cb < CL_CAND ? (nc - cb > 0 ? nc - cb : 0) : CL_CAND;
        __syncthreads();  // the previous task's readers of the LDS arrays are done
        if (lane == 0) {
            sstart = 0;
            lunc = 0;
            lfull = 0;
        }
        if (b != staged_b || cchunk != staged_c) {  // uniform
            staged_b = b;
            staged_c = cchunk;
            float blo[3] = {1e30f, 1e30f, 1e30f}, bhi[3] = {-1e30f, -1e30f, -1e30f};
            const bool from_pf = pf_task == task;  // uniform
            const int tri = lane < nstage ? (from_pf ? pf_tri : lval[c0 + cb + lane]) : -1;
            // entries of an overflowed bin are not triangle ids: left inert
            if (lane < nstage && (unsigned)tri < (unsigned)m.nt) {
                int vid[3];
                if (from_pf && pf_vid_ok) {
                    vid[0] = pf_v0;
                    vid[1] = pf_v1;
                    vid[2] = pf_v2;
                } else {
#pragma unroll
                    for (int i = 0; i < 3; i++) vid[i] = m.tris[3 * (int64_t)tri + i];
                }
                if constexpr (std::is_same<R, float>::value) {
                    if (m.vdtype == GEO_F32) stage_cand_f32in(m, L, tri, vid, b0, cand, lane, blo, bhi, st);
                    else stage_cand<R>(m, L, tri, vid, b0, cand, lane, blo, bhi, st);
                } else {
                    stage_cand<R>(m, L, tri, vid, b0, cand, lane, blo, bhi, st);
                }
            }
            // first task of the next staging unit, and its candidates
            pf_task = -1;
            pf_vid_ok = false;
            const int tn = task_off[b] + (cchunk + 1) * nlc;
            if (tn < t1) {
                const int64_t bn = tn < task_off[b + 1] ? b : advance_block(task_off, d.nblocks, b + 1, tn);
                const int nn = blk_off[bn + 1] - blk_off[bn];
                int64_t d0 = loff[bn], d1 = loff[bn + 1];
                if (d1 > lcap) d1 = lcap;
                if (d0 < 0) d0 = 0;
                if (d0 > d1) d0 = d1;
                const int cbn = ((tn - task_off[bn]) / ((nn + 63) / 64)) * CL_CAND;
                const int rem = (int)(d1 - d0) - cbn;
                pf_n = rem < CL_CAND ? (rem > 0 ? rem : 0) : CL_CAND;
                if (lane < pf_n) pf_tri = lval[d0 + cbn + lane];
                pf_task = tn;
            }
            unsigned long long mine = 0;
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    // lattice position j - 1 of the corner frame is j - 5/2 in the centre frame
                    const float pj = (float)j - 2.5f;
                    const unsigned long long A = __ballot(bhi[a] >= pj);
                    const unsigned long long B = __ballot(blo[a] <= pj);
                    if (lane == 12 * a + j) mine = A;
                    if (lane == 12 * a + 6 + j) mine = B;
                }
            if (lane < 36) bmask[lane] = mine;
        }
        // the links of this task: chunk positions base .. base + 63 of the
        // block's (t, k) order; the links of cell t start at its prefix (my_pre of lane t)
        const int base = lchunk * 64;
        const int cnt = __popc(my_mask);
        __syncthreads();
        if (cnt > 0 && my_pre > base && my_pre < base + 64) {
            atomicOr(&sstart, 1ull << (my_pre - base));
            cellat[my_pre - base] = (unsigned char)lane;
        }
        {
            const unsigned long long before = __ballot(cnt > 0 && my_pre <= base);
            if (lane == 0) cellat[0] = (unsigned char)(before ? 63 - __clzll((long long)before) : 0);
        }
        __syncthreads();
        const int li = base + lane;
        const bool active = li < n;
        int t = 0, k = 13;
        {
            const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
            const int j = 63 - __clzll((long long)((sstart | 1ull) & le));
            t = active ? cellat[j] : 0;
            // the owner cell's mask and prefix, from its lane
            const uint32_t om = (uint32_t)__shfl((int)my_mask, t, 64);
            const int op = __shfl(my_pre, t, 64);
            if (active) k = select_bit(om, li - op);
        }
        int cx, cy, cz;
        dirvec(k, cx, cy, cz);
        const int tl[3] = {t & 3, (t >> 2) & 3, t >> 4};
        sxp[lane] = make_float4((float)tl[0] - 1.5f, (float)tl[1] - 1.5f, (float)tl[2] - 1.5f,
                                __int_as_float((cx + 1) | ((cy + 1) << 8) | ((cz + 1) << 16)));
        lbest[lane] = KEY_MISS;
        // phase 1: candidates whose box meets the link's segment box
        unsigned long long pm = 0;
        if (active) {
            const int slo[3] = {geo_min(tl[0], tl[0] + cx), geo_min(tl[1], tl[1] + cy), geo_min(tl[2], tl[2] + cz)};
            const int shi[3] = {geo_max(tl[0], tl[0] + cx), geo_max(tl[1], tl[1] + cy), geo_max(tl[2], tl[2] + cz)};
            pm = bmask[1 + slo[0]] & bmask[7 + shi[0]] & bmask[13 + slo[1]] & bmask[19 + shi[1]] &
                 bmask[25 + slo[2]] & bmask[31 + shi[2]];
        }
        while (__any(pm != 0)) {  // uniform
            // flatten up to CL_MAXC pairs per link over the wave
            const int pc = __popcll(pm);
            const int cn = pc < CL_MAXC ? pc : CL_MAXC;
            const int inc2 = wave_incl_scan(cn);
            const int pbase = inc2 - cn;
            for (int j = 0; j < cn; j++) {
                const int slot = __ffsll(pm) - 1;
                pm &= pm - 1;
                flat[pbase + j] = (uint16_t)(lane | (slot << 6));
            }
            const int P = __shfl(inc2, 63, 64);
            __syncthreads();
            st.pairs += cn;
            // phase 2: one pair per lane
            for (int p = lane; p < P; p += 64) {
                const int fe = flat[p];
                const int ow = fe & 63;
                const int cidx = fe >> 6;
                const float4 xf = sxp[ow];
                const int cw = __float_as_int(xf.w);
                const R Xp[3] = {(R)xf.x, (R)xf.y, (R)xf.z};
                const R cv[3] = {(R)((cw & 3) - 1), (R)(((cw >> 8) & 3) - 1), (R)(((cw >> 16) & 3) - 1)};
                double tq;
                const int res = pair_test<R>(cand, cidx, Xp, cv, tq, st);
                if (res == 1) {
                    atomicMin(&lbest[ow], hit_key(tq, cand.tri[cidx] & TRI_MASK));  // each link keeps its nearest hit
                } else if (res < 0) {
                    // the exact pass tests this pair alone
                    st.fb++;
                    atomicOr(&lunc, 1ull << ow);
                    const int qi = atomicAdd(pairn, 1);
                    if (qi < pcap)
                        pairq[qi] = make_int2((int)(blk_off[b] + lchunk * 64 + ow), cand.tri[cidx] & TRI_MASK);
                    else
                        atomicOr(&lfull, 1ull << ow);
                }
            }
            __syncthreads();
        }
        const unsigned long long best = lbest[lane];
        const bool unc = (lunc >> lane) & 1ull;
        const bool full = (lfull >> lane) & 1ull;
        if (active) {
            const int64_t pos = (int64_t)blk_off[b] + li;
            if (pos >= 0 && pos < cap) {
                if (ncc == 1) {  // this task holds every candidate of the link
                    link_cell[pos] = (int32_t)(64 * b + t);
                    link_dir[pos] = (uint8_t)k;
                    link_q[pos] = key_q(best);
                    link_tri[pos] = key_tri(best);
                    if (unc) {  // the exact pass folds its pairs into this key
                        keys[pos] = best;
                        enqueue_fix(fixq, fixn, cap, pos, full);
                    }
                } else {
                    if (cchunk == 0) {
                        link_cell[pos] = (int32_t)(64 * b + t);
                        link_dir[pos] = (uint8_t)k;
                    }
                    if (best != KEY_MISS) atomicMin(&keys[pos], best);
                    // bit 0: queued; bit 1: redo over all candidates
                    if (unc && (atomicOr(&mark[pos], 1 | (full ? 2 : 0)) & 1) == 0) enqueue_fix(fixq, fixn, cap, pos, false);
                }
            }
        }
        if (pf_task >= 0 && !pf_vid_ok) {  // uniform
            if (lane < pf_n && (unsigned)pf_tri < (unsigned)m.nt) {
                pf_v0 = m.tris[3 * (int64_t)pf_tri];
                pf_v1 = m.tris[3 * (int64_t)pf_tri + 1];
                pf_v2 = m.tris[3 * (int64_t)pf_tri + 2];
            }
            pf_vid_ok = true;
        }
    }
    if (stats) {
        wave_count(&stats[GEO_STAT_F32_TO_F64], st.fb);
        wave_count(&stats[GEO_STAT_T_F64], st.t64);
        wave_count(&stats[GEO_STAT_STAGED], st.staged);
        wave_count(&stats[GEO_STAT_PAIRS], st.pairs);
        if (threadIdx.x == 0 && st.tasks) atomicAdd((unsigned long long*)&stats[GEO_STAT_TASKS], (unsigned long long)st.tasks);
    }
}

// float32 form: 4 waves per SIMD (128 VGPRs, under 10 KB of LDS per wave)
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) k_cl_q_f32(CL_Q_PARAMS) {
    cl_q_body<float>(CL_Q_ARGS);
}

// float64 form
__global__ void __launch_bounds__(64) k_cl_q_f64(CL_Q_PARAMS) { cl_q_body<double>(CL_Q_ARGS); }

// scaled global coordinate v 2^L - 1/2 (exact), the frame of the exact pass
__device__ __forceinline__ void vert_scaled(const DevMesh& m, int vid, double s, double g[3]) {
    for (int a = 0; a < 3; a++) g[a] = load_coord(m, vid, a) * s - 0.5;
}

// Exact pass, pairs: each queued (link, triangle) pair the filters left
// undecided is tested with exact predicates (one thread per pair) and folded
// into the link's key.
__global__ void k_cl_fix_pairs(DevMesh m, DevLevel d, const int32_t* link_cell, const uint8_t* link_dir,
                               const int2* pairq, const int32_t* pairn, int64_t pcap, int64_t cap,
                               unsigned long long* keys, uint64_t* stats) {
    int64_t np = *pairn;
    if (np > pcap) np = pcap;
    const double s = ldexp(1.0, d.level);
    QStats st;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 e = pairq[i];
        const int64_t pos = e.x;
        const int tri = e.y;
        if (pos < 0 || pos >= cap || (unsigned)tri >= (unsigned)m.nt) continue;
        const int cell = link_cell[pos];
        const int64_t b = cell >> 6;
        const int t = cell & 63;
        int cx, cy, cz;
        dirvec(link_dir[pos], cx, cy, cz);
        const double X[3] = {(double)(4 * d.bcoord[3 * b] + (t & 3)), (double)(4 * d.bcoord[3 * b + 1] + ((t >> 2) & 3)),
                             (double)(4 * d.bcoord[3 * b + 2] + (t >> 4))};
        const double Y[3] = {X[0] + cx, X[1] + cy, X[2] + cz};
        double A[3], B[3], Cc[3];
        vert_scaled(m, m.tris[3 * (int64_t)tri], s, A);
        vert_scaled(m, m.tris[3 * (int64_t)tri + 1], s, B);
        vert_scaled(m, m.tris[3 * (int64_t)tri + 2], s, Cc);
        double tq;
        if (exact_seg_hit(A, B, Cc, X, Y, tq, st)) atomicMin(&keys[pos], hit_key(tq, tri));
    }
    if (stats) wave_count(&stats[GEO_STAT_EXACT], st.ex);
}

// Exact pass, links: every queued link takes q and triangle from its key;
// a link whose undecided pairs did not all fit the pair queue is first
// redone over all candidates of its block with exact predicates (one wave per
// link, lanes split the candidates).
__global__ void __launch_bounds__(64) k_cl_fix(DevMesh m, DevLevel d, const int32_t* loff, const int32_t* lval,
                                               int64_t lcap, const int32_t* link_cell, const uint8_t* link_dir,
                                               const int32_t* fixq, const int32_t* fixn, const int32_t* mark,
                                               int64_t cap, const unsigned long long* keys, float* link_q,
                                               int32_t* link_tri, uint64_t* stats) {
    int64_t nq = *fixn;
    if (nq > cap) nq = cap;
    const double s = ldexp(1.0, d.level);
    QStats st;
    for (int64_t i = blockIdx.x; i < nq; i += gridDim.x) {
        const int32_t qe = fixq[i];
        const int64_t pos = qe & ~FIX_FULL;
        if (pos >= cap) continue;
        const int cell = link_cell[pos];
        const int64_t b = cell >> 6;
        const int t = cell & 63;
        int64_t c0 = loff[b], c1 = loff[b + 1];
        if (c1 > lcap) c1 = lcap;
        if (c0 < 0) c0 = 0;
        const bool multi = c1 - c0 > CL_CAND;
        const bool full = (qe & FIX_FULL) || (multi && (mark[pos] & 2));
        unsigned long long best = keys[pos];
        if (full) {
            best = KEY_MISS;
            int cx, cy, cz;
            dirvec(link_dir[pos], cx, cy, cz);
            const double X[3] = {(double)(4 * d.bcoord[3 * b] + (t & 3)),
                                 (double)(4 * d.bcoord[3 * b + 1] + ((t >> 2) & 3)),
                                 (double)(4 * d.bcoord[3 * b + 2] + (t >> 4))};
            const double Y[3] = {X[0] + cx, X[1] + cy, X[2] + cz};
            const double slo[3] = {fmin(X[0], Y[0]), fmin(X[1], Y[1]), fmin(X[2], Y[2])};
            const double shi[3] = {fmax(X[0], Y[0]), fmax(X[1], Y[1]), fmax(X[2], Y[2])};
            // four candidates per lane and round: their triangle and vertex ids
            // are loaded together, the coordinates just before each test
            for (int64_t cb = c0 + threadIdx.x; cb < c1; cb += 256) {
                int tri[4], vid[4][3];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int64_t c = cb + 64 * u;
                    tri[u] = c < c1 ? lval[c] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    // entries of an overflowed bin are not triangle ids
                    const bool ok = (unsigned)tri[u] < (unsigned)m.nt;
#pragma unroll
                    for (int i2 = 0; i2 < 3; i2++) vid[u][i2] = ok ? m.tris[3 * (int64_t)tri[u] + i2] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (vid[u][0] < 0) continue;
                    double A[3], B[3], Cc[3];
                    vert_scaled(m, vid[u][0], s, A);
                    vert_scaled(m, vid[u][1], s, B);
                    vert_scaled(m, vid[u][2], s, Cc);
                    // boxes apart: no contact (the scaled coordinates are exact)
                    bool apart = false;
#pragma unroll
                    for (int a = 0; a < 3; a++)
                        apart |= fmax(A[a], fmax(B[a], Cc[a])) < slo[a] || fmin(A[a], fmin(B[a], Cc[a])) > shi[a];
                    if (apart) continue;
                    double tq;
                    if (exact_seg_hit(A, B, Cc, X, Y, tq, st)) {
                        const unsigned long long kk = hit_key(tq, tri[u]);
                        best = kk < best ? kk : best;
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long other = __shfl_xor(best, o, 64);
                best = other < best ? other : best;
            }
        }
        if (threadIdx.x == 0) {
            link_q[pos] = key_q(best);
            link_tri[pos] = key_tri(best);
            st.tq++;
        }
    }
    if (stats) {
        wave_count(&stats[GEO_STAT_EXACT], st.ex);
        wave_count(&stats[GEO_STAT_LINKS_EXACT], st.tq);
    }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// capacity of the exact pass's pair queue: pairs beyond it send their link to
// a redo over all candidates
inline int64_t pair_cap(int64_t cap) { return cap < 1 ? 1 : (cap < (1 << 22) ? cap : (1 << 22)); }

size_t geo_cutlinks_ws_bytes(int64_t nb, int64_t cap) {
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    return 2 * al(sizeof(int32_t) * (size_t)nb) + 2 * al(sizeof(int32_t) * ((size_t)nb + 1)) +
           al(geo_scan_partials_bytes(nb)) + al(sizeof(uint32_t) * 64 * (size_t)nb) +
           al(sizeof(unsigned long long) * c) + 2 * al(sizeof(int32_t) * c) + al(3 * sizeof(int32_t)) +
           al(sizeof(int2) * (size_t)pair_cap(cap)) + al(sizeof(int32_t) * (size_t)nb);
}

int launch_cutlinks(const DevMesh& m, const DevLevel& d, const geo_bins* rows, const geo_bins* links, int lattice,
                    int precision, uint32_t* link_mask, int64_t cap, int64_t* d_nlinks, int32_t* link_cell,
                    uint8_t* link_dir, float* link_q, int32_t* link_tri, uint64_t* d_stats, void* ws,
                    size_t ws_bytes, hipStream_t s) {
    const int64_t nb = d.nblocks;
    if (ws_bytes < geo_cutlinks_ws_bytes(nb, cap)) return GEO_ERR_WORKSPACE;
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    char* p = static_cast<char*>(ws);
    int32_t* blk_cnt = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)nb);
    int32_t* blk_off = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nb + 1));
    int32_t* ntask = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)nb);
    int32_t* task_off = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nb + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    p += al(geo_scan_partials_bytes(nb));
    uint32_t* ws_mask = reinterpret_cast<uint32_t*>(p);
    p += al(sizeof(uint32_t) * 64 * (size_t)nb);
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(p);
    p += al(sizeof(unsigned long long) * c);
    int32_t* mark = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * c);
    int32_t* fixq = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * c);
    // fixn[0]: queued links, fixn[1]: queued pairs, fixn[2]: listed multi-chunk blocks
    int32_t* fixn = reinterpret_cast<int32_t*>(p);
    int32_t* pairn = fixn + 1;
    int32_t* mcount = fixn + 2;
    p += al(3 * sizeof(int32_t));
    const int64_t pcap = pair_cap(cap);
    int2* pairq = reinterpret_cast<int2*>(p);
    p += al(sizeof(int2) * (size_t)pcap);
    int32_t* mlist = reinterpret_cast<int32_t*>(p);
    if (nb == 0) return geo_fill_u64(reinterpret_cast<uint64_t*>(d_nlinks), 0, 1, s);
    uint32_t* wmask = link_mask ? link_mask : ws_mask;
    const int64_t nchunk = (nb + 63) / 64;
    const unsigned g = (unsigned)(nchunk < 32768 ? nchunk : 32768);
    k_cl_mask<<<g, 64, 0, s>>>(d, rows->off, rows->val, rows->cap, links->off, lattice, wmask, link_mask ? 1 : 0,
                               blk_cnt, fixn);
    GEO_LAUNCH_CHECK();
    // exact link count (the table's offsets are int32)
    int rc = geo_sum_i32(blk_cnt, nb, d_nlinks, s);
    if (rc != GEO_OK) return rc;
    if ((rc = geo_scan_exclusive(blk_cnt, blk_off, nb, partials, s)) != GEO_OK) return rc;
    const unsigned gb = (unsigned)((nb + 255) / 256 < 65536 ? (nb + 255) / 256 : 65536);
    k_cl_ntask<<<gb, 256, 0, s>>>(nb, blk_off, links->off, links->cap, ntask, mlist, mcount);
    GEO_LAUNCH_CHECK();
    if ((rc = geo_scan_exclusive(ntask, task_off, nb, partials, s)) != GEO_OK) return rc;
    if (cap > 0) {
        k_cl_multi<<<4096, 256, 0, s>>>(mlist, mcount, blk_off, cap, 0, keys, mark, link_q, link_tri);
        GEO_LAUNCH_CHECK();
    }
    // tasks are split into one contiguous range per workgroup; finer ranges
    // balance better; empty ranges exit at once
    const unsigned gq = 65536;
    kt_record(GEO_KT_CUTLINKS_Q, s, false);
    if (precision == GEO_PREC_F32_FALLBACK)
        k_cl_q_f32<<<gq, 64, 0, s>>>(m, d, wmask, links->off, links->val, links->cap, blk_off, task_off, cap,
                                        link_cell, link_dir, link_q, link_tri, keys, mark, fixq, fixn, pairq, pairn, pcap,
                                    d_stats);
    else
        k_cl_q_f64<<<gq, 64, 0, s>>>(m, d, wmask, links->off, links->val, links->cap, blk_off, task_off, cap,
                                         link_cell, link_dir, link_q, link_tri, keys, mark, fixq, fixn, pairq, pairn, pcap,
                                    d_stats);
    kt_record(GEO_KT_CUTLINKS_Q, s, true);
    GEO_LAUNCH_CHECK();
    if (cap > 0) {
        k_cl_multi<<<4096, 256, 0, s>>>(mlist, mcount, blk_off, cap, 1, keys, mark, link_q, link_tri);
        k_cl_fix_pairs<<<256, 256, 0, s>>>(m, d, link_cell, link_dir, pairq, pairn, pcap, cap, keys, d_stats);
        k_cl_fix<<<4096, 64, 0, s>>>(m, d, links->off, links->val, links->cap, link_cell, link_dir, fixq, fixn, mark,
                                     cap, keys, link_q, link_tri, d_stats);
        GEO_LAUNCH_CHECK();
    }
    return GEO_OK;
}
