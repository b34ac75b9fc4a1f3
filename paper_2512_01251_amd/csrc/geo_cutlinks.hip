// Cut links of one level (Methodology, "Boundary Cell Identification",
// "Memory Allocations for Boundary Cells", "Link-Length Computation", Eq. 2).
//
//  k_cl_mask  one wave per block: the solid flags of the block's one-cell
//             halo (6^3 centres) come from the ROWS bins of 36 row lines, so a
//             neighbour centre is classified even where its block does not
//             exist; lane t then forms the link mask of cell t and the wave
//             reduces the block's link count.
//  scan       block counts -> offsets: the table is laid out in the order
//             (block, t, k) without atomics (scan-ordered compaction).
//  k_cl_q     tasks of (64 links x 64 candidates) of a block: the candidates
//             (LINKS bins) are staged in LDS with certified plane coefficients;
//             box tests list the (link, candidate) pairs worth testing, the
//             pairs are flattened over the wave and tested with sign filters in
//             the form's precision, the hit parameter comes from the float64
//             plane, and each link keeps its nearest hit (the paper's minimum
//             over binned faces) through a 64-bit atomic min on a packed
//             (t, triangle) key.  A link with a pair whose signs the filters
//             cannot certify is queued.
//  k_cl_fix   one wave per queued link: exact tests against all candidates.
//  k_cl_final keys -> q and hit triangle.
#include <type_traits>

#include "geo_internal.h"

namespace {

constexpr int CL_CAND = 64;  // candidates staged per round

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

// 6-bit solid vector of centres x0-1 .. x0+4 of one row line
__device__ __forceinline__ unsigned halo_bits(const int32_t* off, const int32_t* val, int64_t cap, int64_t line,
                                              int xm1, int nx) {
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
                int n = v - xm1;
                n = n < 0 ? 0 : (n > 6 ? 6 : n);
                par ^= (1u << n) - 1u;
            } else {
                int a = (v & 0x7fff) - xm1, b = ((v >> 15) & 0x7fff) - xm1;
                a = a < 0 ? 0 : a;
                b = b > 5 ? 5 : b;
                if (a <= b) surf |= ((1u << (b + 1)) - 1u) & ~((1u << a) - 1u);
            }
        }
    }
    unsigned r = (par | surf) & 0x3fu;
    // centres outside the domain are fluid
    for (int p = 0; p < 6; p++) {
        const int x = xm1 + p;
        if (x < 0 || x >= nx) r &= ~(1u << p);
    }
    return r;
}

// link masks of block b: lanes 0..35 classify the 36 halo row lines into
// LDS, then lane t forms the mask of cell t (0 for solid cells)
__device__ __forceinline__ uint32_t block_link_mask(const DevLevel& d, const int32_t* off, const int32_t* val,
                                                    int64_t cap, uint32_t dirs, int64_t b, unsigned* halo) {
    const int L = d.level;
    const int nx = d.n0[0] << L, ny = d.n0[1] << L, nz = d.n0[2] << L;
    const int lane = threadIdx.x;
    const int bx = d.bcoord[3 * b], by = d.bcoord[3 * b + 1], bz = d.bcoord[3 * b + 2];
    __syncthreads();
    if (lane < 36) {
        const int J = lane % 6 - 1, K = lane / 6 - 1;
        const int j = 4 * by + J, k = 4 * bz + K;
        unsigned bits = 0;
        if (j >= 0 && j < ny && k >= 0 && k < nz)
            bits = halo_bits(off, val, cap, (int64_t)j + (int64_t)ny * k, 4 * bx - 1, nx);
        halo[lane] = bits;
    }
    __syncthreads();
    const int I = lane & 3, J = (lane >> 2) & 3, K = lane >> 4;
    // 27-bit neighbourhood word, bit (cx+1) + 3 (cy+1) + 9 (cz+1)
    uint32_t nb = 0;
#pragma unroll
    for (int dz = 0; dz < 3; dz++)
#pragma unroll
        for (int dy = 0; dy < 3; dy++) nb |= ((halo[(J + dy) + 6 * (K + dz)] >> I) & 7u) << (3 * dy + 9 * dz);
    return ((nb >> 13) & 1u) ? 0u : (nb & dirs);
}

__global__ void __launch_bounds__(64) k_cl_mask(DevLevel d, const int32_t* off, const int32_t* val, int64_t cap,
                                                const int32_t* loff, int lattice, uint32_t* link_mask,
                                                int32_t* blk_cnt) {
    __shared__ unsigned halo[36];
    const uint32_t dirs = lattice_dirs(lattice);
    const int lane = threadIdx.x;
    const int64_t nchunks = (d.nblocks + 63) / 64;
    // chunks of 64 blocks: one coalesced read of their candidate counts, then
    // only the blocks with candidates are classified, one per wave step
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
            const int64_t b = b0 + i;
            const uint32_t m = block_link_mask(d, off, val, cap, dirs, b, halo);
            if (link_mask) link_mask[64 * b + lane] = m;
            int c = __popc(m);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            if (lane == 0) blk_cnt[b] = c;
        }
        if (link_mask) {
            unsigned long long empty = __ballot(inb && !has);
            while (empty) {  // uniform
                const int i = __ffsll(empty) - 1;
                empty &= empty - 1;
                link_mask[64 * (b0 + i) + lane] = 0;
            }
        }
    }
}

// ------------------------------------------------------------------------
// candidate records
// ------------------------------------------------------------------------
enum { C_SLOW = 2 };

// The float64 plane used for hit parameters: a copy for the float32 form,
// the candidate's own plane for the float64 form (no second copy in LDS).
template <typename R>
struct PlaneF64 {
    double n_[3], off_;
    __device__ __forceinline__ void set_n(int a, double v) { n_[a] = v; }
    __device__ __forceinline__ void set_off(double v) { off_ = v; }
    template <typename C> __device__ __forceinline__ double n(const C&, int a) const { return n_[a]; }
    template <typename C> __device__ __forceinline__ double off(const C&) const { return off_; }
};
template <>
struct PlaneF64<double> {
    __device__ __forceinline__ void set_n(int, double) {}
    __device__ __forceinline__ void set_off(double) {}
    template <typename C> __device__ __forceinline__ double n(const C& c, int a) const { return c.n[a]; }
    template <typename C> __device__ __forceinline__ double off(const C& c) const { return c.off; }
};

template <typename R>
struct Cand {
    R v[3][3];      // vertices in the block frame (centres of the block at 0..3)
    R n[3];         // plane normal (b - a) x (c - a)
    R off;          // n . a
    R bound;        // |(off - n.P) - orient3d(a,b,c,P)| <= bound for P in [-1,4]^3
    R delta;        // rounding bound of v
    PlaneF64<R> p64;  // float64 plane for the hit parameter (the float64 form's own plane)
    int tri;
};

// bounding box of a staged candidate (float, rounded outward) with flags in lo.w
struct CBox {
    float4 lo;  // xyz: lower corner, w: flags (as float)
    float4 hi;
};

// scaled global coordinate v 2^L - 1/2 (exact)
__device__ __forceinline__ void vert_scaled(const DevMesh& m, int vid, double s, double g[3]) {
    for (int a = 0; a < 3; a++) g[a] = load_coord(m, vid, a) * s - 0.5;
}

__device__ __forceinline__ float down_f(double x) {
    float f = (float)x;
    return (double)f > x ? nextafterf(f, -1e30f) : f;
}
__device__ __forceinline__ float up_f(double x) {
    float f = (float)x;
    return (double)f < x ? nextafterf(f, 1e30f) : f;
}

// Stage one candidate: local float64 coordinates (exact unless flagged slow),
// certified plane coefficients in R, float64 plane, float box.
template <typename R>
__device__ void stage_cand(const DevMesh& m, int L, int tri, const int vid[3], const int b0[3], Cand<R>& C,
                           CBox& B) {
    const double s = ldexp(1.0, L);
    double v[3][3];
    bool exact = true;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        double g[3];
        vert_scaled(m, vid[i], s, g);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double o = (double)b0[a];
            const double sum = g[a] - o;
            const double bb = sum - g[a];
            const double err = (g[a] - (sum - bb)) + (-o - bb);
            if (err != 0.0) exact = false;
            v[i][a] = sum;
        }
    }
    C.tri = tri;
    int flags = exact ? 0 : C_SLOW;
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    double n[3], perm[3];
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    perm[0] = fabs(e1[1] * e2[2]) + fabs(e1[2] * e2[1]);
    perm[1] = fabs(e1[2] * e2[0]) + fabs(e1[0] * e2[2]);
    perm[2] = fabs(e1[0] * e2[1]) + fabs(e1[1] * e2[0]);
    const double u64 = 1.1102230246251565e-16;
    // possibly zero-area: decided exactly by the deferred exact pass
    if (fabs(n[0]) <= 5 * u64 * perm[0] && fabs(n[1]) <= 5 * u64 * perm[1] && fabs(n[2]) <= 5 * u64 * perm[2])
        flags |= C_SLOW;
    const double off = n[0] * v[0][0] + n[1] * v[0][1] + n[2] * v[0][2];
    double sna = 0, n1 = 0, ena = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        sna += fabs(n[a] * v[0][a]);
        n1 += fabs(n[a]);
        ena += 5 * u64 * perm[a] * (fabs(v[0][a]) + 4.0);
    }
#pragma unroll
    for (int a = 0; a < 3; a++) C.p64.set_n(a, n[a]);
    C.p64.set_off(off);
    if constexpr (std::is_same<R, float>::value) {
        const double u32 = 5.9604644775390625e-8;
        float n32[3];
#pragma unroll
        for (int a = 0; a < 3; a++) n32[a] = (float)n[a];
        const float off32 = (float)off;
        const double n321 = fabs((double)n32[0]) + fabs((double)n32[1]) + fabs((double)n32[2]);
        double bound = u32 * fabs(off) + 3.01 * u64 * sna + ena + 4 * u32 * n1 + 4.01 * u32 * (fabs((double)off32) + 4 * n321);
        bound = bound * 1.01 + 1e-30;
#pragma unroll
        for (int a = 0; a < 3; a++) C.n[a] = n32[a];
        C.off = off32;
        C.bound = up_f(bound);
        double dl = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                C.v[i][a] = (float)v[i][a];
                dl = fmax(dl, fabs((double)C.v[i][a] - v[i][a]));
            }
        C.delta = up_f(dl);
    } else {
        double bound = 3.01 * u64 * sna + ena + 4.01 * u64 * (fabs(off) + 4 * n1);
        bound = bound * 1.01 + 1e-300;
#pragma unroll
        for (int a = 0; a < 3; a++) C.n[a] = n[a];
        C.off = off;
        C.bound = bound;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int a = 0; a < 3; a++) C.v[i][a] = v[i][a];
        C.delta = 0;
    }
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = down_f(fmin(v[0][a], fmin(v[1][a], v[2][a])));
        hi[a] = up_f(fmax(v[0][a], fmax(v[1][a], v[2][a])));
    }
    // inexact local coordinates: no box rejection for this candidate
    if (!exact) {
#pragma unroll
        for (int a = 0; a < 3; a++) { lo[a] = -1e30f; hi[a] = 1e30f; }
    }
    B.lo = make_float4(lo[0], lo[1], lo[2], (float)flags);
    // the filtered test never decides such a candidate
    if (flags & C_SLOW) C.bound = (R)INFINITY;
    B.hi = make_float4(hi[0], hi[1], hi[2], 0.0f);
}

struct QStats {
    unsigned fb = 0, ex = 0, tq = 0, staged = 0, pairs = 0, tasks = 0;
};

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

// fast test against a staged candidate: 0 miss, 1 hit (t, terr), -1 not certain
template <typename R>
__device__ __forceinline__ int fast_test(const Cand<R>& C, const R X[3], const R Y[3], R& t, R& terr) {
    const R sX = C.off - C.n[0] * X[0] - C.n[1] * X[1] - C.n[2] * X[2];
    const R sY = C.off - C.n[0] * Y[0] - C.n[1] * Y[1] - C.n[2] * Y[2];
    const R B = C.bound;
    const bool cx = geo_fabs(sX) > B, cy = geo_fabs(sY) > B;
    if (cx && cy && ((sX > 0) == (sY > 0))) return 0;
    if (!cx || !cy) return -1;
    const int e0 = orient3d_filter<R>(X, Y, C.v[0], C.v[1], C.delta);
    const int e1 = orient3d_filter<R>(X, Y, C.v[1], C.v[2], C.delta);
    const int e2 = orient3d_filter<R>(X, Y, C.v[2], C.v[0], C.delta);
    if (e0 == 0 || e1 == 0 || e2 == 0) {
        // a certain miss needs only one pair of strictly opposite signs
        const bool pos = e0 > 0 || e1 > 0 || e2 > 0, neg = e0 < 0 || e1 < 0 || e2 < 0;
        if (pos && neg) return 0;
        return -1;
    }
    if (!((e0 > 0 && e1 > 0 && e2 > 0) || (e0 < 0 && e1 < 0 && e2 < 0))) return 0;
    const R D = sX - sY;
    t = sX / D;
    terr = B * R(2) / geo_fabs(D) + R(4) * Unit<R>::u;
    return 1;
}

// Flattened (link, candidate) pairs, per round up to MAXC per link.  The
// float32 form packs the link's lattice position and direction into the
// entry (one LDS read per pair fewer) and takes 8 per round, keeping the same
// LDS size; the float64 form, with larger candidates in LDS, takes 16.
template <typename R> struct FlatCfg {
    using T = uint32_t;
    static constexpr int MAXC = 8;
    static constexpr bool packed = true;
};
template <> struct FlatCfg<double> {
    using T = uint16_t;
    static constexpr int MAXC = 16;
    static constexpr bool packed = false;
};

// packed nearest-hit key: t in [0,1] as 37-bit fixed point, then the
// triangle id (27 bits); the minimum key is the nearest hit, ties (equal t to
// 2^-37) going to the smallest triangle id
constexpr double Q37 = 137438953471.0;  // 2^37 - 1
constexpr unsigned long long KEY_MISS = ~0ull;
__device__ __forceinline__ unsigned long long hit_key(double t, int tri) {
    const double c = fmin(fmax(t, 0.0), 1.0);
    return ((unsigned long long)(c * Q37 + 0.5) << 27) | (unsigned long long)(unsigned)tri;
}

// tasks per block: ceil(links / 64) x ceil(candidates / 64)
__global__ void k_cl_ntask(int64_t nb, const int32_t* blk_off, const int32_t* loff, int64_t lcap, int32_t* ntask) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const int n = blk_off[b + 1] - blk_off[b];
        int64_t c0 = loff[b], c1 = loff[b + 1];
        if (c1 > lcap) c1 = lcap;
        if (c0 < 0) c0 = 0;
        const int nc = c1 > c0 ? (int)(c1 - c0) : 0;
        ntask[b] = n > 0 ? ((n + 63) / 64) * (nc > 0 ? (nc + CL_CAND - 1) / CL_CAND : 1) : 0;
    }
}

__global__ void k_cl_fill_keys(unsigned long long* keys, int32_t* mark, const int64_t* d_n, int64_t cap) {
    int64_t n = *d_n;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = KEY_MISS;
        mark[i] = 0;
    }
}

__global__ void k_cl_final(const unsigned long long* keys, const int64_t* d_n, int64_t cap, float* link_q,
                           int32_t* link_tri) {
    int64_t n = *d_n;
    if (n > cap) n = cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = keys[i];
        if (k == KEY_MISS) {
            link_q[i] = -1.0f;
            link_tri[i] = -1;
        } else {
            link_q[i] = (float)((double)(k >> 27) / Q37);
            link_tri[i] = (int32_t)(k & ((1ull << 27) - 1));
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

template <typename R>
__global__ void __launch_bounds__(64) k_cl_q(DevMesh m, DevLevel d, const int32_t* roff, const int32_t* rval,
                                             int64_t rcap, const int32_t* loff, const int32_t* lval, int64_t lcap,
                                             int lattice, const int32_t* blk_off, const int32_t* task_off,
                                             int64_t cap, int32_t* link_cell, uint8_t* link_dir,
                                             unsigned long long* keys, int32_t* mark, int32_t* fixq,
                                             int32_t* fixn, uint64_t* stats) {
    __shared__ Cand<R> cand[CL_CAND];
    // box test as bit masks over the staged candidates: for axis a and lattice
    // position j in -1..4, bmask[12a + 1 + j] holds the candidates with
    // hi_a >= j and bmask[12a + 7 + j] those with lo_a <= j
    __shared__ unsigned long long bmask[36];
    __shared__ uint32_t smask[64];
    __shared__ int spre[65];
    __shared__ unsigned halo[36];
    // flattened pairs: owner lane | candidate slot << 6 (| link << 12 when packed)
    __shared__ typename FlatCfg<R>::T flat[64 * FlatCfg<R>::MAXC];
    __shared__ unsigned long long lbest[64];  // nearest hit of each lane's link (packed key)
    __shared__ int sk[64];                    // link of each lane: t | (d + 1) << 8 (2 bits per axis)
    const int L = d.level;
    const int lane = threadIdx.x;
    const uint32_t dirs = lattice_dirs(lattice);
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
    // prefetch of the next staging unit: candidate triangle (at staging) and
    // its vertex ids (at the end of the task), so staging waits for one load
    int pf_task = -1, pf_n = 0;  // first task and candidate count of the prefetched unit
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
        // a block's tasks run candidate chunk by candidate chunk, so that
        // consecutive link chunks reuse the staged candidates
        const int nlc = (n + 63) / 64;
        const int local = task - task_off[b];
        const int cchunk = local / nlc, lchunk = local % nlc;
        const int b0[3] = {4 * d.bcoord[3 * b], 4 * d.bcoord[3 * b + 1], 4 * d.bcoord[3 * b + 2]};
        st.tasks++;
        if (b != b_prev) {  // uniform
            const uint32_t mk = block_link_mask(d, roff, rval, rcap, dirs, b, halo);
            smask[lane] = mk;
            const int c = __popc(mk), incl = wave_incl_scan(c);
            spre[lane] = incl - c;
            if (lane == 63) spre[64] = incl;
            b_prev = b;
        }
        const int cb = cchunk * CL_CAND;
        const int nstage = nc - cb < CL_CAND ? (nc - cb > 0 ? nc - cb : 0) : CL_CAND;
        if (b != staged_b || cchunk != staged_c) {  // uniform
            staged_b = b;
            staged_c = cchunk;
            __syncthreads();
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
                CBox bx;
                stage_cand<R>(m, L, tri, vid, b0, cand[lane], bx);
                blo[0] = bx.lo.x; blo[1] = bx.lo.y; blo[2] = bx.lo.z;
                bhi[0] = bx.hi.x; bhi[1] = bx.hi.y; bhi[2] = bx.hi.z;
                st.staged++;
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
                    const unsigned long long A = __ballot(bhi[a] >= (float)(j - 1));
                    const unsigned long long B = __ballot(blo[a] <= (float)(j - 1));
                    if (lane == 12 * a + j) mine = A;
                    if (lane == 12 * a + 6 + j) mine = B;
                }
            if (lane < 36) bmask[lane] = mine;
        }
        __syncthreads();
        const int li = lchunk * 64 + lane;
        const bool active = li < n;
        int t = 0, k = 13;
        if (active) {
            int lo = 0, hi = 63;  // largest t with spre[t] <= li
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (spre[mid] <= li) lo = mid;
                else hi = mid - 1;
            }
            t = lo;
            int r = li - spre[t];
            uint32_t mm = smask[t];
            for (int q = 0; q < r; q++) mm &= mm - 1u;
            k = __ffs(mm) - 1;
        }
        int cx, cy, cz;
        dirvec(k, cx, cy, cz);
        const int myk = t | ((cx + 1) << 8) | ((cy + 1) << 10) | ((cz + 1) << 12);
        if (!FlatCfg<R>::packed) sk[lane] = myk;
        const int slo[3] = {geo_min(t & 3, (t & 3) + cx), geo_min((t >> 2) & 3, ((t >> 2) & 3) + cy),
                            geo_min(t >> 4, (t >> 4) + cz)};
        const int shi[3] = {geo_max(t & 3, (t & 3) + cx), geo_max((t >> 2) & 3, ((t >> 2) & 3) + cy),
                            geo_max(t >> 4, (t >> 4) + cz)};
        const int64_t lbase = (int64_t)blk_off[b] + lchunk * 64;
        lbest[lane] = KEY_MISS;
        // phase 1: candidates whose box meets the link's segment box
        unsigned long long pm = 0;
        if (active) {
            pm = bmask[1 + slo[0]] & bmask[7 + shi[0]] & bmask[13 + slo[1]] & bmask[19 + shi[1]] &
                 bmask[25 + slo[2]] & bmask[31 + shi[2]];
        }
        while (__any(pm != 0)) {  // uniform
            // flatten up to MAXC pairs per link over the wave
            const int pc = __popcll(pm);
            const int cnt = pc < FlatCfg<R>::MAXC ? pc : FlatCfg<R>::MAXC;
            const int inc2 = wave_incl_scan(cnt);
            const int pbase = inc2 - cnt;
            for (int j = 0; j < cnt; j++) {
                const int slot = __ffsll(pm) - 1;
                pm &= pm - 1;
                flat[pbase + j] = (typename FlatCfg<R>::T)(lane | (slot << 6) | (FlatCfg<R>::packed ? myk << 12 : 0));
            }
            const int P = __shfl(inc2, 63, 64);
            __syncthreads();
            st.pairs += cnt;
            // phase 2: one pair per lane
            for (int p = lane; p < P; p += 64) {
                const int fe = flat[p];
                const int ow = fe & 63;
                const int cidx = (fe >> 6) & 63;
                const int tk = FlatCfg<R>::packed ? (int)(fe >> 12) : sk[ow];
                const int ox = ((tk >> 8) & 3) - 1, oy = ((tk >> 10) & 3) - 1, oz = ((tk >> 12) & 3) - 1;
                const int Xi[3] = {tk & 3, (tk >> 2) & 3, (tk >> 4) & 3};
                const R X[3] = {(R)Xi[0], (R)Xi[1], (R)Xi[2]};
                const R Y[3] = {(R)(Xi[0] + ox), (R)(Xi[1] + oy), (R)(Xi[2] + oz)};
                const Cand<R>& C = cand[cidx];
                R tr = 0, terr = 0;
                const int res = fast_test<R>(C, X, Y, tr, terr);
                unsigned long long kk = KEY_MISS;
                if (res == 1) {
                    // hit parameter from the float64 plane
                    const double n0 = C.p64.n(C, 0), n1 = C.p64.n(C, 1), n2 = C.p64.n(C, 2);
                    const double sX = C.p64.off(C) - n0 * Xi[0] - n1 * Xi[1] - n2 * Xi[2];
                    const double nd = n0 * ox + n1 * oy + n2 * oz;
                    kk = hit_key(sX / nd, C.tri);
                } else if (res < 0) {
                    // not certain: the link is redone exactly by the deferred pass
                    st.fb++;
                    const int64_t pos = lbase + ow;
                    if (pos >= 0 && pos < cap && atomicExch(&mark[pos], 1) == 0) {
                        const int qi = atomicAdd(fixn, 1);
                        if (qi < cap) fixq[qi] = (int32_t)pos;
                    }
                }
                if (kk != KEY_MISS) atomicMin(&lbest[ow], kk);  // each link keeps its nearest hit
            }
            __syncthreads();
        }
        const unsigned long long best = lbest[lane];
        if (active) {
            const int64_t pos = lbase + lane;
            if (pos >= 0 && pos < cap) {
                if (cchunk == 0) {
                    link_cell[pos] = (int32_t)(64 * b + t);
                    link_dir[pos] = (uint8_t)k;
                }
                if (best != KEY_MISS) atomicMin(&keys[pos], best);
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
        wave_count(&stats[GEO_STAT_STAGED], st.staged);
        wave_count(&stats[GEO_STAT_PAIRS], st.pairs);
        if (threadIdx.x == 0 && st.tasks) atomicAdd((unsigned long long*)&stats[GEO_STAT_TASKS], (unsigned long long)st.tasks);
    }
}

// Deferred exact pass: each queued link is tested against all candidates of
// its block with exact predicates (one wave per link, lanes split the
// candidates); the result is folded into its key.
__global__ void __launch_bounds__(64) k_cl_fix(DevMesh m, DevLevel d, const int32_t* loff, const int32_t* lval,
                                               int64_t lcap, const int32_t* link_cell, const uint8_t* link_dir,
                                               const int32_t* fixq, const int32_t* fixn, int64_t cap,
                                               unsigned long long* keys, uint64_t* stats) {
    int64_t nq = *fixn;
    if (nq > cap) nq = cap;
    const double s = ldexp(1.0, d.level);
    QStats st;
    for (int64_t i = blockIdx.x; i < nq; i += gridDim.x) {
        const int64_t pos = fixq[i];
        const int cell = link_cell[pos];
        const int64_t b = cell >> 6;
        const int t = cell & 63;
        int cx, cy, cz;
        dirvec(link_dir[pos], cx, cy, cz);
        const double X[3] = {(double)(4 * d.bcoord[3 * b] + (t & 3)), (double)(4 * d.bcoord[3 * b + 1] + ((t >> 2) & 3)),
                             (double)(4 * d.bcoord[3 * b + 2] + (t >> 4))};
        const double Y[3] = {X[0] + cx, X[1] + cy, X[2] + cz};
        int64_t c0 = loff[b], c1 = loff[b + 1];
        if (c1 > lcap) c1 = lcap;
        if (c0 < 0) c0 = 0;
        const double slo[3] = {fmin(X[0], Y[0]), fmin(X[1], Y[1]), fmin(X[2], Y[2])};
        const double shi[3] = {fmax(X[0], Y[0]), fmax(X[1], Y[1]), fmax(X[2], Y[2])};
        unsigned long long best = KEY_MISS;
        // four candidates per lane and round: their triangle and vertex ids are
        // loaded together, the coordinates just before each test
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
                for (int i = 0; i < 3; i++) vid[u][i] = ok ? m.tris[3 * (int64_t)tri[u] + i] : -1;
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
        if (threadIdx.x == 0 && best != KEY_MISS) atomicMin(&keys[pos], best);
        if (threadIdx.x == 0) st.tq++;
    }
    if (stats) {
        wave_count(&stats[GEO_STAT_EXACT], st.ex);
        wave_count(&stats[GEO_STAT_LINKS_EXACT], st.tq);
    }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t geo_cutlinks_ws_bytes(int64_t nb, int64_t cap) {
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    return 2 * al(sizeof(int32_t) * (size_t)nb) + 2 * al(sizeof(int32_t) * ((size_t)nb + 1)) +
           al(geo_scan_partials_bytes(nb)) + al(sizeof(unsigned long long) * c) + 2 * al(sizeof(int32_t) * c) +
           al(sizeof(int32_t));
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
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(p);
    p += al(sizeof(unsigned long long) * c);
    int32_t* mark = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * c);
    int32_t* fixq = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * c);
    int32_t* fixn = reinterpret_cast<int32_t*>(p);
    if (nb == 0) return geo_fill_u64(reinterpret_cast<uint64_t*>(d_nlinks), 0, 1, s);
    const int64_t nchunk = (nb + 63) / 64;
    const unsigned g = (unsigned)(nchunk < 32768 ? nchunk : 32768);
    k_cl_mask<<<g, 64, 0, s>>>(d, rows->off, rows->val, rows->cap, links->off, lattice, link_mask, blk_cnt);
    GEO_LAUNCH_CHECK();
    // exact link count (the table's offsets are int32)
    int rc = geo_sum_i32(blk_cnt, nb, d_nlinks, s);
    if (rc != GEO_OK) return rc;
    if ((rc = geo_scan_exclusive(blk_cnt, blk_off, nb, partials, s)) != GEO_OK) return rc;
    const unsigned gb = (unsigned)((nb + 255) / 256 < 65536 ? (nb + 255) / 256 : 65536);
    k_cl_ntask<<<gb, 256, 0, s>>>(nb, blk_off, links->off, links->cap, ntask);
    GEO_LAUNCH_CHECK();
    if ((rc = geo_scan_exclusive(ntask, task_off, nb, partials, s)) != GEO_OK) return rc;
    if (cap > 0) {
        k_cl_fill_keys<<<8192, 256, 0, s>>>(keys, mark, d_nlinks, cap);
        if ((rc = geo_fill_i32(fixn, 0, 1, s)) != GEO_OK) return rc;
        GEO_LAUNCH_CHECK();
    }
    // tasks are split into one contiguous range per workgroup; finer ranges
    // balance better (7.2M triangles: 16384 -> 65536 workgroups took the
    // float32 kernel from 4.01 to 3.78 ms); empty ranges exit at once
    const unsigned gq = 65536;
    kt_record(GEO_KT_CUTLINKS_Q, s, false);
    if (precision == GEO_PREC_F32_FALLBACK)
        k_cl_q<float><<<gq, 64, 0, s>>>(m, d, rows->off, rows->val, rows->cap, links->off, links->val, links->cap,
                                        lattice, blk_off, task_off, cap, link_cell, link_dir, keys, mark, fixq, fixn,
                                        d_stats);
    else
        k_cl_q<double><<<gq, 64, 0, s>>>(m, d, rows->off, rows->val, rows->cap, links->off, links->val, links->cap,
                                         lattice, blk_off, task_off, cap, link_cell, link_dir, keys, mark, fixq, fixn,
                                         d_stats);
    kt_record(GEO_KT_CUTLINKS_Q, s, true);
    GEO_LAUNCH_CHECK();
    if (cap > 0) {
        k_cl_fix<<<4096, 64, 0, s>>>(m, d, links->off, links->val, links->cap, link_cell, link_dir, fixq, fixn, cap,
                                     keys, d_stats);
        k_cl_final<<<8192, 256, 0, s>>>(keys, d_nlinks, cap, link_q, link_tri);
        GEO_LAUNCH_CHECK();
    }
    return GEO_OK;
}
