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
//  k_cl_q     one wave per block: the block's candidate triangles (LINKS bins)
//             are staged in LDS with certified plane coefficients; lane i
//             takes link i, tests it against every candidate and keeps the
//             nearest hit (the paper's minimum over binned faces).  Signs that
//             the fast precision cannot certify are recomputed in float64 and
//             then exactly.
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
    unsigned par = 0, surf = 0;
    for (int64_t e = e0; e < e1; e++) {
        const int32_t v = val[e];
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
    unsigned r = (par | surf) & 0x3fu;
    // centres outside the domain are fluid
    for (int p = 0; p < 6; p++) {
        const int x = xm1 + p;
        if (x < 0 || x >= nx) r &= ~(1u << p);
    }
    return r;
}

__global__ void __launch_bounds__(64) k_cl_mask(DevLevel d, const int32_t* off, const int32_t* val, int64_t cap,
                                                int lattice, uint32_t* link_mask, int32_t* blk_cnt) {
    __shared__ unsigned halo[36];
    const int L = d.level;
    const int nx = d.n0[0] << L, ny = d.n0[1] << L, nz = d.n0[2] << L;
    const int lane = threadIdx.x;
    const uint32_t dirs = lattice_dirs(lattice);
    for (int64_t b = blockIdx.x; b < d.nblocks; b += gridDim.x) {
        const int bx = d.bcoord[3 * b], by = d.bcoord[3 * b + 1], bz = d.bcoord[3 * b + 2];
        if (lane < 36) {
            const int J = lane % 6 - 1, K = lane / 6 - 1;
            const int j = 4 * by + J, k = 4 * bz + K;
            unsigned bits = 0;
            if (j >= 0 && j < ny && k >= 0 && k < nz) bits = halo_bits(off, val, cap, (int64_t)j + (int64_t)ny * k, 4 * bx - 1, nx);
            halo[lane] = bits;
        }
        __syncthreads();
        const int I = lane & 3, J = (lane >> 2) & 3, K = lane >> 4;
        uint32_t m = 0;
        if (!((halo[(J + 1) + 6 * (K + 1)] >> (I + 1)) & 1u)) {
            for (int k = 0; k < 27; k++) {
                if (!((dirs >> k) & 1u)) continue;
                int cx, cy, cz;
                dirvec(k, cx, cy, cz);
                if ((halo[(J + 1 + cy) + 6 * (K + 1 + cz)] >> (I + 1 + cx)) & 1u) m |= 1u << k;
            }
        }
        link_mask[64 * b + lane] = m;
        int c = __popc(m);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) blk_cnt[b] = c;
        __syncthreads();
    }
}

__global__ void k_cl_total(const int32_t* blk_off, int64_t nb, int64_t* d_nlinks) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_nlinks = blk_off[nb];
}

// ------------------------------------------------------------------------
// candidate records
// ------------------------------------------------------------------------
enum { C_SKIP = 1, C_SLOW = 2 };

template <typename R>
struct Cand {
    R v[3][3];      // vertices in the block frame (centres of the block at 0..3)
    R n[3];         // plane normal (b - a) x (c - a)
    R off;          // n . a
    R bound;        // |(off - n.P) - orient3d(a,b,c,P)| <= bound for P in [-1,4]^3
    R delta;        // rounding bound of v
    double n64[3];  // float64 plane for refining t
    double off64;
    int tri;
    int flags;
};

// scaled global coordinate v 2^L - 1/2 (exact)
__device__ __forceinline__ void vert_scaled(const DevMesh& m, int vid, double s, double g[3]) {
    for (int a = 0; a < 3; a++) g[a] = load_coord(m, vid, a) * s - 0.5;
}

template <typename R>
__device__ void stage_cand(const DevMesh& m, int L, int tri, const int b0[3], Cand<R>& C) {
    const double s = ldexp(1.0, L);
    double v[3][3];
    bool exact = true;
    for (int i = 0; i < 3; i++) {
        double g[3];
        vert_scaled(m, m.tris[3 * (int64_t)tri + i], s, g);
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
    C.flags = exact ? 0 : C_SLOW;
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
    // degenerate (zero-area) triangles never meet a segment
    if (fabs(n[0]) <= 5 * u64 * perm[0] && fabs(n[1]) <= 5 * u64 * perm[1] && fabs(n[2]) <= 5 * u64 * perm[2]) {
        double g[3][3];
        for (int i = 0; i < 3; i++) vert_scaled(m, m.tris[3 * (int64_t)tri + i], s, g[i]);
        if (orient2d_exact(g[0][1], g[0][2], g[1][1], g[1][2], g[2][1], g[2][2]) == 0 &&
            orient2d_exact(g[0][2], g[0][0], g[1][2], g[1][0], g[2][2], g[2][0]) == 0 &&
            orient2d_exact(g[0][0], g[0][1], g[1][0], g[1][1], g[2][0], g[2][1]) == 0)
            C.flags |= C_SKIP;
    }
    const double off = n[0] * v[0][0] + n[1] * v[0][1] + n[2] * v[0][2];
    double en[3], sna = 0, n1 = 0, ena = 0;
    for (int a = 0; a < 3; a++) {
        en[a] = 5 * u64 * perm[a];
        sna += fabs(n[a] * v[0][a]);
        n1 += fabs(n[a]);
        ena += en[a] * (fabs(v[0][a]) + 4.0);
    }
    for (int a = 0; a < 3; a++) C.n64[a] = n[a];
    C.off64 = off;
    double bound;
    if constexpr (std::is_same<R, float>::value) {
        const double u32 = 5.9604644775390625e-8;
        float n32[3];
        for (int a = 0; a < 3; a++) n32[a] = (float)n[a];
        const float off32 = (float)off;
        double n321 = fabs((double)n32[0]) + fabs((double)n32[1]) + fabs((double)n32[2]);
        bound = u32 * fabs(off) + 3.01 * u64 * sna + ena + 4 * u32 * n1 + 4.01 * u32 * (fabs((double)off32) + 4 * n321);
        bound = bound * 1.01 + 1e-30;
        for (int a = 0; a < 3; a++) C.n[a] = n32[a];
        C.off = off32;
        float bf = (float)bound;
        if ((double)bf < bound) bf = nextafterf(bf, 1e30f);
        C.bound = bf;
        double dl = 0;
        for (int i = 0; i < 3; i++)
            for (int a = 0; a < 3; a++) {
                C.v[i][a] = (float)v[i][a];
                dl = fmax(dl, fabs((double)C.v[i][a] - v[i][a]));
            }
        float df = (float)dl;
        if ((double)df < dl) df = nextafterf(df, 1e30f);
        C.delta = df;
    } else {
        bound = 3.01 * u64 * sna + ena + 4.01 * u64 * (fabs(off) + 4 * n1);
        bound = bound * 1.01 + 1e-300;
        for (int a = 0; a < 3; a++) C.n[a] = n[a];
        C.off = off;
        C.bound = bound;
        for (int i = 0; i < 3; i++)
            for (int a = 0; a < 3; a++) C.v[i][a] = v[i][a];
        C.delta = 0;
    }
}

struct QStats {
    unsigned fb = 0, ex = 0, tq = 0;
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
    for (int k = 0; k < 3; k++) {
        const int u = (k + 1) % 3, w = (k + 2) % 3;
        const int s = o2_sign64(A[u], A[w], B[u], B[w], C[u], C[w], st);
        if (s != 0) { area = s; return k; }
    }
    return -1;
}

__device__ bool in_closed_tri_coplanar(const double* A, const double* B, const double* C, const double* P,
                                       QStats& st) {
    int area;
    const int k = drop_axis(A, B, C, area, st);
    if (k < 0) return false;
    const int u = (k + 1) % 3, w = (k + 2) % 3;
    const double* V[3] = {A, B, C};
    for (int i = 0; i < 3; i++) {
        const double* p = V[i];
        const double* q = V[(i + 1) % 3];
        if (o2_sign64(p[u], p[w], q[u], q[w], P[u], P[w], st) * area < 0) return false;
    }
    return true;
}

// float64 value of orient3d (for hit parameters)
__device__ __forceinline__ double o3_value(const double* a, const double* b, const double* c, const double* d) {
    const double adx = a[0] - d[0], bdx = b[0] - d[0], cdx = c[0] - d[0];
    const double ady = a[1] - d[1], bdy = b[1] - d[1], cdy = c[1] - d[1];
    const double adz = a[2] - d[2], bdz = b[2] - d[2], cdz = c[2] - d[2];
    return adz * (bdx * cdy - cdx * bdy) + bdz * (cdx * ady - adx * cdy) + cdz * (adx * bdy - bdx * ady);
}

// segment X->Y in the plane of T: entry parameter into the closed triangle
__device__ int coplanar_clip(const double* A, const double* B, const double* C, const double* X, const double* Y,
                             double& t, QStats& st) {
    int area;
    const int k = drop_axis(A, B, C, area, st);
    if (k < 0) return 0;
    const int u = (k + 1) % 3, w = (k + 2) % 3;
    const double* V[3] = {A, B, C};
    double lo = 0.0, hi = 1.0;
    for (int i = 0; i < 3; i++) {
        const double* p = V[i];
        const double* q = V[(i + 1) % 3];
        const int g0 = o2_sign64(p[u], p[w], q[u], q[w], X[u], X[w], st) * area;
        const int g1 = o2_sign64(p[u], p[w], q[u], q[w], Y[u], Y[w], st) * area;
        if (g0 < 0 && g1 < 0) return 0;
        if (g0 >= 0 && g1 >= 0) continue;
        const double f0 = area * ((p[u] - X[u]) * (q[w] - X[w]) - (p[w] - X[w]) * (q[u] - X[u]));
        const double f1 = area * ((p[u] - Y[u]) * (q[w] - Y[w]) - (p[w] - Y[w]) * (q[u] - Y[u]));
        const double tt = f0 / (f0 - f1);
        if (g0 < 0) lo = fmax(lo, tt);
        else hi = fmin(hi, tt);
    }
    if (lo > hi) return 0;
    t = lo;
    return 1;
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

template <typename R>
__global__ void __launch_bounds__(64) k_cl_q(DevMesh m, DevLevel d, const int32_t* loff, const int32_t* lval,
                                             int64_t lcap, const uint32_t* link_mask, const int32_t* blk_off,
                                             int64_t cap, int32_t* link_cell, uint8_t* link_dir, float* link_q,
                                             int32_t* link_tri, uint64_t* stats) {
    __shared__ Cand<R> cand[CL_CAND];
    __shared__ uint32_t smask[64];
    __shared__ int spre[65];
    const int L = d.level;
    const double s = ldexp(1.0, L);
    const int lane = threadIdx.x;
    QStats st;
    for (int64_t b = blockIdx.x; b < d.nblocks; b += gridDim.x) {
        const int n = blk_off[b + 1] - blk_off[b];
        if (n == 0) continue;  // uniform across the workgroup
        const int b0[3] = {4 * d.bcoord[3 * b], 4 * d.bcoord[3 * b + 1], 4 * d.bcoord[3 * b + 2]};
        const uint32_t mk = link_mask[64 * b + lane];
        smask[lane] = mk;
        int c = __popc(mk), incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int tt = __shfl_up(incl, o, 64);
            if (lane >= o) incl += tt;
        }
        spre[lane] = incl - c;
        if (lane == 63) spre[64] = incl;
        int64_t c0 = loff[b], c1 = loff[b + 1];
        if (c1 > lcap) c1 = lcap;
        if (c0 > c1) c0 = c1;
        const int nc = (int)(c1 - c0);
        __syncthreads();
        for (int lbase = 0; lbase < n; lbase += 64) {
            const int li = lbase + lane;
            const bool active = li < n;
            int t = 0, k = 0;
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
            const int Xi[3] = {t & 3, (t >> 2) & 3, t >> 4};
            const R X[3] = {(R)Xi[0], (R)Xi[1], (R)Xi[2]};
            const R Y[3] = {(R)(Xi[0] + cx), (R)(Xi[1] + cy), (R)(Xi[2] + cz)};
            double best = 2.0;
            int btri = 0x7fffffff;
            for (int cb = 0; cb < nc; cb += CL_CAND) {
                const int nstage = nc - cb < CL_CAND ? nc - cb : CL_CAND;
                __syncthreads();
                if (lane < nstage) stage_cand<R>(m, L, lval[c0 + cb + lane], b0, cand[lane]);
                __syncthreads();
                if (!active) continue;
                for (int ci = 0; ci < nstage; ci++) {
                    const Cand<R>& C = cand[ci];
                    if (C.flags & C_SKIP) continue;
                    double tq;
                    int res;
                    R tr = 0, terr = 0;
                    res = (C.flags & C_SLOW) ? -1 : fast_test<R>(C, X, Y, tr, terr);
                    if (res < 0) {
                        if constexpr (std::is_same<R, float>::value) st.fb++;
                        double A[3], B[3], Cc[3];
                        vert_scaled(m, m.tris[3 * (int64_t)C.tri], s, A);
                        vert_scaled(m, m.tris[3 * (int64_t)C.tri + 1], s, B);
                        vert_scaled(m, m.tris[3 * (int64_t)C.tri + 2], s, Cc);
                        const double Xg[3] = {(double)(b0[0] + Xi[0]), (double)(b0[1] + Xi[1]), (double)(b0[2] + Xi[2])};
                        const double Yg[3] = {Xg[0] + cx, Xg[1] + cy, Xg[2] + cz};
                        res = exact_seg_hit(A, B, Cc, Xg, Yg, tq, st);
                    } else if (res == 1) {
                        tq = (double)tr;
                        if (terr > (R)2e-6) {
                            // ill-conditioned: refine t with the float64 plane
                            st.tq++;
                            const double sX = C.off64 - C.n64[0] * Xi[0] - C.n64[1] * Xi[1] - C.n64[2] * Xi[2];
                            const double nd = C.n64[0] * cx + C.n64[1] * cy + C.n64[2] * cz;
                            tq = sX / nd;
                            tq = fmin(fmax(tq, 0.0), 1.0);
                        }
                    }
                    if (res == 1 && (tq < best || (tq == best && C.tri < btri))) {
                        best = tq;
                        btri = C.tri;
                    }
                }
            }
            if (active) {
                const int64_t pos = (int64_t)blk_off[b] + li;
                if (pos < cap) {
                    link_cell[pos] = (int32_t)(64 * b + t);
                    link_dir[pos] = (uint8_t)k;
                    link_q[pos] = best <= 1.0 ? (float)best : -1.0f;
                    link_tri[pos] = best <= 1.0 ? btri : -1;
                }
            }
        }
        __syncthreads();
    }
    if (stats) {
        if constexpr (std::is_same<R, float>::value) wave_count(&stats[GEO_STAT_F32_TO_F64], st.fb);
        wave_count(&stats[GEO_STAT_EXACT], st.ex);
        wave_count(&stats[GEO_STAT_Q_F64], st.tq);
    }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t geo_cutlinks_ws_bytes(int64_t nb) {
    return al(sizeof(int32_t) * (size_t)nb) + al(sizeof(int32_t) * ((size_t)nb + 1)) + al(geo_scan_partials_bytes(nb));
}

int launch_cutlinks(const DevMesh& m, const DevLevel& d, const geo_bins* rows, const geo_bins* links, int lattice,
                    int precision, uint32_t* link_mask, int64_t cap, int64_t* d_nlinks, int32_t* link_cell,
                    uint8_t* link_dir, float* link_q, int32_t* link_tri, uint64_t* d_stats, void* ws,
                    size_t ws_bytes, hipStream_t s) {
    const int64_t nb = d.nblocks;
    if (ws_bytes < geo_cutlinks_ws_bytes(nb)) return GEO_ERR_WORKSPACE;
    char* p = static_cast<char*>(ws);
    int32_t* blk_cnt = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)nb);
    int32_t* blk_off = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nb + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    if (nb == 0) return geo_fill_u64(reinterpret_cast<uint64_t*>(d_nlinks), 0, 1, s);
    const unsigned g = (unsigned)(nb < 262144 ? nb : 262144);
    k_cl_mask<<<g, 64, 0, s>>>(d, rows->off, rows->val, rows->cap, lattice, link_mask, blk_cnt);
    GEO_LAUNCH_CHECK();
    int rc = geo_scan_exclusive(blk_cnt, blk_off, nb, partials, s);
    if (rc != GEO_OK) return rc;
    k_cl_total<<<1, 64, 0, s>>>(blk_off, nb, d_nlinks);
    if (precision == GEO_PREC_F32_FALLBACK)
        k_cl_q<float><<<g, 64, 0, s>>>(m, d, links->off, links->val, links->cap, link_mask, blk_off, cap, link_cell,
                                       link_dir, link_q, link_tri, d_stats);
    else
        k_cl_q<double><<<g, 64, 0, s>>>(m, d, links->off, links->val, links->cap, link_mask, blk_off, cap,
                                        link_cell, link_dir, link_q, link_tri, d_stats);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
