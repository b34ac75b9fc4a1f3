// Spatial binning on gfx950 (Methodology, "Spatial Binning").
//
// ROWS bins hold, per x-row line of a level, the exact surface events along
// the line (parity crossings and on-surface intervals); they are built
// triangle-parallel: each triangle visits the row lines inside its yz
// bounding box, decides exactly whether the line meets it, and where along
// the line.  LINKS bins hold, per block, the triangles overlapping the block
// box widened by one cell (the widened bin cover of Algorithm 2).
//
// Both are counting sorts without a global sort: pass 1 appends (key, value)
// pairs with one atomic per wave and counts per key, an exclusive scan turns
// counts into offsets, and a scatter pass places the pairs.
#include <type_traits>

#include "geo_internal.h"

namespace {

// ------------------------------------------------------------------------
// Append of (key, value) pairs.  Each workgroup is one wave; pairs are staged
// in an LDS buffer and flushed with one global reservation per flush (a
// global counter touched once per wave-iteration would serialise at L2).
// The per-key counts are incremented at flush time, and the count a pair
// finds is its rank among its key's pairs, kept beside it: the scatter then
// places it without atomics.
// ------------------------------------------------------------------------
constexpr int APP_BUF = 512;

// Group: pairs whose keys repeat within a flush (link bins: neighbouring
// triangles share blocks) take their ranks with one atomic per key; else one
// atomic per pair (row bins: keys mostly distinct).
template <bool Group>
struct Appender {
    int2* buf;       // LDS [APP_BUF]
    int n;           // pairs staged (identical in every lane)
    int2* pairs;
    int32_t* rank;
    int64_t cap;
    int64_t* d_count;
    int32_t* cnt;

    __device__ __forceinline__ void flush() {
        if (n == 0) return;
        __syncthreads();
        unsigned long long base = 0;
        if (threadIdx.x == 0) base = atomicAdd((unsigned long long*)d_count, (unsigned long long)n);
        base = __shfl(base, 0, 64);
        if constexpr (Group) {
            // Per chunk of 64 pairs, lanes holding the same key form a group;
            // its lowest lane takes the group's ranks with one atomic (atomics
            // on one address serialise).  The atomics of four chunks are in
            // flight together.
            const int lane = threadIdx.x;
            const unsigned long long lt = (1ull << lane) - 1ull;
            for (int i0 = 0; i0 < n; i0 += 256) {
                int2 p[4];
                int lead[4], off[4], cntk[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int i = i0 + 64 * u + lane;
                    const bool valid = i < n;
                    p[u] = valid ? buf[i] : make_int2(-1, 0);
                    lead[u] = -1;
                    off[u] = 0;
                    cntk[u] = 0;
                    unsigned long long rem = __ballot(valid);
                    while (rem) {  // uniform
                        const int l = __ffsll(rem) - 1;
                        const int k = __shfl(p[u].x, l, 64);
                        const unsigned long long same = __ballot(valid && p[u].x == k) & rem;
                        if ((same >> lane) & 1ull) {
                            lead[u] = l;
                            off[u] = __popcll(same & lt);
                        }
                        if (lane == l) cntk[u] = __popcll(same);
                        rem &= ~same;
                    }
                }
                int r[4];
#pragma unroll
                for (int u = 0; u < 4; u++) r[u] = cntk[u] ? atomicAdd(&cnt[p[u].x], cntk[u]) : 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int base_k = __shfl(r[u], lead[u] < 0 ? lane : lead[u], 64);
                    const unsigned long long pos = base + (unsigned long long)(i0 + 64 * u + lane);
                    if (p[u].x >= 0 && pos < (unsigned long long)cap) {
                        pairs[pos] = p[u];
                        rank[pos] = base_k + off[u];
                    }
                }
            }
        } else {
            // four returning atomics in flight per lane before their results are used
            for (int i0 = threadIdx.x; i0 < n; i0 += 256) {
                int2 p[4];
                int r[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int i = i0 + 64 * u;
                    p[u] = i < n ? buf[i] : make_int2(-1, 0);
                }
#pragma unroll
                for (int u = 0; u < 4; u++) r[u] = p[u].x >= 0 ? atomicAdd(&cnt[p[u].x], 1) : 0;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const unsigned long long pos = base + (unsigned long long)(i0 + 64 * u);
                    if (p[u].x >= 0 && pos < (unsigned long long)cap) {
                        pairs[pos] = p[u];
                        rank[pos] = r[u];
                    }
                }
            }
        }
        __syncthreads();
        n = 0;
    }
    // returns the number of pairs added (identical in every lane)
    __device__ __forceinline__ int add(bool has, int key, int32_t val) {
        const unsigned long long mask = __ballot(has);
        if (mask == 0ull) return 0;
        const int k = __popcll(mask);
        if (n + k > APP_BUF) flush();
        if (has) {
            const int lane = __lane_id();
            buf[n + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2(key, val);
        }
        n += k;
        return k;
    }
};

// ------------------------------------------------------------------------
// per-triangle local frame for the row pass
// ------------------------------------------------------------------------
template <typename R>
struct RowTri {
    R v[3][3];    // local coordinates (level-L cell units, centres at integers)
    R delta;      // bound on |v - exact| (0 when exact)
    int o[3];     // integer origin of the local frame
    int idx[3];   // vertex ids in local order (b and c swapped when the yz area is negative)
};

// exact scaled coordinate X = v 2^L - 1/2 of vertex vid, axis a, in float64
__device__ __forceinline__ double scaled64(const DevMesh& m, int vid, int a, double s) {
    return load_coord(m, vid, a) * s - 0.5;
}

// exact float64 local coordinates of T (reloaded from memory)
template <typename R>
__device__ __forceinline__ void local64(const DevMesh& m, const RowTri<R>& T, double s, double v[3][3]) {
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < 3; a++) v[i][a] = scaled64(m, T.idx[i], a, s) - (double)T.o[a];
}

struct Stats {
    unsigned fb = 0, ex = 0;
};

// exact sign of orient2d in the (y,z) plane of local points p, q and (py, pz)
template <typename R>
__device__ __forceinline__ int chain_o2_yz(const DevMesh& m, const RowTri<R>& T, double s, int i, int j,
                                           int py, int pz, Stats& st) {
    int r = orient2d_filter<R>(T.v[i][1], T.v[i][2], T.v[j][1], T.v[j][2], (R)py, (R)pz, T.delta);
    if (r != 0) return r;
    double v[3][3];
    if constexpr (std::is_same<R, float>::value) {
        st.fb++;
        local64(m, T, s, v);
        r = orient2d_filter<double>(v[i][1], v[i][2], v[j][1], v[j][2], (double)py, (double)pz, 0.0);
        if (r != 0) return r;
    } else {
        local64(m, T, s, v);
    }
    st.ex++;
    return orient2d_exact(v[i][1], v[i][2], v[j][1], v[j][2], (double)py, (double)pz);
}

// exact sign of orient3d(v0, v1, v2, P) with local P = (px, py, pz)
template <typename R>
__device__ __forceinline__ int chain_o3(const DevMesh& m, const RowTri<R>& T, double s, int px, int py,
                                        int pz, Stats& st) {
    R P[3] = {(R)px, (R)py, (R)pz};
    int r = orient3d_filter<R>(T.v[0], T.v[1], T.v[2], P, T.delta);
    if (r != 0) return r;
    double v[3][3];
    double P64[3] = {(double)px, (double)py, (double)pz};
    if constexpr (std::is_same<R, float>::value) {
        st.fb++;
        local64(m, T, s, v);
        r = orient3d_filter<double>(v[0], v[1], v[2], P64, 0.0);
        if (r != 0) return r;
    } else {
        local64(m, T, s, v);
    }
    st.ex++;
    return orient3d_exact(v[0], v[1], v[2], P64);
}

// exact sign of orient2d on axes (a0, a1) of the three local vertices
template <typename R>
__device__ __forceinline__ int chain_area(const DevMesh& m, const RowTri<R>& T, double s, int a0, int a1,
                                          Stats& st) {
    int r = orient2d_filter<R>(T.v[0][a0], T.v[0][a1], T.v[1][a0], T.v[1][a1], T.v[2][a0], T.v[2][a1],
                               T.delta);
    if (r != 0) return r;
    double v[3][3];
    local64(m, T, s, v);
    if constexpr (std::is_same<R, float>::value) {
        st.fb++;
        r = orient2d_filter<double>(v[0][a0], v[0][a1], v[1][a0], v[1][a1], v[2][a0], v[2][a1], 0.0);
        if (r != 0) return r;
    }
    st.ex++;
    return orient2d_exact(v[0][a0], v[0][a1], v[1][a0], v[1][a1], v[2][a0], v[2][a1]);
}

// exact sign of orient2d on axes (a0, a1) of local vertices i, j and point (p0, p1)
template <typename R>
__device__ __forceinline__ int chain_o2_axes(const DevMesh& m, const RowTri<R>& T, double s, int i, int j,
                                             int a0, int a1, int p0, int p1, Stats& st) {
    int r = orient2d_filter<R>(T.v[i][a0], T.v[i][a1], T.v[j][a0], T.v[j][a1], (R)p0, (R)p1, T.delta);
    if (r != 0) return r;
    double v[3][3];
    local64(m, T, s, v);
    if constexpr (std::is_same<R, float>::value) {
        st.fb++;
        r = orient2d_filter<double>(v[i][a0], v[i][a1], v[j][a0], v[j][a1], (double)p0, (double)p1, 0.0);
        if (r != 0) return r;
    }
    st.ex++;
    return orient2d_exact(v[i][a0], v[i][a1], v[j][a0], v[j][a1], (double)p0, (double)p1);
}

// Simulation-of-simplicity sign of the yz edge function of u->w at a point
// where it vanishes exactly: the point is moved to (y + e, z + e^2), so
// E changes by -(w_z - u_z) e + (w_y - u_y) e^2.
template <typename R>
__device__ __forceinline__ int sos_tie(const DevMesh& m, const RowTri<R>& T, double s, int i, int j) {
    double v[3][3];
    local64(m, T, s, v);
    const double dz = v[j][2] - v[i][2], dy = v[j][1] - v[i][1];  // exact comparisons via signs
    if (v[j][2] != v[i][2]) return dz > 0 ? -1 : 1;
    if (v[j][1] != v[i][1]) return dy > 0 ? 1 : -1;
    return 0;
}

// vertex ids and coordinates of one triangle, loaded once for every level
struct TriLoad {
    int id[3];
    double x[3][3];
};

__device__ __forceinline__ void tri_load(const DevMesh& m, int64_t t, TriLoad& tl) {
    for (int i = 0; i < 3; i++) tl.id[i] = m.tris[3 * t + i];
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < 3; a++) tl.x[i][a] = load_coord(m, tl.id[i], a);
}

// Set up the local frame of level L.  Returns false for triangles with no line.
template <typename R>
__device__ bool row_setup(const TriLoad& tl, int L, int ny, int nz, bool f32_verts, RowTri<R>& T, int& jlo,
                          int& jhi, int& klo, int& khi) {
    const double s = ldexp(1.0, L);
    const int(&id)[3] = tl.id;
    double X[3][3];  // the same float64 operations as scaled64
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < 3; a++) X[i][a] = tl.x[i][a] * s - 0.5;
    const double ymin = fmin(X[0][1], fmin(X[1][1], X[2][1])), ymax = fmax(X[0][1], fmax(X[1][1], X[2][1]));
    const double zmin = fmin(X[0][2], fmin(X[1][2], X[2][2])), zmax = fmax(X[0][2], fmax(X[1][2], X[2][2]));
    jlo = (int)fmax(ceil(ymin), 0.0);
    jhi = (int)fmin(floor(ymax), (double)(ny - 1));
    klo = (int)fmax(ceil(zmin), 0.0);
    khi = (int)fmin(floor(zmax), (double)(nz - 1));
    if (jlo > jhi || klo > khi) return false;
    // origin: x from vertex 0, y/z from the first line; fall back to 0 on an
    // axis where the translation would not be exact in float64.  Float32
    // vertices within the coordinate contract (0 or [1/4, n0], n0 2^L <=
    // 2^15) need no check: X and X - o span at most 2^14 .. 2^-25, 40 bits.
    int o[3] = {(int)floor(X[0][0]), jlo, klo};
    for (int a = 0; a < 3 && !f32_verts; a++) {
        bool exact = true;
        for (int i = 0; i < 3; i++) {
            // Knuth's two-sum error of X - o: zero iff the difference is exact
            const double sum = X[i][a] - (double)o[a];
            const double bb = sum - X[i][a];
            const double err = (X[i][a] - (sum - bb)) + (-(double)o[a] - bb);
            if (err != 0.0) exact = false;
        }
        if (!exact) o[a] = 0;
    }
    R delta = 0;
    for (int i = 0; i < 3; i++) {
        T.idx[i] = id[i];
        for (int a = 0; a < 3; a++) {
            const double x = X[i][a] - (double)o[a];
            T.v[i][a] = (R)x;
            const double err = fabs((double)T.v[i][a] - x);
            // round the bound up when stored in float
            if ((R)err < err) delta = geo_max(delta, (R)(err * (1.0 + 1e-6)));
            else delta = geo_max(delta, (R)err);
        }
    }
    T.delta = delta;
    for (int a = 0; a < 3; a++) T.o[a] = o[a];
    return true;
}

template <typename R>
__device__ __forceinline__ void swap_bc(RowTri<R>& T) {
    for (int a = 0; a < 3; a++) {
        R tmp = T.v[1][a];
        T.v[1][a] = T.v[2][a];
        T.v[2][a] = tmp;
    }
    int ti = T.idx[1];
    T.idx[1] = T.idx[2];
    T.idx[2] = ti;
}

// events of one (triangle, line) pair; e0: parity event or none, e1: surface interval or none
template <typename R>
__device__ void row_events(const DevMesh& m, const RowTri<R>& T, double s, int mode, int drop, int areaSign,
                           int j, int k, int nx, Stats& st, bool& has0, int32_t& e0, bool& has1, int32_t& e1) {
    has0 = has1 = false;
    const int py = j - T.o[1], pz = k - T.o[2];
    R xmn = geo_min(T.v[0][0], geo_min(T.v[1][0], T.v[2][0])) - T.delta;
    R xmx = geo_max(T.v[0][0], geo_max(T.v[1][0], T.v[2][0])) + T.delta;
    if (mode == 1) {
        // proper yz projection (counter-clockwise after set-up)
        int e[3];
        for (int i = 0; i < 3; i++) {
            e[i] = chain_o2_yz<R>(m, T, s, i, (i + 1) % 3, py, pz, st);
            if (e[i] < 0) return;
        }
        bool sos_in = true;
        for (int i = 0; i < 3; i++)
            if (e[i] == 0 && sos_tie<R>(m, T, s, i, (i + 1) % 3) <= 0) sos_in = false;
        // crossing position: smallest integer c with orient3d(T, (c, py, pz)) <= 0
        // (x_hit <= c); orient3d is n_x (x_hit - x) with n_x > 0.
        const R e1x = T.v[1][0] - T.v[0][0], e1y = T.v[1][1] - T.v[0][1], e1z = T.v[1][2] - T.v[0][2];
        const R e2x = T.v[2][0] - T.v[0][0], e2y = T.v[2][1] - T.v[0][1], e2z = T.v[2][2] - T.v[0][2];
        const R nx_ = e1y * e2z - e1z * e2y, ny_ = e1z * e2x - e1x * e2z, nz_ = e1x * e2y - e1y * e2x;
        const int lo = (int)ceil((double)xmn), hi = (int)ceil((double)xmx);
        R xs = T.v[0][0] - (ny_ * ((R)py - T.v[0][1]) + nz_ * ((R)pz - T.v[0][2])) / nx_;
        int c;
        if (!(xs == xs) || xs < (R)lo) c = lo;
        else if (xs > (R)hi) c = hi;
        else c = (int)ceil((double)xs);
        int sc = chain_o3<R>(m, T, s, c, py, pz, st);
        if (sc > 0) {
            do {
                c++;
                sc = chain_o3<R>(m, T, s, c, py, pz, st);
            } while (sc > 0 && c < hi + 1);
        } else {
            while (c > lo) {
                const int sp = chain_o3<R>(m, T, s, c - 1, py, pz, st);
                if (sp > 0) break;
                c--;
                sc = sp;
            }
        }
        const int g = c + T.o[0];  // global index of the first centre at or right of the crossing
        if (sos_in && g >= 1) {
            has0 = true;
            e0 = g < nx ? g : nx;
        }
        if (sc == 0 && g >= 0 && g < nx) {
            has1 = true;
            e1 = row_surf_entry(g, g);
        }
        return;
    }
    // mode 2: edge-on triangle (zero yz area, non-degenerate).  The line meets
    // it only if the line point is on the projected segment; then every
    // centre of the line inside the closed triangle is on the surface.
    {
        // longest projected edge (any edge with distinct yz endpoints works)
        int bi = 0;
        R best = -1;
        for (int i = 0; i < 3; i++) {
            const int jn = (i + 1) % 3;
            const R l = geo_fabs(T.v[jn][1] - T.v[i][1]) + geo_fabs(T.v[jn][2] - T.v[i][2]);
            if (l > best) { best = l; bi = i; }
        }
        if (chain_o2_yz<R>(m, T, s, bi, (bi + 1) % 3, py, pz, st) != 0) return;
        const int pw = drop == 1 ? py : pz;  // coordinate kept beside x
        bool found = false;
        int first = 0, last = 0;  // local indices; may be negative
        const int lo = (int)ceil((double)xmn), hi = (int)floor((double)xmx);
        for (int c = lo; c <= hi; c++) {
            bool in = true;
            for (int i = 0; i < 3 && in; i++) {
                const int r = chain_o2_axes<R>(m, T, s, i, (i + 1) % 3, 0, drop, c, pw, st);
                if (r * areaSign < 0) in = false;
            }
            if (in) {
                if (!found) first = c;
                found = true;
                last = c;
            } else if (found) {
                break;  // convex: the inside centres are contiguous
            }
        }
        if (found) {
            int gl = first + T.o[0], gh = last + T.o[0];
            gl = gl < 0 ? 0 : gl;
            gh = gh > nx - 1 ? nx - 1 : gh;
            if (gl <= gh) {
                has1 = true;
                e1 = row_surf_entry(gl, gh);
            }
        }
    }
}

// The row-line events of one level for the wave's triangles (live lanes hold
// one loaded triangle each), appended under keys key_base + j + ny k.  Called
// by the whole wave; returns the number of pairs appended.
template <typename R>
__device__ __forceinline__ int rows_level(const DevMesh& m, bool live, const TriLoad& tl, int L, int key_base,
                                          Appender<false>& app, Stats& st, const int n0[3]) {
    const int nx = n0[0] << L, ny = n0[1] << L, nz = n0[2] << L;
    const double s = ldexp(1.0, L);
    RowTri<R> T;
    int jlo = 0, jhi = -1, klo = 0, khi = -1;
    int mode = 0, drop = 0, areaSign = 0;
    if (live && row_setup<R>(tl, L, ny, nz, m.vdtype == GEO_F32, T, jlo, jhi, klo, khi)) {
        const int ayz = chain_area<R>(m, T, s, 1, 2, st);
        if (ayz < 0) swap_bc<R>(T);
        if (ayz != 0) {
            mode = 1;
        } else {
            // edge-on or degenerate: find a plane (x,y) or (x,z) with non-zero area
            const int axy = chain_area<R>(m, T, s, 0, 1, st);
            if (axy != 0) { mode = 2; drop = 1; areaSign = axy; }
            else {
                const int axz = chain_area<R>(m, T, s, 0, 2, st);
                if (axz != 0) { mode = 2; drop = 2; areaSign = axz; }
            }
        }
    }
    const int nj = mode ? jhi - jlo + 1 : 0;
    const int nlines = mode ? nj * (khi - klo + 1) : 0;
    int added = 0;
    for (int it = 0; __any(it < nlines); it++) {
        bool h0 = false, h1 = false;
        int32_t e0 = 0, e1 = 0;
        int key = 0;
        if (it < nlines) {
            const int j = jlo + it % nj, k = klo + it / nj;
            key = key_base + j + ny * k;
            row_events<R>(m, T, s, mode, drop, areaSign, j, k, nx, st, h0, e0, h1, e1);
        }
        added += app.add(h0, key, e0);
        added += app.add(h1, key, e1);
    }
    return added;
}

template <typename R>
__global__ void __launch_bounds__(64) k_rows_pass1(DevMesh m, DevLevel d, int32_t* cnt, int2* pairs, int32_t* rank,
                                                   int64_t cap, int64_t* d_count, uint64_t* stats) {
    __shared__ int2 sbuf[APP_BUF];
    Appender<false> app{sbuf, 0, pairs, rank, cap, d_count, cnt};
    Stats st;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m.nt; base += stride) {
        const int64_t t = base + threadIdx.x;
        TriLoad tl;
        const bool live = t < m.nt;
        if (live) tri_load(m, t, tl);
        rows_level<R>(m, live, tl, d.level, 0, app, st, d.n0);
    }
    app.flush();
    if (stats) {
        if constexpr (std::is_same<R, float>::value) wave_count(&stats[GEO_STAT_F32_TO_F64], st.fb);
        wave_count(&stats[GEO_STAT_EXACT], st.ex);
    }
}

// ROWS bins of levels lmin .. lmin+nlev-1 in one pass: each triangle is
// loaded once and visits its lines of every level in turn; the keys of level
// lmin+l start at rl.base[l].  Pairs share one array and one reservation
// counter (*d_pairs); the pairs needed by each level are counted per wave in
// LDS and added to the level's own counter once at the end.
template <typename R>
__device__ __forceinline__ void rows_levels_body(const DevMesh& m, const DevLevel& d, const RowLevels& rl, int32_t* cnt,
                                                 int2* pairs, int32_t* rank, int64_t cap, int64_t* d_pairs,
                                                 uint64_t* stats) {
    __shared__ int2 sbuf[APP_BUF];
    __shared__ unsigned long long slc[GEO_MAX_LEVELS];
    const int lane = threadIdx.x;
    if (lane < GEO_MAX_LEVELS) slc[lane] = 0;
    __syncthreads();
    Appender<false> app{sbuf, 0, pairs, rank, cap, d_pairs, cnt};
    Stats st;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m.nt; base += stride) {
        const int64_t t = base + lane;
        TriLoad tl;
        const bool live = t < m.nt;
        if (live) tri_load(m, t, tl);
        for (int l = 0; l < rl.nlev; l++) {
            const int added = rows_level<R>(m, live, tl, rl.lmin + l, rl.base[l], app, st, d.n0);
            if (lane == 0 && added) slc[l] += (unsigned long long)added;
        }
    }
    app.flush();
    __syncthreads();
    if (lane < rl.nlev && slc[lane]) atomicAdd(rl.count[lane], slc[lane]);
    if (stats) {
        if constexpr (std::is_same<R, float>::value) wave_count(&stats[GEO_STAT_F32_TO_F64], st.fb);
        wave_count(&stats[GEO_STAT_EXACT], st.ex);
    }
}

// float32 form: 3 waves per SIMD (168 VGPRs; the cap spills 16 B per lane);
// the float64 form keeps its registers (a cap spills it heavily)
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_rows_levels_f32(DevMesh m, DevLevel d, RowLevels rl, int32_t* cnt, int2* pairs, int32_t* rank, int64_t cap,
                  int64_t* d_pairs, uint64_t* stats) {
    rows_levels_body<float>(m, d, rl, cnt, pairs, rank, cap, d_pairs, stats);
}

__global__ void __launch_bounds__(64) k_rows_levels_f64(DevMesh m, DevLevel d, RowLevels rl, int32_t* cnt, int2* pairs,
                                                        int32_t* rank, int64_t cap, int64_t* d_pairs, uint64_t* stats) {
    rows_levels_body<double>(m, d, rl, cnt, pairs, rank, cap, d_pairs, stats);
}

// zero the per-level counters, the shared pair counter and the key counts
__global__ void k_rows_levels_zero(RowLevels rl, int64_t* d_pairs, int32_t* cnt, int64_t nkeys) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 < rl.nlev) *rl.count[i0] = 0ull;
    if (i0 == 0) *d_pairs = 0;
    for (int64_t i = i0; i < nkeys; i += (int64_t)gridDim.x * blockDim.x) cnt[i] = 0;
}

// place the pairs of every level: the level of a pair is found from its key
__global__ void k_rows_levels_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_pairs,
                                      RowLevels rl) {
    __shared__ int sbase[GEO_MAX_LEVELS + 1];
    __shared__ const int32_t* soff[GEO_MAX_LEVELS];
    __shared__ int32_t* sval[GEO_MAX_LEVELS];
    __shared__ int64_t scap[GEO_MAX_LEVELS];
    if (threadIdx.x < GEO_MAX_LEVELS + 1) sbase[threadIdx.x] = rl.base[threadIdx.x];
    if (threadIdx.x < GEO_MAX_LEVELS) {
        soff[threadIdx.x] = rl.off[threadIdx.x];
        sval[threadIdx.x] = rl.val[threadIdx.x];
        scap[threadIdx.x] = rl.cap[threadIdx.x];
    }
    __syncthreads();
    const int64_t n0 = *d_pairs;
    const int64_t n = n0 < cap ? n0 : cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 p = pairs[i];
        int l = 0;
        for (int q = 1; q < rl.nlev; q++) l += p.x >= sbase[q] ? 1 : 0;
        const int64_t pos = (int64_t)soff[l][p.x - sbase[l]] + rank[i];
        if (pos >= 0 && pos < scap[l]) sval[l][pos] = p.y;
    }
}

// ------------------------------------------------------------------------
// LINKS: triangle / widened block box overlap (separating axes, with outward
// margins so that rounding can only add candidates)
// ------------------------------------------------------------------------

// Per-triangle quantities of the separating-axis test.
struct SatTri {
    double v[3][3];
    double e[3][3];  // edges v1-v0, v2-v1, v0-v2
    double n[3];     // e0 x e1 (rounded; any vector is a valid separating axis)
    double nvmin, nvmax;  // min / max over the vertices of n . v
    double nvabs;    // max over the vertices of sum_a |n_a v_a|
    double n1;       // |n|_1
    float ef[3][3];  // e rounded to float, for the edge axes
};

__device__ __forceinline__ void sat_setup(SatTri& T) {
    for (int a = 0; a < 3; a++) {
        T.e[0][a] = T.v[1][a] - T.v[0][a];
        T.e[1][a] = T.v[2][a] - T.v[1][a];
        T.e[2][a] = T.v[0][a] - T.v[2][a];
    }
    T.n[0] = T.e[0][1] * T.e[1][2] - T.e[0][2] * T.e[1][1];
    T.n[1] = T.e[0][2] * T.e[1][0] - T.e[0][0] * T.e[1][2];
    T.n[2] = T.e[0][0] * T.e[1][1] - T.e[0][1] * T.e[1][0];
    T.nvmin = 1e300;
    T.nvmax = -1e300;
    T.nvabs = 0.0;
    for (int i = 0; i < 3; i++) {
        const double p = T.n[0] * T.v[i][0] + T.n[1] * T.v[i][1] + T.n[2] * T.v[i][2];
        T.nvmin = fmin(T.nvmin, p);
        T.nvmax = fmax(T.nvmax, p);
        T.nvabs = fmax(T.nvabs, fabs(T.n[0] * T.v[i][0]) + fabs(T.n[1] * T.v[i][1]) + fabs(T.n[2] * T.v[i][2]));
    }
    T.n1 = fabs(T.n[0]) + fabs(T.n[1]) + fabs(T.n[2]);
    for (int i = 0; i < 3; i++)
        for (int a = 0; a < 3; a++) T.ef[i][a] = (float)T.e[i][a];
}

// Conservative triangle / cube overlap (centre c, half side hs): separating
// axes are the box normals, the triangle normal and the nine edge crosses,
// each with a margin that covers the rounding of the test.  The box normals
// are the candidate range itself (the caller enumerates exactly the blocks
// whose widened box meets the triangle's bounding box); stage one takes the
// triangle normal, stage two the edges.
__device__ bool tri_box_stage1(const double c[3], double hs, const SatTri& T) {
    // the normal axis: projections n . v_i - n . c against the box radius; the
    // margin bounds the rounding of the dot products (4.5 u each side)
    const double nc = T.n[0] * c[0] + T.n[1] * c[1] + T.n[2] * c[2];
    const double err = 5e-16 * (T.nvabs + fabs(T.n[0] * c[0]) + fabs(T.n[1] * c[1]) + fabs(T.n[2] * c[2]));
    const double rn = hs * T.n1 * (1.0 + 1e-9) + 1e-12 * T.n1 + err;
    return !(T.nvmin - nc > rn || T.nvmax - nc < -rn);
}

// The nine edge axes in float.  The vertices relative to the centre,
// w = v - c, are formed in double and rounded once; |w| is at most the
// triangle's extent plus the box's, so each projection x1 w1 + x2 w2 carries
// an absolute error below 4u (|x1| + |x2|) max|w| (u = 2^-24: the roundings
// of w, of the edge components and of the two products and the sum).  The
// radius is widened by 1e-6 max|w| (|x1| + |x2|), more than twice that, and
// by a relative 1e-5 for its own rounding, so an axis is only taken as
// separating where it separates the exact figures; the 1e-30 floor covers
// products that underflow.
__device__ bool tri_box_stage2(const double c[3], double hs, const SatTri& T) {
    float w[3][3];
    float wmax = 0.0f;
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 3; a++) {
            w[k][a] = (float)(T.v[k][a] - c[a]);
            wmax = fmaxf(wmax, fabsf(w[k][a]));
        }
    const float hsf = (float)hs * (1.0f + 1e-5f) + 1e-6f * wmax + 1e-30f;
    // axis = e_box(a) x e(i), nonzero in components b1 = a+1 and b2 = a+2
    for (int i = 0; i < 3; i++) {
        for (int a = 0; a < 3; a++) {
            const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            const float x1 = -T.ef[i][b2], x2 = T.ef[i][b1];
            const float p0 = x1 * w[0][b1] + x2 * w[0][b2];
            const float p1 = x1 * w[1][b1] + x2 * w[1][b2];
            const float p2 = x1 * w[2][b1] + x2 * w[2][b2];
            const float r = hsf * (fabsf(x1) + fabsf(x2));
            const float mn = fminf(p0, fminf(p1, p2)), mx = fmaxf(p0, fmaxf(p1, p2));
            if (mn > r || mx < -r) return false;
        }
    }
    return true;
}

// candidates of a triangle tested (and looked up) together
constexpr int LINKS_U = 4;

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) k_links_pass1(DevMesh m, DevLevel d, int32_t* cnt, int2* pairs, int32_t* rank,
                                                    int64_t cap, int64_t* d_count) {
    __shared__ int2 sbuf[APP_BUF];
    Appender<true> app{sbuf, 0, pairs, rank, cap, d_count, cnt};
    const int L = d.level;
    const double h = ldexp(1.0, -L), bw = 4.0 * h, ibw = ldexp(1.0, L - 2);  // 1 / bw, exact
    const int nb0[3] = {d.n0[0] >> 2, d.n0[1] >> 2, d.n0[2] >> 2};
    const int nbx = nb0[0] << L, nby = nb0[1] << L, nbz = nb0[2] << L;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m.nt; base += stride) {
        const int64_t t = base + threadIdx.x;
        SatTri T;
        double (&v)[3][3] = T.v;
        int lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
        bool live = t < m.nt;
        if (live) {
            for (int i = 0; i < 3; i++) {
                const int vid = m.tris[3 * t + i];
                for (int a = 0; a < 3; a++) v[i][a] = load_coord(m, vid, a);
            }
            sat_setup(T);
            // zero-area triangles never meet a segment: exact test (all three
            // coordinate-plane projections have zero area)
            if (orient2d_filter<double>(v[0][1], v[0][2], v[1][1], v[1][2], v[2][1], v[2][2], 0.0) == 0 &&
                orient2d_filter<double>(v[0][2], v[0][0], v[1][2], v[1][0], v[2][2], v[2][0], 0.0) == 0 &&
                orient2d_filter<double>(v[0][0], v[0][1], v[1][0], v[1][1], v[2][0], v[2][1], 0.0) == 0 &&
                orient2d_exact(v[0][1], v[0][2], v[1][1], v[1][2], v[2][1], v[2][2]) == 0 &&
                orient2d_exact(v[0][2], v[0][0], v[1][2], v[1][0], v[2][2], v[2][0]) == 0 &&
                orient2d_exact(v[0][0], v[0][1], v[1][0], v[1][1], v[2][0], v[2][1]) == 0)
                live = false;
        }
        if (live) {
            const int nb[3] = {nbx, nby, nbz};
            for (int a = 0; a < 3; a++) {
                const double mn = fmin(v[0][a], fmin(v[1][a], v[2][a])), mx = fmax(v[0][a], fmax(v[1][a], v[2][a]));
                // block b's links reach [4bh - h/2, 4bh + 4.5h]: it meets
                // [mn, mx] iff (mn - 4.5h) / bw <= b <= (mx + h/2) / bw (the
                // roundings are monotone and bw is a power of two; the 1e-7
                // only widens the range)
                lo[a] = (int)ceil((mn - 4.5 * h) * ibw - 1e-7);
                hi[a] = (int)floor((mx + 0.5 * h) * ibw + 1e-7);
                lo[a] = lo[a] < 0 ? 0 : lo[a];
                hi[a] = hi[a] > nb[a] - 1 ? nb[a] - 1 : hi[a];
            }
        }
        const int sx = hi[0] - lo[0] + 1, sy = hi[1] - lo[1] + 1, sz = hi[2] - lo[2] + 1;
        const int64_t n = (sx > 0 && sy > 0 && sz > 0) ? (int64_t)sx * sy * sz : 0;
        const double hs = (0.5 * bw + 0.5 * h) * (1.0 + 1e-9);
        // candidate block: box [4bh - h/2, 4(b+1)h + h/2] reached by the
        // block's links, plus a relative margin.  The candidates through both
        // stages, LINKS_U at a time (a triangle has a few: its widened box
        // spans one or two blocks per axis), enumerated x fastest by a cursor;
        // the forest lookups of the LINKS_U candidates descend together, so
        // their dependent loads overlap.
        int cur[3] = {lo[0], lo[1], lo[2]};
        for (int64_t it0 = 0; __any(it0 < n); it0 += LINKS_U) {
            int bb[LINKS_U][3], idx[LINKS_U];
#pragma unroll
            for (int u = 0; u < LINKS_U; u++) {
                idx[u] = -1;
                bb[u][0] = cur[0];
                bb[u][1] = cur[1];
                bb[u][2] = cur[2];
                if (it0 + u < n) {
                    const double c[3] = {(cur[0] + 0.5) * bw, (cur[1] + 0.5) * bw, (cur[2] + 0.5) * bw};
                    if (tri_box_stage1(c, hs, T) && tri_box_stage2(c, hs, T))
                        idx[u] = (cur[0] >> L) + nb0[0] * ((cur[1] >> L) + nb0[1] * (cur[2] >> L));
                }
                if (++cur[0] > hi[0]) {
                    cur[0] = lo[0];
                    if (++cur[1] > hi[1]) {
                        cur[1] = lo[1];
                        ++cur[2];
                    }
                }
            }
            for (int l = 0; l < L; l++) {
                int ch[LINKS_U];
                const int sh = L - 1 - l;
#pragma unroll
                for (int u = 0; u < LINKS_U; u++) ch[u] = idx[u] >= 0 ? d.child[l][idx[u]] : -1;
#pragma unroll
                for (int u = 0; u < LINKS_U; u++)
                    idx[u] = ch[u] < 0 ? -1
                                       : ch[u] + (((bb[u][0] >> sh) & 1) | (((bb[u][1] >> sh) & 1) << 1) |
                                                  (((bb[u][2] >> sh) & 1) << 2));
            }
#pragma unroll
            for (int u = 0; u < LINKS_U; u++) app.add(idx[u] >= 0, idx[u], (int32_t)t);
        }
    }
    app.flush();
}

__global__ void k_bins_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_count,
                               const int32_t* off, int32_t* val) {
    const int64_t n0 = *d_count;
    const int64_t n = n0 < cap ? n0 : cap;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 p = pairs[i];
        const int64_t pos = (int64_t)off[p.x] + rank[i];
        if (pos >= 0 && pos < cap) val[pos] = p.y;
    }
}

__global__ void k_check_mesh(DevMesh m, DevLevel d, uint64_t* stats) {
    // one vertex per thread, its three coordinates in turn (no index division)
    unsigned bad = 0;
    const double top[3] = {(double)d.n0[0], (double)d.n0[1], (double)d.n0[2]};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < m.nv; v += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; a++) {
            const double x = load_coord(m, (int)v, a);
            const bool ok = x == 0.0 || (x >= 0.25 && x <= top[a]);
            bad += ok ? 0u : 1u;
        }
    }
    wave_count(&stats[GEO_STAT_CONTRACT], bad);
}

inline unsigned grid_for(int64_t n, int threads, int64_t maxg = 1 << 16) {
    int64_t g = (n + threads - 1) / threads;
    if (g > maxg) g = maxg;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

int launch_rows_pass1(const DevMesh& m, const DevLevel& d, int precision, int32_t* cnt, int2* pairs,
                      int32_t* rank, int64_t cap, int64_t* d_count, uint64_t* d_stats, hipStream_t s) {
    if (m.nt == 0) return GEO_OK;
    // grid caps measured per form on 7.2M triangles: the float32 pass is
    // fastest at 8192 workgroups, the float64 pass at 2048
    const unsigned g = grid_for(m.nt, 64, precision == GEO_PREC_F32_FALLBACK ? 8192 : 2048);
    kt_record(GEO_KT_ROWS, s, false);
    if (precision == GEO_PREC_F32_FALLBACK)
        k_rows_pass1<float><<<g, 64, 0, s>>>(m, d, cnt, pairs, rank, cap, d_count, d_stats);
    else
        k_rows_pass1<double><<<g, 64, 0, s>>>(m, d, cnt, pairs, rank, cap, d_count, d_stats);
    kt_record(GEO_KT_ROWS, s, true);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_rows_levels(const DevMesh& m, const DevLevel& d, int precision, const RowLevels& rl, int32_t* cnt,
                       int2* pairs, int32_t* rank, int64_t cap, int64_t* d_pairs, uint64_t* d_stats, hipStream_t s) {
    if (m.nt == 0) return GEO_OK;
    // grid caps measured on 7.2M triangles over levels 0..4: 16,384 workgroups
    // for the float32 form (0.645 ms at 8,192), 2,048 for the float64 form
    const unsigned g = grid_for(m.nt, 64, precision == GEO_PREC_F32_FALLBACK ? 16384 : 2048);
    kt_record(GEO_KT_ROWS, s, false);
    if (precision == GEO_PREC_F32_FALLBACK)
        k_rows_levels_f32<<<g, 64, 0, s>>>(m, d, rl, cnt, pairs, rank, cap, d_pairs, d_stats);
    else
        k_rows_levels_f64<<<g, 64, 0, s>>>(m, d, rl, cnt, pairs, rank, cap, d_pairs, d_stats);
    kt_record(GEO_KT_ROWS, s, true);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_rows_levels_zero(const RowLevels& rl, int64_t* d_pairs, int32_t* cnt, int64_t nkeys, hipStream_t s) {
    k_rows_levels_zero<<<grid_for(nkeys, 256, 16384), 256, 0, s>>>(rl, d_pairs, cnt, nkeys);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_rows_levels_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_pairs,
                               const RowLevels& rl, hipStream_t s) {
    if (cap <= 0) return GEO_OK;
    k_rows_levels_scatter<<<grid_for(cap, 256, 8192), 256, 0, s>>>(pairs, rank, cap, d_pairs, rl);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_links_pass1(const DevMesh& m, const DevLevel& d, int32_t* cnt, int2* pairs, int32_t* rank,
                       int64_t cap, int64_t* d_count, hipStream_t s) {
    if (m.nt == 0) return GEO_OK;
    kt_record(GEO_KT_LINKS_BINS, s, false);
    k_links_pass1<<<grid_for(m.nt, 64, 16384), 64, 0, s>>>(m, d, cnt, pairs, rank, cap, d_count);
    kt_record(GEO_KT_LINKS_BINS, s, true);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_bins_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_count,
                        const int32_t* off, int32_t* val, hipStream_t s) {
    if (cap <= 0) return GEO_OK;
    k_bins_scatter<<<grid_for(cap, 256, 8192), 256, 0, s>>>(pairs, rank, cap, d_count, off, val);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int launch_check_mesh(const DevMesh& m, const DevLevel& d, uint64_t* d_stats, hipStream_t s) {
    if (!d_stats || m.nv == 0) return GEO_OK;
    k_check_mesh<<<grid_for(m.nv, 256, 4096), 256, 0, s>>>(m, d, d_stats);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
