// Internal declarations and device helpers of libgeo (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geo.h"

#define GEO_WAVE 64
#define GEO_HD __host__ __device__

// |x| and max/min of floating-point values through the builtins: on the GPU
// |x| is a free source modifier and max/min one instruction each, where a
// compare-and-select costs two (they differ only for -0 and NaN, which no
// bound or decision here depends on)
GEO_HD __forceinline__ double geo_fabs(double x) { return __builtin_fabs(x); }
GEO_HD __forceinline__ float geo_fabs(float x) { return __builtin_fabsf(x); }
template <typename R> GEO_HD __forceinline__ R geo_max(R a, R b) { return a > b ? a : b; }
template <typename R> GEO_HD __forceinline__ R geo_min(R a, R b) { return a < b ? a : b; }
GEO_HD __forceinline__ float geo_max(float a, float b) { return __builtin_fmaxf(a, b); }
GEO_HD __forceinline__ float geo_min(float a, float b) { return __builtin_fminf(a, b); }
GEO_HD __forceinline__ double geo_max(double a, double b) { return __builtin_fmax(a, b); }
GEO_HD __forceinline__ double geo_min(double a, double b) { return __builtin_fmin(a, b); }
// element k of (a0, a1, a2) as a value select, so that arrays stay in registers
// (a select over loads from one array would be folded into a dynamic index)
template <typename R> GEO_HD __forceinline__ R pick3(R a0, R a1, R a2, int k) {
    return k == 0 ? a0 : (k == 1 ? a1 : a2);
}
#define SEL3(a, k) pick3((a)[0], (a)[1], (a)[2], (k))

// --------------------------------------------------------------------------
// kernel-side copies of the level / mesh descriptors (passed by value)
// --------------------------------------------------------------------------
struct DevLevel {
    int n0[3];
    int level;
    int nblocks;
    const int32_t* bcoord;
    const int32_t* child[GEO_MAX_LEVELS];
};

struct DevMesh {
    int nv, nt, vdtype;
    const void* verts;
    const int32_t* tris;
};

static inline DevLevel dev_level(const geo_level* lv) {
    DevLevel d;
    for (int a = 0; a < 3; a++) d.n0[a] = lv->n0[a];
    d.level = lv->level;
    d.nblocks = lv->nblocks;
    d.bcoord = lv->bcoord;
    for (int l = 0; l < GEO_MAX_LEVELS; l++) d.child[l] = l < lv->level ? lv->child[l] : nullptr;
    return d;
}

static inline DevMesh dev_mesh(const geo_mesh* m) {
    DevMesh d;
    d.nv = m->nv;
    d.nt = m->nt;
    d.vdtype = m->vdtype;
    d.verts = m->verts;
    d.tris = m->tris;
    return d;
}

__device__ __forceinline__ double load_coord(const DevMesh& m, int v, int a) {
    return m.vdtype == GEO_F64 ? static_cast<const double*>(m.verts)[3 * (int64_t)v + a]
                               : (double)static_cast<const float*>(m.verts)[3 * (int64_t)v + a];
}

// --------------------------------------------------------------------------
// forest lookup: index of block (bx,by,bz) of level L, -1 if it does not
// exist, -2 if it lies outside the domain.  Walks the child maps from the
// dense level-0 grid down to level L.
// --------------------------------------------------------------------------
__device__ __forceinline__ int forest_lookup(const DevLevel& d, int bx, int by, int bz) {
    const int L = d.level;
    const int nb0x = d.n0[0] >> 2, nb0y = d.n0[1] >> 2, nb0z = d.n0[2] >> 2;
    if (bx < 0 || by < 0 || bz < 0 || bx >= (nb0x << L) || by >= (nb0y << L) || bz >= (nb0z << L))
        return -2;
    int idx = (bx >> L) + nb0x * ((by >> L) + nb0y * (bz >> L));
    for (int l = 0; l < L; l++) {
        const int c = d.child[l][idx];
        if (c < 0) return -1;
        const int sh = L - 1 - l;
        idx = c + (((bx >> sh) & 1) | (((by >> sh) & 1) << 1) | (((bz >> sh) & 1) << 2));
    }
    return idx;
}

// --------------------------------------------------------------------------
// row-line entries
// --------------------------------------------------------------------------
#define ROW_SURF_BIT 0x80000000u
__device__ __forceinline__ int32_t row_surf_entry(int lo, int hi) {
    return (int32_t)(ROW_SURF_BIT | (uint32_t)lo | ((uint32_t)hi << 15));
}

// --------------------------------------------------------------------------
// Exact sign of a polynomial in doubles.
//
// Products of doubles are split exactly into sums of doubles with FMA
// (a*b = p + e, e = fma(a, b, -p), exact barring underflow).  The terms are
// summed exactly in a fixed-point accumulator of eight 32-bit chunks held in
// int64 registers, least significant chunk weighing 2^-192.  This is exact
// when every term is a multiple of 2^-192 and the sum stays below 2^61:
// both hold for products of up to three coordinates that are multiples of
// 2^-64 with magnitudes below 2^16 (the library's coordinate contract).
// --------------------------------------------------------------------------
struct ExactAcc {
    long long c[8];
    GEO_HD __forceinline__ void clear() {
#pragma unroll
        for (int k = 0; k < 8; k++) c[k] = 0;
    }
    GEO_HD __forceinline__ void add(double x) {
        if (x == 0.0) return;
        unsigned long long bits = __builtin_bit_cast(unsigned long long, x);
        const int neg = (int)(bits >> 63);
        const int ef = (int)((bits >> 52) & 0x7ff);
        unsigned long long m = bits & ((1ull << 52) - 1);
        int e;
        if (ef == 0) e = -1074;
        else { m |= 1ull << 52; e = ef - 1075; }
        const int tz = __builtin_ctzll(m);
        m >>= tz;
        e += tz;
        const int s = e + 192;  // bit position of m's lsb in the accumulator
        const int ci = s >> 5, sh = s & 31;
        const unsigned long long lo = m << sh;
        const unsigned long long hi = sh ? (m >> (64 - sh)) : 0ull;
        const long long p0 = (long long)(lo & 0xffffffffull), p1 = (long long)(lo >> 32),
                        p2 = (long long)hi;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            long long v = (k == ci) ? p0 : (k == ci + 1) ? p1 : (k == ci + 2) ? p2 : 0;
            c[k] += neg ? -v : v;
        }
    }
    GEO_HD __forceinline__ void add_prod2(double a, double b) {
        const double p = a * b;
        add(p);
        add(fma(a, b, -p));
    }
    GEO_HD __forceinline__ void sub_prod2(double a, double b) { add_prod2(-a, b); }
    GEO_HD __forceinline__ void add_prod3(double a, double b, double c3) {
        const double p = a * b, e = fma(a, b, -p);
        const double p1 = p * c3, e1 = fma(p, c3, -p1);
        const double p2 = e * c3, e2 = fma(e, c3, -p2);
        add(p1); add(e1); add(p2); add(e2);
    }
    GEO_HD __forceinline__ int sign() {
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const long long carry = c[k] >> 32;  // arithmetic shift: floor division
            c[k] -= carry * 4294967296LL;
            c[k + 1] += carry;
        }
        if (c[7] != 0) return c[7] > 0 ? 1 : -1;
        long long any = 0;
#pragma unroll
        for (int k = 0; k < 7; k++) any |= c[k];
        return any != 0 ? 1 : 0;
    }
};

// orient2d(a,b,c) = det[[ax ay 1],[bx by 1],[cx cy 1]] exactly
GEO_HD __noinline__ static int orient2d_exact(double ax, double ay, double bx, double by,
                                                  double cx, double cy) {
    ExactAcc acc;
    acc.clear();
    acc.add_prod2(ax, by);
    acc.sub_prod2(ax, cy);
    acc.sub_prod2(ay, bx);
    acc.add_prod2(ay, cx);
    acc.add_prod2(bx, cy);
    acc.sub_prod2(by, cx);
    return acc.sign();
}

// det3 of rows p, q, r (raw coordinates), six signed triple products
GEO_HD __forceinline__ void acc_det3(ExactAcc& acc, double s, const double* p, const double* q,
                                         const double* r) {
    acc.add_prod3(s * p[0], q[1], r[2]);
    acc.add_prod3(-s * p[0], q[2], r[1]);
    acc.add_prod3(-s * p[1], q[0], r[2]);
    acc.add_prod3(s * p[1], q[2], r[0]);
    acc.add_prod3(s * p[2], q[0], r[1]);
    acc.add_prod3(-s * p[2], q[1], r[0]);
}

// orient3d(a,b,c,d) = det[a-d; b-d; c-d] = det[[a 1],[b 1],[c 1],[d 1]]
//   = -det3(b,c,d) + det3(a,c,d) - det3(a,b,d) + det3(a,b,c), exactly
GEO_HD __noinline__ static int orient3d_exact(const double* a, const double* b, const double* c,
                                                  const double* d) {
    ExactAcc acc;
    acc.clear();
    acc_det3(acc, -1.0, b, c, d);
    acc_det3(acc, 1.0, a, c, d);
    acc_det3(acc, -1.0, a, b, d);
    acc_det3(acc, 1.0, a, b, c);
    return acc.sign();
}

// --------------------------------------------------------------------------
// Floating-point filters (Shewchuk 1997 forward error bounds: (3+16u)u for
// orient2d and (7+56u)u for orient3d of the permanent; we use 4u and 8u).
// delta: bound on the rounding of each input coordinate (0 when the inputs
// are exact in R); its contribution is bounded from the derivative of the
// determinant.  Return +1/-1 when certain, 0 when not.
// --------------------------------------------------------------------------
template <typename R> struct Unit;
template <> struct Unit<float> { static constexpr float u = 5.9604645e-8f; static constexpr float tiny = 1e-30f; };
template <> struct Unit<double> { static constexpr double u = 1.1102230246251565e-16; static constexpr double tiny = 1e-300; };

template <typename R>
GEO_HD __forceinline__ int orient2d_filter(R ax, R ay, R bx, R by, R cx, R cy, R delta) {
#pragma clang fp contract(off)
    const R acx = ax - cx, acy = ay - cy, bcx = bx - cx, bcy = by - cy;
    const R l = acx * bcy, r = acy * bcx;
    const R det = l - r;
    R bound = R(4) * Unit<R>::u * (geo_fabs(l) + geo_fabs(r)) + Unit<R>::tiny;
    if (delta != R(0)) {
        const R m = geo_max(geo_max(geo_fabs(acx), geo_fabs(acy)), geo_max(geo_fabs(bcx), geo_fabs(bcy))) + R(2) * delta;
        bound += R(8) * delta * m * (R(1) + R(16) * Unit<R>::u) + R(8) * delta * delta;
    }
    return det > bound ? 1 : (det < -bound ? -1 : 0);
}

template <typename R>
GEO_HD __forceinline__ int orient3d_filter(const R* a, const R* b, const R* c, const R* d, R delta) {
#pragma clang fp contract(off)
    const R adx = a[0] - d[0], bdx = b[0] - d[0], cdx = c[0] - d[0];
    const R ady = a[1] - d[1], bdy = b[1] - d[1], cdy = c[1] - d[1];
    const R adz = a[2] - d[2], bdz = b[2] - d[2], cdz = c[2] - d[2];
    const R bdxcdy = bdx * cdy, cdxbdy = cdx * bdy;
    const R cdxady = cdx * ady, adxcdy = adx * cdy;
    const R adxbdy = adx * bdy, bdxady = bdx * ady;
    const R det = adz * (bdxcdy - cdxbdy) + bdz * (cdxady - adxcdy) + cdz * (adxbdy - bdxady);
    const R perm = (geo_fabs(bdxcdy) + geo_fabs(cdxbdy)) * geo_fabs(adz) + (geo_fabs(cdxady) + geo_fabs(adxcdy)) * geo_fabs(bdz) +
                   (geo_fabs(adxbdy) + geo_fabs(bdxady)) * geo_fabs(cdz);
    R bound = R(8) * Unit<R>::u * perm + Unit<R>::tiny;
    if (delta != R(0)) {
        R m = geo_max(geo_max(geo_max(geo_fabs(adx), geo_fabs(bdx)), geo_max(geo_fabs(cdx), geo_fabs(ady))),
                   geo_max(geo_max(geo_fabs(bdy), geo_fabs(cdy)), geo_max(geo_max(geo_fabs(adz), geo_fabs(bdz)), geo_fabs(cdz))));
        m += R(2) * delta;
        bound += R(64) * delta * m * m * (R(1) + R(16) * Unit<R>::u);
    }
    return det > bound ? 1 : (det < -bound ? -1 : 0);
}

// inclusive prefix sum over the 64 lanes of a wave (all lanes active), by
// data-parallel primitives: shifts by 1, 2, 4, 8 within each row of 16 lanes,
// then the last lane of rows 0 and 2 added to rows 1 and 3, and lane 31 to
// rows 2 and 3.  No LDS round trip, unlike a shuffle-based scan.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// statistics: one atomic per wave for a per-lane count
__device__ __forceinline__ void wave_count(uint64_t* ctr, unsigned n) {
    if (!ctr) return;
    unsigned long long tot = n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd((unsigned long long*)ctr, tot);
}

// --------------------------------------------------------------------------
// host-side launchers (defined in the .hip files)
// --------------------------------------------------------------------------
// records the start (stop = false) or stop event of a timed launch when the
// kernel timer is on for that kernel (no-op otherwise)
void kt_record(int kernel, hipStream_t s, bool stop);

// zero *one and p[0..n-1] (one launch)
int geo_zero_counts(uint64_t* one, int32_t* p, int64_t n, hipStream_t s);
int geo_scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* partials,
                       hipStream_t s);
size_t geo_scan_partials_bytes(int64_t n);
int geo_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
int geo_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
int geo_sum_i32(const int32_t* in, int64_t n, int64_t* out, hipStream_t s);

// ROWS bins of several levels built together (levels lmin .. lmin+nlev-1):
// keys of level lmin+l start at base[l] in the joint key space; count, off,
// val and cap are the levels' own bins.
struct RowLevels {
    int nlev, lmin;
    int base[GEO_MAX_LEVELS + 1];
    unsigned long long* count[GEO_MAX_LEVELS];
    const int32_t* off[GEO_MAX_LEVELS];
    int32_t* val[GEO_MAX_LEVELS];
    int64_t cap[GEO_MAX_LEVELS];
};
int launch_rows_levels(const DevMesh& m, const DevLevel& d, int precision, const RowLevels& rl, int32_t* cnt,
                       int2* pairs, int32_t* rank, int64_t cap, int64_t* d_pairs, uint64_t* d_stats, hipStream_t s);
int launch_rows_levels_zero(const RowLevels& rl, int64_t* d_pairs, int32_t* cnt, int64_t nkeys, hipStream_t s);
int launch_rows_levels_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_pairs,
                               const RowLevels& rl, hipStream_t s);
int launch_rows_pass1(const DevMesh& m, const DevLevel& d, int precision, int32_t* cnt,
                      int2* pairs, int32_t* rank, int64_t cap, int64_t* d_count, uint64_t* d_stats,
                      hipStream_t s);
int launch_links_pass1(const DevMesh& m, const DevLevel& d, int32_t* cnt, int2* pairs, int32_t* rank,
                       int64_t cap, int64_t* d_count, hipStream_t s);
int launch_bins_scatter(const int2* pairs, const int32_t* rank, int64_t cap, const int64_t* d_count,
                        const int32_t* off, int32_t* val, hipStream_t s);
int launch_check_mesh(const DevMesh& m, const DevLevel& d, uint64_t* d_stats, hipStream_t s);
size_t geo_dense_ws_bytes(int64_t nb);
int launch_links_dense(int64_t nb, int64_t n_links, const int32_t* link_cell, const uint8_t* link_dir,
                       const float* link_q, const int32_t* link_tri, int lattice, int64_t cap, int32_t* block_map,
                       float* dense_q, int32_t* dense_tri, int64_t* d_nbnd, void* ws, size_t ws_bytes, hipStream_t s);
int launch_block_nbr(const DevLevel& d, int32_t* nbr, hipStream_t s);
int launch_ibb(const DevLevel& d, const uint64_t* solid, const int32_t* block_map, const float* dense_q,
               int64_t nbnd, const int32_t* nbr, int lattice, int interpolate, int dtype, const void* f_post,
               void* f_new, unsigned long long* d_fallback, hipStream_t s);
int launch_solid_change(int64_t n, const uint64_t* prev, const uint64_t* cur, uint64_t* spawned, uint64_t* covered,
                        unsigned long long* d_counts, hipStream_t s);
size_t geo2_bins_ws_bytes(int64_t nkeys);
size_t geo2_refine_ws_bytes(int64_t nb);
size_t geo2_cutlinks_ws_bytes(int64_t nb);
int launch_voxelize(const DevLevel& d, const int32_t* off, const int32_t* val, int64_t cap,
                    uint64_t* solid, hipStream_t s);
int launch_level0(const int32_t n0[3], int32_t* bcoord, hipStream_t s);
int launch_refine(const DevLevel& d, const uint64_t* solid, int n_prop, uint8_t* bclass,
                  uint8_t* refine, int32_t* child_map, int32_t* child_bcoord, int64_t* d_nchild,
                  void* ws, size_t ws_bytes, hipStream_t s);
int launch_cutlinks(const DevMesh& m, const DevLevel& d, const geo_bins* rows, const geo_bins* links,
                    int lattice, int precision, uint32_t* link_mask, int64_t cap, int64_t* d_nlinks,
                    int32_t* link_cell, uint8_t* link_dir, float* link_q, int32_t* link_tri,
                    uint64_t* d_stats, void* ws, size_t ws_bytes, hipStream_t s);
int launch_backward(const DevMesh& m, const DevLevel& d, int64_t n_links, const int32_t* link_cell,
                    const uint8_t* link_dir, const int32_t* link_tri, const float* grad_q,
                    float* grad_verts, hipStream_t s);

#define GEO_LAUNCH_CHECK()                                  \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return GEO_ERR_DEVICE; \
    } while (0)
