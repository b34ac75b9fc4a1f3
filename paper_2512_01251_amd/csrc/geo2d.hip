// The 2D form of the path (the paper notes that its octree discussion holds
// for quadtrees in 2D): cell blocks of 4x4, four children per refined block
// (octant o = ox + 2 oy), closed polygons given as edges, the D2Q9 lattice.
// Each step mirrors its 3D counterpart:
//   ROWS bins   -- per row line of the level, the edges whose closed y range
//                  holds the line (Spatial Binning);
//   LINKS bins  -- per block, the edges meeting the block box grown by half a
//                  cell (the 2D line-AABB overlap case of the appendix);
//   voxelize    -- a centre is solid iff it lies on an edge or the +x ray
//                  from it, lifted to y + eps, crosses an odd number of edges;
//   refinement  -- the 3D rules over the 8-neighbourhood;
//   cut links   -- fluid cell, D2Q9 direction, solid same-level neighbour
//                  centre; q = first crossing along the link.
// Coordinates are handled in level-L cell units (vertices scaled by 2^L,
// exact), where centres are i + 1/2; every sign is exact (floating-point
// filter, then the fixed-point accumulator).
#include "geo_internal.h"

namespace {

struct Dev2Level {
    int n0[2];
    int level;
    int nblocks;
    const int32_t* bcoord;
    const int32_t* child[GEO_MAX_LEVELS];
};

struct Dev2Mesh {
    int nv, ne;
    const double* verts;
    const int32_t* edges;
};

Dev2Level dev2_level(const geo2_level* lv) {
    Dev2Level d;
    d.n0[0] = lv->n0[0];
    d.n0[1] = lv->n0[1];
    d.level = lv->level;
    d.nblocks = lv->nblocks;
    d.bcoord = lv->bcoord;
    for (int l = 0; l < GEO_MAX_LEVELS; l++) d.child[l] = l < lv->level ? lv->child[l] : nullptr;
    return d;
}

Dev2Mesh dev2_mesh(const geo2_mesh* m) {
    Dev2Mesh d;
    d.nv = m->nv;
    d.ne = m->ne;
    d.verts = m->verts;
    d.edges = m->edges;
    return d;
}

// block (bx, by) of level L: its index, -1 if the forest lacks it, -2 outside
__device__ int forest_lookup2(const Dev2Level& d, int bx, int by) {
    const int L = d.level;
    const int nbx0 = d.n0[0] >> 2, nby0 = d.n0[1] >> 2;
    if (bx < 0 || by < 0 || bx >= (nbx0 << L) || by >= (nby0 << L)) return -2;
    int b = (by >> L) * nbx0 + (bx >> L);
    for (int l = 0; l < L; l++) {
        const int c = d.child[l][b];
        if (c < 0) return -1;
        const int s = L - 1 - l;
        b = c + (((bx >> s) & 1) | (((by >> s) & 1) << 1));
    }
    return b;
}

__device__ __forceinline__ int o2(double ax, double ay, double bx, double by, double cx, double cy) {
    const int s = orient2d_filter<double>(ax, ay, bx, by, cx, cy, 0.0);
    return s != 0 ? s : orient2d_exact(ax, ay, bx, by, cx, cy);
}

// edge e in level units; false for a zero-length edge or bad indices
__device__ __forceinline__ bool load_edge(const Dev2Mesh& m, int e, double scale, double* a, double* b) {
    const int i = m.edges[2 * (int64_t)e], j = m.edges[2 * (int64_t)e + 1];
    if (i < 0 || j < 0 || i >= m.nv || j >= m.nv) return false;
    a[0] = m.verts[2 * (int64_t)i] * scale;
    a[1] = m.verts[2 * (int64_t)i + 1] * scale;
    b[0] = m.verts[2 * (int64_t)j] * scale;
    b[1] = m.verts[2 * (int64_t)j + 1] * scale;
    return !(a[0] == b[0] && a[1] == b[1]);
}

// centre (px, py) of row j: solid iff on an edge of the row's bin or odd
// parity of lifted-ray crossings ahead of it
__device__ bool solid_point2(const Dev2Mesh& m, const int32_t* off, const int32_t* val, int64_t cap, double scale,
                             int j, double px, double py) {
    int e0 = off[j], e1 = off[j + 1];
    if (e0 < 0) e0 = 0;
    if (e1 > cap) e1 = (int)cap;
    bool on = false, parity = false;
    for (int q = e0; q < e1; q++) {
        const int e = val[q];
        if (e < 0 || e >= m.ne) continue;
        double a[2], b[2];
        if (!load_edge(m, e, scale, a, b)) continue;
        const double* lo = a[1] < b[1] ? a : b;
        const double* hi = a[1] < b[1] ? b : a;
        if (py < lo[1] || py > hi[1]) continue;
        const int s = o2(lo[0], lo[1], hi[0], hi[1], px, py);
        if (s == 0 && px >= fmin(a[0], b[0]) && px <= fmax(a[0], b[0])) on = true;
        if (a[1] != b[1] && py < hi[1] && s > 0) parity = !parity;
    }
    return on || parity;
}

// --------------------------------------------------------------------------
// bins
// --------------------------------------------------------------------------

// the closed segment [a, b] meets the box [x0, x1] x [y0, y1] (conservative:
// a near miss may count as a meeting)
__device__ bool segment_meets_box(const double* a, const double* b, double x0, double x1, double y0, double y1) {
    if (fmax(a[0], b[0]) < x0 || fmin(a[0], b[0]) > x1 || fmax(a[1], b[1]) < y0 || fmin(a[1], b[1]) > y1) return false;
    const double nx = -(b[1] - a[1]), ny = b[0] - a[0];
    const double cx[4] = {x0, x1, x0, x1}, cy[4] = {y0, y0, y1, y1};
    double lo = 0.0, hi = 0.0, mag = 0.0;
    for (int i = 0; i < 4; i++) {
        const double dx = cx[i] - a[0], dy = cy[i] - a[1];
        const double v = nx * dx + ny * dy;
        lo = i ? fmin(lo, v) : v;
        hi = i ? fmax(hi, v) : v;
        mag = fmax(mag, fabs(nx * dx) + fabs(ny * dy));
    }
    const double margin = 1e-12 * mag + 1e-300;
    return !(lo > margin || hi < -margin);
}

// kind 0 (ROWS): rows j with j + 1/2 in [ymin, ymax]; kind 1 (LINKS): blocks
// whose box grown by 1/2 the segment meets.  FILL = false counts into cnt,
// FILL = true places e at off[key] + cursor[key]++.  One wave per edge, its
// lanes splitting the edge's keys (a long edge covers hundreds of rows).
template <bool FILL>
__global__ void __launch_bounds__(256) k2_bins(Dev2Mesh m, Dev2Level d, int kind, double scale, int32_t* cnt,
                                               const int32_t* off, int32_t* cursor, int32_t* val, int64_t cap) {
    const int64_t ny = (int64_t)d.n0[1] << d.level;
    const int nbx = (d.n0[0] >> 2) << d.level, nby = (d.n0[1] >> 2) << d.level;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t e = wave; e < m.ne; e += nwaves) {
        double a[2], b[2];
        if (!load_edge(m, (int)e, scale, a, b)) continue;
        auto place = [&](int64_t key) {
            if (!FILL) {
                atomicAdd(&cnt[key], 1);
            } else {
                const int64_t p = (int64_t)off[key] + atomicAdd(&cursor[key], 1);
                if (p < cap) val[p] = (int32_t)e;
            }
        };
        if (kind == 0) {
            // clamped before the conversion (no overflow for any input)
            const double y0 = fmin(fmax(fmin(a[1], b[1]) - 0.5, -1.0), (double)ny);
            const double y1 = fmin(fmax(fmax(a[1], b[1]) - 0.5, -1.0), (double)ny);
            int64_t j0 = (int64_t)ceil(y0), j1 = (int64_t)floor(y1);
            if (j0 < 0) j0 = 0;
            if (j1 > ny - 1) j1 = ny - 1;
            for (int64_t j = j0 + lane; j <= j1; j += 64) place(j);
        } else {
            const double x0 = fmin(a[0], b[0]) - 0.5, x1 = fmax(a[0], b[0]) + 0.5;
            const double y0 = fmin(a[1], b[1]) - 0.5, y1 = fmax(a[1], b[1]) + 0.5;
            // blocks whose grown box [4 bx - 1/2, 4 bx + 9/2] meets [x0 + 1/2,
            // x1 - 1/2]: (x0 - 4) / 4 <= bx <= x1 / 4, closed at both ends (the
            // roundings are monotone; the 1e-7 only widens the range)
            int bx0 = (int)fmin(fmax(ceil((x0 - 4.0) / 4.0 - 1e-7), -1.0), (double)nbx);
            int bx1 = (int)fmin(fmax(floor(x1 / 4.0 + 1e-7), -1.0), (double)nbx);
            int by0 = (int)fmin(fmax(ceil((y0 - 4.0) / 4.0 - 1e-7), -1.0), (double)nby);
            int by1 = (int)fmin(fmax(floor(y1 / 4.0 + 1e-7), -1.0), (double)nby);
            if (bx0 < 0) bx0 = 0;
            if (by0 < 0) by0 = 0;
            if (bx1 > nbx - 1) bx1 = nbx - 1;
            if (by1 > nby - 1) by1 = nby - 1;
            const int sx = bx1 - bx0 + 1, sy = by1 - by0 + 1;
            const int64_t n = (sx > 0 && sy > 0) ? (int64_t)sx * sy : 0;
            for (int64_t it = lane; it < n; it += 64) {
                // n < 2^31 here (at most 8192^2 blocks on a level): 32-bit division
                const unsigned u = (unsigned)it, q = u / (unsigned)sx;
                const int bx = bx0 + (int)(u - q * (unsigned)sx), by = by0 + (int)q;
                if (!segment_meets_box(a, b, 4.0 * bx - 0.5, 4.0 * bx + 4.5, 4.0 * by - 0.5, 4.0 * by + 4.5)) continue;
                const int blk = forest_lookup2(d, bx, by);
                if (blk >= 0) place(blk);
            }
        }
    }
}

__global__ void k2_copy_count(const int32_t* off, int64_t nkeys, int64_t* d_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_count = off[nkeys];
}

__global__ void k2_level0(int nbx, int nby, int32_t* bcoord) {
    const int64_t n = (int64_t)nbx * nby;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        bcoord[2 * i] = (int32_t)(i % nbx);
        bcoord[2 * i + 1] = (int32_t)(i / nbx);
    }
}

// --------------------------------------------------------------------------
// voxelization: one thread per cell
// --------------------------------------------------------------------------

__global__ void k2_voxelize(Dev2Mesh m, Dev2Level d, const int32_t* off, const int32_t* val, int64_t cap,
                            double scale, uint16_t* solid) {
    const int64_t ncell = (int64_t)d.nblocks * 16;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = c >> 4;
        const int t = (int)(c & 15);
        const int i = 4 * d.bcoord[2 * b] + (t & 3), j = 4 * d.bcoord[2 * b + 1] + (t >> 2);
        const bool s = solid_point2(m, off, val, cap, scale, j, i + 0.5, j + 0.5);
        // gather the block's 16 bits: lanes of one block are consecutive
        const uint64_t bal = __ballot(s);
        const int lane = threadIdx.x & 63;
        if ((lane & 15) == 0) solid[b] = (uint16_t)((bal >> (lane & 48)) & 0xffff);
    }
}

// --------------------------------------------------------------------------
// refinement (rules as in 3D, 8-neighbourhood)
// --------------------------------------------------------------------------

constexpr int NB8 = 8;

__device__ __forceinline__ void n8_offset(int n, int& ox, int& oy) {
    const int k = n < 4 ? n : n + 1;  // skip the centre of the 3x3 stencil
    ox = k % 3 - 1;
    oy = k / 3 - 1;
}

// neighbour indices (-2 outside the domain, -1 missing), solid-boundary and
// eligibility flags
__global__ void k2_ref_a(Dev2Level d, const uint16_t* solid, int32_t* nbr, uint8_t* sb, uint8_t* elig) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < d.nblocks; b += (int64_t)gridDim.x * blockDim.x) {
        const int bx = d.bcoord[2 * b], by = d.bcoord[2 * b + 1];
        bool fluid_nbr = false, el = true;
        for (int n = 0; n < NB8; n++) {
            int ox, oy;
            n8_offset(n, ox, oy);
            const int k = forest_lookup2(d, bx + ox, by + oy);
            nbr[NB8 * b + n] = k;
            if (k == -1) el = false;
            if (k >= 0 && solid[k] == 0) fluid_nbr = true;
        }
        sb[b] = (uint8_t)(solid[b] != 0 && fluid_nbr);
        elig[b] = (uint8_t)el;
    }
}

__global__ void k2_ref_b(int64_t nb, const uint16_t* solid, const int32_t* nbr, const uint8_t* sb,
                         const uint8_t* elig, uint8_t* mark, uint8_t* bclass) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        bool adj = false;
        for (int n = 0; n < NB8; n++) {
            const int k = nbr[NB8 * b + n];
            if (k >= 0 && sb[k]) adj = true;
        }
        const bool m0 = sb[b] && elig[b];
        const bool mk = m0 || adj;
        mark[b] = (uint8_t)mk;
        bclass[b] = sb[b] ? 2 : (solid[b] ? 1 : ((mk && !m0) ? 3 : 0));
    }
}

__global__ void k2_ref_prop(int64_t nb, const uint16_t* solid, const int32_t* nbr, const uint8_t* mark_in,
                            uint8_t* mark_out, int first) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        bool mk = mark_in[b];
        if (!mk && (solid[b] == 0 || first))
            for (int n = 0; n < NB8; n++) {
                const int k = nbr[NB8 * b + n];
                if (k >= 0 && mark_in[k]) mk = true;
            }
        mark_out[b] = (uint8_t)mk;
    }
}

__global__ void k2_ref_final(int64_t nb, const uint8_t* mark, const uint8_t* elig, uint8_t* refine, int32_t* cnt) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        const bool r = mark[b] && elig[b];
        refine[b] = (uint8_t)r;
        cnt[b] = r ? 4 : 0;
    }
}

__global__ void k2_ref_emit(Dev2Level d, const uint8_t* refine, const int32_t* off, int32_t* child_map,
                            int32_t* child_bcoord, int64_t* d_nchild) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < d.nblocks; b += (int64_t)gridDim.x * blockDim.x) {
        if (!refine[b]) {
            child_map[b] = -1;
            continue;
        }
        const int c = off[b];
        child_map[b] = c;
        for (int o = 0; o < 4; o++) {
            child_bcoord[2 * (int64_t)(c + o)] = 2 * d.bcoord[2 * b] + (o & 1);
            child_bcoord[2 * (int64_t)(c + o) + 1] = 2 * d.bcoord[2 * b + 1] + (o >> 1);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *d_nchild = off[d.nblocks];
}

// --------------------------------------------------------------------------
// cut links: one wave per block; lanes 0..35 classify the 6x6 halo, lanes
// 0..15 are the block's cells
// --------------------------------------------------------------------------

// link masks (bit k: D2Q9 direction k) of the block's cells, from the halo
__device__ uint16_t cell_mask2(const Dev2Mesh& m, const Dev2Level& d, const int32_t* roff, const int32_t* rval,
                               int64_t rcap, double scale, int64_t b, uint8_t* halo) {
    const int lane = threadIdx.x;
    const int nx = d.n0[0] << d.level, ny = d.n0[1] << d.level;
    if (lane < 36) {
        const int I = lane % 6 - 1, J = lane / 6 - 1;
        const int i = 4 * d.bcoord[2 * b] + I, j = 4 * d.bcoord[2 * b + 1] + J;
        bool s = false;
        if (i >= 0 && j >= 0 && i < nx && j < ny) s = solid_point2(m, roff, rval, rcap, scale, j, i + 0.5, j + 0.5);
        halo[lane] = (uint8_t)s;
    }
    __syncthreads();
    uint16_t mk = 0;
    if (lane < 16) {
        const int I = lane & 3, J = lane >> 2;
        if (!halo[(I + 1) + 6 * (J + 1)])
            for (int k = 0; k < 9; k++) {
                if (k == 4) continue;
                if (halo[(I + 1 + k % 3 - 1) + 6 * (J + 1 + k / 3 - 1)]) mk |= (uint16_t)(1u << k);
            }
    }
    __syncthreads();
    return mk;
}

__global__ void __launch_bounds__(64) k2_cl_count(Dev2Mesh m, Dev2Level d, const int32_t* roff, const int32_t* rval,
                                                  int64_t rcap, double scale, uint16_t* mask, int32_t* cnt) {
    __shared__ uint8_t halo[36];
    for (int64_t b = blockIdx.x; b < d.nblocks; b += gridDim.x) {
        const uint16_t mk = cell_mask2(m, d, roff, rval, rcap, scale, b, halo);
        int c = threadIdx.x < 16 ? __popc(mk) : 0;
        if (threadIdx.x < 16) mask[16 * b + threadIdx.x] = mk;
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (threadIdx.x == 0) cnt[b] = c;
    }
}

// first meeting of the link X -> X + c (level units) with the closed segment
// [a, b]: t in (0, 1], or a negative value when they do not meet (X on no edge)
__device__ double link_hit2(const double* a, const double* b, double X0, double X1, double c0, double c1) {
    const double Y0 = X0 + c0, Y1 = X1 + c1;
    const int s1 = o2(a[0], a[1], b[0], b[1], X0, X1);
    const int s2 = o2(a[0], a[1], b[0], b[1], Y0, Y1);
    if (s1 == 0 && s2 == 0) {
        const double dd = c0 * c0 + c1 * c1;
        const double ta = ((a[0] - X0) * c0 + (a[1] - X1) * c1) / dd;
        const double tb = ((b[0] - X0) * c0 + (b[1] - X1) * c1) / dd;
        const double lo = fmin(ta, tb), hi = fmax(ta, tb);
        return (hi < 0.0 || lo > 1.0) ? -1.0 : lo;
    }
    if (s1 * s2 > 0) return -1.0;
    const int s3 = o2(X0, X1, Y0, Y1, a[0], a[1]);
    const int s4 = o2(X0, X1, Y0, Y1, b[0], b[1]);
    if (s3 * s4 > 0) return -1.0;
    const double ex = b[0] - a[0], ey = b[1] - a[1];
    const double num = (a[0] - X0) * ey - (a[1] - X1) * ex;
    const double den = c0 * ey - c1 * ex;
    return num / den;
}

__global__ void __launch_bounds__(64) k2_cl_fill(Dev2Mesh m, Dev2Level d, const int32_t* loff, const int32_t* lval,
                                                 int64_t lcap, double scale, const uint16_t* mask,
                                                 const int32_t* off, int64_t cap, int32_t* link_cell,
                                                 uint8_t* link_dir, float* link_q, int32_t* link_edge) {
    // the block's candidate edges, 64 at a time, staged in LDS by the whole wave
    __shared__ double sa[64][2], sb[64][2];
    __shared__ int sid[64];
    const int lane = threadIdx.x;
    for (int64_t b = blockIdx.x; b < d.nblocks; b += gridDim.x) {
        const uint16_t mk = lane < 16 ? mask[16 * b + lane] : 0;
        // exclusive prefix of the cells' link counts in cell order
        const int c = __popc(mk);
        int incl = c;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if ((lane & 15) >= o) incl += v;
        }
        const int64_t pos0 = (int64_t)off[b] + incl - c;
        if (!__any(mk != 0)) continue;  // uniform
        const double X0 = 4 * d.bcoord[2 * b] + (lane & 3) + 0.5, X1 = 4 * d.bcoord[2 * b + 1] + (lane >> 2) + 0.5;
        int e0 = loff[b], e1 = loff[b + 1];
        if (e0 < 0) e0 = 0;
        if (e1 > lcap) e1 = (int)lcap;
        double best[9];
        int be[9];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            best[k] = 2.0;
            be[k] = -1;
        }
        for (int c0 = e0; c0 < e1; c0 += 64) {  // uniform
            const int nc = e1 - c0 < 64 ? e1 - c0 : 64;
            __syncthreads();
            if (lane < nc) {
                const int e = lval[c0 + lane];
                double a[2], bb[2];
                const bool ok = e >= 0 && e < m.ne && load_edge(m, e, scale, a, bb);
                sid[lane] = ok ? e : -1;
                sa[lane][0] = a[0];
                sa[lane][1] = a[1];
                sb[lane][0] = bb[0];
                sb[lane][1] = bb[1];
            }
            __syncthreads();
            if (mk) {
#pragma unroll
                for (int k = 0; k < 9; k++) {
                    if (!((mk >> k) & 1)) continue;
                    const double cx = k % 3 - 1, cy = k / 3 - 1;
                    for (int q = 0; q < nc; q++) {
                        const int e = sid[q];
                        if (e < 0) continue;
                        const double a[2] = {sa[q][0], sa[q][1]}, bb[2] = {sb[q][0], sb[q][1]};
                        const double t = link_hit2(a, bb, X0, X1, cx, cy);
                        if (t < 0.0) continue;
                        if (t < best[k] || (t == best[k] && e < be[k])) {
                            best[k] = t;
                            be[k] = e;
                        }
                    }
                }
            }
        }
        if (!mk) continue;
        int64_t pos = pos0;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            if (!((mk >> k) & 1)) continue;
            if (pos < cap) {
                link_cell[pos] = (int32_t)(16 * b + lane);
                link_dir[pos] = (uint8_t)k;
                link_q[pos] = be[k] >= 0 ? (float)best[k] : -1.0f;
                link_edge[pos] = be[k];
            }
            pos++;
        }
    }
}

unsigned grid1(int64_t n, int threads, int64_t cap_blocks) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap_blocks) g = cap_blocks;
    return (unsigned)g;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool check2_level(const geo2_level* lv) {
    if (!lv || lv->level < 0 || lv->level >= GEO_MAX_LEVELS || lv->nblocks < 0) return false;
    for (int a = 0; a < 2; a++) {
        if (lv->n0[a] <= 0 || lv->n0[a] % 4 != 0) return false;
        if ((int64_t)lv->n0[a] << lv->level > GEO_MAX_RES) return false;
    }
    if (lv->nblocks > 0 && !lv->bcoord) return false;
    if ((int64_t)lv->nblocks * 16 > INT32_MAX) return false;
    if (lv->nblocks > 0)
        for (int l = 0; l < lv->level; l++)
            if (!lv->child[l]) return false;
    return true;
}

bool check2_mesh(const geo2_mesh* m) {
    if (!m || m->nv < 0 || m->ne < 0) return false;
    if (m->ne > 0 && (!m->verts || !m->edges || m->nv == 0)) return false;
    return (int64_t)m->ne * 2 <= INT32_MAX && (int64_t)m->nv * 2 <= INT32_MAX;
}

bool check2_bins(const geo_bins* b, int kind, int64_t nkeys) {
    return b && b->kind == kind && b->nkeys == nkeys && b->off && b->d_count && b->cap >= 0 && (b->cap == 0 || b->val);
}

int64_t row_keys2(const geo2_level* lv) { return (int64_t)lv->n0[1] << lv->level; }

}  // namespace

size_t geo2_bins_ws_bytes(int64_t nkeys) {
    return 2 * al256(sizeof(int32_t) * (size_t)(nkeys + 1)) + al256(geo_scan_partials_bytes(nkeys));
}

size_t geo2_refine_ws_bytes(int64_t nb) {
    return al256(sizeof(int32_t) * NB8 * (size_t)nb) + 4 * al256((size_t)nb) +
           2 * al256(sizeof(int32_t) * (size_t)(nb + 1)) + al256(geo_scan_partials_bytes(nb));
}

size_t geo2_cutlinks_ws_bytes(int64_t nb) {
    return al256(sizeof(uint16_t) * 16 * (size_t)nb) + 2 * al256(sizeof(int32_t) * (size_t)(nb + 1)) +
           al256(geo_scan_partials_bytes(nb));
}

extern "C" {

int geo2_level0_blocks(const int32_t n0[2], int32_t* bcoord, geo_stream_t stream) {
    if (!n0 || !bcoord) return GEO_ERR_ARG;
    for (int a = 0; a < 2; a++)
        if (n0[a] <= 0 || n0[a] % 4 != 0 || n0[a] > GEO_MAX_RES) return GEO_ERR_ARG;
    const int nbx = n0[0] / 4, nby = n0[1] / 4;
    hipStream_t s = (hipStream_t)stream;
    k2_level0<<<grid1((int64_t)nbx * nby, 256, 4096), 256, 0, s>>>(nbx, nby, bcoord);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo2_build_bins(const geo2_mesh* mesh, const geo2_level* lv, int32_t kind, geo_bins* bins, void* ws,
                    size_t ws_bytes, geo_stream_t stream) {
    if (!check2_mesh(mesh) || !check2_level(lv)) return GEO_ERR_ARG;
    if (kind != GEO_BINS_ROWS && kind != GEO_BINS_LINKS) return GEO_ERR_ARG;
    const int64_t nkeys = kind == GEO_BINS_ROWS ? row_keys2(lv) : (int64_t)lv->nblocks;
    if (!check2_bins(bins, kind, nkeys) || nkeys + 1 > INT32_MAX) return GEO_ERR_ARG;
    if (!ws || ws_bytes < geo2_bins_ws_bytes(nkeys)) return GEO_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* p = static_cast<char*>(ws);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nkeys + 1));
    int32_t* cursor = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nkeys + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    int rc = geo_fill_i32(cnt, 0, nkeys + 1, s);
    if (rc == GEO_OK) rc = geo_fill_i32(cursor, 0, nkeys + 1, s);
    if (rc != GEO_OK) return rc;
    const Dev2Mesh m = dev2_mesh(mesh);
    const Dev2Level d = dev2_level(lv);
    const double scale = ldexp(1.0, lv->level);
    const int kk = kind == GEO_BINS_ROWS ? 0 : 1;
    const unsigned g = grid1((int64_t)mesh->ne * 64, 256, 8192);  // one wave per edge
    if (mesh->ne > 0) k2_bins<false><<<g, 256, 0, s>>>(m, d, kk, scale, cnt, nullptr, nullptr, nullptr, 0);
    GEO_LAUNCH_CHECK();
    rc = geo_scan_exclusive(cnt, bins->off, nkeys, partials, s);
    if (rc != GEO_OK) return rc;
    k2_copy_count<<<1, 64, 0, s>>>(bins->off, nkeys, bins->d_count);
    if (mesh->ne > 0)
        k2_bins<true><<<g, 256, 0, s>>>(m, d, kk, scale, nullptr, bins->off, cursor, bins->val, bins->cap);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo2_voxelize(const geo2_mesh* mesh, const geo2_level* lv, const geo_bins* rows, uint16_t* solid,
                  geo_stream_t stream) {
    if (!check2_mesh(mesh) || !check2_level(lv)) return GEO_ERR_ARG;
    if (!check2_bins(rows, GEO_BINS_ROWS, row_keys2(lv))) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && !solid) return GEO_ERR_ARG;
    if (lv->nblocks == 0) return GEO_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t ncell = (int64_t)lv->nblocks * 16;
    k2_voxelize<<<grid1(ncell, 256, 65536), 256, 0, s>>>(dev2_mesh(mesh), dev2_level(lv), rows->off, rows->val,
                                                        rows->cap, ldexp(1.0, lv->level), solid);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo2_refine_flags(const geo2_level* lv, const uint16_t* solid, int32_t n_prop, uint8_t* bclass, uint8_t* refine,
                      int32_t* child_map, int32_t* child_bcoord, int64_t* d_nchild, void* ws, size_t ws_bytes,
                      geo_stream_t stream) {
    if (!check2_level(lv) || n_prop < 1 || !d_nchild) return GEO_ERR_ARG;
    const int64_t nb = lv->nblocks;
    if (nb > 0 && (!solid || !bclass || !refine || !child_map || !child_bcoord)) return GEO_ERR_ARG;
    if ((int64_t)nb * 4 > INT32_MAX) return GEO_ERR_ARG;
    if (!ws || ws_bytes < geo2_refine_ws_bytes(nb)) return GEO_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* p = static_cast<char*>(ws);
    int32_t* nbr = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * NB8 * (size_t)nb);
    uint8_t* sb = reinterpret_cast<uint8_t*>(p);
    p += al256((size_t)nb);
    uint8_t* elig = reinterpret_cast<uint8_t*>(p);
    p += al256((size_t)nb);
    uint8_t* m0 = reinterpret_cast<uint8_t*>(p);
    p += al256((size_t)nb);
    uint8_t* m1 = reinterpret_cast<uint8_t*>(p);
    p += al256((size_t)nb);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* off = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    const Dev2Level d = dev2_level(lv);
    const unsigned g = grid1(nb, 256, 16384);
    if (nb > 0) {
        k2_ref_a<<<g, 256, 0, s>>>(d, solid, nbr, sb, elig);
        k2_ref_b<<<g, 256, 0, s>>>(nb, solid, nbr, sb, elig, m0, bclass);
        for (int k = 1; k <= n_prop; k++) {
            k2_ref_prop<<<g, 256, 0, s>>>(nb, solid, nbr, m0, m1, k == 1);
            uint8_t* t = m0;
            m0 = m1;
            m1 = t;
        }
        k2_ref_final<<<g, 256, 0, s>>>(nb, m0, elig, refine, cnt);
        GEO_LAUNCH_CHECK();
    }
    const int rc = geo_scan_exclusive(cnt, off, nb, partials, s);
    if (rc != GEO_OK) return rc;
    k2_ref_emit<<<g, 256, 0, s>>>(d, refine, off, child_map, child_bcoord, d_nchild);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

int geo2_cutlinks(const geo2_mesh* mesh, const geo2_level* lv, const geo_bins* rows, const geo_bins* links,
                  int64_t cap, int64_t* d_nlinks, int32_t* link_cell, uint8_t* link_dir, float* link_q,
                  int32_t* link_edge, void* ws, size_t ws_bytes, geo_stream_t stream) {
    if (!check2_mesh(mesh) || !check2_level(lv) || cap < 0 || !d_nlinks) return GEO_ERR_ARG;
    if (!check2_bins(rows, GEO_BINS_ROWS, row_keys2(lv))) return GEO_ERR_ARG;
    if (!check2_bins(links, GEO_BINS_LINKS, lv->nblocks)) return GEO_ERR_ARG;
    if (cap > 0 && (!link_cell || !link_dir || !link_q || !link_edge)) return GEO_ERR_ARG;
    const int64_t nb = lv->nblocks;
    if (!ws || ws_bytes < geo2_cutlinks_ws_bytes(nb)) return GEO_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* p = static_cast<char*>(ws);
    uint16_t* mask = reinterpret_cast<uint16_t*>(p);
    p += al256(sizeof(uint16_t) * 16 * (size_t)nb);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* off = reinterpret_cast<int32_t*>(p);
    p += al256(sizeof(int32_t) * (size_t)(nb + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    const Dev2Mesh m = dev2_mesh(mesh);
    const Dev2Level d = dev2_level(lv);
    const double scale = ldexp(1.0, lv->level);
    const unsigned g = grid1(nb, 1, 65536);
    if (nb > 0) k2_cl_count<<<g, 64, 0, s>>>(m, d, rows->off, rows->val, rows->cap, scale, mask, cnt);
    GEO_LAUNCH_CHECK();
    const int rc = geo_scan_exclusive(cnt, off, nb, partials, s);
    if (rc != GEO_OK) return rc;
    k2_copy_count<<<1, 64, 0, s>>>(off, nb, d_nlinks);
    if (nb > 0)
        k2_cl_fill<<<g, 64, 0, s>>>(m, d, links->off, links->val, links->cap, scale, mask, off, cap, link_cell,
                                    link_dir, link_q, link_edge);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}

}  // extern "C"
