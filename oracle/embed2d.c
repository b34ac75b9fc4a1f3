/* The 2D form of the embedding (the paper's quadtree case: 4x4 cell blocks,
 * four children per refined block, the D2Q9 lattice), written out plainly:
 * brute-force candidate lists, exact orientation signs.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle; shares no code with the GPU
 * library).
 *
 * Geometry: closed polygons given as edges (a, b) of a vertex array [nv][2].
 * A point is solid iff it lies in the closed region they bound: on an edge, or
 * with odd parity of the edges crossed by the +x ray from it, the ray lifted
 * to height y + eps (simulation of simplicity), so that a horizontal edge is
 * never crossed and an edge counts once at a shared vertex.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define P2(V, i) ((V) + 2 * (int64_t)(i))

static inline double centre2(int64_t i, int L) { return ldexp((double)i + 0.5, -L); }

static int degenerate(const double* a, const double* b) { return a[0] == b[0] && a[1] == b[1]; }

/* p on the closed segment [a, b] */
static int on_segment(const double* a, const double* b, const double* p) {
    if (or_orient2d(a[0], a[1], b[0], b[1], p[0], p[1]) != 0) return 0;
    return p[0] >= fmin(a[0], b[0]) && p[0] <= fmax(a[0], b[0]) && p[1] >= fmin(a[1], b[1]) &&
           p[1] <= fmax(a[1], b[1]);
}

/* the lifted +x ray from p crosses [a, b] ahead of p (p on no edge) */
static int ray_crosses2(const double* a, const double* b, const double* p) {
    if (a[1] == b[1]) return 0;
    const double* lo = a[1] < b[1] ? a : b;
    const double* hi = a[1] < b[1] ? b : a;
    if (!(lo[1] <= p[1] && p[1] < hi[1])) return 0;
    /* p left of the upward edge lo -> hi: the crossing lies at larger x */
    return or_orient2d(lo[0], lo[1], hi[0], hi[1], p[0], p[1]) > 0;
}

int or2_solid_point(const double* V, const int32_t* E, const int32_t* cand, int n, const double* p) {
    for (int i = 0; i < n; i++) {
        const double *a = P2(V, E[2 * cand[i]]), *b = P2(V, E[2 * cand[i] + 1]);
        if (!degenerate(a, b) && on_segment(a, b, p)) return 1;
    }
    int parity = 0;
    for (int i = 0; i < n; i++) {
        const double *a = P2(V, E[2 * cand[i]]), *b = P2(V, E[2 * cand[i] + 1]);
        if (!degenerate(a, b)) parity ^= ray_crosses2(a, b, p);
    }
    return parity;
}

/* per row line j of level L (centre height y_j): the edges whose closed y
 * range contains y_j, as CSR lists */
typedef struct {
    int64_t ny;
    int64_t* off;
    int32_t* val;
} rowlists;

static void rows_build(rowlists* R, const double* V, const int32_t* E, int ne, int64_t ny, int L) {
    R->ny = ny;
    R->off = (int64_t*)calloc(ny + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; pass++) {
        int64_t* cur = pass ? (int64_t*)malloc(sizeof(int64_t) * (ny + 1)) : NULL;
        if (pass) memcpy(cur, R->off, sizeof(int64_t) * (ny + 1));
        for (int e = 0; e < ne; e++) {
            const double *a = P2(V, E[2 * e]), *b = P2(V, E[2 * e + 1]);
            if (degenerate(a, b)) continue;
            double y0 = fmin(a[1], b[1]), y1 = fmax(a[1], b[1]);
            /* rows with y_j = (j + 1/2) 2^-L in [y0, y1] */
            int64_t j0 = (int64_t)ceil(ldexp(y0, L) - 0.5), j1 = (int64_t)floor(ldexp(y1, L) - 0.5);
            if (j0 < 0) j0 = 0;
            if (j1 > ny - 1) j1 = ny - 1;
            for (int64_t j = j0; j <= j1; j++) {
                if (!pass) R->off[j + 1]++;
                else R->val[cur[j]++] = e;
            }
        }
        if (!pass) {
            for (int64_t j = 0; j < ny; j++) R->off[j + 1] += R->off[j];
            R->val = (int32_t*)malloc(sizeof(int32_t) * (R->off[ny] > 0 ? R->off[ny] : 1));
        } else {
            free(cur);
        }
    }
}

static void rows_free(rowlists* R) {
    free(R->off);
    free(R->val);
}

/* Classify the cells of level-L blocks (halo = 0: 16 per block, t = I + 4J)
 * or each block's one-cell halo (halo = 1: 36 per block, (I+1) + 6(J+1),
 * I, J in -1..4).  Points outside the domain are fluid. */
void or2_classify_blocks(const double* V, const int32_t* E, int ne, const int32_t* n0, int L, int64_t nb,
                         const int32_t* bcoord, int halo, uint8_t* out) {
    int64_t nx = (int64_t)n0[0] << L, ny = (int64_t)n0[1] << L;
    rowlists R;
    rows_build(&R, V, E, ne, ny, L);
    int lo = halo ? -1 : 0, hi = halo ? 4 : 3, w = hi - lo + 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < nb; b++) {
        uint8_t* o = out + b * (int64_t)w * w;
        for (int J = lo; J <= hi; J++) {
            int64_t j = 4 * (int64_t)bcoord[2 * b + 1] + J;
            for (int I = lo; I <= hi; I++) {
                int64_t i = 4 * (int64_t)bcoord[2 * b] + I;
                int idx = (I - lo) + w * (J - lo);
                if (j < 0 || j >= ny || i < 0 || i >= nx) { o[idx] = 0; continue; }
                double p[2] = {centre2(i, L), centre2(j, L)};
                o[idx] = (uint8_t)or2_solid_point(V, E, R.val + R.off[j], (int)(R.off[j + 1] - R.off[j]), p);
            }
        }
    }
    rows_free(&R);
}

/* ------------------------------------------------------------------------- */
/* refinement (the same rules as in 3D, over the 8-neighbourhood)             */
/* ------------------------------------------------------------------------- */

int64_t or2_refine(const int32_t* n0, int L, int64_t nb, const int32_t* bcoord, const uint8_t* solid, int n_prop,
                   uint8_t* bclass, uint8_t* refine, int32_t* child_map, int32_t* child_bcoord) {
    int64_t dx_ = ((int64_t)n0[0] / 4) << L, dy_ = ((int64_t)n0[1] / 4) << L;
    int32_t* map = (int32_t*)malloc(sizeof(int32_t) * dx_ * dy_);
    for (int64_t i = 0; i < dx_ * dy_; i++) map[i] = -1;
    for (int64_t b = 0; b < nb; b++) map[(int64_t)bcoord[2 * b + 1] * dx_ + bcoord[2 * b]] = (int32_t)b;
    uint8_t *S = calloc(nb, 1), *SB = calloc(nb, 1), *el = calloc(nb, 1), *M = calloc(nb, 1), *Mn = calloc(nb, 1);
    for (int64_t b = 0; b < nb; b++) {
        int s = 0;
        for (int t = 0; t < 16; t++) s |= solid[16 * b + t];
        S[b] = (uint8_t)s;
    }
#define FOR_N8(b, body)                                                                      \
    for (int oy = -1; oy <= 1; oy++)                                                         \
        for (int ox = -1; ox <= 1; ox++) {                                                   \
            if (!ox && !oy) continue;                                                        \
            int64_t x = bcoord[2 * (b)] + ox, y = bcoord[2 * (b) + 1] + oy;                  \
            int in_domain = x >= 0 && y >= 0 && x < dx_ && y < dy_;                          \
            int64_t n = in_domain ? map[y * dx_ + x] : -1;                                   \
            body                                                                             \
        }
    for (int64_t b = 0; b < nb; b++) {
        int sb = 0, e = 1;
        FOR_N8(b, {
            if (in_domain && n < 0) e = 0;
            if (n >= 0 && !S[n]) sb = 1;
        })
        SB[b] = (uint8_t)(S[b] && sb);
        el[b] = (uint8_t)e;
    }
    for (int64_t b = 0; b < nb; b++) {
        int adj = 0;
        FOR_N8(b, { if (n >= 0 && SB[n]) adj = 1; })
        int m0 = SB[b] && el[b];
        M[b] = (uint8_t)(m0 || adj);
        bclass[b] = SB[b] ? 2 : (S[b] ? 1 : ((M[b] && !m0) ? 3 : 0));
    }
    for (int k = 1; k <= n_prop; k++) {
        for (int64_t b = 0; b < nb; b++) {
            int join = 0;
            if (!S[b] || k == 1) { FOR_N8(b, { if (n >= 0 && M[n]) join = 1; }) }
            Mn[b] = (uint8_t)(M[b] || join);
        }
        memcpy(M, Mn, nb);
    }
#undef FOR_N8
    int64_t nch = 0;
    for (int64_t b = 0; b < nb; b++) {
        refine[b] = (uint8_t)(M[b] && el[b]);
        if (refine[b]) {
            child_map[b] = (int32_t)nch;
            for (int o = 0; o < 4; o++) {
                child_bcoord[2 * nch] = 2 * bcoord[2 * b] + (o & 1);
                child_bcoord[2 * nch + 1] = 2 * bcoord[2 * b + 1] + (o >> 1);
                nch++;
            }
        } else {
            child_map[b] = -1;
        }
    }
    free(map); free(S); free(SB); free(el); free(M); free(Mn);
    return nch;
}

/* ------------------------------------------------------------------------- */
/* cut links (D2Q9: k = (cx+1) + 3(cy+1), 4 is the rest direction)            */
/* ------------------------------------------------------------------------- */

/* First point of [X, Y] on the closed segment [a, b] as a fraction t of the
 * link, X on no edge.  Returns 0 when they do not meet. */
static int segment_hit2(const double* a, const double* b, const double* X, const double* Y, long double* t) {
    int o1 = or_orient2d(a[0], a[1], b[0], b[1], X[0], X[1]);
    int o2 = or_orient2d(a[0], a[1], b[0], b[1], Y[0], Y[1]);
    long double dx = (long double)Y[0] - X[0], dy = (long double)Y[1] - X[1];
    if (o1 == 0 && o2 == 0) {
        /* collinear: the segment's span along the link */
        long double dd = dx * dx + dy * dy;
        long double ta = (((long double)a[0] - X[0]) * dx + ((long double)a[1] - X[1]) * dy) / dd;
        long double tb = (((long double)b[0] - X[0]) * dx + ((long double)b[1] - X[1]) * dy) / dd;
        long double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
        if (hi < 0 || lo > 1) return 0;
        *t = lo;
        return 1;
    }
    if ((o1 > 0 && o2 > 0) || (o1 < 0 && o2 < 0)) return 0;
    int o3 = or_orient2d(X[0], X[1], Y[0], Y[1], a[0], a[1]);
    int o4 = or_orient2d(X[0], X[1], Y[0], Y[1], b[0], b[1]);
    if ((o3 > 0 && o4 > 0) || (o3 < 0 && o4 < 0)) return 0;
    long double ex = (long double)b[0] - a[0], ey = (long double)b[1] - a[1];
    long double num = ((long double)a[0] - X[0]) * ey - ((long double)a[1] - X[1]) * ex;
    long double den = dx * ey - dy * ex;
    *t = num / den;
    return 1;
}

/* Cut links of level L (fluid cell, D2Q9 direction, solid same-level
 * neighbour centre), order (block, t, k); q = first crossing of the polygon
 * boundary; edge = the smallest index among the edges whose crossing
 * parameters agree within 1e-12 of the minimum (tied set when more than one).
 * Returns the number of links; entries beyond cap are not written. */
int64_t or2_links(const double* V, const int32_t* E, int ne, const int32_t* n0, int L, int64_t nb,
                  const int32_t* bcoord, int64_t cap, uint16_t* mask_out, int32_t* link_cell, uint8_t* link_dir,
                  double* link_q, int32_t* link_edge, uint8_t* link_tied) {
    uint8_t* halo = (uint8_t*)malloc((size_t)nb * 36 + 1);
    or2_classify_blocks(V, E, ne, n0, L, nb, bcoord, 1, halo);
    int64_t* off = (int64_t*)calloc(nb + 1, sizeof(int64_t));
    for (int64_t b = 0; b < nb; b++) {
        const uint8_t* H = halo + 36 * b;
        for (int t = 0; t < 16; t++) {
            int I = t & 3, J = t >> 2;
            uint16_t m = 0;
            if (!H[(I + 1) + 6 * (J + 1)])
                for (int k = 0; k < 9; k++) {
                    if (k == 4) continue;
                    int cx = k % 3 - 1, cy = k / 3 - 1;
                    if (H[(I + 1 + cx) + 6 * (J + 1 + cy)]) m |= (uint16_t)(1u << k);
                }
            mask_out[16 * b + t] = m;
            off[b + 1] += __builtin_popcount(m);
        }
    }
    for (int64_t b = 0; b < nb; b++) off[b + 1] += off[b];
    double h = ldexp(1.0, -L);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t b = 0; b < nb; b++) {
        int64_t pos = off[b];
        for (int t = 0; t < 16; t++) {
            uint16_t m = mask_out[16 * b + t];
            if (!m) continue;
            double X[2] = {centre2(4 * (int64_t)bcoord[2 * b] + (t & 3), L),
                           centre2(4 * (int64_t)bcoord[2 * b + 1] + (t >> 2), L)};
            for (int k = 0; k < 9; k++) {
                if (!(m >> k & 1)) continue;
                double Y[2] = {X[0] + (k % 3 - 1) * h, X[1] + (k / 3 - 1) * h};
                double lo[2] = {fmin(X[0], Y[0]), fmin(X[1], Y[1])}, hi[2] = {fmax(X[0], Y[0]), fmax(X[1], Y[1])};
                long double best = 2.0L;
                int be = -1, tied = 0;
                for (int e = 0; e < ne; e++) {
                    const double *a = P2(V, E[2 * e]), *c = P2(V, E[2 * e + 1]);
                    if (degenerate(a, c)) continue;
                    if (fmax(a[0], c[0]) < lo[0] || fmin(a[0], c[0]) > hi[0] || fmax(a[1], c[1]) < lo[1] ||
                        fmin(a[1], c[1]) > hi[1])
                        continue;
                    long double tv;
                    if (!segment_hit2(a, c, X, Y, &tv)) continue;
                    if (be < 0 || tv < best - 1e-12L) {
                        tied = be >= 0 && tv > best - 1e-12L;
                        best = tv;
                        be = e;
                    } else if (fabsl(tv - best) <= 1e-12L) {
                        tied = 1;
                        if (tv < best) best = tv;
                    }
                }
                if (pos < cap) {
                    link_cell[pos] = (int32_t)(16 * b + t);
                    link_dir[pos] = (uint8_t)k;
                    link_q[pos] = be >= 0 ? (double)best : -1.0;
                    link_edge[pos] = be;
                    link_tied[pos] = (uint8_t)tied;
                }
                pos++;
            }
        }
    }
    int64_t total = off[nb];
    free(halo);
    free(off);
    return total;
}
