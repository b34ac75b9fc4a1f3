/*
 * CPU oracle of the geometry-embedding hot path (test infrastructure only).
 *
 * Plain definitions, evaluated point by point with the exact predicates of
 * exact.c.  The only acceleration is a uniform bucket grid that lists, for a
 * query point or segment, the triangles whose closed bounding box can contain
 * it; a triangle outside that list can neither contain the point nor be
 * crossed by its +x ray or segment, so the filter never changes a result.
 *
 * Coordinates are base-cell units; level L has cell size h = 2^-L, cell centres
 * at (i + 1/2) h, blocks of 4x4x4 cells, local cell index t = I + 4 J + 16 K
 * (the paper's LINEAR(I, 4), Methodology, "Partial Surface Voxelization").
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define V3(V, i) ((V) + 3 * (int64_t)(i))

/* ------------------------------------------------------------------------- */
/* bucket grids                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    int dim;           /* 2: (y,z) buckets, 3: (x,y,z) buckets */
    double s;          /* bucket edge (base units) */
    int nb[3];
    int64_t* off;      /* CSR offsets */
    int32_t* ids;
} buckets;

static double tri_extent_median(const double* V, const int32_t* T, int nt) {
    int n = nt < 4096 ? nt : 4096;
    if (n == 0) return 1.0;
    double* e = (double*)malloc(sizeof(double) * n);
    for (int k = 0; k < n; k++) {
        int64_t i = (int64_t)k * nt / n;
        double m = 0;
        for (int a = 0; a < 3; a++) {
            double lo = 1e300, hi = -1e300;
            for (int v = 0; v < 3; v++) {
                double x = V3(V, T[3 * i + v])[a];
                lo = x < lo ? x : lo;
                hi = x > hi ? x : hi;
            }
            m = hi - lo > m ? hi - lo : m;
        }
        e[k] = m;
    }
    /* crude median by partial selection */
    for (int i = 0; i <= n / 2; i++)
        for (int j = i + 1; j < n; j++)
            if (e[j] < e[i]) { double t = e[i]; e[i] = e[j]; e[j] = t; }
    double r = e[n / 2];
    free(e);
    return r;
}

static void buckets_build(buckets* B, int dim, const double* V, const int32_t* T, int nt,
                          const int32_t* n0) {
    double med = tri_extent_median(V, T, nt);
    double s = 1.0;
    while (s > med && s > 1.0 / 64) s *= 0.5;
    while (s < 2 * med && s < 4.0) s *= 2.0;
    B->dim = dim;
    B->s = s;
    int ax0 = dim == 2 ? 1 : 0;
    for (int a = 0; a < 3; a++) B->nb[a] = 1;
    for (int a = ax0; a < 3; a++) B->nb[a] = (int)ceil(n0[a] / s) + 1;
    int64_t nbk = (int64_t)B->nb[0] * B->nb[1] * B->nb[2];
    /* a surface fills few cells of a 3D grid: keep the grid to 2^25 buckets */
    while (dim == 3 && nbk > ((int64_t)1 << 25)) {
        s *= 2.0;
        B->s = s;
        for (int a = ax0; a < 3; a++) B->nb[a] = (int)ceil(n0[a] / s) + 1;
        nbk = (int64_t)B->nb[0] * B->nb[1] * B->nb[2];
    }
    int64_t* cnt = (int64_t*)calloc(nbk + 1, sizeof(int64_t));
    int lo[3], hi[3];
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            B->off = (int64_t*)malloc(sizeof(int64_t) * (nbk + 1));
            B->off[0] = 0;
            for (int64_t i = 0; i < nbk; i++) B->off[i + 1] = B->off[i] + cnt[i];
            B->ids = (int32_t*)malloc(sizeof(int32_t) * (B->off[nbk] + 1));
            memset(cnt, 0, sizeof(int64_t) * (nbk + 1));
        }
        for (int t = 0; t < nt; t++) {
            for (int a = 0; a < 3; a++) {
                lo[a] = hi[a] = 0;
                if (a < ax0) continue;
                double mn = 1e300, mx = -1e300;
                for (int v = 0; v < 3; v++) {
                    double x = V3(V, T[3 * t + v])[a];
                    mn = x < mn ? x : mn;
                    mx = x > mx ? x : mx;
                }
                lo[a] = (int)floor(mn / s);
                hi[a] = (int)floor(mx / s);
                if (lo[a] < 0) lo[a] = 0;
                if (hi[a] > B->nb[a] - 1) hi[a] = B->nb[a] - 1;
            }
            for (int z = lo[2]; z <= hi[2]; z++)
                for (int y = lo[1]; y <= hi[1]; y++)
                    for (int x = lo[0]; x <= hi[0]; x++) {
                        int64_t k = ((int64_t)z * B->nb[1] + y) * B->nb[0] + x;
                        if (pass == 0) cnt[k]++;
                        else B->ids[B->off[k] + cnt[k]++] = t;
                    }
        }
    }
    free(cnt);
}

static void buckets_free(buckets* B) {
    free(B->off);
    free(B->ids);
}

static int64_t bucket_of(const buckets* B, const double* p) {
    int c[3] = {0, 0, 0};
    int ax0 = B->dim == 2 ? 1 : 0;
    for (int a = ax0; a < 3; a++) {
        c[a] = (int)floor(p[a] / B->s);
        if (c[a] < 0) c[a] = 0;
        if (c[a] > B->nb[a] - 1) c[a] = B->nb[a] - 1;
    }
    return ((int64_t)c[2] * B->nb[1] + c[1]) * B->nb[0] + c[0];
}

/* triangles whose closed yz bounding box contains (y, z) */
static int line_candidates(const buckets* B, const double* V, const int32_t* T, double y, double z,
                           int32_t** buf, int* cap) {
    double p[3] = {0.0, y, z};
    int64_t k = bucket_of(B, p);
    int n = 0;
    for (int64_t i = B->off[k]; i < B->off[k + 1]; i++) {
        int t = B->ids[i];
        const double *a = V3(V, T[3 * t]), *b = V3(V, T[3 * t + 1]), *c = V3(V, T[3 * t + 2]);
        double ymin = fmin(a[1], fmin(b[1], c[1])), ymax = fmax(a[1], fmax(b[1], c[1]));
        double zmin = fmin(a[2], fmin(b[2], c[2])), zmax = fmax(a[2], fmax(b[2], c[2]));
        if (y < ymin || y > ymax || z < zmin || z > zmax) continue;
        if (n == *cap) {
            *cap = *cap ? 2 * *cap : 64;
            *buf = (int32_t*)realloc(*buf, sizeof(int32_t) * *cap);
        }
        (*buf)[n++] = t;
    }
    return n;
}

/* ------------------------------------------------------------------------- */
/* point classification: solid(p) <=> p in the closed solid                   */
/* ------------------------------------------------------------------------- */

/* p lies on the closed triangle T (non-degenerate T only) */
static int on_triangle(const double* a, const double* b, const double* c, const double* p) {
    if (or_orient3d(a, b, c, p) != 0) return 0;
    return or_point_in_closed_triangle_coplanar(a, b, c, p);
}

/* Sign of the edge function of directed yz-edge u->w at p after the symbolic
 * perturbation p -> (p_y + eps, p_z + eps^2) (simulation of simplicity,
 * Edelsbrunner & Muecke 1990):
 *   E(p+d) = E(p) - (w_z - u_z) eps + (w_y - u_y) eps^2. */
static int sos_edge_sign(const double* u, const double* w, const double* p) {
    int s = or_orient2d(u[1], u[2], w[1], w[2], p[1], p[2]);
    if (s != 0) return s;
    if (w[2] != u[2]) return w[2] > u[2] ? -1 : 1;
    if (w[1] != u[1]) return w[1] > u[1] ? 1 : -1;
    return 0;
}

/* the perturbed +x ray from p crosses T strictly inside its yz projection and
 * ahead of p (p not on T) */
static int ray_crosses(const double* a, const double* b, const double* c, const double* p) {
    int A = or_orient2d(a[1], a[2], b[1], b[2], c[1], c[2]); /* sign of n_x */
    if (A == 0) return 0;                                   /* edge-on or degenerate */
    const double* u[3] = {a, b, c};
    for (int i = 0; i < 3; i++) {
        const double *s = u[i], *w = u[(i + 1) % 3];
        int e = A > 0 ? sos_edge_sign(s, w, p) : sos_edge_sign(w, s, p);
        if (e <= 0) return 0;
    }
    int o = or_orient3d(a, b, c, p); /* = n . (a - p) = n_x (x_hit - p_x) */
    return o != 0 && (o > 0) == (A > 0);
}

int or_solid_point(const double* V, const int32_t* T, const int32_t* cand, int ncand,
                   const double* p) {
    for (int i = 0; i < ncand; i++) {
        int t = cand[i];
        const double *a = V3(V, T[3 * t]), *b = V3(V, T[3 * t + 1]), *c = V3(V, T[3 * t + 2]);
        if (or_triangle_degenerate(a, b, c)) continue;
        if (on_triangle(a, b, c, p)) return 1;
    }
    int parity = 0;
    for (int i = 0; i < ncand; i++) {
        int t = cand[i];
        const double *a = V3(V, T[3 * t]), *b = V3(V, T[3 * t + 1]), *c = V3(V, T[3 * t + 2]);
        parity ^= ray_crosses(a, b, c, p);
    }
    return parity;
}

/* brute force over all triangles (no filter) */
/* wall time of the last bucket build and of the queries that followed it,
 * per entry point call (for the benchmark's CPU baseline) */
static double g_t_build = 0.0, g_t_query = 0.0;

void or_last_timing(double* out) {
    out[0] = g_t_build;
    out[1] = g_t_query;
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void or_solid_points_brute(const double* V, const int32_t* T, int nt, int64_t npts,
                           const double* pts, uint8_t* out) {
    int32_t* all = (int32_t*)malloc(sizeof(int32_t) * (nt > 0 ? nt : 1));
    for (int i = 0; i < nt; i++) all[i] = i;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < npts; k++) out[k] = (uint8_t)or_solid_point(V, T, all, nt, pts + 3 * k);
    free(all);
}

/* filtered by triangles whose yz box contains the point */
void or_solid_points(const double* V, const int32_t* T, int nt, const int32_t* n0, int64_t npts,
                     const double* pts, uint8_t* out) {
    double w0 = omp_get_wtime();
    buckets B;
    buckets_build(&B, 2, V, T, nt, n0);
    double w1 = omp_get_wtime();
#pragma omp parallel
    {
        int32_t* buf = NULL;
        int cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npts; k++) {
            const double* p = pts + 3 * k;
            int n = line_candidates(&B, V, T, p[1], p[2], &buf, &cap);
            out[k] = (uint8_t)or_solid_point(V, T, buf, n, p);
        }
        free(buf);
    }
    g_t_build = w1 - w0;
    g_t_query = omp_get_wtime() - w1;
    buckets_free(&B);
}

static inline double centre(int i, int L) { return ldexp((double)i + 0.5, -L); }

/* Classify every cell of the given level-L blocks (halo = 0: 64 per block,
 * t = I + 4J + 16K) or every point of each block's one-cell halo (halo = 1:
 * 216 per block, index (I+1) + 6 (J+1) + 36 (K+1), I,J,K in -1..4).
 * Points outside the domain are fluid. */
void or_classify_blocks(const double* V, const int32_t* T, int nt, const int32_t* n0, int L,
                        int64_t nb, const int32_t* bcoord, int halo, uint8_t* out) {
    buckets B;
    buckets_build(&B, 2, V, T, nt, n0);
    int lo = halo ? -1 : 0, hi = halo ? 4 : 3, w = hi - lo + 1;
    int64_t ncell[3] = {(int64_t)n0[0] << L, (int64_t)n0[1] << L, (int64_t)n0[2] << L};
#pragma omp parallel
    {
        int32_t* buf = NULL;
        int cap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t b = 0; b < nb; b++) {
            const int32_t* bc = bcoord + 3 * b;
            uint8_t* o = out + b * (int64_t)w * w * w;
            for (int K = lo; K <= hi; K++)
                for (int J = lo; J <= hi; J++) {
                    int64_t j = 4 * (int64_t)bc[1] + J, k = 4 * (int64_t)bc[2] + K;
                    int n = 0;
                    int inside_line = j >= 0 && j < ncell[1] && k >= 0 && k < ncell[2];
                    double y = centre((int)j, L), z = centre((int)k, L);
                    if (inside_line) n = line_candidates(&B, V, T, y, z, &buf, &cap);
                    for (int I = lo; I <= hi; I++) {
                        int64_t i = 4 * (int64_t)bc[0] + I;
                        int idx = (I - lo) + w * (J - lo) + w * w * (K - lo);
                        if (!inside_line || i < 0 || i >= ncell[0]) { o[idx] = 0; continue; }
                        double p[3] = {centre((int)i, L), y, z};
                        o[idx] = (uint8_t)or_solid_point(V, T, buf, n, p);
                    }
                }
        }
        free(buf);
    }
    buckets_free(&B);
}

/* ------------------------------------------------------------------------- */
/* refinement rules (Refinement Flagging and Propagation; Eq. 3)              */
/* ------------------------------------------------------------------------- */

enum { CL_F = 0, CL_S = 1, CL_SB = 2, CL_SA = 3 };

static int64_t dense_index(const int64_t* dims, int64_t x, int64_t y, int64_t z) {
    if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2]) return -1;
    return (z * dims[1] + y) * dims[0] + x;
}

/* solid: per block, 64 cell flags.  Returns the number of children. */
int64_t or_refine(const int32_t* n0, int L, int64_t nb, const int32_t* bcoord,
                  const uint8_t* solid, int n_prop, uint8_t* bclass, uint8_t* refine,
                  int32_t* child_map, int32_t* child_bcoord) {
    int64_t dims[3];
    for (int a = 0; a < 3; a++) dims[a] = ((int64_t)n0[a] / 4) << L;
    int64_t ntot = dims[0] * dims[1] * dims[2];
    int32_t* map = (int32_t*)malloc(sizeof(int32_t) * ntot);
    for (int64_t i = 0; i < ntot; i++) map[i] = -1;
    for (int64_t b = 0; b < nb; b++)
        map[dense_index(dims, bcoord[3 * b], bcoord[3 * b + 1], bcoord[3 * b + 2])] = (int32_t)b;

    uint8_t* S = (uint8_t*)calloc(nb, 1);
    uint8_t* SB = (uint8_t*)calloc(nb, 1);
    uint8_t* elig = (uint8_t*)calloc(nb, 1);
    uint8_t* M = (uint8_t*)calloc(nb, 1);
    uint8_t* Mn = (uint8_t*)calloc(nb, 1);
    for (int64_t b = 0; b < nb; b++) {
        int s = 0;
        for (int t = 0; t < 64; t++) s |= solid[64 * b + t];
        S[b] = (uint8_t)s; /* a block is solid if it has at least one solid cell */
    }
    /* neighbour iteration helper */
#define FOR_NEIGHBOURS(b, body)                                                          \
    for (int dz = -1; dz <= 1; dz++)                                                     \
        for (int dy_ = -1; dy_ <= 1; dy_++)                                              \
            for (int dx = -1; dx <= 1; dx++) {                                           \
                if (!dx && !dy_ && !dz) continue;                                        \
                int64_t nx = bcoord[3 * (b)] + dx, ny = bcoord[3 * (b) + 1] + dy_,       \
                        nz = bcoord[3 * (b) + 2] + dz;                                   \
                int64_t di = dense_index(dims, nx, ny, nz);                              \
                int in_domain = di >= 0;                                                 \
                int64_t n = in_domain ? map[di] : -1;                                    \
                (void)in_domain;                                                         \
                body                                                                     \
            }

    for (int64_t b = 0; b < nb; b++) {
        int sb = 0, el = 1;
        FOR_NEIGHBOURS(b, {
            if (in_domain && n < 0) el = 0;       /* refinement interface */
            if (n >= 0 && !S[n]) sb = 1;          /* fully fluid neighbour */
        })
        SB[b] = (uint8_t)(S[b] && sb);
        elig[b] = (uint8_t)el;
    }
    /* kernel 1 and 2: M1 = (SB & elig) | adjacent-to-SB */
    for (int64_t b = 0; b < nb; b++) {
        int adj = 0;
        FOR_NEIGHBOURS(b, { if (n >= 0 && SB[n]) adj = 1; })
        int m0 = SB[b] && elig[b];
        M[b] = (uint8_t)(m0 || adj);
        bclass[b] = SB[b] ? CL_SB : (S[b] ? CL_S : ((M[b] && !m0) ? CL_SA : CL_F));
    }
    /* kernel 3, n_prop synchronous iterations: fluid blocks, plus solid blocks
     * in the first iteration, join if a neighbour is marked */
    for (int k = 1; k <= n_prop; k++) {
        for (int64_t b = 0; b < nb; b++) {
            int join = 0;
            if (!S[b] || k == 1) { FOR_NEIGHBOURS(b, { if (n >= 0 && M[n]) join = 1; }) }
            Mn[b] = (uint8_t)(M[b] || join);
        }
        memcpy(M, Mn, nb);
    }
    int64_t nchild = 0;
    for (int64_t b = 0; b < nb; b++) {
        refine[b] = (uint8_t)(M[b] && elig[b]);
        if (refine[b]) {
            child_map[b] = (int32_t)nchild;
            for (int o = 0; o < 8; o++) {
                child_bcoord[3 * nchild + 0] = 2 * bcoord[3 * b + 0] + (o & 1);
                child_bcoord[3 * nchild + 1] = 2 * bcoord[3 * b + 1] + ((o >> 1) & 1);
                child_bcoord[3 * nchild + 2] = 2 * bcoord[3 * b + 2] + ((o >> 2) & 1);
                nchild++;
            }
        } else {
            child_map[b] = -1;
        }
    }
#undef FOR_NEIGHBOURS
    free(map); free(S); free(SB); free(elig); free(M); free(Mn);
    return nchild;
}

/* ------------------------------------------------------------------------- */
/* cut links: mask, nearest hit q, hit triangle                               */
/* ------------------------------------------------------------------------- */

/* direction k = (cx+1) + 3(cy+1) + 9(cz+1); 13 is the rest direction */
static inline void dir_vec(int k, int* c) {
    c[0] = k % 3 - 1;
    c[1] = (k / 3) % 3 - 1;
    c[2] = k / 9 - 1;
}

int or_dir_in_lattice(int k, int lattice) {
    if (k == 13 || k < 0 || k > 26) return 0;
    int c[3];
    dir_vec(k, c);
    int n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    return lattice == 27 ? 1 : n2 <= 2;
}

/* candidate triangles whose closed bbox meets the closed box [lo, hi] */
static int box_candidates(const buckets* B, const double* V, const int32_t* T,
                          const double* lo, const double* hi, int32_t** buf, int* cap) {
    int cl[3], ch[3];
    for (int a = 0; a < 3; a++) {
        cl[a] = (int)floor(lo[a] / B->s);
        ch[a] = (int)floor(hi[a] / B->s);
        if (cl[a] < 0) cl[a] = 0;
        if (ch[a] > B->nb[a] - 1) ch[a] = B->nb[a] - 1;
    }
    int n = 0;
    for (int z = cl[2]; z <= ch[2]; z++)
        for (int y = cl[1]; y <= ch[1]; y++)
            for (int x = cl[0]; x <= ch[0]; x++) {
                int64_t k = ((int64_t)z * B->nb[1] + y) * B->nb[0] + x;
                for (int64_t i = B->off[k]; i < B->off[k + 1]; i++) {
                    int t = B->ids[i];
                    int dup = 0;
                    for (int j = 0; j < n; j++) if ((*buf)[j] == t) { dup = 1; break; }
                    if (dup) continue;
                    int ok = 1;
                    for (int a = 0; a < 3 && ok; a++) {
                        double mn = 1e300, mx = -1e300;
                        for (int v = 0; v < 3; v++) {
                            double x_ = V3(V, T[3 * t + v])[a];
                            mn = x_ < mn ? x_ : mn;
                            mx = x_ > mx ? x_ : mx;
                        }
                        if (mx < lo[a] || mn > hi[a]) ok = 0;
                    }
                    if (!ok) continue;
                    if (n == *cap) {
                        *cap = *cap ? 2 * *cap : 64;
                        *buf = (int32_t*)realloc(*buf, sizeof(int32_t) * *cap);
                    }
                    (*buf)[n++] = t;
                }
            }
    return n;
}

/* q = min t in [0,1] with X + t (Y - X) on the surface; returns the hit
 * triangle (smallest index among the exact minimisers) or -1; *tied is set
 * when two or more triangles attain the minimum. */
static int nearest_hit(const double* V, const int32_t* T, const int32_t* cand, int n,
                       const double* X, const double* Y, double* q, int* tied) {
    or_hit best, h;
    int bt = -1;
    *tied = 0;
    for (int i = 0; i < n; i++) {
        int t = cand[i];
        const double *a = V3(V, T[3 * t]), *b = V3(V, T[3 * t + 1]), *c = V3(V, T[3 * t + 2]);
        if (!or_segment_hit(a, b, c, X, Y, &h)) continue;
        if (bt < 0) { best = h; bt = t; continue; }
        int cmp = or_hit_cmp(&h, &best);
        if (cmp < 0) { best = h; bt = t; *tied = 0; }
        else if (cmp == 0) { *tied = 1; if (t < bt) bt = t; }
    }
    *q = bt >= 0 ? or_hit_value(&best) : -1.0;
    return bt;
}

/* Cut-link table at level L (links from fluid cells of the given blocks to
 * solid same-level neighbour centres), in the order (block, t, k).
 * Returns the number of links; entries beyond cap are not written. */
int64_t or_links(const double* V, const int32_t* T, int nt, const int32_t* n0, int L, int64_t nb,
                 const int32_t* bcoord, int lattice, int64_t cap, uint32_t* mask_out,
                 int32_t* link_cell, uint8_t* link_dir, double* link_q, int32_t* link_tri,
                 uint8_t* link_tied) {
    uint8_t* halo = (uint8_t*)malloc((size_t)nb * 216);
    or_classify_blocks(V, T, nt, n0, L, nb, bcoord, 1, halo);
    int64_t* cnt = (int64_t*)calloc(nb + 1, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; b++) {
        const uint8_t* H = halo + 216 * b;
        int64_t c = 0;
        for (int t = 0; t < 64; t++) {
            int I = t & 3, J = (t >> 2) & 3, K = t >> 4;
            uint32_t m = 0;
            if (!H[(I + 1) + 6 * (J + 1) + 36 * (K + 1)]) {
                for (int k = 0; k < 27; k++) {
                    if (!or_dir_in_lattice(k, lattice)) continue;
                    int cv[3];
                    dir_vec(k, cv);
                    if (H[(I + 1 + cv[0]) + 6 * (J + 1 + cv[1]) + 36 * (K + 1 + cv[2])]) m |= 1u << k;
                }
            }
            mask_out[64 * b + t] = m;
            c += __builtin_popcount(m);
        }
        cnt[b] = c;
    }
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (nb + 1));
    off[0] = 0;
    for (int64_t b = 0; b < nb; b++) off[b + 1] = off[b] + cnt[b];
    int64_t total = off[nb];
    buckets B;
    buckets_build(&B, 3, V, T, nt, n0);
    double h = ldexp(1.0, -L);
#pragma omp parallel
    {
        int32_t* buf = NULL;
        int bcap = 0;
#pragma omp for schedule(dynamic, 8)
        for (int64_t b = 0; b < nb; b++) {
            int64_t pos = off[b];
            for (int t = 0; t < 64; t++) {
                uint32_t m = mask_out[64 * b + t];
                if (!m) continue;
                int I = t & 3, J = (t >> 2) & 3, K = t >> 4;
                double X[3] = {centre(4 * bcoord[3 * b] + I, L), centre(4 * bcoord[3 * b + 1] + J, L),
                               centre(4 * bcoord[3 * b + 2] + K, L)};
                for (int k = 0; k < 27; k++) {
                    if (!(m >> k & 1)) continue;
                    int cv[3];
                    dir_vec(k, cv);
                    double Y[3], lo[3], hi[3];
                    for (int a = 0; a < 3; a++) {
                        Y[a] = X[a] + cv[a] * h;
                        lo[a] = fmin(X[a], Y[a]);
                        hi[a] = fmax(X[a], Y[a]);
                    }
                    int n = box_candidates(&B, V, T, lo, hi, &buf, &bcap);
                    double q;
                    int tied;
                    int tri = nearest_hit(V, T, buf, n, X, Y, &q, &tied);
                    if (pos < cap) {
                        link_cell[pos] = (int32_t)(64 * b + t);
                        link_dir[pos] = (uint8_t)k;
                        link_q[pos] = q;
                        link_tri[pos] = tri;
                        link_tied[pos] = (uint8_t)tied;
                    }
                    pos++;
                }
            }
        }
        free(buf);
    }
    buckets_free(&B);
    free(halo); free(cnt); free(off);
    return total;
}

/* q and hit triangle for explicitly given links (cell index triples at level L
 * and directions), e.g. a random sample of a large table. */
void or_q_points(const double* V, const int32_t* T, int nt, const int32_t* n0, int L, int64_t n,
                 const int32_t* cell, const uint8_t* dir, double* q_out, int32_t* tri_out,
                 uint8_t* tied_out) {
    double w0 = omp_get_wtime();
    buckets B;
    buckets_build(&B, 3, V, T, nt, n0);
    double w1 = omp_get_wtime();
    double h = ldexp(1.0, -L);
#pragma omp parallel
    {
        int32_t* buf = NULL;
        int bcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; i++) {
            int cv[3];
            dir_vec(dir[i], cv);
            double X[3], Y[3], lo[3], hi[3];
            for (int a = 0; a < 3; a++) {
                X[a] = centre(cell[3 * i + a], L);
                Y[a] = X[a] + cv[a] * h;
                lo[a] = fmin(X[a], Y[a]);
                hi[a] = fmax(X[a], Y[a]);
            }
            int m = box_candidates(&B, V, T, lo, hi, &buf, &bcap);
            int tied;
            tri_out[i] = nearest_hit(V, T, buf, m, X, Y, &q_out[i], &tied);
            tied_out[i] = (uint8_t)tied;
        }
        free(buf);
    }
    g_t_build = w1 - w0;
    g_t_query = omp_get_wtime() - w1;
    buckets_free(&B);
}

/* For explicitly given links and a triangle named for each: the exact hit
 * parameter of that triangle along the link (-1 when the closed segment
 * misses it), and whether that parameter equals the nearest hit exactly
 * (the named triangle is one of the minimisers).  Checks a hit triangle
 * chosen elsewhere without asking it to be the smallest index at ties. */
void or_q_given(const double* V, const int32_t* T, int nt, const int32_t* n0, int L, int64_t n,
                const int32_t* cell, const uint8_t* dir, const int32_t* given, double* given_q,
                uint8_t* given_is_min) {
    buckets B;
    buckets_build(&B, 3, V, T, nt, n0);
    double h = ldexp(1.0, -L);
#pragma omp parallel
    {
        int32_t* buf = NULL;
        int bcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; i++) {
            int cv[3];
            dir_vec(dir[i], cv);
            double X[3], Y[3], lo[3], hi[3];
            for (int a = 0; a < 3; a++) {
                X[a] = centre(cell[3 * i + a], L);
                Y[a] = X[a] + cv[a] * h;
                lo[a] = fmin(X[a], Y[a]);
                hi[a] = fmax(X[a], Y[a]);
            }
            given_q[i] = -1.0;
            given_is_min[i] = 0;
            int g = given[i];
            if (g < 0 || g >= nt) continue;
            const double *a = V3(V, T[3 * g]), *b = V3(V, T[3 * g + 1]), *c = V3(V, T[3 * g + 2]);
            or_hit hg;
            if (!or_segment_hit(a, b, c, X, Y, &hg)) continue;
            given_q[i] = or_hit_value(&hg);
            /* the nearest hit over the link's candidates */
            int m = box_candidates(&B, V, T, lo, hi, &buf, &bcap);
            int below = 0;
            for (int j = 0; j < m && !below; j++) {
                int t = buf[j];
                or_hit hj;
                const double *ta = V3(V, T[3 * t]), *tb = V3(V, T[3 * t + 1]), *tc = V3(V, T[3 * t + 2]);
                if (or_segment_hit(ta, tb, tc, X, Y, &hj) && or_hit_cmp(&hj, &hg) < 0) below = 1;
            }
            given_is_min[i] = (uint8_t)!below;
        }
        free(buf);
    }
    buckets_free(&B);
}

/* ------------------------------------------------------------------------- */
/* gradient of L = sum_i w_i q_i with respect to the vertices                 */
/* dq/dv_j = lambda_j n / (n . d)  (hit point barycentrics lambda)            */
/* ------------------------------------------------------------------------- */

/* absolute = 1: the same sum with every term replaced by its magnitude,
 * |w_i| |lambda_j n_a / (n . d)| (the scale of the sum's rounding). */
void or_grad(const double* V, const int32_t* T, int nv, const int32_t* n0, int L, int64_t nb,
             const int32_t* bcoord, int64_t nlinks, const int32_t* link_cell,
             const uint8_t* link_dir, const int32_t* link_tri, const double* w, int absolute,
             double* grad) {
    (void)n0; (void)nb;
    memset(grad, 0, sizeof(double) * 3 * (size_t)nv);
    double h = ldexp(1.0, -L);
    for (int64_t i = 0; i < nlinks; i++) {
        int tri = link_tri[i];
        if (tri < 0 || w[i] == 0.0) continue;
        int64_t b = link_cell[i] / 64;
        int t = link_cell[i] % 64;
        int I = t & 3, J = (t >> 2) & 3, K = t >> 4;
        double X[3] = {centre(4 * bcoord[3 * b] + I, L), centre(4 * bcoord[3 * b + 1] + J, L),
                       centre(4 * bcoord[3 * b + 2] + K, L)};
        int cv[3];
        dir_vec(link_dir[i], cv);
        double d[3] = {cv[0] * h, cv[1] * h, cv[2] * h};
        const int32_t* tv = T + 3 * (int64_t)tri;
        const double *a = V3(V, tv[0]), *bb = V3(V, tv[1]), *c = V3(V, tv[2]);
        double e1[3] = {bb[0] - a[0], bb[1] - a[1], bb[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
        double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
        double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
        if (nd == 0.0 || nn == 0.0) continue;
        double q = (n[0] * (a[0] - X[0]) + n[1] * (a[1] - X[1]) + n[2] * (a[2] - X[2])) / nd;
        double H[3] = {X[0] + q * d[0], X[1] + q * d[1], X[2] + q * d[2]};
        const double* P[3] = {a, bb, c};
        double lam[3];
        for (int j = 0; j < 3; j++) {
            const double *u = P[(j + 1) % 3], *v = P[(j + 2) % 3];
            double uu[3] = {u[0] - H[0], u[1] - H[1], u[2] - H[2]};
            double vv[3] = {v[0] - H[0], v[1] - H[1], v[2] - H[2]};
            double cr[3] = {uu[1] * vv[2] - uu[2] * vv[1], uu[2] * vv[0] - uu[0] * vv[2],
                            uu[0] * vv[1] - uu[1] * vv[0]};
            lam[j] = (n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2]) / nn;
        }
        for (int j = 0; j < 3; j++)
            for (int a_ = 0; a_ < 3; a_++) {
                double term = w[i] * lam[j] * n[a_] / nd;
                grad[3 * (int64_t)tv[j] + a_] += absolute ? fabs(term) : term;
            }
    }
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
