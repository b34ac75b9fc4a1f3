/*
 * CPU oracle for the geometry-embedding hot path: test infrastructure only.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library; the GPU path shares no code, header or table with it.
 */
#ifndef GEO_ORACLE_H
#define GEO_ORACLE_H

#include <stdint.h>

#define DY_LIMBS 64

typedef struct {
    int neg;
    int n;
    int exp;
    uint32_t d[DY_LIMBS];
} dy;

typedef struct {
    dy num, den; /* hit parameter t = num / den, den > 0 */
} or_hit;

/* predicates (exact signs) */
int or_orient2d(double ax, double ay, double bx, double by, double cx, double cy);
int or_orient2d_exact(double ax, double ay, double bx, double by, double cx, double cy);
int or_orient3d(const double* a, const double* b, const double* c, const double* d);
int or_orient3d_exact(const double* a, const double* b, const double* c, const double* d);
double or_orient3d_value(const double* a, const double* b, const double* c, const double* d);
int or_triangle_degenerate(const double* a, const double* b, const double* c);
int or_point_in_closed_triangle_coplanar(const double* a, const double* b, const double* c,
                                         const double* p);
int or_segment_hit(const double* a, const double* b, const double* c,
                   const double* X, const double* Y, or_hit* out);
int or_hit_cmp(const or_hit* p, const or_hit* q);
double or_hit_value(const or_hit* h);

/* 2D form (embed2d.c) */
int or2_solid_point(const double* V, const int32_t* E, const int32_t* cand, int n, const double* p);
void or2_classify_blocks(const double* V, const int32_t* E, int ne, const int32_t* n0, int L, int64_t nb,
                         const int32_t* bcoord, int halo, uint8_t* out);
int64_t or2_refine(const int32_t* n0, int L, int64_t nb, const int32_t* bcoord, const uint8_t* solid, int n_prop,
                   uint8_t* bclass, uint8_t* refine, int32_t* child_map, int32_t* child_bcoord);
int64_t or2_links(const double* V, const int32_t* E, int ne, const int32_t* n0, int L, int64_t nb,
                  const int32_t* bcoord, int64_t cap, uint16_t* mask_out, int32_t* link_cell, uint8_t* link_dir,
                  double* link_q, int32_t* link_edge, uint8_t* link_tied);

#endif
