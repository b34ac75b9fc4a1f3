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

#endif
