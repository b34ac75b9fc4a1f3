// Host build of libgeo's predicate helpers (exact accumulator and float
// filters) so that they can be checked on a machine without a GPU.
#include "geo_internal.h"

extern "C" {
int hp_orient2d_exact(double ax, double ay, double bx, double by, double cx, double cy) {
    return orient2d_exact(ax, ay, bx, by, cx, cy);
}
int hp_orient3d_exact(const double* a, const double* b, const double* c, const double* d) {
    return orient3d_exact(a, b, c, d);
}
int hp_orient2d_filter_f64(double ax, double ay, double bx, double by, double cx, double cy) {
    return orient2d_filter<double>(ax, ay, bx, by, cx, cy, 0.0);
}
int hp_orient3d_filter_f64(const double* a, const double* b, const double* c, const double* d) {
    return orient3d_filter<double>(a, b, c, d, 0.0);
}
// float32 filter on rounded inputs with the rounding bound delta
int hp_orient3d_filter_f32(const double* a, const double* b, const double* c, const double* d) {
    float A[3], B[3], Cc[3], D[3];
    double delta = 0;
    for (int k = 0; k < 3; k++) {
        A[k] = (float)a[k]; B[k] = (float)b[k]; Cc[k] = (float)c[k]; D[k] = (float)d[k];
        delta = fmax(delta, fabs((double)A[k] - a[k]));
        delta = fmax(delta, fabs((double)B[k] - b[k]));
        delta = fmax(delta, fabs((double)Cc[k] - c[k]));
        delta = fmax(delta, fabs((double)D[k] - d[k]));
    }
    float df = (float)delta;
    if ((double)df < delta) df = nextafterf(df, 1e30f);
    return orient3d_filter<float>(A, B, Cc, D, df);
}
int hp_orient2d_filter_f32(double ax, double ay, double bx, double by, double cx, double cy) {
    const double in[6] = {ax, ay, bx, by, cx, cy};
    float f[6];
    double delta = 0;
    for (int k = 0; k < 6; k++) {
        f[k] = (float)in[k];
        delta = fmax(delta, fabs((double)f[k] - in[k]));
    }
    float df = (float)delta;
    if ((double)df < delta) df = nextafterf(df, 1e30f);
    return orient2d_filter<float>(f[0], f[1], f[2], f[3], f[4], f[5], df);
}
}
