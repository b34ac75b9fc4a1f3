/*
 * Exact geometric predicates for the CPU oracle (test infrastructure only; the
 * product path never links this file).
 *
 * Every floating-point input is a dyadic rational m * 2^e.  A polynomial in such
 * inputs built from +, -, * is a dyadic rational too, so it can be evaluated
 * exactly with a big integer mantissa and a binary exponent.  This file does
 * exactly that, with schoolbook arithmetic on 32-bit limbs; it is slow and
 * meant to be obviously correct.
 *
 * A fast double-precision evaluation is tried first and trusted only when its
 * magnitude exceeds a deliberately loose error bound (1e-12 of the permanent,
 * several thousand times the bounds proved by Shewchuk, "Adaptive precision
 * floating-point arithmetic and fast robust geometric predicates", 1997:
 * (3+16u)u for orient2d and (7+56u)u for orient3d, u = 2^-53).  Otherwise the
 * sign comes from the exact evaluation.
 *
 * Conventions:
 *   orient2d(a,b,c) = det[[ax ay 1],[bx by 1],[cx cy 1]]  (> 0: a,b,c counter-clockwise)
 *   orient3d(a,b,c,d) = det[a-d; b-d; c-d] = n . (a - d),  n = (b-a) x (c-a)
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>


static void dy_fail(const char* what) {
    fprintf(stderr, "oracle exact arithmetic: %s\n", what);
    abort();
}

static void dy_trim(dy* a) {
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) { a->neg = 0; a->exp = 0; }
}

static void dy_from_double(dy* r, double x) {
    memset(r, 0, sizeof(*r));
    if (x == 0.0) return;
    if (!isfinite(x)) dy_fail("non-finite input");
    int e;
    double f = frexp(fabs(x), &e);              /* |x| = f 2^e, f in [0.5,1) */
    uint64_t m = (uint64_t)ldexp(f, 53);        /* exact: 53-bit integer */
    r->neg = x < 0;
    r->exp = e - 53;
    r->d[0] = (uint32_t)m;
    r->d[1] = (uint32_t)(m >> 32);
    r->n = 2;
    dy_trim(r);
}

/* magnitude of a shifted left by s bits (s >= 0) into r (fresh) */
static void mag_shl(dy* r, const dy* a, int s) {
    int ls = s / 32, bs = s % 32;
    if (a->n + ls + 1 > DY_LIMBS) dy_fail("overflow in shift");
    memset(r->d, 0, sizeof(r->d));
    for (int i = 0; i < a->n; i++) {
        uint64_t v = (uint64_t)a->d[i] << bs;
        r->d[i + ls] |= (uint32_t)v;
        r->d[i + ls + 1] |= (uint32_t)(v >> 32);
    }
    r->n = a->n + ls + 1;
}

static int mag_cmp(const uint32_t* a, int na, const uint32_t* b, int nb) {
    int n = na > nb ? na : nb;
    for (int i = n - 1; i >= 0; i--) {
        uint32_t x = i < na ? a[i] : 0, y = i < nb ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

static void dy_add(dy* r, const dy* a, const dy* b) {
    if (a->n == 0) { *r = *b; return; }
    if (b->n == 0) { *r = *a; return; }
    int e = a->exp < b->exp ? a->exp : b->exp;
    dy A, B;
    mag_shl(&A, a, a->exp - e);
    mag_shl(&B, b, b->exp - e);
    int n = A.n > B.n ? A.n : B.n;
    dy R;
    memset(&R, 0, sizeof(R));
    R.exp = e;
    if (a->neg == b->neg) {
        uint64_t carry = 0;
        if (n + 1 > DY_LIMBS) dy_fail("overflow in add");
        for (int i = 0; i < n; i++) {
            uint64_t s = (uint64_t)(i < A.n ? A.d[i] : 0) + (i < B.n ? B.d[i] : 0) + carry;
            R.d[i] = (uint32_t)s;
            carry = s >> 32;
        }
        R.d[n] = (uint32_t)carry;
        R.n = n + 1;
        R.neg = a->neg;
    } else {
        int c = mag_cmp(A.d, A.n, B.d, B.n);
        if (c == 0) { memset(r, 0, sizeof(*r)); return; }
        const dy* big = c > 0 ? &A : &B;
        const dy* sml = c > 0 ? &B : &A;
        int64_t borrow = 0;
        for (int i = 0; i < n; i++) {
            int64_t s = (int64_t)(i < big->n ? big->d[i] : 0) - (i < sml->n ? sml->d[i] : 0) - borrow;
            borrow = s < 0;
            R.d[i] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
        }
        R.n = n;
        R.neg = c > 0 ? a->neg : b->neg;
    }
    dy_trim(&R);
    *r = R;
}

static void dy_neg(dy* r, const dy* a) {
    *r = *a;
    if (r->n) r->neg = !r->neg;
}

static void dy_sub(dy* r, const dy* a, const dy* b) {
    dy nb;
    dy_neg(&nb, b);
    dy_add(r, a, &nb);
}

static void dy_mul(dy* r, const dy* a, const dy* b) {
    dy R;
    memset(&R, 0, sizeof(R));
    if (a->n == 0 || b->n == 0) { *r = R; return; }
    if (a->n + b->n > DY_LIMBS) dy_fail("overflow in mul");
    for (int i = 0; i < a->n; i++) {
        uint64_t carry = 0;
        for (int j = 0; j < b->n; j++) {
            uint64_t t = (uint64_t)a->d[i] * b->d[j] + R.d[i + j] + carry;
            R.d[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        R.d[i + b->n] = (uint32_t)carry;
    }
    R.n = a->n + b->n;
    R.exp = a->exp + b->exp;
    R.neg = a->neg ^ b->neg;
    dy_trim(&R);
    *r = R;
}

static int dy_sign(const dy* a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

static int dy_cmp(const dy* a, const dy* b) {
    dy d;
    dy_sub(&d, a, b);
    return dy_sign(&d);
}

static double dy_to_double(const dy* a) {
    /* correctly rounded (nearest, ties to even), independent of how the value
     * is stored: take the top 64 significant bits plus a sticky bit */
    if (a->n == 0) return 0.0;
    int top = a->n - 1;
    int lead = 31 - __builtin_clz(a->d[top]);     /* bit index within the top limb */
    int64_t B = (int64_t)32 * top + lead + 1;      /* bit length of the mantissa */
    uint64_t m64 = 0;
    int sticky = 0;
    for (int64_t i = B - 1, k = 0; i >= 0; i--, k++) {
        uint32_t bit = (a->d[i / 32] >> (i % 32)) & 1u;
        if (k < 64) m64 = (m64 << 1) | bit;
        else if (bit) { sticky = 1; break; }
    }
    int64_t used = B < 64 ? B : 64;                /* bits placed in m64 */
    int64_t scale = B - used + a->exp;             /* value ~ m64 * 2^scale */
    /* round m64 (used bits) to 53 bits */
    if (used > 53) {
        int drop = (int)(used - 53);
        uint64_t rem = m64 & ((1ull << drop) - 1), half = 1ull << (drop - 1);
        uint64_t m = m64 >> drop;
        if (rem > half || (rem == half && (sticky || (m & 1)))) m++;
        m64 = m;
        scale += drop;
    }
    double v = ldexp((double)m64, (int)scale);
    return a->neg ? -v : v;
}

/* ------------------------------------------------------------------------- */
/* exact determinants                                                         */
/* ------------------------------------------------------------------------- */

static void det2_exact(dy* r, double ax, double ay, double bx, double by, double cx, double cy) {
    dy A[6], t1, t2, u, v;
    dy_from_double(&A[0], ax); dy_from_double(&A[1], ay);
    dy_from_double(&A[2], bx); dy_from_double(&A[3], by);
    dy_from_double(&A[4], cx); dy_from_double(&A[5], cy);
    dy acx, acy, bcx, bcy;
    dy_sub(&acx, &A[0], &A[4]); dy_sub(&acy, &A[1], &A[5]);
    dy_sub(&bcx, &A[2], &A[4]); dy_sub(&bcy, &A[3], &A[5]);
    dy_mul(&t1, &acx, &bcy);
    dy_mul(&t2, &acy, &bcx);
    dy_sub(&u, &t1, &t2);
    (void)v;
    *r = u;
}

static void det3_exact(dy* r, const double* a, const double* b, const double* c, const double* d) {
    dy P[4][3], D[3][3];
    const double* pts[4] = {a, b, c, d};
    for (int i = 0; i < 4; i++)
        for (int k = 0; k < 3; k++) dy_from_double(&P[i][k], pts[i][k]);
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) dy_sub(&D[i][k], &P[i][k], &P[3][k]);
    /* rows D0=a-d, D1=b-d, D2=c-d; det = D0 . (D1 x D2) */
    dy m1, m2, cr[3], t, acc;
    dy_mul(&m1, &D[1][1], &D[2][2]); dy_mul(&m2, &D[1][2], &D[2][1]); dy_sub(&cr[0], &m1, &m2);
    dy_mul(&m1, &D[1][2], &D[2][0]); dy_mul(&m2, &D[1][0], &D[2][2]); dy_sub(&cr[1], &m1, &m2);
    dy_mul(&m1, &D[1][0], &D[2][1]); dy_mul(&m2, &D[1][1], &D[2][0]); dy_sub(&cr[2], &m1, &m2);
    memset(&acc, 0, sizeof(acc));
    for (int k = 0; k < 3; k++) {
        dy_mul(&t, &D[0][k], &cr[k]);
        dy_add(&acc, &acc, &t);
    }
    *r = acc;
}

int or_orient2d_exact(double ax, double ay, double bx, double by, double cx, double cy) {
    dy r;
    det2_exact(&r, ax, ay, bx, by, cx, cy);
    return dy_sign(&r);
}

int or_orient3d_exact(const double* a, const double* b, const double* c, const double* d) {
    dy r;
    det3_exact(&r, a, b, c, d);
    return dy_sign(&r);
}

double or_orient3d_value(const double* a, const double* b, const double* c, const double* d) {
    dy r;
    det3_exact(&r, a, b, c, d);
    return dy_to_double(&r);
}

#define LOOSE_BOUND 1e-12

int or_orient2d(double ax, double ay, double bx, double by, double cx, double cy) {
    double l = (ax - cx) * (by - cy), r = (ay - cy) * (bx - cx);
    double det = l - r;
    double perm = fabs(l) + fabs(r);
    if (fabs(det) > LOOSE_BOUND * perm) return det > 0 ? 1 : -1;
    return or_orient2d_exact(ax, ay, bx, by, cx, cy);
}

int or_orient3d(const double* a, const double* b, const double* c, const double* d) {
    double adx = a[0] - d[0], ady = a[1] - d[1], adz = a[2] - d[2];
    double bdx = b[0] - d[0], bdy = b[1] - d[1], bdz = b[2] - d[2];
    double cdx = c[0] - d[0], cdy = c[1] - d[1], cdz = c[2] - d[2];
    double det = adx * (bdy * cdz - bdz * cdy) + ady * (bdz * cdx - bdx * cdz)
               + adz * (bdx * cdy - bdy * cdx);
    double perm = fabs(adx) * (fabs(bdy * cdz) + fabs(bdz * cdy))
                + fabs(ady) * (fabs(bdz * cdx) + fabs(bdx * cdz))
                + fabs(adz) * (fabs(bdx * cdy) + fabs(bdy * cdx));
    if (fabs(det) > LOOSE_BOUND * perm) return det > 0 ? 1 : -1;
    return or_orient3d_exact(a, b, c, d);
}

/* ------------------------------------------------------------------------- */
/* closed segment / closed triangle intersection with an exact hit parameter  */
/* ------------------------------------------------------------------------- */

static void hit_set(or_hit* h, const dy* num, const dy* den) {
    h->num = *num;
    h->den = *den;
    if (dy_sign(&h->den) < 0) { dy_neg(&h->num, &h->num); dy_neg(&h->den, &h->den); }
}

int or_hit_cmp(const or_hit* p, const or_hit* q) {
    dy l, r;
    dy_mul(&l, &p->num, &q->den);
    dy_mul(&r, &q->num, &p->den);
    return dy_cmp(&l, &r);
}

/* num/den rounded to the nearest double (ties to even), whatever the
 * representation of the ratio: the float quotient is within 2 ulp, so the
 * nearest of the five neighbouring doubles is found by exact comparison. */
double or_hit_value(const or_hit* h) {
    double q0 = dy_to_double(&h->num) / dy_to_double(&h->den);
    double cand[5];
    cand[2] = q0;
    cand[1] = nextafter(q0, -INFINITY); cand[0] = nextafter(cand[1], -INFINITY);
    cand[3] = nextafter(q0, INFINITY);  cand[4] = nextafter(cand[3], INFINITY);
    int best = -1;
    dy bestabs;
    for (int k = 0; k < 5; k++) {
        dy c, e;
        dy_from_double(&c, cand[k]);
        dy_mul(&e, &c, &h->den);
        dy_sub(&e, &e, &h->num);
        if (e.neg) dy_neg(&e, &e);
        int cmp = best < 0 ? -1 : dy_cmp(&e, &bestabs);
        if (cmp < 0) { best = k; bestabs = e; }
        else if (cmp == 0) {
            /* exact tie between two doubles: keep the even mantissa */
            int64_t bits;
            memcpy(&bits, &cand[k], sizeof bits);
            if ((bits & 1) == 0) { best = k; bestabs = e; }
        }
    }
    return cand[best];
}

/* axis dropped by the in-plane projection of a non-degenerate triangle:
 * one whose exact projected area is non-zero (largest |n_k| tried first). */
static int drop_axis(const double* a, const double* b, const double* c, int* area_sign) {
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                   e1[0] * e2[1] - e1[1] * e2[0]};
    int order[3] = {0, 1, 2};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (fabs(n[order[j]]) > fabs(n[order[i]])) { int t = order[i]; order[i] = order[j]; order[j] = t; }
    for (int r = 0; r < 3; r++) {
        int k = order[r], u = (k + 1) % 3, v = (k + 2) % 3;
        int s = or_orient2d(a[u], a[v], b[u], b[v], c[u], c[v]);
        if (s != 0) { *area_sign = s; return k; }
    }
    return -1; /* degenerate (collinear) triangle */
}

int or_point_in_closed_triangle_coplanar(const double* a, const double* b, const double* c,
                                         const double* p) {
    int A;
    int k = drop_axis(a, b, c, &A);
    if (k < 0) return 0;
    int u = (k + 1) % 3, v = (k + 2) % 3;
    int s0 = or_orient2d(a[u], a[v], b[u], b[v], p[u], p[v]) * A;
    int s1 = or_orient2d(b[u], b[v], c[u], c[v], p[u], p[v]) * A;
    int s2 = or_orient2d(c[u], c[v], a[u], a[v], p[u], p[v]) * A;
    return s0 >= 0 && s1 >= 0 && s2 >= 0;
}

int or_triangle_degenerate(const double* a, const double* b, const double* c) {
    int A;
    return drop_axis(a, b, c, &A) < 0;
}

/* Coplanar segment X->Y against closed T: entry parameter by clipping against
 * the three closed half-planes of the projected triangle. */
static int clip_coplanar(const double* a, const double* b, const double* c,
                         const double* X, const double* Y, or_hit* out) {
    int A;
    int k = drop_axis(a, b, c, &A);
    if (k < 0) return 0;
    int u = (k + 1) % 3, v = (k + 2) % 3;
    const double* P[3] = {a, b, c};
    dy one, zero;
    dy_from_double(&one, 1.0);
    dy_from_double(&zero, 0.0);
    or_hit lo, hi;
    hit_set(&lo, &zero, &one);
    hit_set(&hi, &one, &one);
    for (int i = 0; i < 3; i++) {
        const double* s = P[i];
        const double* w = P[(i + 1) % 3];
        dy f0, f1;
        det2_exact(&f0, s[u], s[v], w[u], w[v], X[u], X[v]);
        det2_exact(&f1, s[u], s[v], w[u], w[v], Y[u], Y[v]);
        if (A < 0) { dy_neg(&f0, &f0); dy_neg(&f1, &f1); }
        int g0 = dy_sign(&f0), g1 = dy_sign(&f1);
        if (g0 < 0 && g1 < 0) return 0;
        if (g0 >= 0 && g1 >= 0) continue;
        dy den;
        dy_sub(&den, &f0, &f1);
        or_hit t;
        hit_set(&t, &f0, &den);              /* f(t) = 0 at t = f0 / (f0 - f1) */
        if (g0 < 0) { if (or_hit_cmp(&t, &lo) > 0) lo = t; }   /* entering */
        else        { if (or_hit_cmp(&t, &hi) < 0) hi = t; }   /* leaving */
    }
    if (or_hit_cmp(&lo, &hi) > 0) return 0;
    *out = lo;
    return 1;
}

int or_segment_hit(const double* a, const double* b, const double* c,
                   const double* X, const double* Y, or_hit* out) {
    if (or_triangle_degenerate(a, b, c)) return 0;
    int sx = or_orient3d(a, b, c, X);
    int sy = or_orient3d(a, b, c, Y);
    if (sx * sy > 0) return 0;
    if (sx == 0 && sy == 0) return clip_coplanar(a, b, c, X, Y, out);
    dy one, zero;
    dy_from_double(&one, 1.0);
    dy_from_double(&zero, 0.0);
    if (sx == 0) {
        if (or_point_in_closed_triangle_coplanar(a, b, c, X)) { hit_set(out, &zero, &one); return 1; }
        return 0;
    }
    if (sy == 0) {
        if (or_point_in_closed_triangle_coplanar(a, b, c, Y)) { hit_set(out, &one, &one); return 1; }
        return 0;
    }
    int v0 = or_orient3d(X, Y, a, b);
    int v1 = or_orient3d(X, Y, b, c);
    int v2 = or_orient3d(X, Y, c, a);
    int pos = v0 > 0 || v1 > 0 || v2 > 0;
    int neg = v0 < 0 || v1 < 0 || v2 < 0;
    if (pos && neg) return 0;
    dy s1, s2, den;
    det3_exact(&s1, a, b, c, X);
    det3_exact(&s2, a, b, c, Y);
    dy_sub(&den, &s1, &s2);
    hit_set(out, &s1, &den);
    return 1;
}
