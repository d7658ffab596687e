/*
 * TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.  Nothing in the product
 * path may link, load or call this file.
 *
 * Exact signs of the 2D and 3D orientation determinants of points with
 * float64 coordinates, computed with exact dyadic big numbers
 * (value = +-integer * 2^exp, integer held in 32-bit limbs).  Every float64 is
 * such a number, sums and products of them are again such numbers, so the
 * determinants below are evaluated without any rounding at all.
 *
 * The paper decides coplanarity and intersection with mixed FP32/FP64
 * arithmetic (Sec. 5.2, last paragraph); the oracle takes the exact reading
 * instead, so that every predicate has one correct answer.
 *
 * A float64 evaluation with a deliberately loose error bound (1e-12 times the
 * permanent, about 1000x Shewchuk's bound for these expressions) returns the
 * sign early when it is certain; every other case is decided exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define XL 240 /* 7680 bits: enough for a degree-3 product of any finite doubles */

typedef struct {
    int neg;
    int n;       /* number of used limbs; 0 means the value is zero */
    int32_t exp; /* value = (-1)^neg * mag * 2^exp */
    uint32_t d[XL];
} xnum;

static void x_fail(const char *what) {
    fprintf(stderr, "oracle exact arithmetic: %s\n", what);
    abort();
}

static void x_trim(xnum *a) {
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) { a->neg = 0; a->exp = 0; }
}

static void x_from_double(xnum *r, double v) {
    if (!(v == v) || isinf(v)) x_fail("non-finite input");
    r->neg = 0; r->n = 0; r->exp = 0;
    if (v == 0.0) return;
    int e;
    double m = frexp(fabs(v), &e);          /* |v| = m 2^e, m in [0.5, 1) */
    uint64_t mi = (uint64_t)ldexp(m, 53);   /* exact: at most 53 significant bits */
    r->neg = v < 0;
    r->exp = e - 53;
    r->d[0] = (uint32_t)mi;
    r->d[1] = (uint32_t)(mi >> 32);
    r->n = 2;
    x_trim(r);
}

/* dst = src.mag << k bits (magnitude only) */
static void mag_shl(uint32_t *dst, int *dn, const uint32_t *src, int sn, int k) {
    int w = k / 32, b = k % 32;
    if (sn + w + 1 > XL) x_fail("limb overflow in shift");
    for (int i = 0; i < w; i++) dst[i] = 0;
    uint32_t carry = 0;
    for (int i = 0; i < sn; i++) {
        uint32_t v = src[i];
        dst[i + w] = b ? ((v << b) | carry) : v;
        carry = b ? (v >> (32 - b)) : 0;
    }
    dst[sn + w] = carry;
    *dn = sn + w + 1;
}

static int mag_cmp(const uint32_t *a, int an, const uint32_t *b, int bn) {
    while (an > 0 && a[an - 1] == 0) an--;
    while (bn > 0 && b[bn - 1] == 0) bn--;
    if (an != bn) return an < bn ? -1 : 1;
    for (int i = an - 1; i >= 0; i--)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

/* r = a + b (signed) */
static void x_add(xnum *r, const xnum *a, const xnum *b) {
    if (a->n == 0) { *r = *b; return; }
    if (b->n == 0) { *r = *a; return; }
    static __thread uint32_t A[XL], B[XL];
    int an, bn;
    int32_t e = a->exp < b->exp ? a->exp : b->exp;
    mag_shl(A, &an, a->d, a->n, a->exp - e);
    mag_shl(B, &bn, b->d, b->n, b->exp - e);
    int n = an > bn ? an : bn;
    for (int i = an; i < n; i++) A[i] = 0;
    for (int i = bn; i < n; i++) B[i] = 0;
    xnum t;
    t.exp = e;
    if (a->neg == b->neg) {
        if (n + 1 > XL) x_fail("limb overflow in add");
        uint64_t c = 0;
        for (int i = 0; i < n; i++) {
            c += (uint64_t)A[i] + B[i];
            t.d[i] = (uint32_t)c;
            c >>= 32;
        }
        t.d[n] = (uint32_t)c;
        t.n = n + 1;
        t.neg = a->neg;
    } else {
        int c = mag_cmp(A, n, B, n);
        if (c == 0) { r->n = 0; r->neg = 0; r->exp = 0; return; }
        const uint32_t *big = c > 0 ? A : B, *small = c > 0 ? B : A;
        int64_t br = 0;
        for (int i = 0; i < n; i++) {
            int64_t v = (int64_t)big[i] - small[i] - br;
            br = v < 0;
            t.d[i] = (uint32_t)(v + (br ? ((int64_t)1 << 32) : 0));
        }
        t.n = n;
        t.neg = c > 0 ? a->neg : b->neg;
    }
    x_trim(&t);
    *r = t;
}

static void x_neg(xnum *r, const xnum *a) {
    *r = *a;
    if (r->n) r->neg = !r->neg;
}

static void x_sub(xnum *r, const xnum *a, const xnum *b) {
    xnum nb;
    x_neg(&nb, b);
    x_add(r, a, &nb);
}

static void x_mul(xnum *r, const xnum *a, const xnum *b) {
    if (a->n == 0 || b->n == 0) { r->n = 0; r->neg = 0; r->exp = 0; return; }
    if (a->n + b->n > XL) x_fail("limb overflow in mul");
    xnum t;
    memset(t.d, 0, sizeof(uint32_t) * (size_t)(a->n + b->n));
    for (int i = 0; i < a->n; i++) {
        uint64_t c = 0;
        for (int j = 0; j < b->n; j++) {
            c += (uint64_t)a->d[i] * b->d[j] + t.d[i + j];
            t.d[i + j] = (uint32_t)c;
            c >>= 32;
        }
        t.d[i + b->n] = (uint32_t)c;
    }
    t.n = a->n + b->n;
    t.exp = a->exp + b->exp;
    t.neg = a->neg ^ b->neg;
    x_trim(&t);
    *r = t;
}

static int x_sign(const xnum *a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

/* exact sign of (a-c) x (b-c) in the plane */
static int orient2d_exact(const double *a, const double *b, const double *c) {
    xnum ax, ay, bx, by, cx, cy, acx, acy, bcx, bcy, l, r, d;
    x_from_double(&ax, a[0]); x_from_double(&ay, a[1]);
    x_from_double(&bx, b[0]); x_from_double(&by, b[1]);
    x_from_double(&cx, c[0]); x_from_double(&cy, c[1]);
    x_sub(&acx, &ax, &cx); x_sub(&acy, &ay, &cy);
    x_sub(&bcx, &bx, &cx); x_sub(&bcy, &by, &cy);
    x_mul(&l, &acx, &bcy);
    x_mul(&r, &acy, &bcx);
    x_sub(&d, &l, &r);
    return x_sign(&d);
}

/* exact sign of det[a-d; b-d; c-d] */
static int orient3d_exact(const double *a, const double *b, const double *c, const double *dp) {
    static __thread xnum P[12], D[9], t1, t2, m1, m2, m3, s, u;
    for (int i = 0; i < 3; i++) {
        x_from_double(&P[i], a[i]);
        x_from_double(&P[3 + i], b[i]);
        x_from_double(&P[6 + i], c[i]);
        x_from_double(&P[9 + i], dp[i]);
    }
    for (int r = 0; r < 3; r++)
        for (int i = 0; i < 3; i++) x_sub(&D[3 * r + i], &P[3 * r + i], &P[9 + i]);
    /* rows: ad = D[0..2], bd = D[3..5], cd = D[6..8] */
    /* m1 = bdy*cdz - bdz*cdy ; m2 = cdy*adz - cdz*ady ; m3 = ady*bdz - adz*bdy */
    x_mul(&t1, &D[4], &D[8]); x_mul(&t2, &D[5], &D[7]); x_sub(&m1, &t1, &t2);
    x_mul(&t1, &D[7], &D[2]); x_mul(&t2, &D[8], &D[1]); x_sub(&m2, &t1, &t2);
    x_mul(&t1, &D[1], &D[5]); x_mul(&t2, &D[2], &D[4]); x_sub(&m3, &t1, &t2);
    x_mul(&t1, &D[0], &m1);
    x_mul(&t2, &D[3], &m2);
    x_add(&s, &t1, &t2);
    x_mul(&t1, &D[6], &m3);
    x_add(&u, &s, &t1);
    return x_sign(&u);
}

int o_orient2d(const double *a, const double *b, const double *c) {
    double acx = a[0] - c[0], acy = a[1] - c[1];
    double bcx = b[0] - c[0], bcy = b[1] - c[1];
    double l = acx * bcy, r = acy * bcx;
    double det = l - r;
    double perm = fabs(l) + fabs(r);
    if (perm > 1e-250 && fabs(det) > 1e-12 * perm) return det > 0 ? 1 : -1;
    return orient2d_exact(a, b, c);
}

int o_orient3d(const double *a, const double *b, const double *c, const double *d) {
    double adx = a[0] - d[0], ady = a[1] - d[1], adz = a[2] - d[2];
    double bdx = b[0] - d[0], bdy = b[1] - d[1], bdz = b[2] - d[2];
    double cdx = c[0] - d[0], cdy = c[1] - d[1], cdz = c[2] - d[2];
    double m1 = bdy * cdz - bdz * cdy;
    double m2 = cdy * adz - cdz * ady;
    double m3 = ady * bdz - adz * bdy;
    double det = adx * m1 + bdx * m2 + cdx * m3;
    double perm = fabs(adx) * (fabs(bdy * cdz) + fabs(bdz * cdy))
                + fabs(bdx) * (fabs(cdy * adz) + fabs(cdz * ady))
                + fabs(cdx) * (fabs(ady * bdz) + fabs(adz * bdy));
    if (perm > 1e-250 && fabs(det) > 1e-12 * perm) return det > 0 ? 1 : -1;
    return orient3d_exact(a, b, c, d);
}

/* exported for the pins: exact answers without the float filter */
int oracle_orient2d_exact(const double *a, const double *b, const double *c) {
    return orient2d_exact(a, b, c);
}
int oracle_orient3d_exact(const double *a, const double *b, const double *c, const double *d) {
    return orient3d_exact(a, b, c, d);
}
int oracle_orient2d(const double *a, const double *b, const double *c) { return o_orient2d(a, b, c); }
int oracle_orient3d(const double *a, const double *b, const double *c, const double *d) {
    return o_orient3d(a, b, c, d);
}
