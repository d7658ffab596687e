/*
 * TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.
 *
 * Self-intersection test for a pair of triangles of one mesh, organised the
 * way the paper organises it (Sec. 5.2 and Appendix 3, "Parallel
 * Self-Intersection Detection" algorithm): count the vertex ids the two
 * triangles share (s), decide whether they are coplanar, then
 *   coplanar, s = 0 : do the two closed triangles overlap in their plane
 *                     (Fig. "coplanar self-intersection cases", case 1);
 *   coplanar, s = 1 : angle-overlap test at the shared vertex (cases 2, 3);
 *   coplanar, s = 2 : same-side test across the shared edge (cases 4, 5);
 *   s = 3           : always reported;
 *   not coplanar, s = 2 : never an intersection (two planes meet only in the
 *                     shared edge);
 *   not coplanar, s = 0 : the triangles meet at all (the paper computes the
 *                     intersection segment with Devillers' method; touching
 *                     counts here);
 *   not coplanar, s = 1 : the triangles meet somewhere other than the shared
 *                     vertex (the paper's "intersection line longer than a
 *                     tolerance"; exact reading: longer than zero).
 * Every sign is exact.  Triangles are assumed non-degenerate; collapses that
 * would create a degenerate triangle are rejected before this test runs.
 */
#include <stdint.h>

#include "oracle_internal.h"

/* project a 3D point by dropping axis k */
static void proj(const double *p, int k, double *out) {
    int a = (k + 1) % 3, b = (k + 2) % 3;
    out[0] = p[a];
    out[1] = p[b];
}

/* an axis whose removal keeps triangle abc non-degenerate */
static int good_axis(const double *a, const double *b, const double *c) {
    for (int k = 2; k >= 0; k--) {
        double pa[2], pb[2], pc[2];
        proj(a, k, pa); proj(b, k, pb); proj(c, k, pc);
        if (o_orient2d(pa, pb, pc) != 0) return k;
    }
    return -1;
}

int o_degenerate(const double *a, const double *b, const double *c) {
    return good_axis(a, b, c) < 0;
}

/* --- 2D helpers (exact) --- */

/* closed segment pq and closed segment rs intersect (2D) */
static int on_seg_collinear(const double *p, const double *q, const double *x) {
    /* x is collinear with p,q: inside the closed segment iff inside its box */
    double lo0 = p[0] < q[0] ? p[0] : q[0], hi0 = p[0] < q[0] ? q[0] : p[0];
    double lo1 = p[1] < q[1] ? p[1] : q[1], hi1 = p[1] < q[1] ? q[1] : p[1];
    return x[0] >= lo0 && x[0] <= hi0 && x[1] >= lo1 && x[1] <= hi1;
}

static int seg_seg_2d(const double *p, const double *q, const double *r, const double *s) {
    int o1 = o_orient2d(p, q, r), o2 = o_orient2d(p, q, s);
    int o3 = o_orient2d(r, s, p), o4 = o_orient2d(r, s, q);
    if (o1 * o2 < 0 && o3 * o4 < 0) return 1;
    if (o1 == 0 && on_seg_collinear(p, q, r)) return 1;
    if (o2 == 0 && on_seg_collinear(p, q, s)) return 1;
    if (o3 == 0 && on_seg_collinear(r, s, p)) return 1;
    if (o4 == 0 && on_seg_collinear(r, s, q)) return 1;
    return 0;
}

/* point x in closed triangle abc (2D, abc non-degenerate) */
static int pt_in_tri_2d(const double *x, const double *a, const double *b, const double *c) {
    int s1 = o_orient2d(a, b, x), s2 = o_orient2d(b, c, x), s3 = o_orient2d(c, a, x);
    int pos = s1 > 0 || s2 > 0 || s3 > 0;
    int neg = s1 < 0 || s2 < 0 || s3 < 0;
    return !(pos && neg);
}

/* coplanar, no shared vertex: closed triangles overlap in the plane */
static int coplanar_overlap(const double P[3][2], const double Q[3][2]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (seg_seg_2d(P[i], P[(i + 1) % 3], Q[j], Q[(j + 1) % 3])) return 1;
    if (pt_in_tri_2d(P[0], Q[0], Q[1], Q[2])) return 1;
    if (pt_in_tri_2d(Q[0], P[0], P[1], P[2])) return 1;
    return 0;
}

/* direction a->x lies in the closed wedge spanned by a->u, a->v (angle < pi) */
static int in_wedge(const double *a, const double *u, const double *v, const double *x) {
    int o = o_orient2d(a, u, v);           /* orientation of the wedge, nonzero */
    int s1 = o_orient2d(a, u, x);          /* sign of (u-a) x (x-a) */
    int s2 = o_orient2d(a, x, v);          /* sign of (x-a) x (v-a) */
    return (s1 == 0 || s1 == o) && (s2 == 0 || s2 == o);
}

/* coplanar, one shared vertex A: T1 = A B C, T2 = A D E.  The triangles meet
 * outside A exactly when their angles at A overlap: an edge direction of one
 * triangle lies inside (or on the boundary of) the angle of the other.  The
 * paper's zero-cross-product special cases are the boundary cases here. */
static int angle_overlap(const double *A, const double *B, const double *C,
                         const double *D, const double *E) {
    if (in_wedge(A, B, C, D) || in_wedge(A, B, C, E)) return 1;
    if (in_wedge(A, D, E, B) || in_wedge(A, D, E, C)) return 1;
    return 0;
}

/* coplanar, shared edge AB, third corners C (T1) and D (T2): the triangles
 * overlap exactly when C and D are strictly on the same side of line AB */
static int same_side(const double *A, const double *B, const double *C, const double *D) {
    int sc = o_orient2d(A, B, C), sd = o_orient2d(A, B, D);
    return sc * sd > 0;
}

/* closed segment pq meets closed (non-degenerate) triangle abc in 3D */
static int seg_tri_3d(const double *p, const double *q,
                      const double *a, const double *b, const double *c) {
    int op = o_orient3d(a, b, c, p), oq = o_orient3d(a, b, c, q);
    if (op * oq > 0) return 0;
    if (op == 0 && oq == 0) {
        int k = good_axis(a, b, c);
        double P2[2], Q2[2], A2[2], B2[2], C2[2];
        proj(p, k, P2); proj(q, k, Q2); proj(a, k, A2); proj(b, k, B2); proj(c, k, C2);
        if (pt_in_tri_2d(P2, A2, B2, C2) || pt_in_tri_2d(Q2, A2, B2, C2)) return 1;
        if (seg_seg_2d(P2, Q2, A2, B2) || seg_seg_2d(P2, Q2, B2, C2) || seg_seg_2d(P2, Q2, C2, A2))
            return 1;
        return 0;
    }
    /* the line pq crosses the plane once, inside the closed segment; it hits
     * the closed triangle iff its orientations against the three edges do not
     * take both strict signs */
    int s1 = o_orient3d(p, q, a, b), s2 = o_orient3d(p, q, b, c), s3 = o_orient3d(p, q, c, a);
    int pos = s1 > 0 || s2 > 0 || s3 > 0;
    int neg = s1 < 0 || s2 < 0 || s3 < 0;
    return !(pos && neg);
}

int o_tri_pair(const double *const P[3], const int32_t ip[3],
               const double *const Q[3], const int32_t iq[3]) {
    /* shared vertex ids; sp[i]=j means P corner i is Q corner j */
    int s = 0, sp[3] = {-1, -1, -1}, sq[3] = {-1, -1, -1};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (ip[i] == iq[j]) { sp[i] = j; sq[j] = i; s++; }
    if (s >= 3) return 1;

    int coplanar = o_orient3d(P[0], P[1], P[2], Q[0]) == 0 &&
                   o_orient3d(P[0], P[1], P[2], Q[1]) == 0 &&
                   o_orient3d(P[0], P[1], P[2], Q[2]) == 0;

    if (coplanar) {
        int k = good_axis(P[0], P[1], P[2]);
        double p2[3][2], q2[3][2];
        for (int i = 0; i < 3; i++) { proj(P[i], k, p2[i]); proj(Q[i], k, q2[i]); }
        if (s == 0) return coplanar_overlap((const double(*)[2])p2, (const double(*)[2])q2);
        if (s == 1) {
            int a = 0;
            while (sp[a] < 0) a++;
            int b = sp[a];
            return angle_overlap(p2[a], p2[(a + 1) % 3], p2[(a + 2) % 3],
                                 q2[(b + 1) % 3], q2[(b + 2) % 3]);
        }
        /* s == 2 */
        int c = 0;
        while (sp[c] >= 0) c++;
        int d = 0;
        while (sq[d] >= 0) d++;
        int a = (c + 1) % 3, b = (c + 2) % 3;
        return same_side(p2[a], p2[b], p2[c], q2[d]);
    }

    if (s == 2) return 0;
    if (s == 0) {
        for (int i = 0; i < 3; i++)
            if (seg_tri_3d(P[i], P[(i + 1) % 3], Q[0], Q[1], Q[2])) return 1;
        for (int j = 0; j < 3; j++)
            if (seg_tri_3d(Q[j], Q[(j + 1) % 3], P[0], P[1], P[2])) return 1;
        return 0;
    }
    /* s == 1: shared corner a of P (= corner b of Q); test the opposite edges */
    int a = 0;
    while (sp[a] < 0) a++;
    int b = sp[a];
    if (seg_tri_3d(P[(a + 1) % 3], P[(a + 2) % 3], Q[0], Q[1], Q[2])) return 1;
    if (seg_tri_3d(Q[(b + 1) % 3], Q[(b + 2) % 3], P[0], P[1], P[2])) return 1;
    return 0;
}
