// Device predicates for the self-intersection test of PaMO (Sec. 5.2 and
// Appendix 3) and for the degeneracy check of generated triangles.
//
// The paper evaluates the test in FP32 with FP64 for coplanarity and the
// intersection line; here every sign is exact:
//   * orient2d / orient3d are first evaluated in float64 with an a-priori
//     error bound (a few times the bounds of Shewchuk 1997, "Adaptive
//     precision floating-point arithmetic and fast robust geometric
//     predicates"); a sign outside the bound is certain;
//   * otherwise the fast instantiation (EX = false) answers UNK and the pair
//     is deferred, and the exact instantiation (EX = true) recomputes the
//     determinant as a floating-point expansion (Shewchuk's two-sum,
//     two-product, grow and scale operations) whose sign is exact as long as
//     no partial product underflows (coordinate differences are 0 or larger
//     than about 1e-90; meshes normalised to [0,1]^3 satisfy this).
//
// Pair test, by the number s of vertex ids the two triangles share:
//   s = 3: reported;  s = 2 (edge AB, third corners C, D): reported only when
//   the four points are coplanar and C, D lie strictly on the same side of AB;
//   s = 1 (corner A, opposite edges BC and DE): reported when segment BC meets
//   triangle ADE or segment DE meets triangle ABC, i.e. the triangles meet
//   somewhere other than A;  s = 0: reported when the closed triangles meet,
//   i.e. some edge of one meets the other.
#pragma once
#include "mesh_dev.hpp"

namespace pamo {

constexpr int UNK = 2;

// ---------------------------------------------------------------- expansions
PAMO_HD __forceinline__ void two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}
PAMO_HD __forceinline__ void fast_two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  y = b - bv;
}
PAMO_HD __forceinline__ void two_diff(double a, double b, double& x, double& y) {
  x = a - b;
  double bv = a - x;
  double av = x + bv;
  double br = bv - b;
  double ar = a - av;
  y = ar + br;
}
PAMO_HD __forceinline__ void two_prod(double a, double b, double& x, double& y) {
  x = a * b;
  y = fma(a, b, -x);
}

// expansions: nonoverlapping components in increasing magnitude, no zeros
// except a lone zero for the value 0

PAMO_HD inline int ex_from_diff(double a, double b, double* h) {
  double x, y;
  two_diff(a, b, x, y);
  int n = 0;
  if (y != 0.0) h[n++] = y;
  if (x != 0.0 || n == 0) h[n++] = x;
  return n;
}

// h = e + b
PAMO_HD inline int ex_grow(int elen, const double* e, double b, double* h) {
  double Q = b;
  int n = 0;
  for (int i = 0; i < elen; i++) {
    double Qn, hh;
    two_sum(Q, e[i], Qn, hh);
    Q = Qn;
    if (hh != 0.0) h[n++] = hh;
  }
  if (Q != 0.0 || n == 0) h[n++] = Q;
  return n;
}

// h = e + f, using t as scratch (both of length >= elen + flen)
PAMO_HD inline int ex_sum(int elen, const double* e, int flen, const double* f, double* h, double* t) {
  int n = elen;
  for (int i = 0; i < elen; i++) h[i] = e[i];
  for (int j = 0; j < flen; j++) {
    int m = ex_grow(n, h, f[j], t);
    for (int i = 0; i < m; i++) h[i] = t[i];
    n = m;
  }
  return n;
}

// h = e * b
PAMO_HD inline int ex_scale(int elen, const double* e, double b, double* h) {
  double Q, hh;
  int n = 0;
  two_prod(e[0], b, Q, hh);
  if (hh != 0.0) h[n++] = hh;
  for (int i = 1; i < elen; i++) {
    double p1, p0, s;
    two_prod(e[i], b, p1, p0);
    two_sum(Q, p0, s, hh);
    if (hh != 0.0) h[n++] = hh;
    fast_two_sum(p1, s, Q, hh);
    if (hh != 0.0) h[n++] = hh;
  }
  if (Q != 0.0 || n == 0) h[n++] = Q;
  return n;
}

// h = e * f (|h| <= 2 elen flen); s1, s2, s3 scratch of that size
PAMO_HD inline int ex_mul(int elen, const double* e, int flen, const double* f, double* h, double* s1,
                             double* s2, double* s3) {
  int n = ex_scale(elen, e, f[0], h);
  for (int j = 1; j < flen; j++) {
    int m = ex_scale(elen, e, f[j], s1);
    int k = ex_sum(n, h, m, s1, s2, s3);
    for (int i = 0; i < k; i++) h[i] = s2[i];
    n = k;
  }
  return n;
}

PAMO_HD __forceinline__ int ex_sign(int n, const double* e) {
  double v = e[n - 1];
  return v > 0.0 ? 1 : (v < 0.0 ? -1 : 0);
}

PAMO_HD inline void ex_negate(int n, double* e) {
  for (int i = 0; i < n; i++) e[i] = -e[i];
}

// exact sign of (a - c) x (b - c)
PAMO_HD inline int orient2d_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  double acx[2], acy[2], bcx[2], bcy[2], l[8], r[8], s1[8], s2[16], s3[16], d[16];
  int nacx = ex_from_diff(ax, cx, acx), nacy = ex_from_diff(ay, cy, acy);
  int nbcx = ex_from_diff(bx, cx, bcx), nbcy = ex_from_diff(by, cy, bcy);
  int nl = ex_mul(nacx, acx, nbcy, bcy, l, s1, s2, s3);
  int nr = ex_mul(nacy, acy, nbcx, bcx, r, s1, s2, s3);
  ex_negate(nr, r);
  int nd = ex_sum(nl, l, nr, r, d, s3);
  return ex_sign(nd, d);
}

// exact sign of det[a-d; b-d; c-d]
PAMO_HD inline __attribute__((noinline)) int orient3d_exact(P3 a, P3 b, P3 c, P3 d) {
  double ad[3][2], bd[3][2], cd[3][2];
  int nad[3], nbd[3], ncd[3];
  const double A[3] = {a.x, a.y, a.z}, B[3] = {b.x, b.y, b.z}, C[3] = {c.x, c.y, c.z}, D[3] = {d.x, d.y, d.z};
  for (int k = 0; k < 3; k++) {
    nad[k] = ex_from_diff(A[k], D[k], ad[k]);
    nbd[k] = ex_from_diff(B[k], D[k], bd[k]);
    ncd[k] = ex_from_diff(C[k], D[k], cd[k]);
  }
  double t1[8], t2[8], m[16], p[64], acc[192], nxt[192], s1[64], s2[192], s3[192];
  int nacc = 0;
  // det = ad_x (bd_y cd_z - bd_z cd_y) + bd_x (cd_y ad_z - cd_z ad_y) + cd_x (ad_y bd_z - ad_z bd_y)
  for (int term = 0; term < 3; term++) {
    const double *u0, *u1, *v0, *v1, *w;
    int nu0, nu1, nv0, nv1, nw;
    if (term == 0) {
      u0 = bd[1]; nu0 = nbd[1]; u1 = cd[2]; nu1 = ncd[2]; v0 = bd[2]; nv0 = nbd[2]; v1 = cd[1]; nv1 = ncd[1];
      w = ad[0]; nw = nad[0];
    } else if (term == 1) {
      u0 = cd[1]; nu0 = ncd[1]; u1 = ad[2]; nu1 = nad[2]; v0 = cd[2]; nv0 = ncd[2]; v1 = ad[1]; nv1 = nad[1];
      w = bd[0]; nw = nbd[0];
    } else {
      u0 = ad[1]; nu0 = nad[1]; u1 = bd[2]; nu1 = nbd[2]; v0 = ad[2]; nv0 = nad[2]; v1 = bd[1]; nv1 = nbd[1];
      w = cd[0]; nw = ncd[0];
    }
    int n1 = ex_mul(nu0, u0, nu1, u1, t1, s1, s2, s3);
    int n2 = ex_mul(nv0, v0, nv1, v1, t2, s1, s2, s3);
    ex_negate(n2, t2);
    int nm = ex_sum(n1, t1, n2, t2, m, s3);
    int np = ex_mul(nm, m, nw, w, p, s1, s2, s3);
    if (nacc == 0) {
      for (int i = 0; i < np; i++) acc[i] = p[i];
      nacc = np;
    } else {
      nacc = ex_sum(nacc, acc, np, p, nxt, s3);
      for (int i = 0; i < nacc; i++) acc[i] = nxt[i];
    }
  }
  return ex_sign(nacc, acc);
}

// ---------------------------------------------------------------- filters
PAMO_HD __forceinline__ int orient2d_filter(double ax, double ay, double bx, double by, double cx, double cy) {
  double l = (ax - cx) * (by - cy);
  double r = (ay - cy) * (bx - cx);
  double det = l - r;
  double perm = fabs(l) + fabs(r);
  double bound = 1e-15 * perm;
  if (perm > 1e-150 && (det > bound || -det > bound)) return det > 0.0 ? 1 : -1;
  return UNK;
}

PAMO_HD __forceinline__ int orient3d_filter(P3 a, P3 b, P3 c, P3 d) {
  double adx = a.x - d.x, ady = a.y - d.y, adz = a.z - d.z;
  double bdx = b.x - d.x, bdy = b.y - d.y, bdz = b.z - d.z;
  double cdx = c.x - d.x, cdy = c.y - d.y, cdz = c.z - d.z;
  double bdycdz = bdy * cdz, bdzcdy = bdz * cdy;
  double cdyadz = cdy * adz, cdzady = cdz * ady;
  double adybdz = ady * bdz, adzbdy = adz * bdy;
  double det = adx * (bdycdz - bdzcdy) + bdx * (cdyadz - cdzady) + cdx * (adybdz - adzbdy);
  double perm = fabs(adx) * (fabs(bdycdz) + fabs(bdzcdy)) + fabs(bdx) * (fabs(cdyadz) + fabs(cdzady)) +
                fabs(cdx) * (fabs(adybdz) + fabs(adzbdy));
  double bound = 2e-15 * perm;
  if (perm > 1e-150 && (det > bound || -det > bound)) return det > 0.0 ? 1 : -1;
  return UNK;
}

template <bool EX>
PAMO_HD __forceinline__ int o3(P3 a, P3 b, P3 c, P3 d) {
  int s = orient3d_filter(a, b, c, d);
  if (EX && s == UNK) s = orient3d_exact(a, b, c, d);
  return s;
}

template <bool EX>
PAMO_HD __forceinline__ int o2(double ax, double ay, double bx, double by, double cx, double cy) {
  int s = orient2d_filter(ax, ay, bx, by, cx, cy);
  if (EX && s == UNK) s = orient2d_exact(ax, ay, bx, by, cx, cy);
  return s;
}

// coordinates after dropping axis k
PAMO_HD __forceinline__ double pu(P3 p, int k) { return k == 0 ? p.y : (k == 1 ? p.z : p.x); }
PAMO_HD __forceinline__ double pv(P3 p, int k) { return k == 0 ? p.z : (k == 1 ? p.x : p.y); }

template <bool EX>
PAMO_HD __forceinline__ int o2k(P3 a, P3 b, P3 c, int k) {
  return o2<EX>(pu(a, k), pv(a, k), pu(b, k), pv(b, k), pu(c, k), pv(c, k));
}

// exact: is the triangle collinear (zero in every axis projection)?
PAMO_HD inline __attribute__((noinline)) bool degenerate_exact(P3 a, P3 b, P3 c) {
  for (int k = 0; k < 3; k++)
    if (o2k<true>(a, b, c, k) != 0) return false;
  return true;
}

// an axis whose projection keeps the (non-degenerate) triangle abc
// non-degenerate; exact
PAMO_HD inline int proj_axis_exact(P3 a, P3 b, P3 c) {
  for (int k = 2; k >= 0; k--)
    if (o2k<true>(a, b, c, k) != 0) return k;
  return 2;
}

// 2D helpers in projection k, exact (only reached for exactly coplanar input)
PAMO_HD inline bool collinear_inside(P3 p, P3 q, P3 x, int k) {
  double lo0 = fmin(pu(p, k), pu(q, k)), hi0 = fmax(pu(p, k), pu(q, k));
  double lo1 = fmin(pv(p, k), pv(q, k)), hi1 = fmax(pv(p, k), pv(q, k));
  return pu(x, k) >= lo0 && pu(x, k) <= hi0 && pv(x, k) >= lo1 && pv(x, k) <= hi1;
}

PAMO_HD inline bool seg_seg_2d(P3 p, P3 q, P3 r, P3 s, int k) {
  int o1 = o2k<true>(p, q, r, k), o2_ = o2k<true>(p, q, s, k);
  int o3_ = o2k<true>(r, s, p, k), o4 = o2k<true>(r, s, q, k);
  if (o1 * o2_ < 0 && o3_ * o4 < 0) return true;
  if (o1 == 0 && collinear_inside(p, q, r, k)) return true;
  if (o2_ == 0 && collinear_inside(p, q, s, k)) return true;
  if (o3_ == 0 && collinear_inside(r, s, p, k)) return true;
  if (o4 == 0 && collinear_inside(r, s, q, k)) return true;
  return false;
}

PAMO_HD inline bool point_in_tri_2d(P3 x, P3 a, P3 b, P3 c, int k) {
  int s1 = o2k<true>(a, b, x, k), s2 = o2k<true>(b, c, x, k), s3 = o2k<true>(c, a, x, k);
  bool pos = s1 > 0 || s2 > 0 || s3 > 0;
  bool neg = s1 < 0 || s2 < 0 || s3 < 0;
  return !(pos && neg);
}

// closed segment pq against closed triangle abc; op, oq = orientation of p, q
// against the plane of abc (as o3(a, b, c, .)).  Returns 0, 1 or UNK.
template <bool EX>
PAMO_HD __forceinline__ int seg_tri_body(P3 p, P3 q, P3 a, P3 b, P3 c, int op, int oq) {
  if (op == UNK || oq == UNK) {
    // a certain strict same side still decides
    return UNK;
  }
  if (op * oq > 0) return 0;
  if (op == 0 && oq == 0) {
    if (!EX) return UNK;
    int k = proj_axis_exact(a, b, c);
    if (point_in_tri_2d(p, a, b, c, k) || point_in_tri_2d(q, a, b, c, k)) return 1;
    if (seg_seg_2d(p, q, a, b, k) || seg_seg_2d(p, q, b, c, k) || seg_seg_2d(p, q, c, a, k)) return 1;
    return 0;
  }
  int s1 = o3<EX>(p, q, a, b);
  int s2 = o3<EX>(p, q, b, c);
  int s3 = o3<EX>(p, q, c, a);
  bool pos = s1 == 1 || s2 == 1 || s3 == 1;
  bool neg = s1 == -1 || s2 == -1 || s3 == -1;
  if (pos && neg) return 0;
  if (s1 == UNK || s2 == UNK || s3 == UNK) return UNK;
  return 1;
}

// the exact form is large and rarely reached: one out-of-line copy; the
// filtered form is small and sits on the hot path: inlined
template <bool EX>
PAMO_HD __attribute__((noinline)) int seg_tri_call(P3 p, P3 q, P3 a, P3 b, P3 c, int op, int oq) {
  return seg_tri_body<EX>(p, q, a, b, c, op, oq);
}
template <bool EX>
PAMO_HD __forceinline__ int seg_tri(P3 p, P3 q, P3 a, P3 b, P3 c, int op, int oq) {
  if (EX) return seg_tri_call<EX>(p, q, a, b, c, op, oq);
  return seg_tri_body<EX>(p, q, a, b, c, op, oq);
}

// element i of a 3-array held in registers, without dynamic indexing
PAMO_HD __forceinline__ double sel3d(double a, double b, double c, int i) { return i == 0 ? a : (i == 1 ? b : c); }
PAMO_HD __forceinline__ P3 sel3(const P3* v, int i) {
  return P3{sel3d(v[0].x, v[1].x, v[2].x, i), sel3d(v[0].y, v[1].y, v[2].y, i), sel3d(v[0].z, v[1].z, v[2].z, i)};
}
PAMO_HD __forceinline__ int sel3i(const int* v, int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }

// Self-intersection predicate for two triangles with corner positions P, Q
// and vertex ids ip, iq.  Returns 0, 1, or (EX = false only) UNK.
template <bool EX>
PAMO_HD inline int tri_pair(const P3* P, const int* ip, const P3* Q, const int* iq) {
  int s = 0, pa = -1, qa = -1, pnot = -1, qnot = -1;
  bool pin[3] = {false, false, false}, qin[3] = {false, false, false};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      if (ip[i] == iq[j]) {
        s++;
        pin[i] = true;
        qin[j] = true;
        pa = i;
        qa = j;
      }
  if (s >= 3) return 1;
  if (s == 2) {
    for (int i = 0; i < 3; i++) {
      if (!pin[i]) pnot = i;
      if (!qin[i]) qnot = i;
    }
    int o = o3<EX>(P[0], P[1], P[2], sel3(Q, qnot));
    if (o == UNK) return UNK;
    if (o != 0) return 0;
    if (!EX) return UNK;  // unreachable: the filter never certifies a zero
    // coplanar: overlap iff the third corners lie strictly on the same side
    int k = proj_axis_exact(P[0], P[1], P[2]);
    P3 A = sel3(P, (pnot + 1) % 3), B = sel3(P, (pnot + 2) % 3);
    int sc = o2k<true>(A, B, sel3(P, pnot), k), sd = o2k<true>(A, B, sel3(Q, qnot), k);
    return sc * sd > 0 ? 1 : 0;
  }
  if (s == 1) {
    // seg BC of P against Q, then seg DE of Q against P (one loop body, so
    // one inlined copy of the segment test)
    const P3 B = sel3(P, (pa + 1) % 3), C = sel3(P, (pa + 2) % 3);
    const P3 D = sel3(Q, (qa + 1) % 3), E = sel3(Q, (qa + 2) % 3);
    bool unk = false;
#pragma unroll 1
    for (int w = 0; w < 2; w++) {
      const P3 p = w ? D : B, q = w ? E : C;
      const P3 a = w ? P[0] : Q[0], b = w ? P[1] : Q[1], c = w ? P[2] : Q[2];
      int r = seg_tri<EX>(p, q, a, b, c, o3<EX>(a, b, c, p), o3<EX>(a, b, c, q));
      if (r == 1) return 1;
      unk |= r == UNK;
    }
    return unk ? UNK : 0;
  }
  // s == 0
  int sp[3], sq[3];
  for (int i = 0; i < 3; i++) sp[i] = o3<EX>(Q[0], Q[1], Q[2], P[i]);
  if ((sp[0] == 1 && sp[1] == 1 && sp[2] == 1) || (sp[0] == -1 && sp[1] == -1 && sp[2] == -1)) return 0;
  for (int j = 0; j < 3; j++) sq[j] = o3<EX>(P[0], P[1], P[2], Q[j]);
  if ((sq[0] == 1 && sq[1] == 1 && sq[2] == 1) || (sq[0] == -1 && sq[1] == -1 && sq[2] == -1)) return 0;
  bool unk = false;
  // the three edges of P against Q, then the three edges of Q against P
#pragma unroll 1
  for (int e = 0; e < 6; e++) {
    const bool w = e >= 3;
    const int i = w ? e - 3 : e, i1 = i == 2 ? 0 : i + 1;
    const P3 p = w ? sel3(Q, i) : sel3(P, i), q = w ? sel3(Q, i1) : sel3(P, i1);
    const P3 a = w ? P[0] : Q[0], b = w ? P[1] : Q[1], c = w ? P[2] : Q[2];
    const int op = w ? sel3i(sq, i) : sel3i(sp, i), oq = w ? sel3i(sq, i1) : sel3i(sp, i1);
    int r = seg_tri<EX>(p, q, a, b, c, op, oq);
    if (r == 1) return 1;
    unk |= r == UNK;
  }
  return unk ? UNK : 0;
}

}  // namespace pamo
