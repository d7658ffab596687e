// Device-side helpers for the half-edge mesh and the per-edge arithmetic of
// the simplification round (PaMO Sec. 5.1, Eq. 1).
//
// Mesh layout in HBM (all arrays indexed by slot, compacted every round):
//   V     double[nv][3]    vertex positions
//   F     int32 [nf][3]    triangle corners, counter-clockwise seen from outside
//   twin  int32 [3 nf]     opposite half-edge; half-edge h = 3f + c runs from
//                          F[f][c] to F[f][(c+1)%3]
//   vh    int32 [nv]       one half-edge leaving each vertex
//   flags uint8 [3 nf]     invalid-edge flags (an edge is flagged when either of
//                          its half-edges is)
// An edge is represented by its smaller half-edge id, which is also its
// unique id inside the 64-bit key.
//
// Floating-point contract: every expression below is evaluated in float64 in
// exactly the order written (the library is built with contraction off), and
// sums over faces run in a fixed order (ascending face slot around one vertex;
// around the smaller endpoint first for an edge), so the results do not depend
// on the thread that computes them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// usable from host code too (unit tests of the arithmetic)
#define PAMO_HD __host__ __device__

#define PAMO_KEY_MAX 0xFFFFFFFFFFFFFFFFull
#define PAMO_SKINNY_K 3.4641016151377544  // 2 sqrt(3): 4 sqrt(3) A = (2 sqrt(3)) |n|

namespace pamo {

// The hardware deals the blocks of a launch to the 8 XCDs in turn (block b to
// XCD b mod 8), and each XCD has its own L2.  This returns a logical block id
// under which every XCD processes one contiguous eighth of the index range, so
// that mesh neighbourhoods gathered by neighbouring elements stay in one L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7, x = b & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// Item of this thread when n items (n known on the device only; the grid has
// a multiple of 8 blocks of `per` items each, at least n items in total) are
// split into 8 contiguous ranges, one per XCD: XCD x takes [x c, (x+1) c),
// c = ceil(n / 8), in the order of its blocks.  Valid when the result < *end.
__device__ __forceinline__ int64_t xcd_item(int64_t n, int per, int within, int64_t* end) {
  const int b = blockIdx.x, x = b & 7;
  const int64_t c = (n + 7) >> 3;
  const int64_t e = (int64_t)(x + 1) * c;
  *end = e < n ? e : n;
  return (int64_t)x * c + (int64_t)(b >> 3) * per + within;
}

PAMO_HD __forceinline__ int he_next(int h) { return h - h % 3 + (h % 3 == 2 ? 0 : h % 3 + 1); }
PAMO_HD __forceinline__ int he_prev(int h) { return h - h % 3 + (h % 3 == 0 ? 2 : h % 3 - 1); }

// rotate to the next half-edge leaving the same vertex
PAMO_HD __forceinline__ int he_rot(const int* __restrict__ twin, int h) { return twin[he_prev(h)]; }

struct P3 {
  double x, y, z;
};

PAMO_HD __forceinline__ P3 ld3(const double* __restrict__ V, int v) {
  return P3{V[3 * (int64_t)v], V[3 * (int64_t)v + 1], V[3 * (int64_t)v + 2]};
}

// Unit-normal plane quadric of triangle p0 p1 p2, 10 upper-triangle entries
// (xx xy xz xw yy yz yw zz zw ww).
PAMO_HD __forceinline__ void face_quadric(P3 p0, P3 p1, P3 p2, double* K) {
  double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  double nx = e1y * e2z - e1z * e2y;
  double ny = e1z * e2x - e1x * e2z;
  double nz = e1x * e2y - e1y * e2x;
  double len = sqrt(nx * nx + ny * ny + nz * nz);
  nx = nx / len;
  ny = ny / len;
  nz = nz / len;
  double d = -(nx * p0.x + ny * p0.y + nz * p0.z);
  K[0] = nx * nx; K[1] = nx * ny; K[2] = nx * nz; K[3] = nx * d;
  K[4] = ny * ny; K[5] = ny * nz; K[6] = ny * d;
  K[7] = nz * nz; K[8] = nz * d;
  K[9] = d * d;
}

// v^T Q v for v = (x, y, z, 1)
PAMO_HD __forceinline__ double quadric_eval(const double* q, P3 v) {
  double qx = q[0] * v.x + q[1] * v.y + q[2] * v.z + q[3];
  double qy = q[1] * v.x + q[4] * v.y + q[5] * v.z + q[6];
  double qz = q[2] * v.x + q[5] * v.y + q[7] * v.z + q[8];
  double qw = q[3] * v.x + q[6] * v.y + q[8] * v.z + q[9];
  return qx * v.x + qy * v.y + qz * v.z + qw;
}

// 1 - C_ijk of Eq. 1: C_ijk = 4 sqrt(3) A / (l01^2 + l12^2 + l20^2)
PAMO_HD __forceinline__ double skinny_term(P3 p0, P3 p1, P3 p2) {
  double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  double e3x = p2.x - p1.x, e3y = p2.y - p1.y, e3z = p2.z - p1.z;
  double nx = e1y * e2z - e1z * e2y;
  double ny = e1z * e2x - e1x * e2z;
  double nz = e1x * e2y - e1y * e2x;
  double nn = sqrt(nx * nx + ny * ny + nz * nz);
  double l01 = e1x * e1x + e1y * e1y + e1z * e1z;
  double l12 = e3x * e3x + e3y * e3y + e3z * e3z;
  double l20 = e2x * e2x + e2y * e2y + e2z * e2z;
  double lsum = l01 + l12 + l20;
  return 1.0 - (PAMO_SKINNY_K * nn) / lsum;
}

// Order-preserving 64-bit key: float32 (round to nearest even) cost in the
// high half, unique edge id in the low half (Sec. 5.1, cost propagation).
PAMO_HD __forceinline__ uint64_t make_key(double cost, uint32_t edge_id) {
  if (cost != cost) return PAMO_KEY_MAX;
  float c = (float)cost;
  uint32_t u;
  __builtin_memcpy(&u, &c, 4);
  uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)o << 32) | (uint64_t)edge_id;
}

// The float64 key mode: a total-order code of the float64 cost (zero of
// either sign as +0, NaN as the largest key); ranks in the order of (code,
// edge id) then replace it (rank_keys).
PAMO_HD __forceinline__ uint64_t cost_code64(double cost) {
  if (cost != cost) return PAMO_KEY_MAX;
  if (cost == 0.0) cost = 0.0;
  uint64_t u;
  __builtin_memcpy(&u, &cost, 8);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// squared distance from p to triangle abc: the closest point found by testing
// which Voronoi region of the triangle's vertices, edges or face holds p, with
// barycentric coordinates from dot products (the published method of
// C. Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5; may be NaN for
// a triangle of zero area)
__device__ __forceinline__ double tri_dist2(P3 p, P3 a, P3 b, P3 c) {
  double abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
  double acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
  double apx = p.x - a.x, apy = p.y - a.y, apz = p.z - a.z;
  double d1 = abx * apx + aby * apy + abz * apz, d2 = acx * apx + acy * apy + acz * apz;
  P3 q;
  if (d1 <= 0.0 && d2 <= 0.0) {
    q = a;
  } else {
    double bpx = p.x - b.x, bpy = p.y - b.y, bpz = p.z - b.z;
    double d3 = abx * bpx + aby * bpy + abz * bpz, d4 = acx * bpx + acy * bpy + acz * bpz;
    double cpx = p.x - c.x, cpy = p.y - c.y, cpz = p.z - c.z;
    double d5 = abx * cpx + aby * cpy + abz * cpz, d6 = acx * cpx + acy * cpy + acz * cpz;
    double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    if (d3 >= 0.0 && d4 <= d3) {
      q = b;
    } else if (d6 >= 0.0 && d5 <= d6) {
      q = c;
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
      double v = d1 / (d1 - d3);
      q = P3{a.x + v * abx, a.y + v * aby, a.z + v * abz};
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
      double v = d2 / (d2 - d6);
      q = P3{a.x + v * acx, a.y + v * acy, a.z + v * acz};
    } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
      double v = (d4 - d3) / ((d4 - d3) + (d5 - d6));
      q = P3{b.x + v * (c.x - b.x), b.y + v * (c.y - b.y), b.z + v * (c.z - b.z)};
    } else {
      double den = 1.0 / (va + vb + vc);
      double v = vb * den, w = vc * den;
      q = P3{a.x + abx * v + acx * w, a.y + aby * v + acy * w, a.z + abz * v + acz * w};
    }
  }
  double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
  return dx * dx + dy * dy + dz * dz;
}

// Sorted insertion of x into a[0..CAP) kept ascending with INT_MAX padding.
// Fully unrolled so the list stays in registers.
template <int CAP>
PAMO_HD __forceinline__ void sorted_insert(int* a, int x) {
#pragma unroll
  for (int i = CAP - 1; i >= 0; --i) {
    int lo = i > 0 ? a[i - 1] : INT32_MIN;
    int m = lo > x ? lo : x;
    a[i] = a[i] < m ? a[i] : m;
  }
}

}  // namespace pamo
