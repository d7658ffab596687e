// The safe projection stage (Sec. 6; Alg. 2; App. 2.2) on the GPU.
//
// Energy (Sec. 6.1, Sec. 6.2): B = k_dis (E_S2M + E_M2S) + k_elas E_elas
// + k_bend E_bend + k_bar sum b(d) over the contact pairs, with
//   E_S2M  = sum_i s0_i |x_i - target_i|^2 (s0 the mixed Voronoi areas of the
//            rest mesh, Meyer et al. 2003; targets the closest input-mesh
//            points, refreshed every few iterations),
//   E_M2S  = A_in / m sum_s d^2(y_s, triangle tri_s at X) (samples y_s on the
//            input mesh, tri_s the closest triangle at the last refresh, the
//            squared distance to its closest vertex, edge or face at X),
//   E_elas = sum_f A0_f / 4 |C_f - I|_F^2, C = B^T G B with G the Gram matrix
//            of the face's two edges and B the inverse of its rest edges in a
//            frame of the rest plane (St. Venant-Kirchhoff, E = 1, nu = 0),
//   E_bend = sum_e |e0| / 2 (theta_e - theta0_e)^2, theta the signed dihedral
//            angle about the edge,
//   b(d)   = -(d - dhat)^2 ln(d / dhat) for point-triangle and edge-edge pairs
//            closer than dhat.
//
// Derivatives: every element (vertex, sample, face, edge stencil, contact
// pair) is one smooth closed form once its closest features are classified
// from the current positions.  Its gradient and Hessian come from hyper-dual
// numbers (f + a e1 + b e2 + c e1 e2, e1^2 = e2^2 = 0): evaluating the element
// with e1 seeded on coordinate i and e2 on coordinate j gives d2f/didj exactly
// (no truncation), so one thread per (element, i <= j) fills the Hessian.
// Each element Hessian is then projected to positive semi-definite (negative
// eigenvalues clamped to zero) by a cyclic Jacobi eigen-decomposition held in
// registers (Golub and Van Loan, Sec. 8.5), and the Newton system is solved
// by conjugate gradients with a 3x3 block-Jacobi preconditioner, matrix-free
// over the element Hessians (fp64 atomics scatter each element's product).
//
// Step bound: additive CCD (Li, Kaufman and Jiang 2021) over the vertex-face
// and edge-edge pairs whose swept boxes overlap; contacts and CCD candidates
// come from one walk over the library's LBVH of (padded or swept) face boxes,
// each face pair visited once and each primitive pair found from the faces
// that own its primitives (a vertex is owned by its smallest incident face, an
// edge by the smaller of its two faces).
#include <algorithm>
#include <cmath>
#include <vector>

#include "project.hpp"
#include "round.hpp"

namespace pamo {
namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

constexpr double TIE = 1e-9;  // closest-triangle ties: the smallest index within this relative margin
constexpr double TIE_ABS = 1e-24;
constexpr double PARALLEL = 1e-20;  // two edges are parallel when |ea x eb|^2 <= PARALLEL |ea|^2 |eb|^2
constexpr int ACCD_MAX_STEPS = 1 << 20;
constexpr double LS_MIN_STEP = 1e-14;  // the line search stops once alpha |p| falls below this length
constexpr int WALK_STACK = 48;  // 3 (D - 1) + 4 entries at most for D <= 14 levels

// ------------------------------------------------------------ hyper-dual numbers
struct HD {
  double v, a, b, ab;
};
__device__ __forceinline__ HD operator+(HD x, HD y) { return {x.v + y.v, x.a + y.a, x.b + y.b, x.ab + y.ab}; }
__device__ __forceinline__ HD operator-(HD x, HD y) { return {x.v - y.v, x.a - y.a, x.b - y.b, x.ab - y.ab}; }
__device__ __forceinline__ HD operator-(HD x) { return {-x.v, -x.a, -x.b, -x.ab}; }
__device__ __forceinline__ HD operator+(HD x, double c) { return {x.v + c, x.a, x.b, x.ab}; }
__device__ __forceinline__ HD operator-(HD x, double c) { return {x.v - c, x.a, x.b, x.ab}; }
__device__ __forceinline__ HD operator*(HD x, HD y) {
  return {x.v * y.v, x.v * y.a + x.a * y.v, x.v * y.b + x.b * y.v, x.v * y.ab + x.a * y.b + x.b * y.a + x.ab * y.v};
}
__device__ __forceinline__ HD operator*(double c, HD x) { return {c * x.v, c * x.a, c * x.b, c * x.ab}; }
// f applied to x, given f(x.v), f'(x.v) and f''(x.v)
__device__ __forceinline__ HD chain(HD x, double f, double f1, double f2) {
  return {f, f1 * x.a, f1 * x.b, f1 * x.ab + f2 * x.a * x.b};
}
__device__ __forceinline__ HD operator/(HD x, HD y) {
  const double r = 1.0 / y.v;
  return x * chain(y, r, -r * r, 2.0 * r * r * r);
}
__device__ __forceinline__ HD operator/(HD x, double c) { return {x.v / c, x.a / c, x.b / c, x.ab / c}; }

__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ HD f_sqrt(HD x) {
  const double s = sqrt(x.v);
  return chain(x, s, 0.5 / s, -0.25 / (s * x.v));
}
__device__ __forceinline__ double f_log(double x) { return log(x); }
__device__ __forceinline__ HD f_log(HD x) { return chain(x, log(x.v), 1.0 / x.v, -1.0 / (x.v * x.v)); }
__device__ __forceinline__ double f_atan2(double y, double x) { return atan2(y, x); }
// d atan2(y, x) = (x dy - y dx) / r^2; the mixed part differentiates that
// quotient once more
__device__ __forceinline__ HD f_atan2(HD y, HD x) {
  const double r2 = x.v * x.v + y.v * y.v;
  const double na = x.v * y.a - y.v * x.a, nb = x.v * y.b - y.v * x.b;
  const double nab = x.b * y.a + x.v * y.ab - y.b * x.a - y.v * x.ab;
  const double r2b = 2.0 * (x.v * x.b + y.v * y.b);
  return {atan2(y.v, x.v), na / r2, nb / r2, (nab * r2 - na * r2b) / (r2 * r2)};
}

template <class T>
__device__ __forceinline__ T cst(double c);
template <>
__device__ __forceinline__ double cst<double>(double c) {
  return c;
}
template <>
__device__ __forceinline__ HD cst<HD>(double c) {
  return {c, 0.0, 0.0, 0.0};
}

template <class T>
struct V3 {
  T x, y, z;
};
template <class T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T>
__device__ __forceinline__ V3<T> ld3(const T* z, int i) {
  return {z[3 * i], z[3 * i + 1], z[3 * i + 2]};
}
using D3 = V3<double>;
__device__ __forceinline__ D3 ldX(const double* X, int v) {
  return {X[3 * (int64_t)v], X[3 * (int64_t)v + 1], X[3 * (int64_t)v + 2]};
}

// ------------------------------------------------------------ closest features
// Closest feature of triangle abc to p (regions of Ericson, Real-Time Collision
// Detection, Sec. 5.1.5): 0 the face, 1 edge ab, 2 edge bc, 3 edge ca, 4 vertex
// a, 5 vertex b, 6 vertex c.
__device__ int pt_feature(D3 p, D3 a, D3 b, D3 c) {
  const D3 ab = b - a, ac = c - a, ap = p - a;
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) return 4;
  const D3 bp = p - b;
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) return 5;
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return 1;
  const D3 cp = p - c;
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return 6;
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 3;
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) return 2;
  return 0;
}

// end r of the segment that point p (0, 1 on the first, 2, 3 on the second)
// is not on; with p and r known at compile time the points stay in registers
__host__ __device__ constexpr int ee_other(int p, int r) { return p < 2 ? 2 + r : r; }

// Closest features of segments P0P1 and P2P3: 0 inside both (not parallel):
// line against line; 1 + p point p against the other segment's line; 5 + 2 p
// + r point p against end r of the other segment.  The interior case is the
// stationary point of the squared distance over both segment parameters when
// it lies inside (0, 1)^2, else the nearest of the four point-segment
// distances.
__device__ int ee_feature(const D3* P) {
  const D3 ea = P[1] - P[0], eb = P[3] - P[2], w = P[0] - P[2];
  const D3 n = cross(ea, eb);
  const double A = dot(ea, ea), B = dot(ea, eb), C = dot(eb, eb), Dv = dot(ea, w), E = dot(eb, w);
  if (dot(n, n) > PARALLEL * A * C) {
    const double den = A * C - B * B;
    const double s = (B * E - C * Dv) / den, t = (A * E - B * Dv) / den;
    if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) return 0;
  }
  double best = INFINITY;
  int code = 0;
#pragma unroll
  for (int p = 0; p < 4; p++) {
    const D3 u = P[ee_other(p, 0)], v = P[ee_other(p, 1)];
    const D3 ab = v - u, pu = P[p] - u;
    double t = dot(pu, ab) / fmax(dot(ab, ab), 1e-300);
    t = fmin(fmax(t, 0.0), 1.0);
    const D3 q{u.x + t * ab.x, u.y + t * ab.y, u.z + t * ab.z};
    const D3 d = P[p] - q;
    const double d2 = dot(d, d);
    if (d2 < best) {
      best = d2;
      code = t <= 0.0 ? 5 + 2 * p : (t >= 1.0 ? 6 + 2 * p : 1 + p);
    }
  }
  return code;
}

// ------------------------------------------------------------ distances by feature
template <class T>
__device__ __forceinline__ T d2_pp(V3<T> p, V3<T> a) {
  const V3<T> d = p - a;
  return dot(d, d);
}
template <class T>
__device__ __forceinline__ T d2_pl(V3<T> p, V3<T> a, V3<T> b) {
  const V3<T> e = b - a;
  const V3<T> c = cross(p - a, e);
  return dot(c, c) / dot(e, e);
}
template <class T>
__device__ __forceinline__ T d2_pf(V3<T> p, V3<T> a, V3<T> b, V3<T> c) {
  const V3<T> n = cross(b - a, c - a);
  const T s = dot(p - a, n);
  return s * s / dot(n, n);
}
template <class T>
__device__ __forceinline__ T d2_ll(V3<T> a0, V3<T> a1, V3<T> b0, V3<T> b1) {
  const V3<T> n = cross(a1 - a0, b1 - b0);
  const T s = dot(b0 - a0, n);
  return s * s / dot(n, n);
}
template <class T>
__device__ T pt_d2(int code, V3<T> p, V3<T> a, V3<T> b, V3<T> c) {
  switch (code) {
    case 0: return d2_pf(p, a, b, c);
    case 1: return d2_pl(p, a, b);
    case 2: return d2_pl(p, b, c);
    case 3: return d2_pl(p, c, a);
    case 4: return d2_pp(p, a);
    case 5: return d2_pp(p, b);
    default: return d2_pp(p, c);
  }
}
// (one case per feature code, so that no point is indexed at run time)
template <class T>
__device__ T ee_d2(int code, const V3<T>* P) {
  switch (code) {
    case 0: return d2_ll(P[0], P[1], P[2], P[3]);
    case 1: return d2_pl(P[0], P[ee_other(0, 0)], P[ee_other(0, 1)]);
    case 2: return d2_pl(P[1], P[ee_other(1, 0)], P[ee_other(1, 1)]);
    case 3: return d2_pl(P[2], P[ee_other(2, 0)], P[ee_other(2, 1)]);
    case 4: return d2_pl(P[3], P[ee_other(3, 0)], P[ee_other(3, 1)]);
    case 5: return d2_pp(P[0], P[ee_other(0, 0)]);
    case 6: return d2_pp(P[0], P[ee_other(0, 1)]);
    case 7: return d2_pp(P[1], P[ee_other(1, 0)]);
    case 8: return d2_pp(P[1], P[ee_other(1, 1)]);
    case 9: return d2_pp(P[2], P[ee_other(2, 0)]);
    case 10: return d2_pp(P[2], P[ee_other(2, 1)]);
    case 11: return d2_pp(P[3], P[ee_other(3, 0)]);
    default: return d2_pp(P[3], P[ee_other(3, 1)]);
  }
}
__device__ __forceinline__ double pt_dist2(D3 p, D3 a, D3 b, D3 c) { return pt_d2<double>(pt_feature(p, a, b, c), p, a, b, c); }
__device__ __forceinline__ double ee_dist2(const D3* P) { return ee_d2<double>(ee_feature(P), P); }

// ------------------------------------------------------------ element energies
template <class T>
__device__ T elastic_e(const T* z, const double* Bi, double A0) {
  const V3<T> x0 = ld3(z, 0), x1 = ld3(z, 1), x2 = ld3(z, 2);
  const V3<T> d0 = x1 - x0, d1 = x2 - x0;
  const T g00 = dot(d0, d0), g01 = dot(d0, d1), g11 = dot(d1, d1);
  const double b00 = Bi[0], b01 = Bi[1], b10 = Bi[2], b11 = Bi[3];
  // C = B^T G B
  const T gb00 = b00 * g00 + b10 * g01, gb01 = b01 * g00 + b11 * g01;
  const T gb10 = b00 * g01 + b10 * g11, gb11 = b01 * g01 + b11 * g11;
  const T c00 = b00 * gb00 + b10 * gb10, c01 = b00 * gb01 + b10 * gb11, c11 = b01 * gb01 + b11 * gb11;
  const T e00 = c00 - 1.0, e11 = c11 - 1.0;
  return (0.25 * A0) * (e00 * e00 + 2.0 * (c01 * c01) + e11 * e11);
}

// signed angle between the normals of faces (i, j, k) and (j, i, l) about i -> j
template <class T>
__device__ T dihedral(V3<T> xi, V3<T> xj, V3<T> xk, V3<T> xl) {
  const V3<T> e = xj - xi;
  const V3<T> n1 = cross(e, xk - xi);
  const V3<T> n2 = cross(xi - xj, xl - xj);
  const T el = f_sqrt(dot(e, e));
  return f_atan2(dot(cross(n1, n2), e) / el, dot(n1, n2));
}

template <class T>
__device__ T bend_e(const T* z, double th0, double l0) {
  const T d = dihedral(ld3(z, 0), ld3(z, 1), ld3(z, 2), ld3(z, 3)) - th0;
  return (0.5 * l0) * (d * d);
}

template <class T>
__device__ T barrier_e(T d2, double dhat) {
  const T d = f_sqrt(d2);
  const T t = d - dhat;
  return -(t * t) * f_log(d / dhat);
}

// ------------------------------------------------------------ element sets
enum Kind { K_M2S = 0, K_EL = 1, K_BEND = 2, K_PT = 3, K_EE = 4, K_KINDS = 5 };
template <int K>
struct KT {
  static constexpr int NV = (K == K_M2S || K == K_EL) ? 3 : 4;
  static constexpr int N = 3 * NV;
  static constexpr int NP = N * (N + 1) / 2;
};

struct Elems {
  const int* ids = nullptr;  // NV vertex ids per element
  int n = 0;                 // elements (also the stride of the SoA arrays)
  double w = 0.0;            // weight of the term in B
  const double* Y = nullptr;     // samples (M2S)
  const double* Binv = nullptr;  // elastic rest data
  const double* A0 = nullptr;
  const double* th0 = nullptr;   // bending rest data
  const double* l0 = nullptr;
  double dhat = 0.0;
  double* H = nullptr;    // weighted Hessians, SoA [N * N][n]
  double* g = nullptr;    // weighted gradients, SoA [N][n]
  double* val = nullptr;  // unweighted energies [n]
};

template <int K>
__device__ __forceinline__ void elem_load(const Elems& E, const double* __restrict__ X, int e, double* x) {
#pragma unroll
  for (int i = 0; i < KT<K>::NV; i++) {
    const int64_t v = E.ids[KT<K>::NV * (int64_t)e + i];
    x[3 * i] = X[3 * v];
    x[3 * i + 1] = X[3 * v + 1];
    x[3 * i + 2] = X[3 * v + 2];
  }
}

template <int K>
__device__ __forceinline__ int elem_code(const Elems& E, int e, const double* x) {
  if (K == K_M2S) {
    const D3 y{E.Y[3 * (int64_t)e], E.Y[3 * (int64_t)e + 1], E.Y[3 * (int64_t)e + 2]};
    return pt_feature(y, ld3(x, 0), ld3(x, 1), ld3(x, 2));
  }
  if (K == K_PT) return pt_feature(ld3(x, 0), ld3(x, 1), ld3(x, 2), ld3(x, 3));
  if (K == K_EE) {
    const D3 P[4] = {ld3(x, 0), ld3(x, 1), ld3(x, 2), ld3(x, 3)};
    return ee_feature(P);
  }
  return 0;
}

template <int K, class T>
__device__ __forceinline__ T elem_energy(const Elems& E, int e, const T* z, int code) {
  if constexpr (K == K_M2S) {
    const V3<T> y{cst<T>(E.Y[3 * (int64_t)e]), cst<T>(E.Y[3 * (int64_t)e + 1]), cst<T>(E.Y[3 * (int64_t)e + 2])};
    return pt_d2<T>(code, y, ld3(z, 0), ld3(z, 1), ld3(z, 2));
  } else if constexpr (K == K_EL) {
    return elastic_e<T>(z, E.Binv + 4 * (int64_t)e, E.A0[e]);
  } else if constexpr (K == K_BEND) {
    return bend_e<T>(z, E.th0[e], E.l0[e]);
  } else if constexpr (K == K_PT) {
    return barrier_e<T>(pt_d2<T>(code, ld3(z, 0), ld3(z, 1), ld3(z, 2), ld3(z, 3)), E.dhat);
  } else {
    const V3<T> P[4] = {ld3(z, 0), ld3(z, 1), ld3(z, 2), ld3(z, 3)};
    return barrier_e<T>(ee_d2<T>(code, P), E.dhat);
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_elem_value(Elems E, const double* __restrict__ X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E.n) return;
  double x[KT<K>::N];
  elem_load<K>(E, X, e, x);
  E.val[e] = elem_energy<K, double>(E, e, x, elem_code<K>(E, e, x));
}

// one thread per (element, Hessian entry i <= j), entries outermost so that a
// wave writes one entry of 64 consecutive elements
template <int K>
__global__ __launch_bounds__(256) void k_elem_deriv(Elems E, const double* __restrict__ X) {
  constexpr int N = KT<K>::N;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid >= (int64_t)KT<K>::NP * E.n) return;
  int q = (int)(tid / E.n);
  const int e = (int)(tid - (int64_t)q * E.n);
  int i = 0;
  while (q >= N - i) {
    q -= N - i;
    i++;
  }
  const int j = i + q;
  double x[N];
  elem_load<K>(E, X, e, x);
  const int code = elem_code<K>(E, e, x);
  HD z[N];
#pragma unroll
  for (int k = 0; k < N; k++) z[k] = HD{x[k], k == i ? 1.0 : 0.0, k == j ? 1.0 : 0.0, 0.0};
  const HD r = elem_energy<K, HD>(E, e, z, code);
  const int64_t n = E.n;
  E.H[(int64_t)(i * N + j) * n + e] = E.w * r.ab;
  E.H[(int64_t)(j * N + i) * n + e] = E.w * r.ab;
  if (i == j) E.g[(int64_t)i * n + e] = E.w * r.a;
}

// Cyclic Jacobi on one symmetric N x N matrix in registers (upper triangle
// kept), then the PSD part sum_k max(lambda_k, 0) q_k q_k^T written back.
template <int N>
__device__ __forceinline__ constexpr int ut(int i, int j) {
  return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
}

// Sixteen lanes per matrix: lane r holds row r of the matrix and row r of the
// accumulated rotation Q.  Parallel cyclic Jacobi (round-robin ordering, as
// in Golub and Van Loan, Sec. 8.5.5): a sweep is M - 1 steps (M = N rounded up
// to even), each applying M / 2 rotations on disjoint index pairs at once, so
// one exchange of rows between partner lanes serves them all; columns and Q
// rotate locally.  Step st pairs M - 1 with st and st + k with st - k (mod
// M - 1); an index >= N is a dummy whose pair does not rotate.  The final PSD
// part sum_k max(lambda_k, 0) q_k q_k^T is written row by row.
constexpr int PSD_G = 16;
__host__ __device__ constexpr int rr_a(int M, int st, int k) { return k == 0 ? M - 1 : (st + k) % (M - 1); }
__host__ __device__ constexpr int rr_b(int M, int st, int k) { return k == 0 ? st : (st - k + (M - 1)) % (M - 1); }

template <int N>
__global__ __launch_bounds__(256) void k_elem_psd(double* __restrict__ H, int n) {
  static_assert(N <= PSD_G, "one lane per row");
  constexpr int M = N + (N & 1), R = M - 1;
  const int lane = threadIdx.x & (PSD_G - 1);
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / PSD_G;
  if (grp >= n) return;  // whole groups leave together
  const int64_t e = grp;
  const bool row = lane < N;
  // the lane's row of the accumulated rotations lives in LDS (column k of the
  // block's rows at qs[k][threadIdx.x]: consecutive lanes, consecutive banks);
  // in registers it would hold the kernel to one wave a SIMD
  __shared__ double qs[N][256];
  double* q = &qs[0][threadIdx.x];
  // the lane's row of A J for its partner to read, and the rotation of the
  // lane's pair at its smaller lane, exchanged through LDS (fewer and wider
  // operations than lane shuffles); the 16 lanes of a group are in one wave
  __shared__ double rw[N][256];
  __shared__ double csb[2][256];
  const int gbase = threadIdx.x & ~(PSD_G - 1);
  double a[N];
#pragma unroll
  for (int k = 0; k < N; k++) {
    a[k] = row ? 0.5 * (H[(int64_t)(lane * N + k) * n + e] + H[(int64_t)(k * N + lane) * n + e]) : 0.0;
    q[256 * k] = (row && k == lane) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 30; sweep++) {
    double off = 0.0, all = 0.0;
#pragma unroll
    for (int k = 0; k < N; k++) {
      all += a[k] * a[k];
      if (k != lane) off += a[k] * a[k];
    }
#pragma unroll
    for (int d = PSD_G / 2; d >= 1; d >>= 1) {
      off += __shfl_xor(off, d, PSD_G);
      all += __shfl_xor(all, d, PSD_G);
    }
    if (!(off > 1e-32 * all)) break;
#pragma unroll
    for (int st = 0; st < R; st++) {
      const int partner = lane == M - 1 ? st : (lane == st ? M - 1 : (lane < R ? (2 * st - lane + 2 * R) % R : lane));
      const bool act = row && partner < N && partner != lane;
      const bool isp = lane < partner;
      double mydiag = 0.0, myoff = 0.0;
#pragma unroll
      for (int k = 0; k < N; k++) {
        mydiag = k == lane ? a[k] : mydiag;
        myoff = k == partner ? a[k] : myoff;
      }
      const double pdiag = __shfl(mydiag, partner, PSD_G);
      const double poff = __shfl(myoff, partner, PSD_G);
      // the rotation of this lane's pair: both lanes compute it from the same
      // three values (the off-diagonal entry as the smaller lane p holds it),
      // so they get the same bits without sending the rotation across
      const double app = isp ? mydiag : pdiag, aqq = isp ? pdiag : mydiag, apq = isp ? myoff : poff;
      double c = 1.0, sn = 0.0, t = 0.0;
      if (act && apq != 0.0) {
        const double th = (aqq - app) / (2.0 * apq);
        t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        c = 1.0 / sqrt(t * t + 1.0);
        sn = t * c;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the last step's reads are done
      if (act && isp) {
        csb[0][threadIdx.x] = c;
        csb[1][threadIdx.x] = sn;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // columns of every pair (A J) and rows of Q, with each pair's rotation
#pragma unroll
      for (int k = 0; k < M / 2; k++) {
        const int pa = rr_a(M, st, k), pb = rr_b(M, st, k);
        const int pp = pa < pb ? pa : pb, qq = pa < pb ? pb : pa;
        if (qq >= N) continue;
        const double ck = csb[0][gbase + pp], sk = csb[1][gbase + pp];
        const double arp = a[pp], arq = a[qq];
        a[pp] = ck * arp - sk * arq;
        a[qq] = sk * arp + ck * arq;
        const double qrp = q[256 * pp], qrq = q[256 * qq];
        q[256 * pp] = ck * qrp - sk * qrq;
        q[256 * qq] = sk * qrp + ck * qrq;
      }
      // rows (J^T (A J)) from the partner's row
#pragma unroll
      for (int k = 0; k < N; k++) rw[k][threadIdx.x] = a[k];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      double o[N];
#pragma unroll
      for (int k = 0; k < N; k++) o[k] = rw[k][gbase + partner];
      if (act) {
        if (isp) {
#pragma unroll
          for (int k = 0; k < N; k++)
            a[k] = k == lane ? app - t * apq : (k == partner ? 0.0 : c * a[k] - sn * o[k]);
        } else {
#pragma unroll
          for (int k = 0; k < N; k++)
            a[k] = k == lane ? aqq + t * apq : (k == partner ? 0.0 : sn * o[k] + c * a[k]);
        }
      }
    }
  }
  double lam[N], qr[N];
#pragma unroll
  for (int k = 0; k < N; k++) {
    lam[k] = fmax(__shfl(a[k], k, PSD_G), 0.0);
    qr[k] = q[256 * k];
  }
#pragma unroll
  for (int j = 0; j < N; j++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < N; k++) s += lam[k] * qr[k] * __shfl(qr[k], j, PSD_G);
    if (row) H[(int64_t)(lane * N + j) * n + e] = s;
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_elem_grad(Elems E, double* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E.n) return;
#pragma unroll
  for (int i = 0; i < KT<K>::N; i++) {
    const int64_t v = E.ids[KT<K>::NV * (int64_t)e + i / 3];
    unsafeAtomicAdd(&grad[3 * v + i % 3], E.g[(int64_t)i * E.n + e]);
  }
}

// ------------------------------------------------------------ vertex term and setup
__global__ void k_s2m_value(const double* __restrict__ X, const double* __restrict__ tg, const double* __restrict__ s0,
                            int nv, double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double dx = X[3 * i] - tg[3 * i], dy = X[3 * i + 1] - tg[3 * i + 1], dz = X[3 * i + 2] - tg[3 * i + 2];
  val[i] = s0[i] * (dx * dx + dy * dy + dz * dz);
}

// gradient and diagonal blocks start with the vertex term: 2 k s0 (x - t), 2 k s0 I
__global__ void k_s2m_init(const double* __restrict__ X, const double* __restrict__ tg, const double* __restrict__ s0,
                           int nv, double k, double* __restrict__ grad, double* __restrict__ Dblk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double w = 2.0 * k * s0[i];
  for (int c = 0; c < 3; c++) grad[3 * i + c] = w * (X[3 * i + c] - tg[3 * i + c]);
  for (int c = 0; c < 9; c++) Dblk[9 * i + c] = (c % 4 == 0) ? w : 0.0;
}

// inverse of each 3x3 block (adjugate over determinant)
__global__ void k_block_inv(const double* __restrict__ D, int nv, double* __restrict__ Di) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double* a = D + 9 * (int64_t)i;
  double* o = Di + 9 * (int64_t)i;
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  const double r = 1.0 / det;
  o[0] = c00 * r;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * r;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * r;
  o[3] = c01 * r;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * r;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * r;
  o[6] = c02 * r;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * r;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * r;
}

// mixed Voronoi area of each corner, added into its vertex
__global__ void k_voronoi(const double* __restrict__ X, const int* __restrict__ F, int nf, double* __restrict__ s0) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int id[3];
  D3 P[3];
  for (int c = 0; c < 3; c++) {
    id[c] = F[3 * (int64_t)f + c];
    P[c] = ldX(X, id[c]);
  }
  const D3 n = cross(P[1] - P[0], P[2] - P[0]);
  const double A = 0.5 * sqrt(dot(n, n));
  double dt[3], cot[3];
  for (int c = 0; c < 3; c++) {
    const D3 u = P[(c + 1) % 3] - P[c], w = P[(c + 2) % 3] - P[c];
    const D3 x = cross(u, w);
    dt[c] = dot(u, w);
    cot[c] = dt[c] / sqrt(dot(x, x));
  }
  const bool obtuse = dt[0] < 0.0 || dt[1] < 0.0 || dt[2] < 0.0;
  for (int c = 0; c < 3; c++) {
    double a;
    if (obtuse) {
      a = dt[c] < 0.0 ? A / 2.0 : A / 4.0;
    } else {
      const int q = (c + 1) % 3, r = (c + 2) % 3;
      const D3 pr = P[r] - P[c], pq = P[q] - P[c];
      a = (dot(pr, pr) * cot[q] + dot(pq, pq) * cot[r]) / 8.0;
    }
    unsafeAtomicAdd(&s0[id[c]], a);
  }
}

// per face: area and the inverse of its rest edge matrix in a frame of its plane
__global__ void k_rest_faces(const double* __restrict__ X, const int* __restrict__ F, int nf, double* __restrict__ Binv,
                             double* __restrict__ A0) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const D3 p0 = ldX(X, F[3 * f]), p1 = ldX(X, F[3 * f + 1]), p2 = ldX(X, F[3 * f + 2]);
  const D3 e1 = p1 - p0, e2 = p2 - p0;
  const double l1 = sqrt(dot(e1, e1));
  const D3 u{e1.x / l1, e1.y / l1, e1.z / l1};
  const D3 n = cross(e1, e2);
  const double nl = sqrt(dot(n, n));
  const D3 w = cross(D3{n.x / nl, n.y / nl, n.z / nl}, u);
  const double m01 = dot(u, e2), m11 = dot(w, e2);
  // inverse of [[l1, m01], [0, m11]]
  Binv[4 * f] = 1.0 / l1;
  Binv[4 * f + 1] = -m01 / (l1 * m11);
  Binv[4 * f + 2] = 0.0;
  Binv[4 * f + 3] = 1.0 / m11;
  A0[f] = 0.5 * nl;
}

__global__ void k_edge_flags(const int* __restrict__ twin, int nh, uint8_t* __restrict__ fl,
                             uint8_t* __restrict__ hown) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  const int t = twin[h];
  fl[h] = h < t;
  hown[h] = (h / 3) < (t / 3);
}

// each edge once: stencil (i, j, k, l), rest angle and rest length
__global__ void k_stencils(const int* __restrict__ list, int ne, const int* __restrict__ F, const int* __restrict__ twin,
                           const double* __restrict__ X, int* __restrict__ st, double* __restrict__ th0,
                           double* __restrict__ l0) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int h = list[e], t = twin[h];
  const int f = h / 3, c = h % 3, g = t / 3, d = t % 3;
  const int i = F[3 * f + c], j = F[3 * f + (c + 1) % 3], k = F[3 * f + (c + 2) % 3], l = F[3 * g + (d + 2) % 3];
  st[4 * e] = i;
  st[4 * e + 1] = j;
  st[4 * e + 2] = k;
  st[4 * e + 3] = l;
  const D3 xi = ldX(X, i), xj = ldX(X, j);
  th0[e] = dihedral<double>(xi, xj, ldX(X, k), ldX(X, l));
  const D3 d3 = xj - xi;
  l0[e] = sqrt(dot(d3, d3));
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_vown(const int* __restrict__ F, int nf, int* __restrict__ vown) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  for (int c = 0; c < 3; c++) atomicMin(&vown[F[3 * f + c]], f);
}

__global__ void k_gather_tri(const int* __restrict__ F, const int* __restrict__ tri, int m, int* __restrict__ ids) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int f = tri[s];
  for (int c = 0; c < 3; c++) ids[3 * s + c] = F[3 * f + c];
}

// ------------------------------------------------------------ sums
constexpr int SUM_T = 256, SUM_ITEMS = 8;
__device__ double block_sum(double x) {
  __shared__ double sh[SUM_T];
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int d = SUM_T / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
// partial[b] = sum of a[i] (times b[i] when given) over block b's items
__global__ __launch_bounds__(SUM_T) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                       int64_t n, double* __restrict__ part,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  const int64_t base = (int64_t)blockIdx.x * SUM_T * SUM_ITEMS;
  double s = 0.0;
  for (int k = 0; k < SUM_ITEMS; k++) {
    const int64_t i = base + (int64_t)k * SUM_T + threadIdx.x;
    if (i < n) s += b ? a[i] * b[i] : a[i];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
inline unsigned sum_blocks(int64_t n) { return nblk(n, SUM_T * SUM_ITEMS); }
__device__ double sum_parts(const double* __restrict__ part, int nb) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += SUM_T) s += part[i];
  return block_sum(s);
}
__global__ __launch_bounds__(SUM_T) void k_sum_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  const double s = sum_parts(part, nb);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------ fused launches
// The element kinds of one evaluation in one launch: blocks [blk[k],
// blk[k+1]) serve kind k (0 the vertex term, then K_M2S .. K_EE + 1).
constexpr int NSEG = K_KINDS + 1;
struct KindRanges {
  Elems E[K_KINDS];
  const double* s0;
  const double* tg;
  double* sval;  // vertex term values
  int nv;
  const int* cnt;  // device contact counts (point-face, edge-edge)
  int blk[NSEG + 1];
};
__device__ __forceinline__ int kind_of_block(const KindRanges& a, int b, int* local) {
  int k = 0;
  while (k < NSEG - 1 && b >= a.blk[k + 1]) k++;
  *local = (b - a.blk[k]) * 256 + (int)threadIdx.x;
  return k;
}
template <int K>
__device__ __forceinline__ void value_one(const Elems& E, int e, const double* __restrict__ X) {
  double x[KT<K>::N];
  elem_load<K>(E, X, e, x);
  E.val[e] = elem_energy<K, double>(E, e, x, elem_code<K>(E, e, x));
}
// every element's unweighted energy; contacts up to their device counts
__global__ __launch_bounds__(256) void k_values_all(KindRanges a, const double* __restrict__ X) {
  int i;
  const int k = kind_of_block(a, blockIdx.x, &i);
  switch (k) {
    case 0:
      if (i < a.nv) {
        const double dx = X[3 * i] - a.tg[3 * i], dy = X[3 * i + 1] - a.tg[3 * i + 1], dz = X[3 * i + 2] - a.tg[3 * i + 2];
        a.sval[i] = a.s0[i] * (dx * dx + dy * dy + dz * dz);
      }
      break;
    case 1 + K_M2S:
      if (i < a.E[K_M2S].n) value_one<K_M2S>(a.E[K_M2S], i, X);
      break;
    case 1 + K_EL:
      if (i < a.E[K_EL].n) value_one<K_EL>(a.E[K_EL], i, X);
      break;
    case 1 + K_BEND:
      if (i < a.E[K_BEND].n) value_one<K_BEND>(a.E[K_BEND], i, X);
      break;
    case 1 + K_PT:
      if (i < min(a.cnt[0], a.E[K_PT].n)) value_one<K_PT>(a.E[K_PT], i, X);
      break;
    default:
      if (i < min(a.cnt[1], a.E[K_EE].n)) value_one<K_EE>(a.E[K_EE], i, X);
      break;
  }
}
// partial sums of NSEG value arrays (blockIdx.y the segment; counts from the
// host, or for the contact segments from the device); every block writes
// its partial, zero past the segment's end
struct SegSums {
  const double* v[NSEG];
  int n[NSEG];
  const int* cnt;
  double* part;
  int stride;
};
__global__ __launch_bounds__(SUM_T) void k_sum_seg(SegSums a) {
  const int k = blockIdx.y;
  int n = a.n[k];
  if (k >= 1 + K_PT) n = min(n, a.cnt[k - 1 - K_PT]);
  const int64_t base = (int64_t)blockIdx.x * SUM_T * SUM_ITEMS;
  double s = 0.0;
  if (base < n)
    for (int j = 0; j < SUM_ITEMS; j++) {
      const int64_t i = base + (int64_t)j * SUM_T + threadIdx.x;
      if (i < n) s += a.v[k][i];
    }
  s = block_sum(s);
  if (threadIdx.x == 0) a.part[(int64_t)k * a.stride + blockIdx.x] = s;
}
__global__ __launch_bounds__(SUM_T) void k_sum_seg_final(const double* __restrict__ part, int nb, int stride,
                                                         double* __restrict__ sums) {
  const double s = sum_parts(part + (int64_t)blockIdx.x * stride, nb);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// ------------------------------------------------------------ block-sparse Hessian
// After the element Hessians are projected, their 3x3 vertex blocks are
// summed into one block-sparse matrix (rows by vertex, a 3x3 block per vertex
// pair that shares an element): the products of the CG loop then read each
// block once and need no atomics.  Entries: [0, nv) the vertex term's
// diagonal blocks, then NV^2 blocks per element of each kind.
struct EntryRanges {
  Elems E[K_KINDS];
  int64_t off[NSEG + 1];
  const double* s0;
  double k2;  // 2 k_dis
  int nv;
};
__device__ __forceinline__ int entry_decode(const EntryRanges& r, int64_t id, int* e, int* a, int* b) {
  if (id < r.off[1]) {
    *e = (int)id;
    *a = *b = 0;
    return 0;
  }
  int k = 1;
  while (k < NSEG && id >= r.off[k + 1]) k++;
  const int nv = k == 1 + K_M2S || k == 1 + K_EL ? 3 : 4;
  const int64_t loc = id - r.off[k];
  *e = (int)(loc / (nv * nv));
  const int ab = (int)(loc - (int64_t)*e * nv * nv);
  *a = ab / nv;
  *b = ab % nv;
  return k;
}
__device__ __forceinline__ const Elems& kind_elems(const EntryRanges& r, int k) { return r.E[k - 1]; }

__global__ void k_bsr_keys(EntryRanges r, int bits, uint64_t* __restrict__ keys, int* __restrict__ vals) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (id >= r.off[NSEG]) return;
  int e, a, b;
  const int k = entry_decode(r, id, &e, &a, &b);
  int64_t i, j;
  if (k == 0) {
    i = j = e;
  } else {
    const Elems& E = kind_elems(r, k);
    const int nv = k == 1 + K_M2S || k == 1 + K_EL ? 3 : 4;
    i = E.ids[nv * (int64_t)e + a];
    j = E.ids[nv * (int64_t)e + b];
  }
  keys[id] = ((uint64_t)i << bits) | (uint64_t)j;
  vals[id] = (int)id;
}
__global__ void k_bsr_flags(const uint64_t* __restrict__ keys, int64_t n, uint8_t* __restrict__ fl) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) fl[k] = k == 0 || keys[k] != keys[k - 1];
}
__global__ void k_bsr_starts(const uint8_t* __restrict__ fl, const int* __restrict__ excl, int64_t n,
                             int* __restrict__ ustart) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n && fl[k]) ustart[excl[k]] = (int)k;
}
// one thread per block: its column, its row's start, and the sum of its
// entries' 3x3 blocks in sorted (key, entry) order
__global__ void k_bsr_fill(EntryRanges r, const uint64_t* __restrict__ keys, const int* __restrict__ vals,
                           const int* __restrict__ ustart, const int* __restrict__ nslot, int64_t n, int bits,
                           int* __restrict__ rowptr, int* __restrict__ col, double* __restrict__ B) {
  const int ns = *nslot;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int64_t beg = ustart[k], end = k + 1 < ns ? ustart[k + 1] : n;
  const uint64_t key = keys[beg];
  const int i = (int)(key >> bits);
  col[k] = (int)(key & ((1ull << bits) - 1));
  if (k == 0 || (int)(keys[ustart[k - 1]] >> bits) != i) rowptr[i] = k;
  if (k == ns - 1) rowptr[r.nv] = ns;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t p = beg; p < end; p++) {
    int e, a, b;
    const int kind = entry_decode(r, vals[p], &e, &a, &b);
    if (kind == 0) {
      const double w = r.k2 * r.s0[e];
      acc[0] += w;
      acc[4] += w;
      acc[8] += w;
      continue;
    }
    const Elems& E = kind_elems(r, kind);
    const int N = kind == 1 + K_M2S || kind == 1 + K_EL ? 9 : 12;
    for (int rr = 0; rr < 3; rr++)
      for (int c = 0; c < 3; c++) acc[3 * rr + c] += E.H[(int64_t)((3 * a + rr) * N + 3 * b + c) * E.n + e];
  }
  for (int q = 0; q < 9; q++) B[9 * (int64_t)k + q] = acc[q];
}
// the diagonal block of each row into Dblk
__global__ void k_bsr_diag(const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ B,
                           int nv, double* __restrict__ Dblk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  for (int k = rowptr[i]; k < rowptr[i + 1]; k++)
    if (col[k] == i)
      for (int q = 0; q < 9; q++) Dblk[9 * (int64_t)i + q] = B[9 * (int64_t)k + q];
}
// out = H v, one thread per output component
__global__ __launch_bounds__(256) void k_bsr_spmv(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                  const double* __restrict__ B, int nv, const double* __restrict__ v,
                                                  double* __restrict__ out, const int* __restrict__ done) {
  if (done && *done) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * nv) return;
  const int i = t / 3, r = t - 3 * i;
  double s = 0.0;
  for (int k = rowptr[i]; k < rowptr[i + 1]; k++) {
    const int64_t j = col[k];
    const double* b = B + 9 * (int64_t)k + 3 * r;
    s += b[0] * v[3 * j] + b[1] * v[3 * j + 1] + b[2] * v[3 * j + 2];
  }
  out[t] = s;
}

// ------------------------------------------------------------ conjugate gradients
// rzs[i & 1]: r.z after i iterations (the two latest, so that a kernel can
// write the new one while its other blocks still read the one before)
struct CgState {
  double rzs[2], rr, bb, tol;
  int it, max_it, done, pad;
};
__global__ void k_cg_start(const double* __restrict__ pr, const double* __restrict__ pz, int nb, CgState* st) {
  // partial sums of r.r (= b.b) in pr, of r.z in pz
  const double rr = sum_parts(pr, nb);
  const double rz = sum_parts(pz, nb);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->bb = rr;
    st->rzs[0] = rz;
    st->it = 0;
    st->done = !(sqrt(rr) > st->tol * sqrt(rr)) || st->max_it <= 0;
  }
}
// x = 0, r = -g, z = D^-1 r, p = z
__global__ void k_cg_init(const double* __restrict__ g, const double* __restrict__ Di, int nv, double* __restrict__ x,
                          double* __restrict__ r, double* __restrict__ z, double* __restrict__ p,
                          double* __restrict__ Ap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double rv[3];
  for (int c = 0; c < 3; c++) {
    x[3 * i + c] = 0.0;
    Ap[3 * i + c] = 0.0;
    rv[c] = -g[3 * i + c];
    r[3 * i + c] = rv[c];
  }
  const double* d = Di + 9 * (int64_t)i;
  for (int c = 0; c < 3; c++) {
    const double zc = d[3 * c] * rv[0] + d[3 * c + 1] * rv[1] + d[3 * c + 2] * rv[2];
    z[3 * i + c] = zc;
    p[3 * i + c] = zc;
  }
}

// Sums for the CG kernels, whose blocks are single waves (CG_T = 64): a small
// system's few thousand rows then spread over many CUs, and a block's sum
// needs no barrier.  The kernels of an iteration pass their dot products on as
// per-block partial sums, and every block of the next kernel adds them up
// itself, in the same order (so all get the same value): no block waits for
// the others, and no device-scope fence is needed inside a kernel (on this
// chip such a fence writes back and invalidates the L2).
constexpr int CG_T = 64;
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}
constexpr int CG_PRE = 8;  // blocks of a Hessian row loaded ahead in k_cg_dir

__device__ double sum_parts_wave(const double* __restrict__ part, int nb) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += CG_T) s += part[i];
  return wave_sum(s);
}

// Iteration i, first half: the stopping test on r after i iterations (i > 0:
// its r.r and r.z from the step's partials), then the new direction pn = z +
// beta p (beta = 0 at i = 0, so pn = z), Apn = H pn (one thread per output
// component, reading pn at the block's columns as z + beta p) and the partial
// sums of pn.Apn.  pn is a separate array from p, since other blocks still
// read p while this one writes pn.
__global__ __launch_bounds__(CG_T) void k_cg_dir(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                 const double* __restrict__ B, int nv, const double* __restrict__ z,
                                                 const double* __restrict__ p, double* __restrict__ pn,
                                                 double* __restrict__ Ap, double* __restrict__ part,
                                                 const double* __restrict__ pz, const double* __restrict__ pr,
                                                 int nbv, int i, CgState* st) {
  // the row's first CG_PRE blocks and their columns of z and p do not depend
  // on beta: their loads go out together with those of the scalars
  const int t = blockIdx.x * CG_T + threadIdx.x;
  const bool live = t < 3 * nv;
  const int v = t / 3, r = t - 3 * v;
  int k0 = 0, k1 = 0;
  if (live) {
    k0 = rowptr[v];
    k1 = rowptr[v + 1];
  }
  double bq[CG_PRE][3], zq[CG_PRE][3], pq[CG_PRE][3];
#pragma unroll
  for (int q = 0; q < CG_PRE; q++) {
    const int k = k0 + q < k1 ? k0 + q : k0;  // a valid slot when the row has one
    const int64_t j = live && k0 < k1 ? col[k] : 0;
    const double* b = B + 9 * (int64_t)(live && k0 < k1 ? k : 0) + 3 * r;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      bq[q][c] = live && k0 < k1 ? b[c] : 0.0;
      zq[q][c] = z[3 * j + c];
      pq[q][c] = p[3 * j + c];
    }
  }
  if (st->done) return;
  double beta = 0.0;
  if (i > 0) {
    const double rz = sum_parts_wave(pz, nbv);
    const double rr = sum_parts_wave(pr, nbv);
    const bool fin = !(sqrt(rr) > st->tol * sqrt(st->bb)) || i >= st->max_it;
    if (fin) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr = rr;
        st->it = i;
        st->done = 1;
      }
      return;
    }
    beta = rz / st->rzs[(i - 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->rzs[i & 1] = rz;
      st->rr = rr;
    }
  }
  double dot = 0.0;
  if (live) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < CG_PRE; q++) {
      if (k0 + q < k1) {
        const double v0 = zq[q][0] + beta * pq[q][0];
        const double v1 = zq[q][1] + beta * pq[q][1];
        const double v2 = zq[q][2] + beta * pq[q][2];
        s += bq[q][0] * v0 + bq[q][1] * v1 + bq[q][2] * v2;
      }
    }
    for (int k = k0 + CG_PRE; k < k1; k++) {
      const int64_t j = col[k];
      const double* b = B + 9 * (int64_t)k + 3 * r;
      const double v0 = z[3 * j] + beta * p[3 * j];
      const double v1 = z[3 * j + 1] + beta * p[3 * j + 1];
      const double v2 = z[3 * j + 2] + beta * p[3 * j + 2];
      s += b[0] * v0 + b[1] * v1 + b[2] * v2;
    }
    Ap[t] = s;
    const double pt = z[t] + beta * p[t];
    pn[t] = pt;
    dot = pt * s;
  }
  dot = wave_sum(dot);
  if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// Iteration i, second half: alpha = (r.z) / (p.Ap) from the first half's
// partials, x += alpha p, r -= alpha Ap, z = D^-1 r, and the partial sums of
// r.z and r.r for the next iteration's first half.
__global__ __launch_bounds__(CG_T) void k_cg_step(double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ z, const double* __restrict__ p,
                                                  const double* __restrict__ Ap, const double* __restrict__ Di,
                                                  int nv, const double* __restrict__ part, int nbd,
                                                  double* __restrict__ pz, double* __restrict__ pr, int i,
                                                  const CgState* st) {
  // the vertex's own entries do not depend on alpha: loaded with the scalars
  const int v = blockIdx.x * CG_T + threadIdx.x;
  const bool live = v < nv;
  double xv[3], rv[3], pv[3], av[3], d[9];
  const int w = live ? v : 0;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    xv[c] = x[3 * w + c];
    rv[c] = r[3 * w + c];
    pv[c] = p[3 * w + c];
    av[c] = Ap[3 * w + c];
  }
#pragma unroll
  for (int c = 0; c < 9; c++) d[c] = Di[9 * (int64_t)w + c];
  if (st->done) return;
  const double a = st->rzs[i & 1] / sum_parts_wave(part, nbd);
  double srz = 0.0, srr = 0.0;
  if (live) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      x[3 * v + c] = xv[c] + a * pv[c];
      rv[c] = rv[c] - a * av[c];
      r[3 * v + c] = rv[c];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const double zc = d[3 * c] * rv[0] + d[3 * c + 1] * rv[1] + d[3 * c + 2] * rv[2];
      z[3 * v + c] = zc;
      srz += rv[c] * zc;
      srr += rv[c] * rv[c];
    }
  }
  srz = wave_sum(srz);
  srr = wave_sum(srr);
  if (threadIdx.x == 0) {
    pz[blockIdx.x] = srz;
    pr[blockIdx.x] = srr;
  }
}

__global__ void k_axpy_pos(const double* __restrict__ X, const double* __restrict__ P, double a, int64_t n,
                           double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[i] + a * P[i];
}

// ------------------------------------------------------------ surface samples
__global__ void k_face_area(const double* __restrict__ V, const int* __restrict__ F, int nf, double* __restrict__ a) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const D3 p0 = ldX(V, F[3 * f]), p1 = ldX(V, F[3 * f + 1]), p2 = ldX(V, F[3 * f + 2]);
  const D3 n = cross(p1 - p0, p2 - p0);
  a[f] = 0.5 * sqrt(dot(n, n));
}
constexpr int SCAN_T = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_T * SCAN_ITEMS;
// inclusive scan inside tiles of SCAN_TILE; tile totals to tsum
__global__ __launch_bounds__(SCAN_T) void k_scan_tile(double* __restrict__ a, int n, double* __restrict__ tsum) {
  __shared__ double sh[SCAN_T];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  double v[SCAN_ITEMS];
  double run = 0.0;
  for (int k = 0; k < SCAN_ITEMS; k++) {
    run += (base + k < n) ? a[base + k] : 0.0;
    v[k] = run;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int d = 1; d < SCAN_T; d <<= 1) {  // inclusive scan of the thread totals
    const double o = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += o;
    __syncthreads();
  }
  const double off = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
  for (int k = 0; k < SCAN_ITEMS; k++)
    if (base + k < n) a[base + k] = v[k] + off;
  if (threadIdx.x == SCAN_T - 1) tsum[blockIdx.x] = sh[SCAN_T - 1];
}
__global__ void k_scan_top(double* __restrict__ tsum, int nt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double run = 0.0;
  for (int i = 0; i < nt; i++) {
    const double t = tsum[i];
    tsum[i] = run;
    run += t;
  }
}
__global__ void k_scan_add(double* __restrict__ a, int n, const double* __restrict__ tsum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += tsum[i / SCAN_TILE];
}
__global__ void k_sample(const double* __restrict__ V, const int* __restrict__ F, int nf, const double* __restrict__ cum,
                         const double* __restrict__ U, int64_t m, double* __restrict__ Y) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= m) return;
  const double u0 = U[3 * s], u1 = U[3 * s + 1], u2 = U[3 * s + 2];
  const double key = u0 * cum[nf - 1];
  int lo = 0, hi = nf;  // first index with cum > key
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cum[mid] > key) hi = mid;
    else lo = mid + 1;
  }
  const int f = lo < nf ? lo : nf - 1;
  const double r = sqrt(u1);
  const double w0 = 1.0 - r, w1 = r * (1.0 - u2), w2 = r * u2;
  const D3 a = ldX(V, F[3 * f]), b = ldX(V, F[3 * f + 1]), c = ldX(V, F[3 * f + 2]);
  Y[3 * s] = w0 * a.x + w1 * b.x + w2 * c.x;
  Y[3 * s + 1] = w0 * a.y + w1 * b.y + w2 * c.y;
  Y[3 * s + 2] = w0 * a.z + w1 * b.z + w2 * c.z;
}

// ------------------------------------------------------------ boxes and tree walks
__device__ __forceinline__ void round_out(double lo, double hi, float* b, int k) {
  float fl = (float)lo, fh = (float)hi;
  if ((double)fl > lo) fl = nextafterf(fl, -INFINITY);
  if ((double)fh < hi) fh = nextafterf(fh, INFINITY);
  b[k] = fl;
  b[k + 3] = fh;
}
// face boxes grown by pad, or swept over the step P (pad 0), rounded outward
__global__ void k_boxes(const double* __restrict__ X, const double* __restrict__ P, const int* __restrict__ F, int nf,
                        double pad, float* __restrict__ box) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int c = 0; c < 3; c++) {
    const int64_t v = F[3 * f + c];
    for (int k = 0; k < 3; k++) {
      const double x = X[3 * v + k];
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
      if (P) {
        const double y = x + P[3 * v + k];
        lo[k] = fmin(lo[k], y);
        hi[k] = fmax(hi[k], y);
      }
    }
  }
  float b[6];
  for (int k = 0; k < 3; k++) round_out(lo[k] - pad, hi[k] + pad, b, k);
  for (int k = 0; k < 6; k++) box[6 * (int64_t)f + k] = b[k];
}

__device__ __forceinline__ int child_hits(const BvhNode& nd, const float* b) {
  const float lx[4] = {nd.lx.x, nd.lx.y, nd.lx.z, nd.lx.w}, ly[4] = {nd.ly.x, nd.ly.y, nd.ly.z, nd.ly.w};
  const float lz[4] = {nd.lz.x, nd.lz.y, nd.lz.z, nd.lz.w}, hx[4] = {nd.hx.x, nd.hx.y, nd.hx.z, nd.hx.w};
  const float hy[4] = {nd.hy.x, nd.hy.y, nd.hy.z, nd.hy.w}, hz[4] = {nd.hz.x, nd.hz.y, nd.hz.z, nd.hz.w};
  int m = 0;
  for (int c = 0; c < 4; c++)
    m |= (lx[c] <= b[3] && b[0] <= hx[c] && ly[c] <= b[4] && b[1] <= hy[c] && lz[c] <= b[5] && b[2] <= hz[c]) << c;
  return m;
}

struct WalkArgs {
  const BvhNode* nodes;
  int D, nf;
  const float* box;
  const double* X;
  const double* P;  // null: contact detection; else the step (CCD)
  const int* F;
  const int* vown;
  const uint8_t* hown;
  double pad, dhat2, s;
  int4* pt;
  int4* ee;
  int* cnt;  // [0] point-face contacts, [1] edge-edge contacts, [2] stack overflow, [3] face pairs
  int cap;
  int2* fpair;  // face pairs whose boxes meet
  int fcap;
  unsigned long long* step;  // bits of the smallest CCD step (non-negative doubles order like their bits)
};

// exact primitive box test: boxes of the start positions grown by pad, or of
// the start and end positions (the same double arithmetic as the oracle's)
__device__ __forceinline__ bool prim_boxes_meet(const WalkArgs& a, const int* p, int np, const int* q, int nq) {
  for (int k = 0; k < 3; k++) {
    double lo1 = INFINITY, hi1 = -INFINITY, lo2 = INFINITY, hi2 = -INFINITY;
    for (int i = 0; i < np; i++) {
      const double x = a.X[3 * (int64_t)p[i] + k];
      lo1 = fmin(lo1, x);
      hi1 = fmax(hi1, x);
      if (a.P) {
        const double y = x + a.P[3 * (int64_t)p[i] + k];
        lo1 = fmin(lo1, y);
        hi1 = fmax(hi1, y);
      }
    }
    for (int i = 0; i < nq; i++) {
      const double x = a.X[3 * (int64_t)q[i] + k];
      lo2 = fmin(lo2, x);
      hi2 = fmax(hi2, x);
      if (a.P) {
        const double y = x + a.P[3 * (int64_t)q[i] + k];
        lo2 = fmin(lo2, y);
        hi2 = fmax(hi2, y);
      }
    }
    if (!(lo1 - a.pad <= hi2 + a.pad && lo2 - a.pad <= hi1 + a.pad)) return false;
  }
  return true;
}

// Additive CCD of one pair (ids[0..3]: point and triangle, or two edges):
// the step in [0, 1] up to which the pair keeps at least the fraction s of its
// starting distance.
template <bool PT>
__device__ double accd_pair(const WalkArgs& a, const int* ids) {
  D3 x[4], p[4];
  for (int i = 0; i < 4; i++) {
    x[i] = ldX(a.X, ids[i]);
    p[i] = ldX(a.P, ids[i]);
  }
  D3 mean{((p[0].x + p[1].x) + p[2].x) + p[3].x, ((p[0].y + p[1].y) + p[2].y) + p[3].y,
          ((p[0].z + p[1].z) + p[2].z) + p[3].z};
  mean = D3{mean.x / 4.0, mean.y / 4.0, mean.z / 4.0};
  double nrm[4];
  for (int i = 0; i < 4; i++) {
    p[i] = p[i] - mean;
    nrm[i] = sqrt(p[i].x * p[i].x + p[i].y * p[i].y + p[i].z * p[i].z);
  }
  const double lp = PT ? nrm[0] + fmax(fmax(nrm[1], nrm[2]), nrm[3]) : fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]);
  if (lp == 0.0) return 1.0;
  auto dist = [&]() { return sqrt(PT ? pt_dist2(x[0], x[1], x[2], x[3]) : ee_dist2(x)); };
  double d = dist();
  if (d == 0.0) return 0.0;
  const double g = a.s * d;
  double t = 0.0, tl = (1.0 - a.s) * d / lp;
  for (int it = 0; it < ACCD_MAX_STEPS; it++) {
    for (int i = 0; i < 4; i++) x[i] = D3{x[i].x + tl * p[i].x, x[i].y + tl * p[i].y, x[i].z + tl * p[i].z};
    d = dist();
    if (t > 0.0 && d < g) return t;
    t += tl;
    if (t > 1.0) return 1.0;
    tl = 0.9 * d / lp;
  }
  return t;
}

__device__ void on_pt(const WalkArgs& a, int v, const int* f) {
  if (v == f[0] || v == f[1] || v == f[2]) return;
  if (!prim_boxes_meet(a, &v, 1, f, 3)) return;
  const int ids[4] = {v, f[0], f[1], f[2]};
  if (a.P) {
    const double t = accd_pair<true>(a, ids);
    if (t < 1.0) atomicMin(a.step, (unsigned long long)__double_as_longlong(t));
    return;
  }
  if (pt_dist2(ldX(a.X, v), ldX(a.X, f[0]), ldX(a.X, f[1]), ldX(a.X, f[2])) < a.dhat2) {
    const int k = atomicAdd(&a.cnt[0], 1);
    if (k < a.cap) a.pt[k] = make_int4(v, f[0], f[1], f[2]);
  }
}

__device__ void on_ee(const WalkArgs& a, const int* e1, const int* e2) {
  if (e1[0] == e2[0] || e1[0] == e2[1] || e1[1] == e2[0] || e1[1] == e2[1]) return;
  if (!prim_boxes_meet(a, e1, 2, e2, 2)) return;
  const int ids[4] = {e1[0], e1[1], e2[0], e2[1]};
  if (a.P) {
    const double t = accd_pair<false>(a, ids);
    if (t < 1.0) atomicMin(a.step, (unsigned long long)__double_as_longlong(t));
    return;
  }
  const D3 P[4] = {ldX(a.X, ids[0]), ldX(a.X, ids[1]), ldX(a.X, ids[2]), ldX(a.X, ids[3])};
  if (ee_dist2(P) < a.dhat2) {
    const int k = atomicAdd(&a.cnt[1], 1);
    if (k < a.cap) a.ee[k] = make_int4(ids[0], ids[1], ids[2], ids[3]);
  }
}

// Slot s of face pair (t, u): 0-2 the vertex of corner s of t against face u,
// 3-5 the vertex of corner s - 3 of u against face t, 6-14 edge (s - 6) / 3
// of t against edge (s - 6) % 3 of u; a slot counts only when the faces own
// its primitives, so every primitive pair is tested once.
constexpr int PAIR_SLOTS = 15;
__device__ void pair_slot(const WalkArgs& a, int t, int u, int slot) {
  if (slot < 6) {
    const int f = slot < 3 ? t : u, g = slot < 3 ? u : t;
    const int v = a.F[3 * f + slot % 3];
    if (a.vown[v] != f) return;
    const int fg[3] = {a.F[3 * g], a.F[3 * g + 1], a.F[3 * g + 2]};
    on_pt(a, v, fg);
    return;
  }
  const int c = (slot - 6) / 3, d = (slot - 6) % 3;
  if (!a.hown[3 * t + c] || !a.hown[3 * u + d]) return;
  const int e1[2] = {a.F[3 * t + c], a.F[3 * t + (c + 1) % 3]};
  const int e2[2] = {a.F[3 * u + d], a.F[3 * u + (d + 1) % 3]};
  on_ee(a, e1, e2);
}

// every (face pair, slot) of the collected pairs, over a grid of any size
__global__ __launch_bounds__(256) void k_pair_slots(WalkArgs a) {
  const int64_t n = (int64_t)min(a.cnt[3], a.fcap) * PAIR_SLOTS;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(i / PAIR_SLOTS), slot = (int)(i - (int64_t)f * PAIR_SLOTS);
    const int2 pr = a.fpair[f];
    pair_slot(a, pr.x, pr.y, slot);
  }
}

__device__ __forceinline__ void emit_pair(const WalkArgs& a, int t, int u) {
  const int k = atomicAdd(&a.cnt[3], 1);
  if (k < a.fcap) a.fpair[k] = make_int2(t, u);
}

// One thread per leaf slot i (faces in Hilbert order, so a wave walks nearby
// parts of the tree): every face in a later slot whose box meets this face's
// box, each face pair once.  The walk keeps no stack in memory: per level, the
// children still to visit are four bits of one 64-bit mask (levels below 14),
// and backtracking goes to the deepest level with a bit left, whose node is
// an ancestor of the current one (parent of node k is (k - 1) / 4).  Children
// whose leaves all come at or before slot i are skipped: child c of node k at
// level L holds slots [(4 k' + c) 4^(D-L-1), (4 k' + c + 1) 4^(D-L-1)), k' its
// index within the level.
__device__ __forceinline__ int later_mask(int node, int L, int D, int i) {
  const int64_t k = node - ((((int64_t)1) << (2 * L)) - 1) / 3;
  const int sh = 2 * (D - L - 1);
  int m = 0;
  for (int c = 0; c < 4; c++) m |= (((4 * k + c + 1) << sh) > (int64_t)i + 1) << c;
  return m;
}

__global__ __launch_bounds__(256) void k_walk(WalkArgs a, const int* __restrict__ sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nf) return;
  const int t = sorted[i];
  float b[6];
  for (int k = 0; k < 6; k++) b[k] = a.box[6 * (int64_t)t + k];
  int node = 0, L = 0;
  uint64_t pend = 0;
  for (;;) {
    const BvhNode nd = a.nodes[node];
    const int m = child_hits(nd, b) & later_mask(node, L, a.D, i);
    if (L == a.D - 1) {
      // the leaf hits of every lane at this step go out with one atomic for
      // the wave (a lane's count, at most 4, is summed over the lanes below it
      // bit by bit from three ballots)
      const int lf[4] = {nd.leaf.x, nd.leaf.y, nd.leaf.z, nd.leaf.w};
      const int mine = __popc(m);
      const uint64_t below = (1ull << (threadIdx.x & 63)) - 1;
      int pre = 0, tot = 0;
#pragma unroll
      for (int bit = 0; bit < 3; bit++) {
        const uint64_t bb = __ballot((mine >> bit) & 1);
        pre += __popcll(bb & below) << bit;
        tot += __popcll(bb) << bit;
      }
      const uint64_t act = __ballot(1);
      const int leader = __ffsll((long long)act) - 1;
      int base = 0;
      if ((threadIdx.x & 63) == leader && tot) base = atomicAdd(&a.cnt[3], tot);
      base = __shfl(base, leader, 64);
      int k = base + pre;
      for (int c = 0; c < 4; c++)
        if ((m >> c) & 1) {
          if (k < a.fcap) a.fpair[k] = make_int2(t, lf[c]);
          k++;
        }
    } else {
      pend |= (uint64_t)m << (4 * L);
    }
    if (!pend) break;
    const int Lp = (63 - __clzll((long long)pend)) >> 2;
    const int c = __ffs((int)((pend >> (4 * Lp)) & 15)) - 1;
    pend &= ~(1ull << (4 * Lp + c));
    int anc = node;
    for (int l = L; l > Lp; l--) anc = (anc - 1) >> 2;
    node = 4 * anc + 1 + c;
    L = Lp + 1;
  }
}

// brute force when the tree has fewer than two faces
__global__ void k_walk_small(WalkArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int t = 0; t < a.nf; t++)
      for (int u = t + 1; u < a.nf; u++) emit_pair(a, t, u);
}

// squared distance from q to a float box (a lower bound for its triangles)
__device__ __forceinline__ double box_d2(const BvhNode& nd, int c, D3 q) {
  const float lo[3] = {c == 0 ? nd.lx.x : c == 1 ? nd.lx.y : c == 2 ? nd.lx.z : nd.lx.w,
                       c == 0 ? nd.ly.x : c == 1 ? nd.ly.y : c == 2 ? nd.ly.z : nd.ly.w,
                       c == 0 ? nd.lz.x : c == 1 ? nd.lz.y : c == 2 ? nd.lz.z : nd.lz.w};
  const float hi[3] = {c == 0 ? nd.hx.x : c == 1 ? nd.hx.y : c == 2 ? nd.hx.z : nd.hx.w,
                       c == 0 ? nd.hy.x : c == 1 ? nd.hy.y : c == 2 ? nd.hy.z : nd.hy.w,
                       c == 0 ? nd.hz.x : c == 1 ? nd.hz.y : c == 2 ? nd.hz.z : nd.hz.w};
  if (!(lo[0] <= hi[0])) return INFINITY;  // absent child
  const double qq[3] = {q.x, q.y, q.z};
  double s = 0.0;
  for (int k = 0; k < 3; k++) {
    const double d = fmax(fmax((double)lo[k] - qq[k], qq[k] - (double)hi[k]), 0.0);
    s += d * d;
  }
  return s;
}

__device__ __forceinline__ double face_d2(const double* V, const int* F, int f, D3 q) {
  return pt_dist2(q, ldX(V, F[3 * f]), ldX(V, F[3 * f + 1]), ldX(V, F[3 * f + 2]));
}

// Closest triangle of the tree's mesh to each query point (queries taken in
// the order `order` gives, Morton order of the points, so a wave walks nearby
// parts of the tree): a best-first walk for the smallest squared distance,
// then a walk for the smallest triangle index within the tie margin of it;
// optionally the closest point on that triangle.
__device__ __forceinline__ double tie_bound(double best) { return best * (1.0 + TIE) + TIE_ABS; }

__global__ __launch_bounds__(256) void k_nearest(const BvhNode* __restrict__ nodes, int D, int ntree,
                                                 const double* __restrict__ V, const int* __restrict__ F,
                                                 const double* __restrict__ Q, const int* __restrict__ order, int nq,
                                                 double* __restrict__ target, int* __restrict__ tri,
                                                 int* __restrict__ err) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= nq) return;
  const int i = order ? order[qi] : qi;
  const D3 q = ldX(Q, i);
  double best = INFINITY;
  int bestf = 0;
  if (ntree < 2) {
    for (int f = 0; f < ntree; f++) best = fmin(best, face_d2(V, F, f, q));
  } else {
    for (int pass = 0; pass < 2; pass++) {
      const double bound0 = tie_bound(best);
      int st[WALK_STACK];
      double sd[WALK_STACK];
      int sp = 0;
      st[sp] = 0;
      sd[sp++] = 0.0;
      while (sp > 0) {
        sp--;
        const int ent = st[sp];
        const double bound = pass == 0 ? best : bound0;
        if (sd[sp] > bound) continue;
        const int node = ent & ((1 << 27) - 1), L = ent >> 27;
        const BvhNode nd = nodes[node];
        double cd[4];
        for (int c = 0; c < 4; c++) cd[c] = box_d2(nd, c, q);
        if (L == D - 1) {
          const int lf[4] = {nd.leaf.x, nd.leaf.y, nd.leaf.z, nd.leaf.w};
          for (int c = 0; c < 4; c++) {
            if (lf[c] < 0 || cd[c] > (pass == 0 ? best : bound0)) continue;
            const double d = face_d2(V, F, lf[c], q);
            if (pass == 0) {
              if (d < best) best = d;
            } else if (d <= bound0 && (bestf < 0 || lf[c] < bestf)) {
              bestf = lf[c];
            }
          }
        } else {
          // push the far children first so the nearest is taken next
          int ord[4] = {0, 1, 2, 3};
          for (int x = 1; x < 4; x++)
            for (int y = x; y > 0 && cd[ord[y]] > cd[ord[y - 1]]; y--) {
              const int tmp = ord[y];
              ord[y] = ord[y - 1];
              ord[y - 1] = tmp;
            }
          for (int x = 0; x < 4; x++) {
            const int c = ord[x];
            if (cd[c] > bound) continue;
            if (sp < WALK_STACK) {
              st[sp] = (4 * node + 1 + c) | ((L + 1) << 27);
              sd[sp++] = cd[c];
            } else {
              atomicOr(err, PAMO_EBIT_STACK);
            }
          }
        }
      }
      if (pass == 0) bestf = -1;
    }
    if (bestf < 0) bestf = 0;
  }
  if (tri) tri[i] = bestf;
  if (target) {
    const D3 a = ldX(V, F[3 * bestf]), b = ldX(V, F[3 * bestf + 1]), c = ldX(V, F[3 * bestf + 2]);
    const int code = pt_feature(q, a, b, c);
    D3 r;
    if (code == 0) {
      const D3 n = cross(b - a, c - a);
      const double s = dot(q - a, n) / dot(n, n);
      r = D3{q.x - s * n.x, q.y - s * n.y, q.z - s * n.z};
    } else if (code <= 3) {
      const D3 u = code == 1 ? a : code == 2 ? b : c, v = code == 1 ? b : code == 2 ? c : a;
      const D3 e = v - u;
      double t = dot(q - u, e) / fmax(dot(e, e), 1e-300);
      t = fmin(fmax(t, 0.0), 1.0);
      r = D3{u.x + t * e.x, u.y + t * e.y, u.z + t * e.z};
    } else {
      r = code == 4 ? a : code == 5 ? b : c;
    }
    target[3 * (int64_t)i] = r.x;
    target[3 * (int64_t)i + 1] = r.y;
    target[3 * (int64_t)i + 2] = r.z;
  }
}

// Morton codes of points (in [0,1]^3, 10 bits a coordinate) for the query order
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
  x &= 1023;
  x = (x | (x << 16)) & 0x030000FF;
  x = (x | (x << 8)) & 0x0300F00F;
  x = (x | (x << 4)) & 0x030C30C3;
  x = (x | (x << 2)) & 0x09249249;
  return x;
}
__global__ void k_point_codes(const double* __restrict__ P, int n, uint32_t* __restrict__ code, int* __restrict__ id) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c3[3];
  for (int k = 0; k < 3; k++) {
    const double c = fmin(fmax(P[3 * (int64_t)i + k], 0.0), 1.0);
    const int x = (int)(c * 1024.0);
    c3[k] = (uint32_t)(x > 1023 ? 1023 : x);
  }
  code[i] = (spread10(c3[0]) << 2) | (spread10(c3[1]) << 1) | spread10(c3[2]);
  id[i] = i;
}

// ------------------------------------------------------------ host side
void check_launch() { PAMO_HIP(hipGetLastError()); }

template <class T>
void read(hipStream_t s, T* host, const T* dev, size_t n) {
  PAMO_HIP(hipMemcpyAsync(host, dev, n * sizeof(T), hipMemcpyDeviceToHost, s));
  PAMO_HIP(hipStreamSynchronize(s));
}

// The projection problem on one stream: rest data, targets, contacts, the
// element terms of the current evaluation and the CG vectors.
struct Projection {
  Workspace& ws;
  hipStream_t s;
  pamo_project_options o;
  int nv, nf, ne = 0, m;
  // a leaf order of the faces carried from walk to walk: the vertices move
  // little between two walks, so the sorted order of an earlier walk still
  // gives a tight tree (any order gives a correct one); sorted afresh every
  // LEAF_RESORT walks
  static constexpr int LEAF_RESORT = 16;
  int* lord = nullptr;
  int lord_age = LEAF_RESORT;
  const int* F;
  const double* X0;
  const double* Y;
  double area_in;
  double *s0, *Binv, *A0, *th0, *l0;
  int *st, *vown, *twin, *vh;
  uint8_t* hown;
  double* targets;
  int* tri;
  int* m2s_ids;
  int4 *pt = nullptr, *ee = nullptr;
  int cap = 0, npt = 0, nee = 0;
  int2* fpair = nullptr;
  int fcap = 0;
  int* cnt;
  Elems E[K_KINDS];
  double *grad, *Dblk, *Dinv, *cx, *cr, *cz, *cp, *cAp, *part, *part2, *sums;
  CgState* cg;
  int *rowptr = nullptr, *bcol = nullptr;
  double* bval = nullptr;
  double* evsum;
  int* evcnt;
  unsigned long long* stepbits;
  int* err;

  Projection(Workspace& w, hipStream_t st_, const pamo_project_options& opt) : ws(w), s(st_), o(opt) {}

  void setup(const double* X0_, int nv_, const int* F_, int nf_, const double* Y_, int m_, double area) {
    X0 = X0_;
    nv = nv_;
    F = F_;
    nf = nf_;
    Y = Y_;
    m = m_;
    area_in = area;
    const int nh = 3 * nf;
    err = ws.get<int>("pj.err", 4);
    cnt = ws.get<int>("pj.cnt", 4);
    PAMO_HIP(hipMemsetAsync(err, 0, 4 * sizeof(int), s));
    // adjacency: twins, then each edge once
    twin = ws.get<int>("pj.twin", nh);
    vh = ws.get<int>("pj.vh", nv);
    MeshView mv{};
    mv.V = const_cast<double*>(X0);
    mv.F = const_cast<int*>(F);
    mv.twin = twin;
    mv.vh = vh;
    mv.nv = nv;
    mv.nf = nf;
    launch_adjacency(ws, s, mv, err);
    uint8_t* efl = ws.get<uint8_t>("pj.efl", nh);
    hown = ws.get<uint8_t>("pj.hown", nh);
    hipLaunchKernelGGL(k_edge_flags, dim3(nblk(nh)), dim3(256), 0, s, (const int*)twin, nh, efl, hown);
    int* elist = ws.get<int>("pj.elist", nh);
    compact_flags(ws, s, efl, nh, elist, cnt);
    int h_err = 0;
    read(s, &h_err, err, 1);
    if (h_err) throw ProjectMeshError("the mesh to project is not closed, manifold and consistently oriented");
    read(s, &ne, cnt, 1);
    st = ws.get<int>("pj.st", 4 * (int64_t)ne);
    th0 = ws.get<double>("pj.th0", ne);
    l0 = ws.get<double>("pj.l0", ne);
    hipLaunchKernelGGL(k_stencils, dim3(nblk(ne)), dim3(256), 0, s, (const int*)elist, ne, F, (const int*)twin, X0, st,
                       th0, l0);
    vown = ws.get<int>("pj.vown", nv);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(nv)), dim3(256), 0, s, vown, nv, INT32_MAX);
    hipLaunchKernelGGL(k_vown, dim3(nblk(nf)), dim3(256), 0, s, F, nf, vown);
    s0 = ws.get<double>("pj.s0", nv);
    hipLaunchKernelGGL(k_fill_f64, dim3(nblk(nv)), dim3(256), 0, s, s0, (int64_t)nv, 0.0);
    hipLaunchKernelGGL(k_voronoi, dim3(nblk(nf)), dim3(256), 0, s, X0, F, nf, s0);
    Binv = ws.get<double>("pj.binv", 4 * (int64_t)nf);
    A0 = ws.get<double>("pj.a0", nf);
    hipLaunchKernelGGL(k_rest_faces, dim3(nblk(nf)), dim3(256), 0, s, X0, F, nf, Binv, A0);
    targets = ws.get<double>("pj.targets", 3 * (int64_t)nv);
    tri = ws.get<int>("pj.tri", std::max(m, 1));
    m2s_ids = ws.get<int>("pj.m2sids", 3 * (int64_t)std::max(m, 1));
    grad = ws.get<double>("pj.grad", 3 * (int64_t)nv);
    Dblk = ws.get<double>("pj.dblk", 9 * (int64_t)nv);
    Dinv = ws.get<double>("pj.dinv", 9 * (int64_t)nv);
    cx = ws.get<double>("pj.cx", 3 * (int64_t)nv);
    cr = ws.get<double>("pj.cr", 3 * (int64_t)nv);
    cz = ws.get<double>("pj.cz", 3 * (int64_t)nv);
    cp = ws.get<double>("pj.cp", 3 * (int64_t)nv);
    cAp = ws.get<double>("pj.cap", 3 * (int64_t)nv);
    part = ws.get<double>("pj.part", sum_blocks(3 * (int64_t)nv));
    part2 = ws.get<double>("pj.part2", sum_blocks(3 * (int64_t)nv));
    sums = ws.get<double>("pj.sums", 8);
    cg = ws.get<CgState>("pj.cg", 1);
    evsum = ws.get<double>("pj.evsum", 10);  // 8 sums, then the 4 counts
    evcnt = reinterpret_cast<int*>(evsum + 8);
    stepbits = ws.get<unsigned long long>("pj.step", 1);
    // element sets that do not change
    E[K_M2S].ids = m2s_ids;
    E[K_M2S].n = m;
    E[K_M2S].Y = Y;
    E[K_M2S].w = o.k_dis * area_in / (double)std::max(m, 1);
    E[K_EL].ids = F;
    E[K_EL].n = nf;
    E[K_EL].Binv = Binv;
    E[K_EL].A0 = A0;
    E[K_EL].w = o.k_elas;
    E[K_BEND].ids = st;
    E[K_BEND].n = ne;
    E[K_BEND].th0 = th0;
    E[K_BEND].l0 = l0;
    E[K_BEND].w = o.k_bend;
    E[K_PT].dhat = E[K_EE].dhat = o.dhat;
    E[K_PT].w = E[K_EE].w = o.k_bar;
    const char* vn[K_KINDS] = {"pj.v0", "pj.v1", "pj.v2", "pj.v3", "pj.v4"};
    for (int k = 0; k < K_KINDS; k++)
      if (k < K_PT) E[k].val = ws.get<double>(vn[k], std::max(E[k].n, 1));
    grow_contacts(std::max(4096, 2 * nf));
    grow_pairs(std::max(1 << 16, 32 * nf));
    check_launch();
  }

  void grow_contacts(int c) {
    cap = c;
    pt = ws.get<int4>("pj.pt", cap);
    ee = ws.get<int4>("pj.ee", cap);
    E[K_PT].val = ws.get<double>("pj.v3", cap);
    E[K_EE].val = ws.get<double>("pj.v4", cap);
  }

  void use_targets(const double* tg, const int* tr) {
    if (tg != targets)
      PAMO_HIP(hipMemcpyAsync(targets, tg, 3 * (size_t)nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (m > 0) {
      if (tr != tri) PAMO_HIP(hipMemcpyAsync(tri, tr, (size_t)m * sizeof(int), hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_gather_tri, dim3(nblk(m)), dim3(256), 0, s, F, (const int*)tri, m, m2s_ids);
    }
    check_launch();
  }

  void walk(const double* X, const double* P, double pad) {
    float* box = ws.get<float>("pj.box", 6 * (int64_t)nf);
    hipLaunchKernelGGL(k_boxes, dim3(nblk(nf)), dim3(256), 0, s, X, P, F, nf, pad, box);
    const bool reuse = lord && lord_age < LEAF_RESORT;
    Bvh b = build_bvh(ws, s, box, nf, reuse ? lord : nullptr);
    if (reuse) {
      lord_age++;
    } else if (nf >= 2) {
      lord = ws.get<int>("pj.lord", nf);
      PAMO_HIP(hipMemcpyAsync(lord, b.sorted, (size_t)nf * sizeof(int), hipMemcpyDeviceToDevice, s));
      lord_age = 1;
    }
    WalkArgs a{};
    a.nodes = b.nodes;
    a.D = b.D;
    a.nf = nf;
    a.box = box;
    a.X = X;
    a.P = P;
    a.F = F;
    a.vown = vown;
    a.hown = hown;
    a.pad = pad;
    a.dhat2 = o.dhat * o.dhat;
    a.s = o.accd_s;
    a.pt = pt;
    a.ee = ee;
    a.cnt = cnt;
    a.cap = cap;
    a.step = stepbits;
    a.fpair = fpair;
    a.fcap = fcap;
    if (nf >= 2) hipLaunchKernelGGL(k_walk, dim3(nblk(nf, 64)), dim3(64), 0, s, a, b.sorted);  // one-wave blocks
    else hipLaunchKernelGGL(k_walk_small, dim3(1), dim3(1), 0, s, a);
    hipLaunchKernelGGL(k_pair_slots, dim3(4096), dim3(256), 0, s, a);  // about one slot per thread
    check_launch();
  }

  void grow_pairs(int c) {
    fcap = c;
    fpair = ws.get<int2>("pj.fpair", fcap);
  }

  // the additive-CCD step along P from X (at most 1)
  double ccd(const double* X, const double* P) {
    const double one = 1.0;
    unsigned long long bits;
    __builtin_memcpy(&bits, &one, 8);
    PAMO_HIP(hipMemcpyAsync(stepbits, &bits, 8, hipMemcpyHostToDevice, s));
    for (;;) {
      PAMO_HIP(hipMemsetAsync(cnt, 0, 4 * sizeof(int), s));
      walk(X, P, 0.0);
      int h[4];
      read(s, h, cnt, 4);
      if (h[3] <= fcap) break;
      grow_pairs(h[3] + h[3] / 2);
      PAMO_HIP(hipMemcpyAsync(stepbits, &bits, 8, hipMemcpyHostToDevice, s));
    }
    read(s, &bits, stepbits, 1);
    double t;
    __builtin_memcpy(&t, &bits, 8);
    return t;
  }

  // the kinds' launch ranges (contacts sized by their capacity)
  // the kinds' launch ranges, one thread per element (contacts sized by their
  // capacity)
  KindRanges ranges(bool contacts_by_cap) {
    KindRanges r{};
    for (int k = 0; k < K_KINDS; k++) r.E[k] = E[k];
    if (contacts_by_cap) r.E[K_PT].n = r.E[K_EE].n = cap;
    r.s0 = s0;
    r.tg = targets;
    r.sval = ws.get<double>("pj.s2mval", nv);
    r.nv = nv;
    r.cnt = cnt;
    const int n[NSEG] = {nv, r.E[K_M2S].n, r.E[K_EL].n, r.E[K_BEND].n, r.E[K_PT].n, r.E[K_EE].n};
    r.blk[0] = 0;
    for (int k = 0; k < NSEG; k++) r.blk[k + 1] = r.blk[k] + (n[k] > 0 ? (int)nblk(n[k]) : 0);
    return r;
  }

  // the five terms (unweighted) and B at X; contacts are detected at X first.
  // One read-back: the sums and the contact counts together.
  void energy(const double* X, double* parts) {
    for (;;) {
      PAMO_HIP(hipMemsetAsync(cnt, 0, 4 * sizeof(int), s));
      walk(X, nullptr, o.dhat);
      E[K_PT].ids = (const int*)pt;
      E[K_EE].ids = (const int*)ee;
      KindRanges r = ranges(true);
      hipLaunchKernelGGL(k_values_all, dim3(r.blk[NSEG]), dim3(256), 0, s, r, X);
      SegSums ss{};
      const int n[NSEG] = {nv, E[K_M2S].n, E[K_EL].n, E[K_BEND].n, cap, cap};
      const double* v[NSEG] = {r.sval, E[K_M2S].val, E[K_EL].val, E[K_BEND].val, E[K_PT].val, E[K_EE].val};
      int most = 1;
      for (int k = 0; k < NSEG; k++) {
        ss.v[k] = v[k];
        ss.n[k] = n[k];
        most = std::max(most, n[k]);
      }
      const unsigned nb = sum_blocks(most);
      ss.cnt = cnt;
      ss.stride = (int)nb;
      ss.part = ws.get<double>("pj.segpart", (int64_t)NSEG * nb);
      hipLaunchKernelGGL(k_sum_seg, dim3(nb, NSEG), dim3(SUM_T), 0, s, ss);
      hipLaunchKernelGGL(k_sum_seg_final, dim3(NSEG), dim3(SUM_T), 0, s, (const double*)ss.part, (int)nb, (int)nb,
                         evsum);
      PAMO_HIP(hipMemcpyAsync(evcnt, cnt, 4 * sizeof(int), hipMemcpyDeviceToDevice, s));
      check_launch();
      struct {
        double sum[8];
        int cnt[4];
      } h;
      read(s, reinterpret_cast<char*>(&h), reinterpret_cast<const char*>(evsum), sizeof(h));
      if (h.cnt[3] > fcap) {
        grow_pairs(h.cnt[3] + h.cnt[3] / 2);
        continue;
      }
      if (h.cnt[0] > cap || h.cnt[1] > cap) {
        grow_contacts(std::max(h.cnt[0], h.cnt[1]) + std::max(h.cnt[0], h.cnt[1]) / 2);
        continue;
      }
      npt = h.cnt[0];
      nee = h.cnt[1];
      E[K_PT].n = npt;
      E[K_EE].n = nee;
      parts[0] = h.sum[0];
      parts[1] = area_in / (double)std::max(m, 1) * h.sum[1 + K_M2S];
      parts[2] = h.sum[1 + K_EL];
      parts[3] = h.sum[1 + K_BEND];
      parts[4] = h.sum[1 + K_PT] + h.sum[1 + K_EE];
      parts[5] = o.k_dis * (parts[0] + parts[1]) + o.k_elas * parts[2] + o.k_bend * parts[3] + o.k_bar * parts[4];
      return;
    }
  }

  template <int K>
  void derivs_of(const double* X, const char* hn, const char* gn) {
    Elems& e = E[K];
    if (e.n == 0) return;
    constexpr int N = KT<K>::N;
    e.H = ws.get<double>(hn, (int64_t)N * N * e.n);
    e.g = ws.get<double>(gn, (int64_t)N * e.n);
    hipLaunchKernelGGL(k_elem_deriv<K>, dim3(nblk((int64_t)KT<K>::NP * e.n)), dim3(256), 0, s, e, X);
    hipLaunchKernelGGL(k_elem_psd<N>, dim3(nblk((int64_t)PSD_G * e.n)), dim3(256), 0, s, e.H, e.n);
    hipLaunchKernelGGL(k_elem_grad<K>, dim3(nblk(e.n)), dim3(256), 0, s, e, grad);
    check_launch();
  }

  // gradient of B and the projected element Hessians at X (contacts as last
  // detected, which must be at X)
  void derivs(const double* X) {
    hipLaunchKernelGGL(k_s2m_init, dim3(nblk(nv)), dim3(256), 0, s, X, (const double*)targets, (const double*)s0, nv,
                       o.k_dis, grad, Dblk);
    derivs_of<K_M2S>(X, "pj.h0", "pj.g0");
    derivs_of<K_EL>(X, "pj.h1", "pj.g1");
    derivs_of<K_BEND>(X, "pj.h2", "pj.g2");
    derivs_of<K_PT>(X, "pj.h3", "pj.g3");
    derivs_of<K_EE>(X, "pj.h4", "pj.g4");
    assemble();
    hipLaunchKernelGGL(k_bsr_diag, dim3(nblk(nv)), dim3(256), 0, s, (const int*)rowptr, (const int*)bcol,
                       (const double*)bval, nv, Dblk);
    hipLaunchKernelGGL(k_block_inv, dim3(nblk(nv)), dim3(256), 0, s, (const double*)Dblk, nv, Dinv);
    check_launch();
  }

  // the block-sparse Hessian from the projected element Hessians
  void assemble() {
    EntryRanges r{};
    for (int k = 0; k < K_KINDS; k++) r.E[k] = E[k];
    r.s0 = s0;
    r.k2 = 2.0 * o.k_dis;
    r.nv = nv;
    const int64_t per[NSEG] = {(int64_t)nv, 9LL * E[K_M2S].n, 9LL * E[K_EL].n, 16LL * E[K_BEND].n,
                               16LL * E[K_PT].n, 16LL * E[K_EE].n};
    r.off[0] = 0;
    for (int k = 0; k < NSEG; k++) r.off[k + 1] = r.off[k] + per[k];
    const int64_t n = r.off[NSEG];
    if (n > INT32_MAX) throw std::runtime_error("Hessian pattern too large");
    int bits = 1;
    while ((1 << bits) < nv) bits++;
    uint64_t* keys = ws.get<uint64_t>("pj.bkeys", n);
    int* vals = ws.get<int>("pj.bvals", n);
    uint8_t* fl = ws.get<uint8_t>("pj.bflags", n);
    int* excl = ws.get<int>("pj.bexcl", n);
    int* ustart = ws.get<int>("pj.bstart", n);
    int* nslot = ws.get<int>("pj.bnslot", 1);
    rowptr = ws.get<int>("pj.browptr", (int64_t)nv + 1);
    bcol = ws.get<int>("pj.bcol", n);
    bval = ws.get<double>("pj.bval", 9 * n);
    hipLaunchKernelGGL(k_bsr_keys, dim3(nblk(n)), dim3(256), 0, s, r, bits, keys, vals);
    radix_sort_u64(ws, s, keys, vals, n, 2 * bits);
    hipLaunchKernelGGL(k_bsr_flags, dim3(nblk(n)), dim3(256), 0, s, (const uint64_t*)keys, n, fl);
    run_flag_scan(ws, s, fl, n, excl, nslot);
    hipLaunchKernelGGL(k_bsr_starts, dim3(nblk(n)), dim3(256), 0, s, (const uint8_t*)fl, (const int*)excl, n, ustart);
    hipLaunchKernelGGL(k_bsr_fill, dim3(nblk(n)), dim3(256), 0, s, r, (const uint64_t*)keys, (const int*)vals,
                       (const int*)ustart, (const int*)nslot, n, bits, rowptr, bcol, bval);
    check_launch();
  }

  // out = H v (after derivs)
  void matvec(const double* v, double* out, const int* done) {
    hipLaunchKernelGGL(k_bsr_spmv, dim3(nblk(3 * (int64_t)nv)), dim3(256), 0, s, (const int*)rowptr, (const int*)bcol,
                       (const double*)bval, nv, v, out, done);
    check_launch();
  }

  // p from H p = -grad (after derivs); returns the CG iterations.  Two
  // launches per iteration (direction with its product, then the update);
  // the host looks at the stopping flag every 8.
  int solve(double* dir) {
    const int64_t n3 = 3 * (int64_t)nv;
    const unsigned nb = sum_blocks(n3);
    const unsigned nbv = nblk(nv, CG_T);
    const unsigned nbd = nblk(n3, CG_T);
    double* pz = ws.get<double>("pj.cgpz", nbv);
    double* pr = ws.get<double>("pj.cgpr", nbv);
    double* pp = ws.get<double>("pj.cgpp", nbd);
    double* p2 = ws.get<double>("pj.cgp2", n3);  // the other direction buffer
    CgState h{};
    h.tol = o.cg_tol;
    h.max_it = o.cg_max;
    PAMO_HIP(hipMemcpyAsync(cg, &h, sizeof(h), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_cg_init, dim3(nblk(nv)), dim3(256), 0, s, (const double*)grad, (const double*)Dinv, nv, cx, cr,
                       cz, cp, cAp);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(SUM_T), 0, s, (const double*)cr, (const double*)cr, n3, part,
                       (const int*)nullptr);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(SUM_T), 0, s, (const double*)cr, (const double*)cz, n3, part2,
                       (const int*)nullptr);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(SUM_T), 0, s, (const double*)part, (const double*)part2, (int)nb, cg);
    double* pa = cp;  // this iteration's direction goes into pb
    double* pb = p2;
    for (int it = 0;;) {
      for (int k = 0; k < 8; k++, it++) {
        hipLaunchKernelGGL(k_cg_dir, dim3(nbd), dim3(CG_T), 0, s, (const int*)rowptr, (const int*)bcol,
                           (const double*)bval, nv, (const double*)cz, (const double*)pa, pb, cAp, pp,
                           (const double*)pz, (const double*)pr, (int)nbv, it, cg);
        hipLaunchKernelGGL(k_cg_step, dim3(nbv), dim3(CG_T), 0, s, cx, cr, cz, (const double*)pb, (const double*)cAp,
                           (const double*)Dinv, nv, (const double*)pp, (int)nbd, pz, pr, it, (const CgState*)cg);
        std::swap(pa, pb);
      }
      check_launch();
      read(s, &h, cg, 1);
      if (h.done) break;
    }
    PAMO_HIP(hipMemcpyAsync(dir, cx, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    return h.it;
  }
};

double dot_dev(Workspace& ws, hipStream_t s, const double* a, const double* b, int64_t n) {
  const unsigned nb = sum_blocks(n);
  double* part = ws.get<double>("pj.dpart", nb);
  double* out = ws.get<double>("pj.dsum", 1);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(SUM_T), 0, s, a, b, n, part, (const int*)nullptr);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(SUM_T), 0, s, (const double*)part, (int)nb, out);
  double v;
  read(s, &v, out, 1);
  return v;
}

double surface_area(Workspace& ws, hipStream_t s, const double* V, const int* F, int nf) {
  double* a = ws.get<double>("pj.area", std::max(nf, 1));
  hipLaunchKernelGGL(k_face_area, dim3(nblk(nf)), dim3(256), 0, s, V, F, nf, a);
  check_launch();
  return dot_dev(ws, s, a, nullptr, nf);
}

}  // namespace

double project_sample(Workspace& ws, hipStream_t s, const double* V, int nv, const int* F, int nf, const double* U,
                      int64_t m, double* Y) {
  (void)nv;
  double* cum = ws.get<double>("pj.cum", std::max(nf, 1));
  const int nt = (nf + SCAN_TILE - 1) / SCAN_TILE;
  double* tsum = ws.get<double>("pj.tsum", std::max(nt, 1));
  hipLaunchKernelGGL(k_face_area, dim3(nblk(nf)), dim3(256), 0, s, V, F, nf, cum);
  hipLaunchKernelGGL(k_scan_tile, dim3(std::max(nt, 1)), dim3(SCAN_T), 0, s, cum, nf, tsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(64), 0, s, tsum, nt);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk(nf)), dim3(256), 0, s, cum, nf, (const double*)tsum);
  if (m > 0) hipLaunchKernelGGL(k_sample, dim3(nblk(m)), dim3(256), 0, s, V, F, nf, (const double*)cum, U, m, Y);
  check_launch();
  double total;
  read(s, &total, cum + (nf - 1), 1);
  return total;
}

void project_targets(Workspace& ws, hipStream_t s, const double* X, int nv, const int* F, int nf, const double* Vin,
                     int nvin, const int* Fin, int nfin, const double* Y, int m, double* targets, int* tri) {
  (void)nvin;
  int* err = ws.get<int>("pj.terr", 1);
  PAMO_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
  float* box = ws.get<float>("pj.tbox", 6 * (int64_t)std::max(nfin, nf));
  hipLaunchKernelGGL(k_boxes, dim3(nblk(nfin)), dim3(256), 0, s, Vin, (const double*)nullptr, Fin, nfin, 0.0, box);
  // query orders: the points sorted by Morton code
  auto point_order = [&](const double* P, int n, const char* kn, const char* in) {
    uint32_t* code = ws.get<uint32_t>(kn, std::max(n, 1));
    int* id = ws.get<int>(in, std::max(n, 1));
    hipLaunchKernelGGL(k_point_codes, dim3(nblk(n)), dim3(256), 0, s, P, n, code, id);
    radix_sort_u32(ws, s, code, id, n, 30);
    return (const int*)id;
  };
  const int* vorder = point_order(X, nv, "pj.vcode", "pj.vord");
  const int* sorder = m > 0 ? point_order(Y, m, "pj.scode", "pj.sord") : nullptr;
  Bvh b = build_bvh(ws, s, box, nfin, nullptr);
  // one-wave blocks: a few thousand long walks spread over all the CUs
  hipLaunchKernelGGL(k_nearest, dim3(nblk(nv, 64)), dim3(64), 0, s, (const BvhNode*)b.nodes, b.D, nfin, Vin, Fin, X,
                     vorder, nv, targets, (int*)nullptr, err);
  if (m > 0) {
    hipLaunchKernelGGL(k_boxes, dim3(nblk(nf)), dim3(256), 0, s, X, (const double*)nullptr, F, nf, 0.0, box);
    Bvh c = build_bvh(ws, s, box, nf, nullptr);
    hipLaunchKernelGGL(k_nearest, dim3(nblk(m, 64)), dim3(64), 0, s, (const BvhNode*)c.nodes, c.D, nf, X, F, Y, sorder, m,
                       (double*)nullptr, tri, err);
  }
  check_launch();
  int h = 0;
  read(s, &h, err, 1);
  if (h) throw std::runtime_error("closest-point walk: traversal stack overflow");
}

void project_eval(Workspace& ws, hipStream_t s, const double* X0, const double* X, int nv, const int* F, int nf,
                  const double* targets, const double* Y, const int* tri, int m, double area_in,
                  const pamo_project_options& o, ProjectEvalOut& out) {
  Projection P(ws, s, o);
  P.setup(X0, nv, F, nf, Y, m, area_in);
  P.use_targets(targets, tri);
  P.energy(X, out.parts);
  out.npt = P.npt;
  out.nee = P.nee;
  if (!(out.grad || out.Hv || out.dir)) return;
  P.derivs(X);
  if (out.grad)
    PAMO_HIP(hipMemcpyAsync(out.grad, P.grad, 3 * (size_t)nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (out.Hv && out.v) P.matvec(out.v, out.Hv, nullptr);
  if (out.dir) {
    out.cg_iters = P.solve(out.dir);
    if (out.want_step) out.step = P.ccd(X, out.dir);
  }
  PAMO_HIP(hipStreamSynchronize(s));
}

void project_run(Workspace& ws, hipStream_t s, const double* X0, int nv, const int* F, int nf, const double* Vin,
                 int nvin, const int* Fin, int nfin, const double* Y, int m, const pamo_project_options& o,
                 double* Xout, double* log, pamo_project_stats* stats) {
  const double area_in = surface_area(ws, s, Vin, Fin, nfin);
  Projection P(ws, s, o);
  P.setup(X0, nv, F, nf, Y, m, area_in);
  const int64_t n3 = 3 * (int64_t)nv;
  double* X = Xout;
  double* Xt = ws.get<double>("pj.xt", n3);
  double* dir = ws.get<double>("pj.dir", n3);
  if (X != X0) PAMO_HIP(hipMemcpyAsync(X, X0, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  pamo_project_stats st{};
  double parts[6], trial[6];
  double B0 = 0.0;
  bool have = false;     // contacts and B0 are those of X
  bool stalled = false;  // this window's targets gave no decrease: X stays until the next refresh
  for (int t = 0; t < o.iterations; t++) {
    if (t % o.refresh == 0) {
      project_targets(ws, s, X, nv, F, nf, Vin, nvin, Fin, nfin, Y, m, P.targets, P.tri);
      P.use_targets(P.targets, P.tri);
      have = false;
      stalled = false;
    }
    st.iterations++;
    if (stalled) {
      if (log) {
        double* r = log + 8 * (int64_t)t;
        for (int k = 0; k < 8; k++) r[k] = 0.0;
        r[0] = B0;
        r[5] = (double)P.npt;
        r[6] = (double)P.nee;
      }
      continue;
    }
    if (!have) {
      P.energy(X, parts);
      B0 = parts[5];
    }
    if (t == 0) st.B_first = B0;
    st.max_pt = std::max<int64_t>(st.max_pt, P.npt);
    st.max_ee = std::max<int64_t>(st.max_ee, P.nee);
    const int64_t npt = P.npt, nee = P.nee;
    const double Bstart = B0;
    P.derivs(X);
    const double gnorm = std::sqrt(dot_dev(ws, s, P.grad, P.grad, n3));
    const int it = P.solve(dir);
    const double pnorm = std::sqrt(dot_dev(ws, s, dir, dir, n3));
    const double accd = P.ccd(X, dir);
    double alpha = std::min(1.0, accd);
    bool moved = false;
    int h = 0;
    for (h = 0; h < o.ls_max; h++) {
      if (alpha * pnorm < LS_MIN_STEP) break;
      hipLaunchKernelGGL(k_axpy_pos, dim3(nblk(n3)), dim3(256), 0, s, (const double*)X, (const double*)dir, alpha, n3,
                         Xt);
      check_launch();
      P.energy(Xt, trial);
      if (trial[5] < B0) {
        PAMO_HIP(hipMemcpyAsync(X, Xt, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
        B0 = trial[5];
        moved = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!moved && h >= o.ls_max) h = o.ls_max - 1;
    have = moved;
    stalled = !moved;
    st.cg_iters += it;
    st.halvings += h;
    st.stalled += !moved;
    if (log) {
      double* r = log + 8 * (int64_t)t;
      r[0] = Bstart;
      r[1] = accd;
      r[2] = moved ? alpha : 0.0;
      r[3] = h;
      r[4] = it;
      r[5] = (double)npt;
      r[6] = (double)nee;
      r[7] = gnorm;
    }
  }
  st.B_last = B0;
  PAMO_HIP(hipStreamSynchronize(s));
  if (stats) *stats = st;
}

}  // namespace pamo
