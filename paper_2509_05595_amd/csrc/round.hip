// Per-round kernels of parallel intersection-free QEM simplification
// (PaMO Sec. 5.1 and 5.3), one thread per vertex, edge or candidate.
//
// Every per-element result is a pure function of the pre-round mesh, so the
// kernels need no atomics except the idempotent marks of the check/undo loop:
//   quadrics      vertex:    Q_v = sum of plane quadrics of its faces, ascending face slot
//   cost_keys     edge:      placement + Eq. 1 cost + 64-bit key (both half-edges)
//   vertex_min    vertex:    m_v = min key of its edges, gathered over the stored star
//                            (the pull form of the paper's AtomicMin propagation)
//   select        vertex:    the edge m_v names is chosen iff its key is the minimum
//                            of m_w over the closed neighbourhood of the edge
//   local_check   candidate: link condition, exact degeneracy, normal flip
//   apply/undo    candidate: tentative collapse and its exact reversal
//   commit        candidate: twin rewiring of the two removed faces
//   compaction    face/vertex: stable, order-preserving
#include "internal.hpp"
#include "exact_dev.hpp"
#include "round.hpp"

namespace pamo {

namespace {

constexpr int RING_GUARD = 1 << 15;  // a vertex star longer than this is treated as corrupt

__device__ __forceinline__ void set_err(int* err, int bit) { atomicOr(err, bit); }

// visit the outgoing half-edges of the vertex at the origin of h0
template <class Fn>
__device__ __forceinline__ bool walk_star(const int* __restrict__ twin, int h0, Fn&& fn) {
  if (h0 < 0) return false;
  int h = h0, guard = 0;
  do {
    fn(h);
    h = twin[he_prev(h)];
    if (++guard > RING_GUARD || h < 0) return false;
  } while (h != h0);
  return true;
}

__device__ __forceinline__ int dest(const int* __restrict__ F, int h) { return F[he_next(h)]; }

// histogram of reasons 0..4 over the active lanes of a wave: one atomic per
// value present
__device__ __forceinline__ void wave_hist(int r, int* hist) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v <= 4; v++) {
    unsigned long long b = __ballot(r == v);
    if (b && lane == __ffsll((long long)b) - 1) atomicAdd(&hist[v], __popcll(b));
  }
}

// pop the smallest entry of an ascending register list
template <int CAP>
__device__ __forceinline__ int pop_front(int* a) {
  int f = a[0];
#pragma unroll
  for (int i = 0; i < CAP - 1; i++) a[i] = a[i + 1];
  a[CAP - 1] = INT32_MAX;
  return f;
}

// ------------------------------------------------------------ adjacency
__global__ void k_he_keys(const int* __restrict__ F, int nf, int nv, int bits, uint64_t* keys, int* vals, int* err) {
  int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 3 * nf) return;
  int a = F[h], b = F[he_next(h)];
  if (a < 0 || a >= nv || b < 0 || b >= nv) {
    set_err(err, PAMO_EBIT_INDEX);
    a = b = 0;
  }
  if (a == b) set_err(err, PAMO_EBIT_DEGENERATE);
  uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  keys[h] = ((uint64_t)lo << bits) | hi;
  vals[h] = h;
}

__global__ void k_pair_twins(const uint64_t* __restrict__ keys, const int* __restrict__ vals, int n,
                             const int* __restrict__ F, int* twin, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i];
  if (i > 0 && keys[i - 1] == k) return;  // not the first of its group
  int len = 1;
  while (i + len < n && keys[i + len] == k && len < 3) len++;
  if (len != 2) {
    set_err(err, PAMO_EBIT_EDGE);
    twin[vals[i]] = -1;
    return;
  }
  int h1 = vals[i], h2 = vals[i + 1];
  // opposite directions: h1 = a->b, h2 = b->a
  if (F[h1] != F[he_next(h2)] || F[he_next(h1)] != F[h2]) {
    set_err(err, PAMO_EBIT_ORIENT);
    return;
  }
  twin[h1] = h2;
  twin[h2] = h1;
}

__global__ void k_vertex_he(const int* __restrict__ F, int nf, int* vh, int* deg) {
  int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 3 * nf) return;
  int v = F[h];
  vh[v] = h;  // any leaving half-edge will do
  atomicAdd(&deg[v], 1);
}

// every vertex must be used and its star must be one fan around it
__global__ void k_check_vertices(const int* __restrict__ twin, const int* __restrict__ vh,
                                 const int* __restrict__ deg, int nv, int* err) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int d = deg[v];
  if (d == 0) {
    set_err(err, PAMO_EBIT_VERTEX);
    return;
  }
  int h0 = vh[v], h = h0, cnt = 0;
  do {
    int p = twin[he_prev(h)];
    cnt++;
    if (p < 0 || cnt > d) break;
    h = p;
  } while (h != h0);
  if (cnt != d || h != h0) set_err(err, PAMO_EBIT_VERTEX);
}

// ------------------------------------------------------------ quadrics
// One thread per vertex: walk the star once (sorted half-edge list in
// registers), then sum the face quadrics in ascending face slot, four faces
// at a time with their loads issued together.
__global__ __launch_bounds__(256) void k_quadrics(MeshView m, double* __restrict__ Q, int* err) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.nv) return;
  constexpr int CAP = VSTAR;
  int hl[CAP];
#pragma unroll
  for (int i = 0; i < CAP; i++) hl[i] = INT32_MAX;
  int n = 0;
  P3 lo{INFINITY, INFINITY, INFINITY}, hi{-INFINITY, -INFINITY, -INFINITY};
  const bool stars = m.vstar != nullptr;
  bool ok = walk_star(m.twin, m.vh[v], [&](int h) {
    if (n < CAP) sorted_insert<CAP>(hl, h);
    n++;
  });
  if (!ok) {
    set_err(err, PAMO_EBIT_RING);
    return;
  }
  if (stars) {
    int4* o = reinterpret_cast<int4*>(m.vstar + (int64_t)VSTAR * v);
#pragma unroll
    for (int i = 0; i < CAP / 4; i++) o[i] = make_int4(hl[4 * i], hl[4 * i + 1], hl[4 * i + 2], hl[4 * i + 3]);
    m.vdeg[v] = n;
  }
  double q[10];
#pragma unroll
  for (int i = 0; i < 10; i++) q[i] = 0.0;
  auto add_face = [&](P3 p0, P3 p1, P3 p2) {
    double K[10];
    face_quadric(p0, p1, p2, K);
    if (stars) {  // box of the closed 1-ring: every corner of the star
      lo.x = fmin(lo.x, fmin(fmin(p0.x, p1.x), p2.x));
      lo.y = fmin(lo.y, fmin(fmin(p0.y, p1.y), p2.y));
      lo.z = fmin(lo.z, fmin(fmin(p0.z, p1.z), p2.z));
      hi.x = fmax(hi.x, fmax(fmax(p0.x, p1.x), p2.x));
      hi.y = fmax(hi.y, fmax(fmax(p0.y, p1.y), p2.y));
      hi.z = fmax(hi.z, fmax(fmax(p0.z, p1.z), p2.z));
    }
#pragma unroll
    for (int i = 0; i < 10; i++) q[i] = q[i] + K[i];
  };
  if (n <= CAP) {
    const P3 pv = ld3(m.V, v);
#pragma unroll
    for (int j = 0; j < CAP / 4; j++) {
      if (4 * j >= n) break;
      P3 p[4][3];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        // corner g % 3 of face g / 3 is v itself: only the other two are loaded
        const int g = 4 * j + k < n ? hl[4 * j + k] : hl[0];
        const int f = g / 3, ci = g - 3 * f;
        int c[3];
#pragma unroll
        for (int i = 0; i < 3; i++) c[i] = m.F[3 * (int64_t)f + i];
        const int c1 = ci == 2 ? 0 : ci + 1, c2 = ci == 0 ? 2 : ci - 1;
        const P3 q1 = ld3(m.V, c1 == 0 ? c[0] : c1 == 1 ? c[1] : c[2]);
        const P3 q2 = ld3(m.V, c2 == 0 ? c[0] : c2 == 1 ? c[1] : c[2]);
#pragma unroll
        for (int i = 0; i < 3; i++) p[k][i] = i == ci ? pv : i == c1 ? q1 : q2;
      }
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (4 * j + k < n) add_face(p[k][0], p[k][1], p[k][2]);
    }
  } else {
    int last = -1;
    for (int k = 0; k < n; k++) {
      int best = INT32_MAX;
      walk_star(m.twin, m.vh[v], [&](int h) {
        int g = h / 3;
        if (g > last && g < best) best = g;
      });
      last = best;
      add_face(ld3(m.V, m.F[3 * best]), ld3(m.V, m.F[3 * best + 1]), ld3(m.V, m.F[3 * best + 2]));
    }
  }
#pragma unroll
  for (int i = 0; i < 10; i++) Q[10 * (int64_t)v + i] = q[i];
  if (stars) {
    double* bx = m.vbox + 6 * (int64_t)v;
    bx[0] = lo.x; bx[1] = lo.y; bx[2] = lo.z;
    bx[3] = hi.x; bx[4] = hi.y; bx[5] = hi.z;
  }
}

// ------------------------------------------------------------ edge evaluation
// Edge h with endpoints s < r, the half-edges leaving them, its two faces and
// the box of every vertex of star(s) u star(r).  fast: both stars were stored
// by the quadrics kernel of this round (at most VSTAR faces each), so neither
// box nor ring needs a walk.
struct EdgeStars {
  int s, r, hs, hr, f1, f2, ns, nr;
  bool fast;
  P3 lo, hi;
};

__device__ __forceinline__ bool edge_stars(const MeshView& m, int h, EdgeStars& E) {
  const int t = m.twin[h];
  const int a = m.F[h], b = m.F[he_next(h)];
  E.s = a < b ? a : b;
  E.r = a < b ? b : a;
  E.hs = a < b ? h : t;
  E.hr = a < b ? t : h;
  E.f1 = h / 3;
  E.f2 = t / 3;
  E.fast = false;
  E.ns = E.nr = 0;
  if (m.vstar) {
    E.ns = m.vdeg[E.s];
    E.nr = m.vdeg[E.r];
    E.fast = E.ns <= VSTAR && E.nr <= VSTAR;
  }
  if (E.fast) {
    const double* bs = m.vbox + 6 * (int64_t)E.s;
    const double* br = m.vbox + 6 * (int64_t)E.r;
    E.lo = P3{fmin(bs[0], br[0]), fmin(bs[1], br[1]), fmin(bs[2], br[2])};
    E.hi = P3{fmax(bs[3], br[3]), fmax(bs[4], br[4]), fmax(bs[5], br[5])};
    return true;
  }
  E.lo = P3{INFINITY, INFINITY, INFINITY};
  E.hi = P3{-INFINITY, -INFINITY, -INFINITY};
  auto visit = [&](int g) {
    P3 p = ld3(m.V, dest(m.F, g));
    E.lo.x = fmin(E.lo.x, p.x); E.lo.y = fmin(E.lo.y, p.y); E.lo.z = fmin(E.lo.z, p.z);
    E.hi.x = fmax(E.hi.x, p.x); E.hi.y = fmax(E.hi.y, p.y); E.hi.z = fmax(E.hi.z, p.z);
  };
  bool ok = walk_star(m.twin, E.hs, visit);
  return ok && walk_star(m.twin, E.hr, visit);
}

// The faces of star(v) (v = E.s with hv = E.hs, or r with E.hr) other than
// the edge's two faces, in ascending face slot, by repeated scans of the star
// for the next larger slot (the path for stars that were not stored).
template <class Fn>
__device__ __forceinline__ void star_ascending(const MeshView& m, const EdgeStars& E, int hv, Fn fn) {
  int last = -1;
  for (;;) {
    int best = INT32_MAX;
    walk_star(m.twin, hv, [&](int g) {
      int f = g / 3;
      if (f > last && f < best) best = f;
    });
    if (best == INT32_MAX) break;
    last = best;
    if (best != E.f1 && best != E.f2) fn(best);
  }
}

// placement of the merged vertex (quadric minimiser by Cramer's rule when the
// system is well conditioned and the minimiser is inside the ring box, else
// the best of midpoint, p_s, p_r)
__device__ __forceinline__ P3 placement(const double* q, P3 ps, P3 pr, P3 lo, P3 hi) {
  double a00 = q[0], a01 = q[1], a02 = q[2], a11 = q[4], a12 = q[5], a22 = q[7];
  double r0 = -q[3], r1 = -q[6], r2 = -q[8];
  double c00 = a11 * a22 - a12 * a12;
  double c01 = a01 * a22 - a12 * a02;
  double c02 = a01 * a12 - a11 * a02;
  double det = a00 * c00 - a01 * c01 + a02 * c02;
  double tr3 = (a00 + a11 + a22) / 3.0;
  double thr = 1e-10 * (tr3 * tr3 * tr3);
  if (fabs(det) > thr) {
    double dx = r0 * c00 - a01 * (r1 * a22 - a12 * r2) + a02 * (r1 * a12 - a11 * r2);
    double dy = a00 * (r1 * a22 - a12 * r2) - r0 * c01 + a02 * (a01 * r2 - r1 * a02);
    double dz = a00 * (a11 * r2 - r1 * a12) - a01 * (a01 * r2 - r1 * a02) + r0 * c02;
    P3 v{dx / det, dy / det, dz / det};
    if (v.x >= lo.x && v.x <= hi.x && v.y >= lo.y && v.y <= hi.y && v.z >= lo.z && v.z <= hi.z) return v;
  }
  P3 mid{(ps.x + pr.x) * 0.5, (ps.y + pr.y) * 0.5, (ps.z + pr.z) * 0.5};
  P3 best = mid;
  double qb = quadric_eval(q, mid);
  double qs = quadric_eval(q, ps);
  if (qs < qb) {
    best = ps;
    qb = qs;
  }
  double qr = quadric_eval(q, pr);
  if (qr < qb) best = pr;
  return best;
}

__device__ __forceinline__ P3 corner_after(const MeshView& m, int f, int c, int s, int r, P3 vbar) {
  int v = m.F[3 * f + c];
  return (v == s || v == r) ? vbar : ld3(m.V, v);
}

// The stored star of v (n <= VSTAR slots) without the slots of faces x1 and
// x2: returns how many are left; c8 gets the first eight of them (logical
// slot i sits at physical slot i, i + 1 or i + 2), q1 < q2 the excluded
// physical slots (VSTAR when absent).  One 64-byte load.
__device__ __forceinline__ int star_compact8(const MeshView& m, int v, int n, int x1, int x2, int* c8, int& q1,
                                             int& q2) {
  const int4* s4 = reinterpret_cast<const int4*>(m.vstar + (int64_t)VSTAR * v);
  int raw[VSTAR];
#pragma unroll
  for (int q = 0; q < VSTAR / 4; q++) {
    const int4 x = s4[q];
    raw[4 * q] = x.x; raw[4 * q + 1] = x.y; raw[4 * q + 2] = x.z; raw[4 * q + 3] = x.w;
  }
  q1 = VSTAR;
  q2 = VSTAR;
  int cnt = n;
  if (x1 >= 0 || x2 >= 0) {
#pragma unroll
    for (int i = 0; i < VSTAR; i++) {
      const int f = raw[i] / 3;
      const bool ex = i < n && (f == x1 || f == x2);
      q2 = ex && q1 < VSTAR && q2 == VSTAR ? i : q2;
      q1 = ex && q1 == VSTAR ? i : q1;
    }
    cnt = n - (q1 < VSTAR) - (q2 < VSTAR);
  }
#pragma unroll
  for (int i = 0; i < 8; i++) c8[i] = i < q1 ? raw[i] : i + 1 < q2 ? raw[i + 1] : raw[i + 2];
  return cnt;
}

// logical slot i (>= 8) of the star of v: a reload of the slot
__device__ __forceinline__ int star_slot(const MeshView& m, int v, int i, int q1, int q2, bool use) {
  int phys = i;
  phys += phys >= q1;
  phys += phys >= q2;
  return m.vstar[(int64_t)VSTAR * v + (use ? phys : 0)];
}

// chunk j (four slots) of a compacted star
__device__ __forceinline__ void star_chunk(const MeshView& m, int v, int j, int cnt, const int* c8, int q1, int q2,
                                           int pad, int* g, bool* use) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int i = 4 * j + k;
    use[k] = i < cnt;
    const int e = j < 2 ? (j == 0 ? c8[k] : c8[4 + k]) : star_slot(m, v, i, q1, q2, use[k]);
    g[k] = use[k] ? e : pad;
  }
}

// The stored star of v (n <= VSTAR half-edges leaving v, ascending) without
// those in faces x1 and x2, four at a time: fn(g, use) gets four half-edges;
// slots past the end carry `pad` (a half-edge that is safe to read through)
// and use = false.  The excluded slots are located once in the star's 64-byte
// line and skipped, so the chunks are full (a valence-6 star around an edge is
// one chunk of four); the first two chunks come from the registers holding
// the line.  The callee issues its loads for all four before acting on any,
// so a star costs a few load latencies instead of one per face of a twin walk.
template <class Fn>
__device__ __forceinline__ void star_chunks(const MeshView& m, int v, int n, int x1, int x2, int pad, Fn fn) {
  int c8[8], q1, q2;
  const int cnt = star_compact8(m, v, n, x1, x2, c8, q1, q2);
  for (int j = 0; 4 * j < cnt; j++) {
    int g[4];
    bool use[4];
    star_chunk(m, v, j, cnt, c8, q1, q2, pad, g, use);
    fn(g, use);
  }
}

// The whole stored star of v in registers: g[i] for i < n, slot 0 beyond
// (n >= 1), one 64-byte load.
__device__ __forceinline__ void star_all(const MeshView& m, int v, int n, int* g) {
  const int4* st = reinterpret_cast<const int4*>(m.vstar + (int64_t)VSTAR * v);
  int raw[VSTAR];
#pragma unroll
  for (int q = 0; q < VSTAR / 4; q++) {
    const int4 x = st[q];
    raw[4 * q] = x.x; raw[4 * q + 1] = x.y; raw[4 * q + 2] = x.z; raw[4 * q + 3] = x.w;
  }
#pragma unroll
  for (int i = 0; i < VSTAR; i++) g[i] = i < n ? raw[i] : raw[0];
}

// both stars of an edge stored (inside a round, before the tentative apply)
__device__ __forceinline__ bool stars_stored(const MeshView& m, int s, int r, int& ns, int& nr) {
  if (!m.vstar) return false;
  ns = m.vdeg[s];
  nr = m.vdeg[r];
  return ns <= VSTAR && nr <= VSTAR;
}

// S plus the skinny terms of the faces of the stored star of v (E.fast), in
// slot order.  Four slots at a time, branch-free: every load of the four
// faces (corner ids, then corner positions) is issued before any arithmetic,
// slots past the star or holding the edge's faces read face f1 and add
// nothing.  Same terms in the same order as star_ascending.
__device__ __forceinline__ double skinny_sum_star(const MeshView& m, const EdgeStars& E, int v, int n, P3 vb,
                                                  double S) {
  star_chunks(m, v, n, E.f1, E.f2, E.hs, [&](const int* g, const bool* use) {
    // corner g % 3 of face g / 3 is v and moves to vb (no other corner is s
    // or r); only the other two corners are loaded
    P3 p[4][3];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int f = g[k] / 3, ci = g[k] - 3 * f;
      int c[3];
#pragma unroll
      for (int i = 0; i < 3; i++) c[i] = m.F[3 * (int64_t)f + i];
      const int c1 = ci == 2 ? 0 : ci + 1, c2 = ci == 0 ? 2 : ci - 1;
      const P3 q1 = ld3(m.V, c1 == 0 ? c[0] : c1 == 1 ? c[1] : c[2]);
      const P3 q2 = ld3(m.V, c2 == 0 ? c[0] : c2 == 1 ? c[1] : c[2]);
#pragma unroll
      for (int i = 0; i < 3; i++) p[k][i] = i == ci ? vb : i == c1 ? q1 : q2;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const double t = skinny_term(p[k][0], p[k][1], p[k][2]);
      S = use[k] ? S + t : S;
    }
  });
  return S;
}

// cost (Eq. 1) and placement of edge E; the skinny terms are summed over the
// faces around s, then those around r, each in ascending face slot
__device__ __forceinline__ double edge_cost(const MeshView& m, const double* __restrict__ Q, const EdgeStars& E,
                                            double w_e, double w_s, P3& vbar) {
  const int s = E.s, r = E.r;
  double q[10];
#pragma unroll
  for (int i = 0; i < 10; i++) q[i] = Q[10 * (int64_t)s + i] + Q[10 * (int64_t)r + i];
  P3 ps = ld3(m.V, s), pr = ld3(m.V, r);
  vbar = placement(q, ps, pr, E.lo, E.hi);
  double dx = ps.x - pr.x, dy = ps.y - pr.y, dz = ps.z - pr.z;
  double lab = sqrt(dx * dx + dy * dy + dz * dz);
  double S = 0.0;
  const P3 vb = vbar;
  if (E.fast) {
    S = skinny_sum_star(m, E, s, E.ns, vb, S);
    S = skinny_sum_star(m, E, r, E.nr, vb, S);
  } else {
    auto add = [&](int f) {
      S = S + skinny_term(corner_after(m, f, 0, s, r, vb), corner_after(m, f, 1, s, r, vb),
                          corner_after(m, f, 2, s, r, vb));
    };
    star_ascending(m, E, E.hs, add);
    star_ascending(m, E, E.hr, add);
  }
  return quadric_eval(q, vbar) + w_e * lab + w_s * S;
}

// the placement of edge E alone (the same arithmetic as edge_cost)
__device__ __forceinline__ P3 edge_placement(const MeshView& m, const double* __restrict__ Q, const EdgeStars& E) {
  double q[10];
#pragma unroll
  for (int i = 0; i < 10; i++) q[i] = Q[10 * (int64_t)E.s + i] + Q[10 * (int64_t)E.r + i];
  return placement(q, ld3(m.V, E.s), ld3(m.V, E.r), E.lo, E.hi);
}

// ------------------------------------------------------------ local checks
__device__ __forceinline__ bool degenerate(P3 a, P3 b, P3 c) {
  // certain nonzero in some projection -> not degenerate
  for (int k = 0; k < 3; k++) {
    int s = orient2d_filter(pu(a, k), pv(a, k), pu(b, k), pv(b, k), pu(c, k), pv(c, k));
    if (s != UNK) return false;
  }
  return degenerate_exact(a, b, c);
}

// link condition Lk(a) n Lk(b) = Lk(ab) on a closed manifold: the only
// common neighbours are the two apexes, and the edge is not inside a
// tetrahedron component (both endpoints of valence 3)
__device__ __forceinline__ bool link_ok(const MeshView& m, int h) {
  constexpr int CAP = 16;
  int na[CAP];
#pragma unroll
  for (int i = 0; i < CAP; i++) na[i] = -1;
  int vala = 0;
  walk_star(m.twin, h, [&](int g) {
    int w = dest(m.F, g);
#pragma unroll
    for (int i = 0; i < CAP; i++)
      if (i == vala) na[i] = w;
    vala++;
  });
  int valb = 0, common = 0;
  walk_star(m.twin, m.twin[h], [&](int g) {
    int w = dest(m.F, g);
    valb++;
    bool in = false;
    if (vala <= CAP) {
#pragma unroll
      for (int i = 0; i < CAP; i++) in |= na[i] == w;
    } else {
      walk_star(m.twin, h, [&](int g2) { in |= dest(m.F, g2) == w; });
    }
    common += in;
  });
  return common == 2 && !(vala == 3 && valb == 3);
}

// the same test from the stored stars: N(v) = far ends of the half-edges
// leaving v, each neighbour once.  In two parts, so that a caller can issue
// the loads and do other work before it needs the answer.
struct LinkStars {
  int na, nb;
  int wa[VSTAR], wb[VSTAR];
};

__device__ __forceinline__ void link_stars_load(const MeshView& m, int a, int na, int b, int nb, LinkStars& L) {
  int ga[VSTAR], gb[VSTAR];
  star_all(m, a, na, ga);
  star_all(m, b, nb, gb);
  L.na = na;
  L.nb = nb;
#pragma unroll
  for (int i = 0; i < VSTAR; i++) {
    L.wa[i] = m.F[he_next(ga[i])];
    L.wb[i] = m.F[he_next(gb[i])];
  }
}

__device__ __forceinline__ bool link_stars_holds(const LinkStars& L) {
  int common = 0;
#pragma unroll
  for (int j = 0; j < VSTAR; j++) {
    bool in = false;
#pragma unroll
    for (int i = 0; i < VSTAR; i++) in |= i < L.na && L.wa[i] == L.wb[j];
    common += j < L.nb && in;
  }
  return common == 2 && !(L.na == 3 && L.nb == 3);
}

__device__ __forceinline__ bool link_ok_stars(const MeshView& m, int a, int na, int b, int nb) {
  LinkStars L;
  link_stars_load(m, a, na, b, nb, L);
  return link_stars_holds(L);
}

// the link condition for the edge of h, from the stored stars when they fit
__device__ __forceinline__ bool link_holds(const MeshView& m, int h) {
  int na = 0, nb = 0;
  const int a0 = m.F[h], b0 = m.F[he_next(h)];
  const bool fast = stars_stored(m, a0, b0, na, nb);
  return fast ? link_ok_stars(m, a0, na, b0, nb) : link_ok(m, h);
}

// triangle o0 o1 o2 becomes p0 p1 p2: degenerate, or its normal turned by 90
// degrees or more
__device__ __forceinline__ bool turned(P3 o0, P3 o1, P3 o2, P3 p0, P3 p1, P3 p2) {
  if (degenerate(p0, p1, p2)) return true;
  double ax = o1.x - o0.x, ay = o1.y - o0.y, az = o1.z - o0.z;
  double bx = o2.x - o0.x, by = o2.y - o0.y, bz = o2.z - o0.z;
  double nox = ay * bz - az * by, noy = az * bx - ax * bz, noz = ax * by - ay * bx;
  double cx = p1.x - p0.x, cy = p1.y - p0.y, cz = p1.z - p0.z;
  double dx = p2.x - p0.x, dy = p2.y - p0.y, dz = p2.z - p0.z;
  double nnx = cy * dz - cz * dy, nny = cz * dx - cx * dz, nnz = cx * dy - cy * dx;
  double dot = nox * nnx + noy * nny + noz * nnz;
  return !(dot > 0.0);
}

// the same test with the filters alone: 1 turned (or degenerate with its
// normal not kept), 0 kept and certainly not degenerate, 2 undecided (every
// projection of p0 p1 p2 within the filter's error bound of zero)
__device__ __forceinline__ int turned_filter(P3 o0, P3 o1, P3 o2, P3 p0, P3 p1, P3 p2) {
  double ax = o1.x - o0.x, ay = o1.y - o0.y, az = o1.z - o0.z;
  double bx = o2.x - o0.x, by = o2.y - o0.y, bz = o2.z - o0.z;
  double nox = ay * bz - az * by, noy = az * bx - ax * bz, noz = ax * by - ay * bx;
  double cx = p1.x - p0.x, cy = p1.y - p0.y, cz = p1.z - p0.z;
  double dx = p2.x - p0.x, dy = p2.y - p0.y, dz = p2.z - p0.z;
  double nnx = cy * dz - cz * dy, nny = cz * dx - cx * dz, nnz = cx * dy - cy * dx;
  double dot = nox * nnx + noy * nny + noz * nnz;
  if (!(dot > 0.0)) return 1;
  for (int k = 0; k < 3; k++)
    if (orient2d_filter(pu(p0, k), pv(p0, k), pu(p1, k), pv(p1, k), pu(p2, k), pv(p2, k)) != UNK) return 0;
  return 2;
}

// the four faces of a chunk of the stored star around a vertex at pc (corner
// g % 3 of each is that vertex and moves to vbar; no other corner is s or r,
// and the other two are loaded).  Every load is issued before any test.
// `bad` is set when a face is turned; with EXACT the degeneracy test is exact,
// else its filters alone decide and `und` is set for a face they leave
// undecided.
template <bool EXACT>
__device__ __forceinline__ void flip_faces(const MeshView& m, const int* g, const bool* use, P3 pc, P3 vbar,
                                           bool& bad, bool& und) {
  constexpr int K = 4;
  P3 o[K][3];
  int ci[K];
  bool u[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int gk = g[k];
    u[k] = use[k];
    const int f = gk / 3;
    ci[k] = gk - 3 * f;
    int c[3];
#pragma unroll
    for (int i = 0; i < 3; i++) c[i] = m.F[3 * (int64_t)f + i];
    const int c1 = ci[k] == 2 ? 0 : ci[k] + 1, c2 = ci[k] == 0 ? 2 : ci[k] - 1;
    const P3 q1 = ld3(m.V, c1 == 0 ? c[0] : c1 == 1 ? c[1] : c[2]);
    const P3 q2 = ld3(m.V, c2 == 0 ? c[0] : c2 == 1 ? c[1] : c[2]);
#pragma unroll
    for (int i = 0; i < 3; i++) o[k][i] = i == ci[k] ? pc : i == c1 ? q1 : q2;
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    if (!u[k] || bad) continue;
    P3 p[3];
#pragma unroll
    for (int i = 0; i < 3; i++) p[i] = i == ci[k] ? vbar : o[k][i];
    if constexpr (EXACT) {
      bad = turned(o[k][0], o[k][1], o[k][2], p[0], p[1], p[2]);
    } else {
      const int t = turned_filter(o[k][0], o[k][1], o[k][2], p[0], p[1], p[2]);
      bad = t == 1;
      und |= t == 2;
    }
  }
}

// the flip test over both stored stars on the filters alone: 0 no face
// turned, 1 some face turned, 2 none certainly turned but some undecided
__device__ __forceinline__ int flipped_filter(const MeshView& m, const EdgeStars& E, P3 vbar) {
  bool bad = false, und = false;
  const P3 ps = ld3(m.V, E.s), pr = ld3(m.V, E.r);
  star_chunks(m, E.s, E.ns, E.f1, E.f2, E.hs,
              [&](const int* g, const bool* use) { flip_faces<false>(m, g, use, ps, vbar, bad, und); });
  star_chunks(m, E.r, E.nr, E.f1, E.f2, E.hs,
              [&](const int* g, const bool* use) { flip_faces<false>(m, g, use, pr, vbar, bad, und); });
  return bad ? 1 : und ? 2 : 0;
}

// some generated triangle (corners after the collapse to vbar) degenerate or
// with its normal turned by 90 degrees or more against the original
__device__ __forceinline__ bool flipped_after(const MeshView& m, const EdgeStars& E, P3 vbar) {
  const int s = E.s, r = E.r;
  bool bad = false, und = false;
  if (E.fast) {
    const P3 ps = ld3(m.V, s), pr = ld3(m.V, r);
    star_chunks(m, s, E.ns, E.f1, E.f2, E.hs,
                [&](const int* g, const bool* use) { flip_faces<true>(m, g, use, ps, vbar, bad, und); });
    star_chunks(m, r, E.nr, E.f1, E.f2, E.hs,
                [&](const int* g, const bool* use) { flip_faces<true>(m, g, use, pr, vbar, bad, und); });
  } else {
    auto chk = [&](int f) {
      if (bad) return;
      P3 o0 = ld3(m.V, m.F[3 * f]), o1 = ld3(m.V, m.F[3 * f + 1]), o2 = ld3(m.V, m.F[3 * f + 2]);
      bad = turned(o0, o1, o2, corner_after(m, f, 0, s, r, vbar), corner_after(m, f, 1, s, r, vbar),
                   corner_after(m, f, 2, s, r, vbar));
    };
    star_ascending(m, E, E.hs, chk);
    star_ascending(m, E, E.hr, chk);
  }
  return bad;
}

// R7 for the edge of h: 0 passes, 1 link condition, 2 a generated triangle
// degenerate or flipped; vbar gets the placement (when the link holds)
__device__ __forceinline__ uint8_t local_reason(const MeshView& m, const double* __restrict__ Q, double w_e,
                                                double w_s, int h, P3& vbar, int* err) {
  EdgeStars E;
  const bool ok = edge_stars(m, h, E);
  const P3 vb = edge_placement(m, Q, E);  // the cost itself is not needed here
  if (E.fast) {
    // the link test's loads are in flight while the flip test runs; a
    // candidate failing the link test keeps reason 1 and no placement
    LinkStars L;
    const bool a_is_s = m.F[h] == E.s;
    link_stars_load(m, a_is_s ? E.s : E.r, a_is_s ? E.ns : E.nr, a_is_s ? E.r : E.s, a_is_s ? E.nr : E.ns, L);
    const bool flipped = flipped_after(m, E, vb);
    if (!link_stars_holds(L)) return 1;
    vbar = vb;
    return flipped ? 2 : 0;
  }
  if (!link_holds(m, h)) return 1;
  if (!ok) set_err(err, PAMO_EBIT_RING);
  vbar = vb;
  return flipped_after(m, E, vb) ? 2 : 0;
}

// The local checks of one candidate split over LC = 2 consecutive lanes
// (stored stars only).  Both lanes load the edge, its stars and the placement
// (the same addresses, merged by the memory pipeline); lane `part` then
// compares half of b's neighbours against a's and tests the faces of one star
// (lane 0 the star of s, lane 1 that of r).  The pair sums the common
// neighbours and ORs the flip results: the same decisions as local_reason,
// with its two stars' chains of loads side by side.  (Four lanes, two faces
// of every chunk each, were no faster on single meshes and slower on
// batches.)  The
// degeneracy test runs on its filters only; a candidate that needs the exact
// test (or whose stars are not stored) gets REASON_LATE and is decided by
// local_reason in a second kernel, which keeps the exact arithmetic's
// registers and scratch out of this one.
constexpr int LC = 2;
constexpr uint8_t REASON_LATE = 5;

// common neighbours of a and b over the slots j of b's star with j % LC == part
__device__ __forceinline__ int link_common_part(const MeshView& m, int a, int na, int b, int nb, int part) {
  int ga[VSTAR];
  star_all(m, a, na, ga);
  int wa[VSTAR], wb[VSTAR / LC];
#pragma unroll
  for (int i = 0; i < VSTAR; i++) wa[i] = m.F[he_next(ga[i])];
#pragma unroll
  for (int q = 0; q < VSTAR / LC; q++) {
    const int j = LC * q + part;
    wb[q] = m.F[he_next(m.vstar[(int64_t)VSTAR * b + (j < nb ? j : 0)])];
  }
  int common = 0;
#pragma unroll
  for (int q = 0; q < VSTAR / LC; q++) {
    bool in = false;
#pragma unroll
    for (int i = 0; i < VSTAR; i++) in |= i < na && wa[i] == wb[q];
    common += LC * q + part < nb && in;
  }
  return common;
}

// the flip test over the faces of the star of s (part 0) or r (part 1), on
// the filters (0 none turned, 1 some face turned, 2 none certainly turned,
// some undecided)
__device__ __forceinline__ int flipped_part(const MeshView& m, const EdgeStars& E, P3 vbar, int part) {
  const bool on_s = part == 0;
  const int v = on_s ? E.s : E.r;
  const P3 pc = ld3(m.V, v);
  bool bad = false, und = false;
  star_chunks(m, v, on_s ? E.ns : E.nr, E.f1, E.f2, E.hs,
              [&](const int* g, const bool* use) { flip_faces<false>(m, g, use, pc, vbar, bad, und); });
  return bad ? 1 : und ? 2 : 0;
}

// ------------------------------------------------------------ cost + keys
// One thread per edge: each wave gathers the representative half-edges
// (h < twin h) of its PW consecutive half-edges into an LDS queue and then
// evaluates them with the lanes busy (one thread per half-edge would leave
// half the lanes idle).  PW = 256 (two edges per lane) on large meshes; on
// small ones PW = 64 (at most one edge per lane) puts four times as many waves
// on the chip, since there the latency of one lane's loads sets the time.
constexpr int64_t CK_SMALL_NH = 1 << 21;

// PRE: the link/flip pre-filter, an edge failing the local checks of R7 gets
// the largest key (from the placement just computed).  lex: the key is the
// float64 cost's order code (ranked afterwards).  Keys go to both half-edges;
// the vertex minima are gathered from them by the next kernel (no atomics).
template <int PW, bool PRE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRE ? 2 : 1))) void k_cost_keys(MeshView m, const double* __restrict__ Q, double w_e, double w_s,
                                                   double cost_max, const uint8_t* __restrict__ demote,
                                                   const uint8_t* __restrict__ mesh_done, uint64_t* __restrict__ key,
                                                   int* err, bool lex, int* __restrict__ late, int* __restrict__ nlate) {
  __shared__ int queue[4][PW];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nh = 3 * (int64_t)m.nf;
  const int64_t base = ((int64_t)xcd_block() * 4 + w) * PW;
  int count = 0;
#pragma unroll
  for (int j = 0; j < PW / 64; j++) {
    const int64_t h = base + 64 * j + lane;
    const bool rep = h < nh && h < m.twin[h];
    const unsigned long long b = __ballot(rep);
    if (rep) queue[w][count + __popcll(b & ((1ull << lane) - 1))] = (int)h;
    count += __popcll(b);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int i = lane; i < count; i += 64) {
    const int h = queue[w][i];
    const int t = m.twin[h];
    uint64_t k = PAMO_KEY_MAX;
    bool skip = m.flags[h] || m.flags[t] || (demote && (demote[h] || demote[t])) ||
                (mesh_done && mesh_done[m.fmesh[h / 3]]);
    if (!skip) {
      EdgeStars E;
      if (!edge_stars(m, h, E)) {
        set_err(err, PAMO_EBIT_RING);
      } else {
        P3 vbar;
        double cost = edge_cost(m, Q, E, w_e, w_s, vbar);
        k = cost > cost_max ? PAMO_KEY_MAX                                 // above the cost target: never chosen
            : lex        ? cost_code64(cost)
                         : make_key(cost, (uint32_t)h);
        if (PRE && k != PAMO_KEY_MAX) {
          // the flip test on its filters; an edge they leave undecided (or
          // whose stars are not stored) is listed for k_prefilter_late, which
          // keeps the exact arithmetic's registers out of this kernel
          const int fl = !link_holds(m, h) ? 1 : E.fast ? flipped_filter(m, E, vbar) : 2;
          if (fl == 1) k = PAMO_KEY_MAX;
          if (fl == 2) late[atomicAdd(nlate, 1)] = h;
        }
      }
    }
    key[h] = k;
    key[t] = k;
  }
}

// the listed edges of the pre-filter: the exact flip test, failing edges unkeyed
__global__ __launch_bounds__(256) void k_prefilter_late(MeshView m, const double* __restrict__ Q,
                                                        const int* __restrict__ late, const int* __restrict__ nlate,
                                                        uint64_t* __restrict__ key) {
  const int n = *nlate;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int h = late[i];
    EdgeStars E;
    edge_stars(m, h, E);
    if (flipped_after(m, E, edge_placement(m, Q, E))) {
      key[h] = PAMO_KEY_MAX;
      key[m.twin[h]] = PAMO_KEY_MAX;
    }
  }
}

// float64 key mode: the edges (by their lower half-edge, ascending) and their
// codes; a stable sort of the codes then gives each keyed edge its rank in the
// order of (float64 cost, edge id), stored in the high half of its key (the
// edge id below, so keys stay unique and the batch cap's high-half order holds)
__global__ void k_edge_flags(int nh, const int* __restrict__ twin, uint8_t* __restrict__ flag) {
  int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < nh) flag[h] = h < twin[h];
}

__global__ void k_gather_codes(int ne, const int* __restrict__ count, int* __restrict__ edges,
                               const uint64_t* __restrict__ key, uint64_t* __restrict__ codes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  if (i < *count) {
    codes[i] = key[edges[i]];
  } else {  // past the edges found (an open mesh has fewer): sorts last, ranks nothing
    codes[i] = PAMO_KEY_MAX;
    edges[i] = -1;
  }
}

__global__ void k_assign_ranks(int ne, const int* __restrict__ edges, const uint64_t* __restrict__ codes,
                               const int* __restrict__ twin, uint64_t* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne || codes[i] == PAMO_KEY_MAX) return;
  const int h = edges[i];
  const uint64_t k = ((uint64_t)i << 32) | (uint32_t)h;
  key[h] = k;
  key[twin[h]] = k;
}

// ------------------------------------------------------------ selection
// vmin[v]: smallest key of the edges at v (each is one half-edge leaving v)
__global__ __launch_bounds__(256) void k_vertex_min(MeshView m, const uint64_t* __restrict__ key,
                                                    uint64_t* __restrict__ vmin) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= m.nv) return;
  uint64_t best = PAMO_KEY_MAX;
  const int n = m.vstar ? m.vdeg[v] : VSTAR + 1;
  if (n <= VSTAR) {
    star_chunks(m, v, n, -1, -1, 0, [&](const int* g, const bool* use) {
      uint64_t k[4];
#pragma unroll
      for (int i = 0; i < 4; i++) k[i] = key[g[i]];
#pragma unroll
      for (int i = 0; i < 4; i++) best = use[i] && k[i] < best ? k[i] : best;
    });
  } else {
    walk_star(m.twin, m.vh[v], [&](int h) {
      uint64_t k = key[h];
      best = k < best ? k : best;
    });
  }
  vmin[v] = best;
}

// e = (a, b) is chosen iff its key is the minimum over the vertex minima of
// {a, b} u N(a) u N(b), i.e. no edge sharing a ring triangle has a smaller key
__device__ __forceinline__ uint8_t select_edge(const MeshView& m, const uint64_t* __restrict__ key,
                                               const uint64_t* __restrict__ vmin, int h) {
  uint8_t ok = 0;
  uint64_t k = key[h];
  if (k != PAMO_KEY_MAX && h < m.twin[h]) {
    int a = m.F[h], b = m.F[he_next(h)];
    if (vmin[a] == k && vmin[b] == k) {
      bool local_min = true;
      int na = 0, nb = 0;
      if (stars_stored(m, a, b, na, nb)) {
        // N(v): the far ends of the half-edges leaving v
        auto side = [&](int v, int n) {
          int g[VSTAR];
          star_all(m, v, n, g);
          int w[VSTAR];
#pragma unroll
          for (int i = 0; i < VSTAR; i++) w[i] = m.F[he_next(g[i])];
          uint64_t mw[VSTAR];
#pragma unroll
          for (int i = 0; i < VSTAR; i++) mw[i] = vmin[w[i]];
#pragma unroll
          for (int i = 0; i < VSTAR; i++) local_min = local_min && !(mw[i] < k);
        };
        side(a, na);
        side(b, nb);
      } else {
        auto nbr = [&](int g) {
          if (vmin[dest(m.F, g)] < k) local_min = false;
        };
        walk_star(m.twin, h, nbr);
        if (local_min) walk_star(m.twin, m.twin[h], nbr);
      }
      ok = local_min;
    }
  }
  return ok;
}

// A chosen edge holds the minimum key at both its ends, and a key carries its
// edge's lower half-edge in its low 32 bits: so each vertex tests the one edge
// its minimum names (from the edge's origin end only, once per edge), instead
// of every half-edge testing itself.  sel must be zero on entry.
constexpr int SELECT_PAIR_NV = 1 << 18;  // two lanes per vertex up to this many vertices

// SL = 2: two lanes per vertex; with stored stars, lane 0 gathers the
// neighbour minima around a, lane 1 those around b, and the pair ANDs the
// answers (shorter chains on small meshes; on large ones the second lane's
// loads cost more than they hide, and SL = 1 runs both sides on one lane).
template <int SL>
__global__ __launch_bounds__(256) void k_select(MeshView m, const uint64_t* __restrict__ key,
                                                const uint64_t* __restrict__ vmin, uint8_t* __restrict__ sel) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int v = (int)(t / SL), part = (int)(t % SL);
  if (v >= m.nv) return;  // every lane of the vertex
  const uint64_t k = vmin[v];
  if (k == PAMO_KEY_MAX) return;
  const int h = (int)(uint32_t)k;
  if (m.F[h] != v) return;  // the other end tests it
  if (key[h] != k || !(h < m.twin[h])) return;
  const int a = v, b = m.F[he_next(h)];
  if (vmin[b] != k) return;
  int na = 0, nb = 0;
  if (SL == 2 && stars_stored(m, a, b, na, nb)) {
    const int u = part ? b : a, n = part ? nb : na;
    int g[VSTAR];
    star_all(m, u, n, g);
    int w[VSTAR];
#pragma unroll
    for (int i = 0; i < VSTAR; i++) w[i] = m.F[he_next(g[i])];
    uint64_t mw[VSTAR];
#pragma unroll
    for (int i = 0; i < VSTAR; i++) mw[i] = vmin[w[i]];
    int low = 1;
#pragma unroll
    for (int i = 0; i < VSTAR; i++) low = low && !(mw[i] < k);
    low &= __shfl_xor(low, 1);
    if (part == 0 && low) sel[h] = 1;
  } else if (part == 0 && select_edge(m, key, vmin, h)) {
    sel[h] = 1;
  }
}

// Re-selection after candidates were set aside (both half-edges of each got
// the largest key).  A set-aside edge (a, b) changes only the vertex minima
// of a and b, so a selection changes only for edges with an endpoint u in
// {a, b} u N(a) u N(b), and such an edge can be chosen only if its key is
// vmin[u]: each such u has one edge to evaluate again, the one its minimum
// names (a key carries its edge's lower half-edge in the low 32 bits).  Every
// other edge keeps its flag of the selection before (candidates' closed
// neighbourhoods hold no endpoint of another candidate,
// so no two set-aside edges share a vertex either).  Work items run
// grid-stride over the list of set-aside edges: two per edge for the minima,
// 2 + 2 VSTAR per edge for the re-evaluation (its two ends, then the far end
// of each stored half-edge leaving them; the ends of larger stars walk their
// neighbours themselves).
__global__ __launch_bounds__(256) void k_demoted_vmin(MeshView m, const uint64_t* __restrict__ key,
                                                      const int* __restrict__ dlist, const int* __restrict__ nd,
                                                      uint64_t* __restrict__ vmin, uint8_t* __restrict__ sel) {
  const int64_t n = 2 * (int64_t)*nd;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int h = dlist[i >> 1];
    const int v = (i & 1) ? m.F[he_next(h)] : m.F[h];
    if (!(i & 1)) sel[h] = 0;
    uint64_t best = PAMO_KEY_MAX;
    const int deg = m.vdeg[v];
    if (deg <= VSTAR) {
      int g[VSTAR];
      star_all(m, v, deg, g);
      uint64_t k[VSTAR];
#pragma unroll
      for (int q = 0; q < VSTAR; q++) k[q] = key[g[q]];
#pragma unroll
      for (int q = 0; q < VSTAR; q++) best = k[q] < best ? k[q] : best;
    } else {
      walk_star(m.twin, m.vh[v], [&](int g) {
        const uint64_t k = key[g];
        best = k < best ? k : best;
      });
    }
    vmin[v] = best;
  }
}

constexpr int RESEL_ITEMS = 2 + 2 * VSTAR;

__global__ __launch_bounds__(256) void k_reselect(MeshView m, const uint64_t* __restrict__ key,
                                                  const int* __restrict__ dlist, const int* __restrict__ nd,
                                                  const uint64_t* __restrict__ vmin, uint8_t* __restrict__ sel) {
  const int64_t n = RESEL_ITEMS * (int64_t)*nd;
  auto again = [&](int u) {  // the edge holding u's minimum: the key's low 32 bits
    const uint64_t k = vmin[u];
    if (k == PAMO_KEY_MAX) return;
    const int e = (int)(uint32_t)k;
    sel[e] = select_edge(m, key, vmin, e);
  };
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int h = dlist[i / RESEL_ITEMS];
    const int j = (int)(i % RESEL_ITEMS);
    const int end = j < 2 ? j : (j - 2) / VSTAR;  // 0: a, 1: b
    const int v = end ? m.F[he_next(h)] : m.F[h];
    const int deg = m.vdeg[v];
    if (j < 2) {
      again(v);
      if (deg > VSTAR) walk_star(m.twin, m.vh[v], [&](int g) { again(dest(m.F, g)); });
    } else {
      const int slot = (j - 2) % VSTAR;
      if (deg <= VSTAR && slot < deg) again(dest(m.F, m.vstar[(int64_t)VSTAR * v + slot]));
    }
  }
}

__global__ __launch_bounds__(256) void k_local_check(MeshView m, const double* __restrict__ Q, double w_e,
                                                     double w_s, const int* __restrict__ cand,
                                                     const int* __restrict__ ncand, const uint64_t* __restrict__ key,
                                                     uint8_t* __restrict__ reason, double* __restrict__ vbar_out,
                                                     uint64_t* __restrict__ ckey, int* err, int* __restrict__ hist) {
  int64_t ce;  // XCD-contiguous ranges of the candidate list, LC lanes per candidate
  const int c = (int)xcd_item(*ncand, blockDim.x / LC, threadIdx.x / LC, &ce);
  const int part = threadIdx.x % LC;
  if (c >= ce) return;  // the whole group
  const int h = cand[c];
  P3 vbar{0, 0, 0};
  uint8_t rs = 0;
  EdgeStars E;
  edge_stars(m, h, E);
  if (E.fast) {  // uniform over the group
    const P3 vb = edge_placement(m, Q, E);
    const bool a_is_s = m.F[h] == E.s;
    const int na = a_is_s ? E.ns : E.nr, nb = a_is_s ? E.nr : E.ns;
    int common = link_common_part(m, a_is_s ? E.s : E.r, na, a_is_s ? E.r : E.s, nb, part);
    const int fl = flipped_part(m, E, vb, part);
    int bad = fl == 1, und = fl == 2;
#pragma unroll
    for (int o = 1; o < LC; o <<= 1) {
      common += __shfl_xor(common, o);
      bad |= __shfl_xor(bad, o);
      und |= __shfl_xor(und, o);
    }
    // a candidate failing the link test keeps reason 1 and no placement
    const bool link = common == 2 && !(na == 3 && nb == 3);
    rs = !link ? 1 : bad ? 2 : und ? REASON_LATE : 0;
    if (link) vbar = vb;
  } else {
    rs = REASON_LATE;
  }
  if (part == 0) {
    ckey[c] = key[h];
    reason[c] = rs;
    vbar_out[3 * (int64_t)c] = vbar.x;
    vbar_out[3 * (int64_t)c + 1] = vbar.y;
    vbar_out[3 * (int64_t)c + 2] = vbar.z;
  }
  wave_hist(part == 0 ? rs : -1, hist);
}

// the candidates left to the exact tests (REASON_LATE), one lane each
__global__ __launch_bounds__(256) void k_local_late(MeshView m, const double* __restrict__ Q, double w_e, double w_s,
                                                    const int* __restrict__ cand, const int* __restrict__ ncand,
                                                    uint8_t* __restrict__ reason, double* __restrict__ vbar_out,
                                                    int* err, int* __restrict__ hist) {
  int64_t ce;
  const int c = (int)xcd_item(*ncand, blockDim.x, threadIdx.x, &ce);
  if (c >= ce) return;
  int rs = -1;
  if (reason[c] == REASON_LATE) {
    P3 vbar{0, 0, 0};
    rs = local_reason(m, Q, w_e, w_s, cand[c], vbar, err);
    reason[c] = rs;
    vbar_out[3 * (int64_t)c] = vbar.x;
    vbar_out[3 * (int64_t)c + 1] = vbar.y;
    vbar_out[3 * (int64_t)c + 2] = vbar.z;
  }
  wave_hist(rs, hist);
}

// candidates passing the local checks whose key exceeds the threshold are
// capped (exact face target)
__global__ void k_cap(const int* __restrict__ ncand, const uint64_t* __restrict__ ckey, const uint64_t* __restrict__ thr,
                      uint8_t* __restrict__ reason) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= *ncand) return;
  if (reason[c] == 0 && ckey[c] > *thr) reason[c] = 4;
}

__global__ void k_pass_keys(const int* __restrict__ ncand, const uint64_t* __restrict__ ckey,
                            const uint8_t* __restrict__ reason, uint64_t* __restrict__ out, int* __restrict__ idx) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= *ncand) return;
  out[c] = reason[c] == 0 ? ckey[c] : PAMO_KEY_MAX;
  idx[c] = c;
}

__global__ void k_pick(const uint64_t* __restrict__ sorted, int64_t k, uint64_t* __restrict__ thr) { *thr = sorted[k]; }

// ------------------------------------------------------------ boxes
__device__ __forceinline__ float f_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
__device__ __forceinline__ float f_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

// float32 box of face f, rounded outward (shifted to its mesh's cell in a batch)
__device__ __forceinline__ void face_box_f32(const MeshView& m, int f, float* b) {
  P3 p0 = ld3(m.V, m.F[3 * f]), p1 = ld3(m.V, m.F[3 * f + 1]), p2 = ld3(m.V, m.F[3 * f + 2]);
  double ox = 0, oy = 0, oz = 0;
  if (m.fmesh) mesh_shift(m.fmesh[f], ox, oy, oz);
  b[0] = f_down(fmin(fmin(p0.x, p1.x), p2.x) + ox);
  b[1] = f_down(fmin(fmin(p0.y, p1.y), p2.y) + oy);
  b[2] = f_down(fmin(fmin(p0.z, p1.z), p2.z) + oz);
  b[3] = f_up(fmax(fmax(p0.x, p1.x), p2.x) + ox);
  b[4] = f_up(fmax(fmax(p0.y, p1.y), p2.y) + oy);
  b[5] = f_up(fmax(fmax(p0.z, p1.z), p2.z) + oz);
}

__global__ __launch_bounds__(256) void k_face_boxes(MeshView m, float* __restrict__ box) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= m.nf) return;
  float b[6];
  face_box_f32(m, f, b);
#pragma unroll
  for (int i = 0; i < 6; i++) box[6 * (int64_t)f + i] = b[i];
}

// ------------------------------------------------------------ apply / undo
// Tentatively collapse every candidate with reason 0: the merged vertex keeps
// the smaller id s and moves to vbar, corners of the larger id r are
// relabelled s, the two faces of the edge die.  Faces of star(a) u star(b)
// get owner = candidate; their boxes grow to cover the new geometry too.
// Two lanes per candidate: with stored stars each takes one side of the edge.
constexpr int AP = 2;
__global__ __launch_bounds__(256) void k_apply(MeshView m, const int* __restrict__ cand, const int* __restrict__ ncand,
                                               const uint8_t* __restrict__ reason, const double* __restrict__ vbar,
                                               double* __restrict__ oldpos, int* __restrict__ owner,
                                               uint8_t* __restrict__ falive, float* __restrict__ box) {
  int64_t ce;  // XCD-contiguous ranges of the candidate list, AP lanes per candidate
  const int c = (int)xcd_item(*ncand, blockDim.x / AP, threadIdx.x / AP, &ce);
  const int part = threadIdx.x % AP;
  if (c >= ce || reason[c] != 0) return;
  int h = cand[c];
  int t = m.twin[h];
  int a = m.F[h], b = m.F[he_next(h)];
  int s = a < b ? a : b, r = a < b ? b : a;
  int hr = a == r ? h : t;  // leaves r
  int f1 = h / 3, f2 = t / 3;
  int ns = 0, nr = 0;
  const P3 vb{vbar[3 * (int64_t)c], vbar[3 * (int64_t)c + 1], vbar[3 * (int64_t)c + 2]};
  const bool fast = stars_stored(m, s, r, ns, nr);
  if (fast) {
    // from the stored stars: ownership, relabelling r -> s and the grown
    // boxes, four faces at a time (the corners read are the pre-apply ones,
    // mapped r -> s and placed at vbar where they are s)
    double ox = 0, oy = 0, oz = 0;
    if (m.fmesh) mesh_shift(m.fmesh[f1], ox, oy, oz);
    auto side = [&](const int* g, const bool* use, bool relabel) {
      int f[4];
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = g[k] / 3;
      // corner g % 3 of the face is s or r and moves to vbar; no other
      // corner is s or r; the other two are loaded
      P3 p[4][3];
      float ob[4][6];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int ci = g[k] - 3 * f[k];
        int c[3];
#pragma unroll
        for (int i = 0; i < 3; i++) c[i] = m.F[3 * (int64_t)f[k] + i];
        const int c1 = ci == 2 ? 0 : ci + 1, c2 = ci == 0 ? 2 : ci - 1;
        const P3 q1 = ld3(m.V, c1 == 0 ? c[0] : c1 == 1 ? c[1] : c[2]);
        const P3 q2 = ld3(m.V, c2 == 0 ? c[0] : c2 == 1 ? c[1] : c[2]);
#pragma unroll
        for (int i = 0; i < 3; i++) p[k][i] = i == ci ? vb : i == c1 ? q1 : q2;
#pragma unroll
        for (int i = 0; i < 6; i++) ob[k][i] = box[6 * (int64_t)f[k] + i];
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (!use[k]) continue;
        owner[f[k]] = c;
        if (relabel) m.F[g[k]] = s;  // the corner of r in this face
        float* bx = box + 6 * (int64_t)f[k];
        bx[0] = fminf(ob[k][0], f_down(fmin(fmin(p[k][0].x, p[k][1].x), p[k][2].x) + ox));
        bx[1] = fminf(ob[k][1], f_down(fmin(fmin(p[k][0].y, p[k][1].y), p[k][2].y) + oy));
        bx[2] = fminf(ob[k][2], f_down(fmin(fmin(p[k][0].z, p[k][1].z), p[k][2].z) + oz));
        bx[3] = fmaxf(ob[k][3], f_up(fmax(fmax(p[k][0].x, p[k][1].x), p[k][2].x) + ox));
        bx[4] = fmaxf(ob[k][4], f_up(fmax(fmax(p[k][0].y, p[k][1].y), p[k][2].y) + oy));
        bx[5] = fmaxf(ob[k][5], f_up(fmax(fmax(p[k][0].z, p[k][1].z), p[k][2].z) + oz));
      }
    };
    // lane 0 the faces around s, lane 1 those around r (relabelled): the two
    // sets are disjoint, and neither reads a position the other writes
    const bool on_r = part == 1;
    star_chunks(m, on_r ? r : s, on_r ? nr : ns, f1, f2, h,
                [&](const int* g, const bool* use) { side(g, use, on_r); });
    if (on_r) return;
    owner[f1] = c;
    owner[f2] = c;
  } else if (part == 1) {
    return;
  } else {
    auto own = [&](int g) { owner[g / 3] = c; };
    walk_star(m.twin, h, own);
    walk_star(m.twin, t, own);
    walk_star(m.twin, hr, [&](int g) {
      int f = g / 3;
      if (f != f1 && f != f2) m.F[g] = s;  // corner g % 3 of face f held r
    });
  }
  for (int k = 0; k < 3; k++) oldpos[3 * (int64_t)c + k] = m.V[3 * (int64_t)s + k];
  m.V[3 * (int64_t)s] = vb.x;
  m.V[3 * (int64_t)s + 1] = vb.y;
  m.V[3 * (int64_t)s + 2] = vb.z;
  falive[f1] = 0;
  falive[f2] = 0;
  if (fast) return;
  // union boxes of the faces around s (now the merged vertex)
  int hs = a == s ? h : t;
  auto grow = [&](int g) {
    int f = g / 3;
    if (f == f1 || f == f2) return;
    float nb[6];
    face_box_f32(m, f, nb);
    float* bx = box + 6 * (int64_t)f;
    bx[0] = fminf(bx[0], nb[0]); bx[1] = fminf(bx[1], nb[1]); bx[2] = fminf(bx[2], nb[2]);
    bx[3] = fmaxf(bx[3], nb[3]); bx[4] = fmaxf(bx[4], nb[4]); bx[5] = fmaxf(bx[5], nb[5]);
  };
  walk_star(m.twin, hs, grow);
  walk_star(m.twin, hr, grow);
}

// undo the collapses marked in check iteration `iter`
__global__ __launch_bounds__(256) void k_undo(MeshView m, const int* __restrict__ cand, const int* __restrict__ ncand,
                                              const int* __restrict__ undone, int iter,
                                              const double* __restrict__ oldpos, uint8_t* __restrict__ falive) {
  int64_t ce;  // XCD-contiguous ranges of the candidate list
  const int c = (int)xcd_item(*ncand, blockDim.x, threadIdx.x, &ce);
  if (c >= ce || undone[c] != iter) return;
  int h = cand[c];
  int t = m.twin[h];
  int a = m.F[h], b = m.F[he_next(h)];
  // corners of f1 = h/3 and f2 = t/3 were never relabelled, so a, b are the
  // original endpoints
  int s = a < b ? a : b, r = a < b ? b : a;
  int hr = a == r ? h : t;
  int f1 = h / 3, f2 = t / 3;
  int ns, nr;
  if (stars_stored(m, s, r, ns, nr)) {
    star_chunks(m, r, nr, f1, f2, h, [&](const int* g, const bool* use) {
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (use[k]) m.F[g[k]] = r;
    });
  } else {
    walk_star(m.twin, hr, [&](int g) {
      int f = g / 3;
      if (f != f1 && f != f2) m.F[g] = r;
    });
  }
  for (int k = 0; k < 3; k++) m.V[3 * (int64_t)s + k] = oldpos[3 * (int64_t)c + k];
  falive[f1] = 1;
  falive[f2] = 1;
}

__global__ void k_changed_faces(int nf, const int* __restrict__ owner, const uint8_t* __restrict__ falive,
                                const int* __restrict__ undone, int iter, const int* __restrict__ order,
                                uint8_t* __restrict__ pred) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nf) return;
  int f = order ? order[j] : j;
  int o = owner[f];
  uint8_t p = 0;
  if (o >= 0) {
    if (iter == 0)
      p = falive[f];  // faces changed by an applied collapse
    else
      p = undone[o] == iter;  // faces restored by the undo of iteration iter
  }
  pred[j] = p;
}

// ------------------------------------------------------------ commit
// Make the surviving collapses permanent: rewire the twins across the two
// removed faces, fix the leaving half-edges of the merged vertex and the two
// apexes, retire r.  Undone candidates get reason 3.
__global__ __launch_bounds__(256) void k_commit(MeshView m, const int* __restrict__ cand, const int* __restrict__ ncand,
                                                uint8_t* __restrict__ reason, const int* __restrict__ undone,
                                                uint8_t* __restrict__ valive, GateIn gin) {
  if (gin.flag) {
    const bool shut = *gin.nundo > 0 || *gin.ncandp > gin.cap || *gin.err != 0 || (gin.npass && *gin.npass == 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *gin.flag = shut ? 1 : 0;
    if (shut) return;
  }
  int64_t ce;  // XCD-contiguous ranges of the candidate list
  const int c = (int)xcd_item(*ncand, blockDim.x, threadIdx.x, &ce);
  if (c >= ce || reason[c] != 0) return;
  if (undone[c]) {
    reason[c] = 3;
    return;
  }
  int h1 = cand[c];
  int h2 = m.twin[h1];
  int a = m.F[h1], b = m.F[he_next(h1)];
  int r = a < b ? b : a;
  int o1 = m.twin[he_next(h1)];  // x -> b
  int o2 = m.twin[he_prev(h1)];  // a -> x
  int o3 = m.twin[he_next(h2)];  // y -> a
  int o4 = m.twin[he_prev(h2)];  // b -> y
  m.twin[o1] = o2;
  m.twin[o2] = o1;
  m.twin[o3] = o4;
  m.twin[o4] = o3;
  int s = a < b ? a : b;
  m.vh[s] = o2;            // leaves the merged vertex
  m.vh[m.F[o1]] = o1;      // leaves x
  m.vh[m.F[o3]] = o3;      // leaves y
  valive[r] = 0;
}

__global__ void k_flags(MeshView m, const int* __restrict__ cand, const int* __restrict__ ncand,
                        const uint8_t* __restrict__ reason, int* __restrict__ hist, const int* __restrict__ gate) {
  if (gate && *gate) return;
  int64_t ce;  // XCD-contiguous ranges of the candidate list
  const int c = (int)xcd_item(*ncand, blockDim.x, threadIdx.x, &ce);
  if (c >= ce) return;
  uint8_t rs = reason[c];
  if (rs >= 1 && rs <= 3) {
    int h = cand[c];
    m.flags[h] = 1;
    m.flags[m.twin[h]] = 1;
  }
  if (hist) wave_hist(rs, hist);
}

__global__ void k_reason_hist(const int* __restrict__ ncand, const uint8_t* __restrict__ reason, int* __restrict__ hist) {
  __shared__ int local[8];
  if (threadIdx.x < 8) local[threadIdx.x] = 0;
  __syncthreads();
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < *ncand) atomicAdd(&local[reason[c] & 7], 1);
  __syncthreads();
  if (threadIdx.x < 8 && local[threadIdx.x]) atomicAdd(&hist[threadIdx.x], local[threadIdx.x]);
}

// ------------------------------------------------------------ compaction
__device__ __forceinline__ void compact_face(MeshView src, MeshView dst, const uint8_t* __restrict__ falive,
                                                     const int* __restrict__ fmap, const int* __restrict__ vmap,
                                                     int* err, const int* __restrict__ gate,
                                                     uint8_t* __restrict__ sel) {
  if (gate && *gate) return;
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= src.nf || !falive[f]) return;
  int g = fmap[f];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    int h = 3 * f + k;
    int v = vmap[src.F[h]];
    int t = src.twin[h];
    int tf = t >= 0 ? fmap[t / 3] : -1;
    if (v < 0 || tf < 0) {  // a live face pointing at a removed vertex or face
      atomicOr(err, PAMO_EBIT_RING);
      v = 0;
      tf = g;
    }
    dst.F[3 * g + k] = v;
    dst.twin[3 * g + k] = 3 * tf + (t >= 0 ? t % 3 : k);
    dst.flags[3 * g + k] = src.flags[h];
    if (sel) sel[3 * g + k] = 0;  // the next round's selection flags start cleared
  }
  if (src.fmesh) dst.fmesh[g] = src.fmesh[f];
  if (src.ovl) dst.ovl[g] = src.ovl[f];
}

__device__ __forceinline__ void compact_vertex(MeshView src, MeshView dst, const uint8_t* __restrict__ valive,
                                                     const int* __restrict__ vmap, const int* __restrict__ fmap,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= src.nv || !valive[v]) return;
  int w = vmap[v];
  for (int k = 0; k < 3; k++) dst.V[3 * (int64_t)w + k] = src.V[3 * (int64_t)v + k];
  int h = src.vh[v];
  dst.vh[w] = 3 * fmap[h / 3] + h % 3;
  if (src.vmesh) dst.vmesh[w] = src.vmesh[v];
}

// faces and vertices in one launch (thread i compacts face i and vertex i);
// ord (optional): the surviving faces in leaf order, old ids -> new ids
__global__ void k_compact(MeshView src, MeshView dst, const uint8_t* __restrict__ falive,
                          const uint8_t* __restrict__ valive, const int* __restrict__ fmap,
                          const int* __restrict__ vmap, int* err, const int* __restrict__ gate, int* __restrict__ ord,
                          const int* __restrict__ nord, uint8_t* __restrict__ sel) {
  compact_face(src, dst, falive, fmap, vmap, err, gate, sel);
  compact_vertex(src, dst, valive, vmap, fmap, gate);
  if (ord && !(gate && *gate)) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *nord) ord[i] = fmap[ord[i]];
  }
}

__global__ void k_remap_order(const int* __restrict__ order, int n, const uint8_t* __restrict__ falive,
                              const int* __restrict__ fmap, int* __restrict__ tmp, uint8_t* __restrict__ pred) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int f = order[j];
  bool keep = falive[f] != 0;
  tmp[j] = keep ? fmap[f] : -1;
  pred[j] = keep;
}

__global__ void k_clear_u8(uint8_t* __restrict__ p, int64_t n, const int* __restrict__ gate) {
  if (gate && *gate) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_flags_or(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] |= src[i];
}

// faces changed by a committed collapse take the overlap count measured on
// the round's tentative mesh
__global__ void k_ovl_commit(int nf, const int* __restrict__ owner, const uint8_t* __restrict__ falive,
                             const int* __restrict__ undone, const int* __restrict__ ovl_new, int* __restrict__ ovl,
                             const int* __restrict__ gate) {
  if (gate && *gate) return;
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf || !falive[f]) return;
  int o = owner[f];
  if (o >= 0 && undone[o] == 0) ovl[f] = ovl_new[f];
}

// state of a round's check/undo loop: every face alive and unowned with its
// box, nothing undone, every vertex alive
__global__ void k_round_prep(MeshView m, float* __restrict__ box, uint8_t* __restrict__ falive,
                             int* __restrict__ owner, int ncand, int* __restrict__ undone,
                             uint8_t* __restrict__ valive) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m.nf) {
    falive[i] = 1;
    owner[i] = -1;
    if (box) face_box_f32(m, i, box + 6 * (int64_t)i);
  }
  if (i < ncand) undone[i] = 0;
  if (i < m.nv && valive) valive[i] = 1;
}

// state of a check/undo loop: every face alive and unowned, nothing undone
__global__ void k_check_reset(int nf, uint8_t* __restrict__ falive, int* __restrict__ owner, int ncand,
                              int* __restrict__ undone) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) {
    falive[i] = 1;
    owner[i] = -1;
  }
  if (i < ncand) undone[i] = 0;
}

// ------------------------------------------------------------ batches
__global__ void k_mesh_tally(const int* __restrict__ cand, const int* __restrict__ ncand, const int* __restrict__ fmesh,
                             const uint8_t* __restrict__ reason_local, const uint8_t* __restrict__ reason_final,
                             const int* __restrict__ undone, int* ncand_m, int* npass_m, int* commits_m, int* hist_m,
                             int* undo_m, const int* __restrict__ gate) {
  if (gate && *gate) return;
  // Candidates are sorted by half-edge and meshes occupy contiguous face
  // ranges, so the lanes of a wave nearly always share one mesh: the counts
  // are reduced per (wave, mesh) and added with one atomic each (one atomic
  // per candidate on the same few counters serialised the kernel).
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = c < *ncand;
  const int m = valid ? fmesh[cand[c] / 3] : -1;
  const bool pass = valid && reason_local && reason_local[c] == 0;
  const int r = valid && reason_final ? (reason_final[c] & 7) : -1;
  if (valid && undo_m && undone && undone[c]) atomicMax(&undo_m[m], undone[c]);  // rare
  unsigned long long left = __ballot(valid);
  while (left) {
    const int leader = __ffsll((long long)left) - 1;
    const int mm = __shfl(m, leader, 64);
    const unsigned long long same = __ballot(valid && m == mm);
    const int nc = __popcll(same);
    const int np = __popcll(__ballot(pass && m == mm));
    int hv = 0;
    if (hist_m || commits_m) {
      // lane k (< 8) takes the count of reason k
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const int ck = __popcll(__ballot(r == k && m == mm));
        hv = lane == k ? ck : hv;
      }
    }
    if (lane == leader) {
      if (ncand_m) atomicAdd(&ncand_m[mm], nc);
      if (npass_m && np) atomicAdd(&npass_m[mm], np);
    }
    const int c0 = __shfl(hv, 0, 64);
    if (lane == leader && commits_m && reason_final && c0) atomicAdd(&commits_m[mm], c0);
    if (hist_m && reason_final && lane < 8 && hv) atomicAdd(&hist_m[8 * mm + lane], hv);
    left &= ~same;
  }
}

// candidates sorted by (mesh, key, index): rank inside the mesh's segment
__global__ void k_cap_batch(const int* __restrict__ ncand, const int* __restrict__ sidx, const int* __restrict__ cand,
                            const int* __restrict__ fmesh, const int* __restrict__ seg, const int* __restrict__ need_m,
                            uint8_t* __restrict__ reason) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *ncand) return;
  int c = sidx[p];
  int m = fmesh[cand[c] / 3];
  if (reason[c] == 0 && p - seg[m] >= need_m[m]) reason[c] = 4;
}

// sort key of a candidate for the per-mesh cap: (mesh, cost), passing
// candidates before the others; a stable sort keeps ascending candidate index
// (= ascending edge id) among equal costs, as the single-mesh key does
__global__ void k_cap_batch_keys(const int* __restrict__ ncand, const int* __restrict__ cand,
                                 const int* __restrict__ fmesh, const uint64_t* __restrict__ ckey,
                                 const uint8_t* __restrict__ reason, uint64_t* __restrict__ out,
                                 int* __restrict__ idx) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= *ncand) return;
  uint64_t cost = reason[c] == 0 ? (ckey[c] >> 32) : (1ull << 32);
  uint64_t m = (uint64_t)fmesh[cand[c] / 3];
  out[c] = (m << 33) | cost;
  idx[c] = c;
}

__global__ void k_flags_clear_batch(MeshView m, const int* __restrict__ commits_m, const int* __restrict__ gate) {
  if (gate && *gate) return;
  int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 3 * m.nf) return;
  if (commits_m[m.fmesh[h / 3]] > 0) m.flags[h] = 0;
}

__device__ __forceinline__ int seg_of(const int* __restrict__ off, int nmesh, int i) {
  int lo = 0, hi = nmesh - 1;  // largest m with off[m] <= i
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void k_batch_ids(const int* __restrict__ f_off, const int* __restrict__ v_off, int nmesh, int nf, int nv,
                            int* __restrict__ F, int* __restrict__ fmesh, int* __restrict__ vmesh, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) {
    int m = seg_of(f_off, nmesh, i);
    fmesh[i] = m;
    int o = v_off[m], nvm = v_off[m + 1] - o;
    for (int k = 0; k < 3; k++) {
      int l = F[3 * i + k];
      if (l < 0 || l >= nvm) atomicOr(err, PAMO_EBIT_INDEX);
      F[3 * i + k] = l + o;
    }
  }
  if (i < nv) vmesh[i] = seg_of(v_off, nmesh, i);
}

// per-mesh face and vertex offsets after a compaction, from the exclusive
// prefix counts of the surviving faces and vertices (one launch for both)
__global__ void k_batch_offsets2(const int* __restrict__ fexcl, const int* __restrict__ ftotal, int nf,
                                 int* __restrict__ f_off, const int* __restrict__ vexcl,
                                 const int* __restrict__ vtotal, int nv, int* __restrict__ v_off, int nmesh,
                                 const int* __restrict__ gate) {
  if (gate && *gate) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= nmesh) {
    const int o = f_off[i];
    f_off[i] = o >= nf ? *ftotal : fexcl[o];
  } else if (i <= 2 * nmesh + 1) {
    const int m = i - nmesh - 1;
    const int o = v_off[m];
    v_off[m] = o >= nv ? *vtotal : vexcl[o];
  }
}

__global__ void k_batch_offsets(const int* __restrict__ excl, const int* __restrict__ total, int* __restrict__ off,
                                int nmesh, int n) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > nmesh) return;
  int o = off[m];
  off[m] = o >= n ? *total : excl[o];
}

__global__ void k_batch_output(MeshView mv, const int* __restrict__ f_off, const int* __restrict__ v_off,
                               const int* __restrict__ f_out_off, const int* __restrict__ v_out_off, int nmesh,
                               double* __restrict__ V_out, int* __restrict__ F_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < mv.nf) {
    int m = mv.fmesh[i];
    int lf = i - f_off[m];
    for (int k = 0; k < 3; k++) F_out[3 * (int64_t)(f_out_off[m] + lf) + k] = mv.F[3 * i + k] - v_off[m];
  }
  if (i < mv.nv) {
    int m = mv.vmesh[i];
    int lv = i - v_off[m];
    for (int k = 0; k < 3; k++) V_out[3 * (int64_t)(v_out_off[m] + lv) + k] = mv.V[3 * (int64_t)i + k];
  }
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }
// grids for xcd_item: a multiple of 8 blocks
inline unsigned nblk8(int64_t n, int t = 256) { return (nblk(n, t) + 7u) & ~7u; }

}  // namespace

// ============================================================ host wrappers
void round_reserve(Workspace& ws, int64_t nv, int64_t nf, int64_t ncand, int nmesh, bool key_mode) {
  const int64_t nh = 3 * nf;
  ws.get<uint64_t>("adj.keys", nh);
  ws.get<int>("adj.vals", nh);
  ws.get<int>("adj.deg", nv);
  ws.get<uint8_t>("sel", nh);
  ws.get<uint64_t>("cap.keys", ncand);
  ws.get<int>("cap.idx", ncand);
  ws.get<uint64_t>("cap.thr", 1);
  ws.get<uint8_t>("qpred", nf);
  ws.get<int>("cmp.fmap", nf);
  ws.get<int>("cmp.vmap", nv);
  ws.get<int>("cmp.fexcl", nf);
  ws.get<int>("cmp.vexcl", nv);
  ws.get<int>("ord.tmp", nf);
  ws.get<uint8_t>("ord.pred", nf);
  if (nmesh > 1) {
    ws.get<uint64_t>("capb.keys", ncand);
    ws.get<int>("capb.idx", ncand);
    ws.get<int>("capb.seg", nmesh + 1);
    ws.get<int>("bo.excl", std::max(nf, nv));
    ws.get<int>("bo.total", 1);
  }
  if (key_mode) {
    const int64_t ne = nh / 2;
    ws.get<uint8_t>("rk.flag", nh);
    ws.get<int>("rk.edges", ne + 1);
    ws.get<int>("rk.count", 1);
    ws.get<uint64_t>("rk.codes", ne + 1);
  }
}

void launch_adjacency(Workspace& ws, hipStream_t s, MeshView m, int* err) {
  int64_t nh = 3 * (int64_t)m.nf;
  uint64_t* keys = ws.get<uint64_t>("adj.keys", nh);
  int* vals = ws.get<int>("adj.vals", nh);
  int* deg = ws.get<int>("adj.deg", m.nv);
  int bits = 1;
  while ((1ll << bits) < m.nv) bits++;
  hipLaunchKernelGGL(k_he_keys, dim3(nblk(nh)), dim3(256), 0, s, (const int*)m.F, m.nf, m.nv, bits, keys, vals, err);
  radix_sort_u64(ws, s, keys, vals, nh, 2 * bits);
  fill_i32(s, m.twin, nh, -1);
  hipLaunchKernelGGL(k_pair_twins, dim3(nblk(nh)), dim3(256), 0, s, (const uint64_t*)keys, (const int*)vals, (int)nh,
                     (const int*)m.F, m.twin, err);
  fill_i32(s, deg, m.nv, 0);
  hipLaunchKernelGGL(k_vertex_he, dim3(nblk(nh)), dim3(256), 0, s, (const int*)m.F, m.nf, m.vh, deg);
  PAMO_HIP(hipGetLastError());
}

void launch_check_vertices(Workspace& ws, hipStream_t s, MeshView m, int* err) {
  int* deg = ws.get<int>("adj.deg", m.nv);
  hipLaunchKernelGGL(k_check_vertices, dim3(nblk(m.nv)), dim3(256), 0, s, (const int*)m.twin, (const int*)m.vh,
                     (const int*)deg, m.nv, err);
  PAMO_HIP(hipGetLastError());
}

void launch_quadrics(hipStream_t s, MeshView m, double* Q, int* err) {
  hipLaunchKernelGGL(k_quadrics, dim3(nblk(m.nv)), dim3(256), 0, s, m, Q, err);
  PAMO_HIP(hipGetLastError());
}

void launch_cost_keys(Workspace& ws, hipStream_t s, MeshView m, const double* Q, double w_e, double w_s,
                      const uint8_t* demote, const uint8_t* mesh_done, uint64_t* key, int* err, double cost_target,
                      bool prefilter, bool lex) {
  const int64_t nh = 3 * (int64_t)m.nf;
  const double cost_max = cost_target > 0 ? cost_target : INFINITY;
  int* late = nullptr;
  int* nlate = nullptr;
  if (prefilter) {  // at most one entry per edge
    late = ws.get<int>("ck.late", nh / 2 + 1);
    nlate = ws.get<int>("ck.nlate", 1);
    fill_i32(s, nlate, 1, 0);
  }
  auto go = [&](auto kern, int pw) {
    hipLaunchKernelGGL(kern, dim3(nblk(nh, 4 * pw)), dim3(256), 0, s, m, Q, w_e, w_s, cost_max, demote, mesh_done,
                       key, err, lex, late, nlate);
  };
  if (nh <= CK_SMALL_NH)
    prefilter ? go(k_cost_keys<64, true>, 64) : go(k_cost_keys<64, false>, 64);
  else
    prefilter ? go(k_cost_keys<256, true>, 256) : go(k_cost_keys<256, false>, 256);
  if (prefilter)
    hipLaunchKernelGGL(k_prefilter_late, dim3(16), dim3(256), 0, s, m, Q, (const int*)late, (const int*)nlate, key);
  PAMO_HIP(hipGetLastError());
}

void launch_rank_keys(Workspace& ws, hipStream_t s, MeshView m, uint64_t* key) {
  const int64_t nh = 3 * (int64_t)m.nf;
  const int64_t ne = nh / 2;  // every edge of a closed mesh has two half-edges
  uint8_t* flag = ws.get<uint8_t>("rk.flag", nh);
  int* edges = ws.get<int>("rk.edges", ne + 1);
  int* count = ws.get<int>("rk.count", 1);
  uint64_t* codes = ws.get<uint64_t>("rk.codes", ne + 1);
  hipLaunchKernelGGL(k_edge_flags, dim3(nblk(nh)), dim3(256), 0, s, (int)nh, (const int*)m.twin, flag);
  compact_flags(ws, s, flag, nh, edges, count);
  hipLaunchKernelGGL(k_gather_codes, dim3(nblk(ne)), dim3(256), 0, s, (int)ne, (const int*)count, edges,
                     (const uint64_t*)key, codes);
  radix_sort_u64(ws, s, codes, edges, ne, 64);  // stable: equal codes keep ascending edge id
  hipLaunchKernelGGL(k_assign_ranks, dim3(nblk(ne)), dim3(256), 0, s, (int)ne, (const int*)edges,
                     (const uint64_t*)codes, (const int*)m.twin, key);
  PAMO_HIP(hipGetLastError());
}

void launch_select(Workspace& ws, hipStream_t s, MeshView m, const uint64_t* key, uint64_t* vmin, int* cand,
                   int* ncand, bool sel_clear) {
  int64_t nh = 3 * (int64_t)m.nf;
  uint8_t* sel = ws.get<uint8_t>("sel", nh);
  hipLaunchKernelGGL(k_vertex_min, dim3(nblk(m.nv)), dim3(256), 0, s, m, key, vmin);
  if (!sel_clear) fill_u8(s, sel, nh, 0);
  if (m.nv <= SELECT_PAIR_NV)
    hipLaunchKernelGGL(k_select<2>, dim3(nblk(2 * (int64_t)m.nv)), dim3(256), 0, s, m, key, (const uint64_t*)vmin,
                       sel);
  else
    hipLaunchKernelGGL(k_select<1>, dim3(nblk(m.nv)), dim3(256), 0, s, m, key, (const uint64_t*)vmin, sel);
  compact_flags(ws, s, sel, nh, cand, ncand);
  PAMO_HIP(hipGetLastError());
}

void launch_reselect(Workspace& ws, hipStream_t s, MeshView m, const uint64_t* key, uint64_t* vmin, const int* dlist,
                     const int* nd, int bound, int* cand, int* ncand) {
  int64_t nh = 3 * (int64_t)m.nf;
  uint8_t* sel = ws.get<uint8_t>("sel", nh);  // the flags of the selection before
  const unsigned g1 = std::min(nblk(2 * (int64_t)bound), 1024u);
  const unsigned g2 = std::min(nblk(RESEL_ITEMS * (int64_t)bound), 2048u);
  hipLaunchKernelGGL(k_demoted_vmin, dim3(g1), dim3(256), 0, s, m, key, dlist, nd, vmin, sel);
  hipLaunchKernelGGL(k_reselect, dim3(g2), dim3(256), 0, s, m, key, dlist, nd, (const uint64_t*)vmin, sel);
  compact_flags(ws, s, sel, nh, cand, ncand);
  PAMO_HIP(hipGetLastError());
}

void launch_local_check(hipStream_t s, MeshView m, const double* Q, double w_e, double w_s, const int* cand,
                        const int* ncand, int cand_bound, const uint64_t* key, uint8_t* reason, double* vbar,
                        uint64_t* ckey, int* err, int* hist) {
  hipLaunchKernelGGL(k_local_check, dim3(nblk8((int64_t)cand_bound * LC)), dim3(256), 0, s, m, Q, w_e, w_s, cand,
                     ncand, key, reason, vbar, ckey, err, hist);
  hipLaunchKernelGGL(k_local_late, dim3(nblk8(cand_bound)), dim3(256), 0, s, m, Q, w_e, w_s, cand, ncand, reason, vbar,
                     err, hist);
  PAMO_HIP(hipGetLastError());
}

void launch_cap(Workspace& ws, hipStream_t s, const int* ncand, int nc_host, const uint64_t* ckey, uint8_t* reason,
                int64_t need) {
  uint64_t* k = ws.get<uint64_t>("cap.keys", nc_host);
  int* idx = ws.get<int>("cap.idx", nc_host);
  uint64_t* thr = ws.get<uint64_t>("cap.thr", 1);
  hipLaunchKernelGGL(k_pass_keys, dim3(nblk(nc_host)), dim3(256), 0, s, ncand, ckey, (const uint8_t*)reason, k, idx);
  radix_sort_u64(ws, s, k, idx, nc_host, 64);
  hipLaunchKernelGGL(k_pick, dim3(1), dim3(1), 0, s, (const uint64_t*)k, need - 1, thr);
  hipLaunchKernelGGL(k_cap, dim3(nblk(nc_host)), dim3(256), 0, s, ncand, ckey, (const uint64_t*)thr, reason);
  PAMO_HIP(hipGetLastError());
}

void launch_face_boxes(hipStream_t s, MeshView m, float* box) {
  hipLaunchKernelGGL(k_face_boxes, dim3(nblk(m.nf)), dim3(256), 0, s, m, box);
  PAMO_HIP(hipGetLastError());
}

void launch_apply(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, const uint8_t* reason,
                  const double* vbar, double* oldpos, int* owner, uint8_t* falive, float* box) {
  // one-wave blocks: the candidates' serial gathers spread over more CUs
  hipLaunchKernelGGL(k_apply, dim3(nblk8((int64_t)cand_bound * AP, 64)), dim3(64), 0, s, m, cand, ncand, reason,
                     vbar, oldpos, owner, falive, box);
  PAMO_HIP(hipGetLastError());
}

void launch_undo(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, const int* undone,
                 int iter, const double* oldpos, uint8_t* falive) {
  hipLaunchKernelGGL(k_undo, dim3(nblk8(cand_bound)), dim3(256), 0, s, m, cand, ncand, undone, iter, oldpos, falive);
  PAMO_HIP(hipGetLastError());
}

void launch_face_list(Workspace& ws, hipStream_t s, int nf, const int* owner, const uint8_t* falive,
                      const int* undone, int iter, const int* order, int* list, int* count) {
  uint8_t* pred = ws.get<uint8_t>("qpred", nf);
  hipLaunchKernelGGL(k_changed_faces, dim3(nblk(nf)), dim3(256), 0, s, nf, owner, falive, undone, iter, order, pred);
  if (order)
    compact_flags_map(ws, s, pred, nf, order, list, count);
  else
    compact_flags(ws, s, pred, nf, list, count);
  PAMO_HIP(hipGetLastError());
}

void launch_commit(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, uint8_t* reason,
                   const int* undone, uint8_t* valive, GateIn gin) {
  hipLaunchKernelGGL(k_commit, dim3(nblk8(cand_bound, 64)), dim3(64), 0, s, m, cand, ncand, reason, undone, valive,
                     gin);  // one-wave blocks, as k_apply
  PAMO_HIP(hipGetLastError());
}

void launch_flags(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound,
                  const uint8_t* reason, int* hist, const int* gate) {
  hipLaunchKernelGGL(k_flags, dim3(nblk8(cand_bound)), dim3(256), 0, s, m, cand, ncand, reason, hist, gate);
  PAMO_HIP(hipGetLastError());
}

void launch_clear_u8(hipStream_t s, uint8_t* p, int64_t n, const int* gate) {
  if (n <= 0) return;
  int64_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_clear_u8, dim3((unsigned)(b > 65536 ? 65536 : b)), dim3(256), 0, s, p, n, gate);
  PAMO_HIP(hipGetLastError());
}

void launch_reason_hist(hipStream_t s, const int* ncand, int cand_bound, const uint8_t* reason, int* hist) {
  hipLaunchKernelGGL(k_reason_hist, dim3(nblk(cand_bound)), dim3(256), 0, s, ncand, reason, hist);
  PAMO_HIP(hipGetLastError());
}

void launch_compact(Workspace& ws, hipStream_t s, MeshView src, MeshView dst, const uint8_t* falive,
                    const uint8_t* valive, int* nf_new, int* nv_new, int* err, const int* gate, const int* order,
                    int* order_out, int* nord, int* f_off, int* v_off, int nmesh, uint8_t* sel) {
  int* fmap = ws.get<int>("cmp.fmap", src.nf);
  int* vmap = ws.get<int>("cmp.vmap", src.nv);
  // face ranks, vertex ranks and the surviving faces in leaf order in one
  // scan (the order segment up to 1,024 tiles of 4,096; beyond, on its own);
  // batches also take the exclusive counts for their per-mesh offsets
  const bool fuse = order && src.nf <= 1024ll * 4096;
  FlagSegment sg[3];
  sg[0].flag = falive; sg[0].n = src.nf; sg[0].rank = fmap; sg[0].total = nf_new;
  sg[1].flag = valive; sg[1].n = src.nv; sg[1].rank = vmap; sg[1].total = nv_new;
  if (f_off) {
    sg[0].excl = ws.get<int>("cmp.fexcl", src.nf);
    sg[1].excl = ws.get<int>("cmp.vexcl", src.nv);
  }
  if (fuse) {
    sg[2].flag = falive; sg[2].gather = order; sg[2].n = src.nf; sg[2].list = order_out; sg[2].total = nord;
  }
  rank_segments(ws, s, sg, fuse ? 3 : 2);
  hipLaunchKernelGGL(k_compact, dim3(nblk(src.nf > src.nv ? src.nf : src.nv)), dim3(256), 0, s, src, dst, falive,
                     valive, (const int*)fmap, (const int*)vmap, err, gate, fuse ? order_out : nullptr,
                     (const int*)nord, sel);
  if (f_off)
    hipLaunchKernelGGL(k_batch_offsets2, dim3(nblk(2 * (int64_t)nmesh + 2)), dim3(256), 0, s, (const int*)sg[0].excl,
                       (const int*)nf_new, src.nf, f_off, (const int*)sg[1].excl, (const int*)nv_new, src.nv, v_off,
                       nmesh, gate);
  PAMO_HIP(hipGetLastError());
  if (order && !fuse) launch_remap_order(ws, s, order, src.nf, falive, fmap, order_out, nord);
}

void launch_remap_order(Workspace& ws, hipStream_t s, const int* order, int nf_old, const uint8_t* falive,
                        const int* fmap, int* out, int* count) {
  int* tmp = ws.get<int>("ord.tmp", nf_old);
  uint8_t* pred = ws.get<uint8_t>("ord.pred", nf_old);
  hipLaunchKernelGGL(k_remap_order, dim3(nblk(nf_old)), dim3(256), 0, s, order, nf_old, falive, fmap, tmp, pred);
  compact_flags_map(ws, s, pred, nf_old, tmp, out, count);
  PAMO_HIP(hipGetLastError());
}

void launch_ovl_commit(hipStream_t s, int nf, const int* owner, const uint8_t* falive, const int* undone,
                       const int* ovl_new, int* ovl, const int* gate) {
  hipLaunchKernelGGL(k_ovl_commit, dim3(nblk(nf)), dim3(256), 0, s, nf, owner, falive, undone, ovl_new, ovl, gate);
  PAMO_HIP(hipGetLastError());
}

void launch_round_prep(hipStream_t s, MeshView m, float* box, uint8_t* falive, int* owner, int ncand, int* undone,
                       uint8_t* valive) {
  int n = m.nf > ncand ? m.nf : ncand;
  n = n > m.nv ? n : m.nv;
  hipLaunchKernelGGL(k_round_prep, dim3(nblk(n)), dim3(256), 0, s, m, box, falive, owner, ncand, undone, valive);
  PAMO_HIP(hipGetLastError());
}

void launch_check_reset(hipStream_t s, int nf, uint8_t* falive, int* owner, int ncand, int* undone) {
  int n = nf > ncand ? nf : ncand;
  hipLaunchKernelGGL(k_check_reset, dim3(nblk(n)), dim3(256), 0, s, nf, falive, owner, ncand, undone);
  PAMO_HIP(hipGetLastError());
}

void launch_mesh_tally(hipStream_t s, const int* cand, const int* ncand, int bound, const int* fmesh,
                       const uint8_t* reason_local, const uint8_t* reason_final, const int* undone, int* ncand_m,
                       int* npass_m, int* commits_m, int* hist_m, int* undo_m, const int* gate) {
  hipLaunchKernelGGL(k_mesh_tally, dim3(nblk(bound)), dim3(256), 0, s, cand, ncand, fmesh, reason_local, reason_final,
                     undone, ncand_m, npass_m, commits_m, hist_m, undo_m, gate);
  PAMO_HIP(hipGetLastError());
}

void launch_cap_batch(Workspace& ws, hipStream_t s, const int* ncand, int nc_host, const int* cand,
                      const int* fmesh, const uint64_t* ckey, uint8_t* reason, const int* need_m,
                      const int* ncand_m, int nmesh) {
  int mbits = 1;
  while ((1ll << mbits) < nmesh) mbits++;
  uint64_t* k = ws.get<uint64_t>("capb.keys", nc_host);
  int* idx = ws.get<int>("capb.idx", nc_host);
  int* seg = ws.get<int>("capb.seg", nmesh + 1);
  hipLaunchKernelGGL(k_cap_batch_keys, dim3(nblk(nc_host)), dim3(256), 0, s, ncand, cand, fmesh, ckey,
                     (const uint8_t*)reason, k, idx);
  radix_sort_u64(ws, s, k, idx, nc_host, 33 + mbits);
  scan_exclusive(ws, s, ncand_m, seg, nmesh, nullptr);
  hipLaunchKernelGGL(k_cap_batch, dim3(nblk(nc_host)), dim3(256), 0, s, ncand, (const int*)idx, cand, fmesh,
                     (const int*)seg, need_m, reason);
  PAMO_HIP(hipGetLastError());
}

void launch_flags_clear_batch(hipStream_t s, MeshView m, const int* commits_m, const int* gate) {
  hipLaunchKernelGGL(k_flags_clear_batch, dim3(nblk(3 * (int64_t)m.nf)), dim3(256), 0, s, m, commits_m, gate);
  PAMO_HIP(hipGetLastError());
}

void launch_batch_ids(hipStream_t s, const int* f_off, const int* v_off, int nmesh, int nf, int nv, int* F,
                      int* fmesh, int* vmesh, int* err) {
  int n = nf > nv ? nf : nv;
  hipLaunchKernelGGL(k_batch_ids, dim3(nblk(n)), dim3(256), 0, s, f_off, v_off, nmesh, nf, nv, F, fmesh, vmesh, err);
  PAMO_HIP(hipGetLastError());
}

void launch_batch_offsets(Workspace& ws, hipStream_t s, const uint8_t* alive, int n, int* off, int nmesh) {
  int* excl = ws.get<int>("bo.excl", n);
  int* total = ws.get<int>("bo.total", 1);
  run_flag_scan(ws, s, alive, n, excl, total);
  hipLaunchKernelGGL(k_batch_offsets, dim3(nblk(nmesh + 1)), dim3(256), 0, s, (const int*)excl, (const int*)total, off,
                     nmesh, n);
  PAMO_HIP(hipGetLastError());
}

void launch_batch_output(hipStream_t s, MeshView m, const int* f_off, const int* v_off, const int* f_out_off,
                         const int* v_out_off, int nmesh, double* V_out, int* F_out) {
  int n = m.nf > m.nv ? m.nf : m.nv;
  hipLaunchKernelGGL(k_batch_output, dim3(nblk(n)), dim3(256), 0, s, m, f_off, v_off, f_out_off, v_out_off, nmesh,
                     V_out, F_out);
  PAMO_HIP(hipGetLastError());
}

void launch_flags_or(hipStream_t s, uint8_t* dst, const uint8_t* src, int64_t n) {
  hipLaunchKernelGGL(k_flags_or, dim3(nblk(n)), dim3(256), 0, s, dst, src, n);
  PAMO_HIP(hipGetLastError());
}

}  // namespace pamo
