// The remeshing stage's volume-to-mesh step (Sec. 4.2): Dual Marching Cubes on
// a grid of float64 values, with the manifold fix for ambiguous faces shared by
// two cubes.
//
// Grid point (i, j, k) holds s = S[(i r + j) r + k] - iso and sits at
// ((i + 1/2) / r, (j + 1/2) / r, (k + 1/2) / r); it is positive when s >= 0.
// Cube (i, j, k) spans the points (i..i+1, j..j+1, k..k+1); corner c has bit 0
// for +x, bit 1 for +y, bit 2 for +z.  Cube edge 4 a + u + 2 v runs along axis
// a, u and v being its coordinates on the other two axes, lower axis first.
//
// Patches: per face, the crossed edges are joined where the surface crosses
// the face: two crossed edges are joined to each other; on an ambiguous face
// (four crossed edges) the two edges at each positive corner are joined, or,
// when the face is flipped, the two at each negative corner.  The connected
// sets of crossed edges are the cube's patches, numbered by their smallest
// edge.  A face shared by two cubes is flipped (in both) when each cube,
// unflipped, has one patch holding all four of its edges: that pair of
// patches would otherwise be joined by four quads along one dual edge.
//
// Vertices: one per patch, the mean of its edges' crossing points (summed in
// ascending edge order), numbered by cube (x outermost), then patch.  The
// crossing sits at the fraction t = s0 / (s0 - s1) of the edge, or, with
// beta > 0, at 1 / (1 + exp(-beta (t - 1/2))) (Appendix 2.1).
// Quads: one per crossed grid edge whose four neighbouring cubes exist,
// ordered by axis then grid point; its vertices go counter-clockwise round
// the axis seen from the axis's positive side, reversed when the lower end is
// positive, so the normal points to the positive side.
//
// Quad division by the envelope of the grid edge (Appendix 2.1): with p+ and
// p- the edge's positive and negative ends and l, r the quad neighbours of
// vertex v, v is concave when (v - p+) . ((l - p+) x (r - p+)) < 0 or
// (v - p-) . ((l - p-) x (r - p-)) > 0.  Concave vertices on one diagonal
// only: the split along it; on both: four triangles around an extra vertex at
// the edge's crossing point (numbered after the patch vertices, in quad
// order); none: the split whose smallest angle is larger (through the first
// vertex on a tie).
//
// Kernels: one thread per grid point (sign byte); one per cube (configuration,
// crossed or not); one per grid point (its three edges: crossed and interior
// or not); compactions of the crossed cubes and of the crossed edges; one
// thread per crossed cube (flips, patches), a scan of their patch counts, one
// per crossed cube (positions, into scratch); one per crossed edge (its
// division), a scan of the four-triangle quads; then the positions copied
// out and one thread per crossed edge (extra vertex, triangles).  The patch
// structure of a cube is found once, by a small union-find, and kept as two
// bits per edge.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "remesh.hpp"

namespace pamo {
namespace {

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

struct DGrid {
  const double* S;
  int r;
  double iso;
  double beta;  // > 0: smoothed crossing fraction
};

__device__ __forceinline__ double gval(const DGrid& g, int i, int j, int k) {
  return g.S[((int64_t)i * g.r + j) * g.r + k] - g.iso;
}

// the sign of every grid point (1: s >= 0), one byte each
__global__ void k_dmc_sign(DGrid g, uint8_t* __restrict__ sg) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x < (int64_t)g.r * g.r * g.r) sg[x] = g.S[x] - g.iso >= 0.0 ? 1 : 0;
}

__device__ __forceinline__ uint32_t cube_config(const uint8_t* sg, int r, int i, int j, int k) {
  uint32_t c = 0;
  for (int b = 0; b < 8; b++)
    c |= (uint32_t)sg[((int64_t)(i + (b & 1)) * r + j + ((b >> 1) & 1)) * r + k + ((b >> 2) & 1)] << b;
  return c;
}

// the two axes other than a, lower first
__device__ __forceinline__ int lo_axis(int a) { return a == 0 ? 1 : 0; }
__device__ __forceinline__ int hi_axis(int a) { return a == 2 ? 1 : 2; }

// id of the cube edge along axis a whose lower corner is c0
__device__ __forceinline__ int edge_of(int a, int c0) {
  return 4 * a + ((c0 >> lo_axis(a)) & 1) + 2 * ((c0 >> hi_axis(a)) & 1);
}

// lower corner of cube edge e
__device__ __forceinline__ int edge_corner(int e) {
  const int a = e >> 2;
  return ((e & 1) << lo_axis(a)) | (((e >> 1) & 1) << hi_axis(a));
}

// corners of face (a, w) in cyclic order and the edge from corner t to t + 1
__device__ __forceinline__ void face_ring(int a, int w, int c[4], int ed[4]) {
  const int p = lo_axis(a), q = hi_axis(a);
  c[0] = w << a;
  c[1] = c[0] | (1 << p);
  c[2] = c[1] | (1 << q);
  c[3] = c[0] | (1 << q);
  ed[0] = edge_of(p, c[0]);
  ed[1] = edge_of(q, c[1]);
  ed[2] = edge_of(p, c[3]);
  ed[3] = edge_of(q, c[0]);
}

__device__ __forceinline__ int root(const int* par, int x) {
  while (par[x] != x) x = par[x];
  return x;
}

__device__ __forceinline__ void join(int* par, int x, int y) {
  x = root(par, x);
  y = root(par, y);
  if (x != y) par[x > y ? x : y] = x < y ? x : y;
}

// patch of each cube edge (-1: not crossed); returns the number of patches
__device__ int cube_patches(uint32_t cfg, uint32_t flips, int pid[12]) {
  int par[12];
  for (int e = 0; e < 12; e++) par[e] = e;
  for (int f = 0; f < 6; f++) {
    int c[4], ed[4];
    face_ring(f >> 1, f & 1, c, ed);
    int nx = 0, x0 = -1, x1 = -1;
    for (int t = 0; t < 4; t++) {
      if (((cfg >> c[t]) & 1) != ((cfg >> c[(t + 1) & 3]) & 1)) {
        nx++;
        if (x0 < 0)
          x0 = ed[t];
        else
          x1 = ed[t];
      }
    }
    if (nx == 2) {
      join(par, x0, x1);
    } else if (nx == 4) {
      const uint32_t side = (flips >> f) & 1 ? 0u : 1u;
      for (int t = 0; t < 4; t++)
        if (((cfg >> c[t]) & 1) == side) join(par, ed[(t + 3) & 3], ed[t]);  // the edges meeting at corner t
    }
  }
  int label[12];
  for (int e = 0; e < 12; e++) label[e] = -1;
  int n = 0;
  for (int e = 0; e < 12; e++) {
    const int c0 = edge_corner(e), c1 = c0 | (1 << (e >> 2));
    if (((cfg >> c0) & 1) == ((cfg >> c1) & 1)) {
      pid[e] = -1;
      continue;
    }
    const int rt = root(par, e);
    if (label[rt] < 0) label[rt] = n++;
    pid[e] = label[rt];
  }
  return n;
}

// one unflipped patch holds all four edges of face f
__device__ bool holds_face(uint32_t cfg, int f) {
  int c[4], ed[4];
  face_ring(f >> 1, f & 1, c, ed);
  for (int t = 0; t < 4; t++)
    if (((cfg >> c[t]) & 1) == ((cfg >> c[(t + 1) & 3]) & 1)) return false;
  int pid[12];
  cube_patches(cfg, 0, pid);
  return pid[ed[0]] == pid[ed[1]] && pid[ed[0]] == pid[ed[2]] && pid[ed[0]] == pid[ed[3]];
}

// per cube: its configuration, and whether the surface crosses it
__global__ void k_dmc_active(const uint8_t* __restrict__ sg, int r, uint8_t* __restrict__ cfgs,
                             uint8_t* __restrict__ act) {
  const int m = r - 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m * m) return;
  const int k = idx % m, j = idx / m % m, i = idx / (m * m);
  const uint32_t cfg = cube_config(sg, r, i, j, k);
  cfgs[idx] = (uint8_t)cfg;
  act[idx] = cfg != 0 && cfg != 255;
}

// per crossed cube (ascending list): the number of patches and, in pmap, the
// patch of each crossed edge e in bits 2e..2e+1 (a cube has at most four
// patches: each is a cycle of at least three of the twelve edges)
__global__ void k_dmc_cubes(const uint8_t* __restrict__ cfgs, int m, const int32_t* __restrict__ clist, int nc,
                            uint32_t* __restrict__ pmap, int32_t* __restrict__ cntl) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int64_t idx = clist[q];
  const int k = (int)(idx % m), j = (int)(idx / m % m), i = (int)(idx / ((int64_t)m * m));
  const uint32_t cfg = cfgs[idx];
  uint32_t flips = 0;
  for (int f = 0; f < 6; f++) {
    const int a = f >> 1, w = f & 1;
    int n[3] = {i, j, k};
    n[a] += w ? 1 : -1;
    if (n[a] < 0 || n[a] > m - 1) continue;
    if (holds_face(cfg, f) && holds_face(cfgs[((int64_t)n[0] * m + n[1]) * m + n[2]], f ^ 1)) flips |= 1u << f;
  }
  int pid[12];
  cntl[q] = cube_patches(cfg, flips, pid);
  uint32_t pm = 0;
  for (int e = 0; e < 12; e++)
    if (pid[e] > 0) pm |= (uint32_t)pid[e] << (2 * e);
  pmap[idx] = pm;
}

__global__ void k_dmc_verts(DGrid g, const uint8_t* __restrict__ cfgs, const int32_t* __restrict__ clist, int nc,
                            const uint32_t* __restrict__ pmap, const int32_t* __restrict__ cntl,
                            const int32_t* __restrict__ vbl, int32_t* __restrict__ vbase, double* __restrict__ V) {
  const int m = g.r - 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int64_t idx = clist[q];
  const int np = cntl[q];
  const int k = (int)(idx % m), j = (int)(idx / m % m), i = (int)(idx / ((int64_t)m * m));
  const uint32_t cfg = cfgs[idx], pm = pmap[idx];
  double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0}, sz[4] = {0, 0, 0, 0};
  int ne[4] = {0, 0, 0, 0};
  const double rr = (double)g.r;
  for (int e = 0; e < 12; e++) {
    const int a = e >> 2, c0 = edge_corner(e);
    if (((cfg >> c0) & 1) == ((cfg >> (c0 | (1 << a))) & 1)) continue;
    const int p = (pm >> (2 * e)) & 3;
    const int i0 = i + (c0 & 1), j0 = j + ((c0 >> 1) & 1), k0 = k + ((c0 >> 2) & 1);
    const double s0 = gval(g, i0, j0, k0);
    const double s1 = gval(g, i0 + (a == 0), j0 + (a == 1), k0 + (a == 2));
    double t = s0 / (s0 - s1);
    if (g.beta > 0.0) t = 1.0 / (1.0 + exp(-g.beta * (t - 0.5)));
    double q[3] = {(double)i0 + 0.5, (double)j0 + 0.5, (double)k0 + 0.5};
    q[a] = q[a] + t;
    sx[p] += q[0] / rr;
    sy[p] += q[1] / rr;
    sz[p] += q[2] / rr;
    ne[p]++;
  }
  const int64_t b = vbl[q];
  vbase[idx] = (int32_t)b;
  for (int p = 0; p < np; p++) {
    V[(b + p) * 3 + 0] = sx[p] / (double)ne[p];
    V[(b + p) * 3 + 1] = sy[p] / (double)ne[p];
    V[(b + p) * 3 + 2] = sz[p] / (double)ne[p];
  }
}

// one thread per grid point, its three edges towards +x, +y, +z (flag of the
// edge along axis a at a r^3 + point); res <= 512 keeps the indices in int32
__global__ void k_dmc_qflags(const uint8_t* __restrict__ sg, int r, uint8_t* __restrict__ flag) {
  const int n3 = r * r * r;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int gp[3] = {p / (r * r), p / r % r, p % r};
  const int step[3] = {r * r, r, 1};
  const uint8_t s0 = sg[p];
  for (int a = 0; a < 3; a++) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const bool in = gp[a] <= r - 2 && gp[b] >= 1 && gp[b] <= r - 2 && gp[c] >= 1 && gp[c] <= r - 2;
    flag[a * n3 + p] = in && s0 != sg[p + step[a]] ? 1 : 0;
  }
}

// the crossing point of grid edge (i0, j0, k0) -> +axis a (fraction from the
// lower end, smoothed when beta > 0), as for the patch vertices
__device__ __forceinline__ void edge_crossing(const DGrid& g, int i0, int j0, int k0, int a, double* out) {
  const double s0 = gval(g, i0, j0, k0);
  const double s1 = gval(g, i0 + (a == 0), j0 + (a == 1), k0 + (a == 2));
  double t = s0 / (s0 - s1);
  if (g.beta > 0.0) t = 1.0 / (1.0 + exp(-g.beta * (t - 0.5)));
  double q[3] = {(double)i0 + 0.5, (double)j0 + 0.5, (double)k0 + 0.5};
  q[a] = q[a] + t;
  const double rr = (double)g.r;
  out[0] = q[0] / rr;
  out[1] = q[1] / rr;
  out[2] = q[2] / rr;
}

// the quad of crossed grid edge x (axis a = x / r^3): its four vertices in
// order (normal towards the positive end), the grid point of its lower end
__device__ __forceinline__ void quad_ring(int r, const uint8_t* __restrict__ sg, const uint32_t* __restrict__ pmap,
                                          const int32_t* __restrict__ vbase, int64_t x, int ring[4], int gp[3],
                                          int& a, bool& lower_pos) {
  const int64_t n3 = (int64_t)r * r * r, pt = x % n3;
  a = (int)(x / n3);
  gp[0] = (int)(pt / ((int64_t)r * r));
  gp[1] = (int)(pt / r % r);
  gp[2] = (int)(pt % r);
  const int m = r - 1;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int db[4] = {-1, 0, 0, -1}, dc[4] = {-1, -1, 0, 0};
  for (int t = 0; t < 4; t++) {
    int cu[3] = {gp[0], gp[1], gp[2]};
    cu[b] += db[t];
    cu[c] += dc[t];
    const int lb = -db[t], lc = -dc[t];  // the grid edge's place in the cube
    const int u = b < c ? lb : lc, v = b < c ? lc : lb;
    const int64_t ci = ((int64_t)cu[0] * m + cu[1]) * m + cu[2];
    ring[t] = vbase[ci] + (int)((pmap[ci] >> (2 * (4 * a + u + 2 * v))) & 3);
  }
  lower_pos = sg[pt] != 0;
  if (lower_pos) {
    const int t1 = ring[1];
    ring[1] = ring[3];
    ring[3] = t1;
  }
}

// (v - p) . ((l - p) x (r - p)), in this order of operations
__device__ __forceinline__ double triple(const double* v, const double* l, const double* r, const double* p) {
  const double ax = l[0] - p[0], ay = l[1] - p[1], az = l[2] - p[2];
  const double bx = r[0] - p[0], by = r[1] - p[1], bz = r[2] - p[2];
  const double cx = ay * bz - az * by;
  const double cy = az * bx - ax * bz;
  const double cz = ax * by - ay * bx;
  return (v[0] - p[0]) * cx + (v[1] - p[1]) * cy + (v[2] - p[2]) * cz;
}

// the largest cosine of the angles of triangle pqr (1 where an edge has zero length)
__device__ __forceinline__ double worst_cos(const double* p, const double* q, const double* r) {
  const double* A[3] = {p, q, r};
  double out = -2.0;
  for (int i = 0; i < 3; i++) {
    const double* a = A[i];
    const double* b = A[(i + 1) % 3];
    const double* c = A[(i + 2) % 3];
    const double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    const double wx = c[0] - a[0], wy = c[1] - a[1], wz = c[2] - a[2];
    const double uu = ux * ux + uy * uy + uz * uz;
    const double ww = wx * wx + wy * wy + wz * wz;
    const double cs = uu == 0.0 || ww == 0.0 ? 1.0 : (ux * wx + uy * wy + uz * wz) / (sqrt(uu) * sqrt(ww));
    out = cs > out ? cs : out;
  }
  return out;
}

// division of every crossed grid edge's quad: 0 along v0 v2, 1 along v1 v3,
// 2 four triangles around an extra vertex on the edge (four[q] = 1)
__global__ void k_dmc_qdiv(int r, const uint8_t* __restrict__ sg, const uint32_t* __restrict__ pmap,
                           const int32_t* __restrict__ vbase, const int32_t* __restrict__ qlist, int nq,
                           const double* __restrict__ V, uint8_t* __restrict__ kind, uint8_t* __restrict__ four) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int ring[4], gp[3], a;
  bool lower_pos;
  quad_ring(r, sg, pmap, vbase, qlist[q], ring, gp, a, lower_pos);
  double p[4][3];
  for (int t = 0; t < 4; t++)
    for (int k = 0; k < 3; k++) p[t][k] = V[(int64_t)ring[t] * 3 + k];
  double e0[3], e1[3];
  const double rr = (double)r;
  for (int k = 0; k < 3; k++) {
    e0[k] = ((double)gp[k] + 0.5) / rr;
    e1[k] = ((double)(gp[k] + (k == a)) + 0.5) / rr;
  }
  const double* pp = lower_pos ? e0 : e1;
  const double* pn = lower_pos ? e1 : e0;
  bool conc[4];
  for (int i = 0; i < 4; i++) {
    const double* l = p[(i + 3) & 3];
    const double* rt = p[(i + 1) & 3];
    conc[i] = triple(p[i], l, rt, pp) < 0.0 || triple(p[i], l, rt, pn) > 0.0;
  }
  const bool on_a = conc[0] || conc[2], on_b = conc[1] || conc[3];
  uint8_t k;
  if (on_a && on_b) {
    k = 2;
  } else if (on_a) {
    k = 0;
  } else if (on_b) {
    k = 1;
  } else {
    const double a1 = worst_cos(p[0], p[1], p[2]), a2 = worst_cos(p[0], p[2], p[3]);
    const double b1 = worst_cos(p[0], p[1], p[3]), b2 = worst_cos(p[1], p[2], p[3]);
    const double wa = a1 > a2 ? a1 : a2, wb = b1 > b2 ? b1 : b2;
    k = wa <= wb ? 0 : 1;
  }
  kind[q] = k;
  four[q] = k == 2;
}

// the triangles of every crossed grid edge's quad, from triangle 2 q + 2
// rank[q] on (rank: four-triangle quads before it), and the extra vertex of a
// four-triangle quad at nv_patch + rank[q]
__global__ void k_dmc_quads(DGrid g, const uint8_t* __restrict__ sg, const uint32_t* __restrict__ pmap,
                            const int32_t* __restrict__ vbase, const int32_t* __restrict__ qlist, int nq,
                            const uint8_t* __restrict__ kind, const int32_t* __restrict__ rank, int nv_patch,
                            double* __restrict__ V, int32_t* __restrict__ F) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int ring[4], gp[3], a;
  bool lower_pos;
  quad_ring(g.r, sg, pmap, vbase, qlist[q], ring, gp, a, lower_pos);
  const int rk = rank[q];
  const int64_t o = ((int64_t)q + rk) * 6;
  const uint8_t k = kind[q];
  if (k == 0) {
    F[o + 0] = ring[0], F[o + 1] = ring[1], F[o + 2] = ring[2];
    F[o + 3] = ring[0], F[o + 4] = ring[2], F[o + 5] = ring[3];
  } else if (k == 1) {
    F[o + 0] = ring[0], F[o + 1] = ring[1], F[o + 2] = ring[3];
    F[o + 3] = ring[1], F[o + 4] = ring[2], F[o + 5] = ring[3];
  } else {
    const int ve = nv_patch + rk;
    edge_crossing(g, gp[0], gp[1], gp[2], a, V + (int64_t)ve * 3);
    for (int t = 0; t < 4; t++) {
      F[o + 3 * t + 0] = ring[t];
      F[o + 3 * t + 1] = ring[(t + 1) & 3];
      F[o + 3 * t + 2] = ve;
    }
  }
}

__global__ void k_add_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] += v;
}

int32_t read_i32(hipStream_t s, const int32_t* p) {
  int32_t h = 0;
  PAMO_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, s));
  PAMO_HIP(hipStreamSynchronize(s));
  return h;
}

// ascending indices of the set flags of flags[0..n) into out; returns their
// number.  The compaction takes at most 2^26 items a call, so longer inputs go
// in chunks, each chunk's local indices then offset by its start.
int32_t compact_long(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* out, int32_t* tot) {
  constexpr int64_t CHUNK = (int64_t)1 << 26;
  int32_t count = 0;
  for (int64_t off = 0; off < n; off += CHUNK) {
    const int64_t len = n - off < CHUNK ? n - off : CHUNK;
    compact_flags(ws, s, flags + off, len, out + count, tot);
    const int32_t c = read_i32(s, tot);
    if (off > 0 && c > 0)
      hipLaunchKernelGGL(k_add_i32, dim3(blocks(c)), dim3(256), 0, s, out + count, c, (int32_t)off);
    count += c;
  }
  PAMO_HIP(hipGetLastError());
  return count;
}

}  // namespace

bool dualmc_run(Workspace& ws, hipStream_t s, const double* S, int res, double iso, double beta, double* V,
                int64_t vcap, int32_t* F, int64_t fcap, int64_t* nv, int64_t* nf) {
  *nv = *nf = 0;
  if (res < 2) return true;
  DGrid g{S, res, iso, beta};
  const int m = res - 1;
  const int64_t npt = (int64_t)res * res * res, ncube = (int64_t)m * m * m, nedge = 3 * npt;
  uint8_t* sg = ws.get<uint8_t>("dmc.sign", npt);
  uint8_t* cfgs = ws.get<uint8_t>("dmc.cfg", ncube);
  uint8_t* act = ws.get<uint8_t>("dmc.act", ncube);
  int32_t* clist = ws.get<int32_t>("dmc.clist", ncube);
  uint8_t* qflag = ws.get<uint8_t>("dmc.qflag", nedge);
  int32_t* qlist = ws.get<int32_t>("dmc.qlist", nedge);
  int32_t* tot = ws.get<int32_t>("dmc.tot", 3);
  hipLaunchKernelGGL(k_dmc_sign, dim3(blocks(npt)), dim3(256), 0, s, g, sg);
  hipLaunchKernelGGL(k_dmc_active, dim3(blocks(ncube)), dim3(256), 0, s, (const uint8_t*)sg, res, cfgs, act);
  hipLaunchKernelGGL(k_dmc_qflags, dim3(blocks(npt)), dim3(256), 0, s, (const uint8_t*)sg, res, qflag);
  PAMO_HIP(hipGetLastError());
  int nc, nq;
  if (nedge <= ((int64_t)1 << 26)) {  // one compaction each, one read-back
    compact_flags(ws, s, act, ncube, clist, tot);
    compact_flags(ws, s, qflag, nedge, qlist, tot + 1);
    int32_t h[2] = {0, 0};
    PAMO_HIP(hipMemcpyAsync(h, tot, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PAMO_HIP(hipStreamSynchronize(s));
    nc = h[0];
    nq = h[1];
  } else {
    nc = compact_long(ws, s, act, ncube, clist, tot);
    nq = compact_long(ws, s, qflag, nedge, qlist, tot + 1);
  }
  if (nc == 0) return nq == 0;  // a crossed grid edge lies in crossed cubes
  uint32_t* pmap = ws.get<uint32_t>("dmc.pmap", ncube);
  int32_t* vbase = ws.get<int32_t>("dmc.vbase", ncube);
  int32_t* cntl = ws.get<int32_t>("dmc.cntl", nc);
  int32_t* vbl = ws.get<int32_t>("dmc.vbl", nc);
  hipLaunchKernelGGL(k_dmc_cubes, dim3(blocks(nc)), dim3(256), 0, s, (const uint8_t*)cfgs, m,
                     (const int32_t*)clist, nc, pmap, cntl);
  scan_exclusive(ws, s, cntl, vbl, nc, tot + 2);
  PAMO_HIP(hipGetLastError());
  const int32_t nvp = read_i32(s, tot + 2);
  // patch vertices into scratch first: the quads' division needs them, and
  // the sizes (extra vertices, four-triangle quads) must be known before any
  // output is written
  double* vt = ws.get<double>("dmc.vtmp", 3 * (int64_t)nvp);
  hipLaunchKernelGGL(k_dmc_verts, dim3(blocks(nc)), dim3(256), 0, s, g, (const uint8_t*)cfgs, (const int32_t*)clist,
                     nc, (const uint32_t*)pmap, (const int32_t*)cntl, (const int32_t*)vbl, vbase, vt);
  int32_t n4 = 0;
  uint8_t* kind = ws.get<uint8_t>("dmc.kind", nq);
  int32_t* rank = ws.get<int32_t>("dmc.rank", nq);
  if (nq > 0) {
    if (nq > ((int64_t)1 << 26)) throw std::runtime_error("more than 2^26 quads");
    uint8_t* four = ws.get<uint8_t>("dmc.four", nq);
    hipLaunchKernelGGL(k_dmc_qdiv, dim3(blocks(nq)), dim3(256), 0, s, res, (const uint8_t*)sg, (const uint32_t*)pmap,
                       (const int32_t*)vbase, (const int32_t*)qlist, nq, (const double*)vt, kind, four);
    run_flag_scan(ws, s, four, nq, rank, tot + 2);
    PAMO_HIP(hipGetLastError());
    n4 = read_i32(s, tot + 2);
  }
  *nv = (int64_t)nvp + n4;
  *nf = 2 * ((int64_t)nq + n4);
  if (*nv > vcap || *nf > fcap) return false;
  if (nvp > 0) PAMO_HIP(hipMemcpyAsync(V, vt, 3 * (size_t)nvp * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (nq > 0)
    hipLaunchKernelGGL(k_dmc_quads, dim3(blocks(nq)), dim3(256), 0, s, g, (const uint8_t*)sg, (const uint32_t*)pmap,
                       (const int32_t*)vbase, (const int32_t*)qlist, nq, (const uint8_t*)kind, (const int32_t*)rank,
                       nvp, V, F);
  PAMO_HIP(hipGetLastError());
  return true;
}

}  // namespace pamo
