// The remeshing stage's mesh-to-volume step (Sec. 4.1): the unsigned
// distance field of a triangle soup at the voxel centres of an R^3 grid over
// [0,1]^3, kept only inside a narrow band around the surface.
//
// The paper filters triangle-voxel pairs level by level over a hierarchy of
// grids, keeping a pair when the voxel's bounding sphere meets the band
// around the triangle, then evaluates the remaining pairs exactly.  Here the
// hierarchy has two levels: tiles of UT^3 voxels (one wave), paired with a
// triangle when the tile's bounding sphere meets the band (a point-triangle
// distance), and the voxels of each tile against the triangles paired with
// it, staged through LDS.  The filter is conservative, so each value is the
// minimum over all triangles whenever that minimum lies inside the band.
#include <math.h>

#include "internal.hpp"
#include "mesh_dev.hpp"
#include "remesh.hpp"
#include "round.hpp"

namespace pamo {

namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

constexpr int UT = 4;              // voxels per tile edge: a tile is 64 voxels, one wave
constexpr int64_t TILE_CAP = 1 << 20;  // tiles one triangle may visit (its banded box)

__device__ __forceinline__ double seg_dist2(P3 p, P3 a, P3 b) {
  double abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
  double l2 = abx * abx + aby * aby + abz * abz;
  double t = l2 > 0.0 ? ((p.x - a.x) * abx + (p.y - a.y) * aby + (p.z - a.z) * abz) / l2 : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  double dx = p.x - (a.x + t * abx), dy = p.y - (a.y + t * aby), dz = p.z - (a.z + t * abz);
  return dx * dx + dy * dy + dz * dz;
}

// squared distance to a triangle of the soup; a triangle of (nearly) zero
// area, whose region tests round unreliably, is taken as its three edges
__device__ __forceinline__ double soup_dist2(P3 p, P3 a, P3 b, P3 c) {
  const double abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
  const double acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
  const double nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
  const double n2 = nx * nx + ny * ny + nz * nz;
  const double l2 = (abx * abx + aby * aby + abz * abz) * (acx * acx + acy * acy + acz * acz);
  if (n2 > 1e-20 * l2) {
    const double d = tri_dist2(p, a, b, c);
    if (d == d) return d;
  }
  const double e0 = seg_dist2(p, a, b), e1 = seg_dist2(p, b, c), e2 = seg_dist2(p, c, a);
  const double d = e0 < e1 ? e0 : e1;
  return d < e2 ? d : e2;
}

struct Grid {
  int res;        // voxels per axis
  int nt;         // tiles per axis
  double band;    // band width
  double slack;   // added to the tile test so that rounding can only keep more pairs
};

__device__ __forceinline__ double centre(const Grid& g, int i) { return (i + 0.5) / g.res; }

// the tile range of triangle t's box grown by the band, and the tile test
template <class Fn>
__device__ __forceinline__ bool tri_tiles(const Grid& g, P3 a, P3 b, P3 c, Fn&& fn) {
  const double lo[3] = {fmin(a.x, fmin(b.x, c.x)), fmin(a.y, fmin(b.y, c.y)), fmin(a.z, fmin(b.z, c.z))};
  const double hi[3] = {fmax(a.x, fmax(b.x, c.x)), fmax(a.y, fmax(b.y, c.y)), fmax(a.z, fmax(b.z, c.z))};
  int t0[3], t1[3];
  int64_t vol = 1;
  for (int k = 0; k < 3; k++) {
    // voxel centres (i + 1/2) / R within [lo - band, hi + band], one voxel of margin
    double v0 = floor((lo[k] - g.band) * g.res - 0.5) - 1.0, v1 = ceil((hi[k] + g.band) * g.res - 0.5) + 1.0;
    v0 = v0 < 0.0 ? 0.0 : v0;
    v1 = v1 > g.res - 1.0 ? g.res - 1.0 : v1;
    if (!(v0 <= v1)) return true;  // no voxel near it (or a non-finite corner)
    t0[k] = (int)v0 / UT;
    t1[k] = (int)v1 / UT;
    vol *= t1[k] - t0[k] + 1;
  }
  if (vol > TILE_CAP) return false;
  // the sphere around a tile's UT^3 centre positions
  const double rad = 0.8660254037844387 * (UT - 1) / g.res;
  const double lim = g.band + rad + g.slack;
  const double lim2 = lim * lim;
  for (int x = t0[0]; x <= t1[0]; x++)
    for (int y = t0[1]; y <= t1[1]; y++)
      for (int z = t0[2]; z <= t1[2]; z++) {
        const P3 q{(UT * x + 0.5 * (UT - 1) + 0.5) / g.res, (UT * y + 0.5 * (UT - 1) + 0.5) / g.res,
                   (UT * z + 0.5 * (UT - 1) + 0.5) / g.res};
        if (soup_dist2(q, a, b, c) <= lim2) fn(((int64_t)x * g.nt + y) * g.nt + z);
      }
  return true;
}

__device__ __forceinline__ void tri_corners(const double* __restrict__ V, const int* __restrict__ F, int t, P3& a,
                                            P3& b, P3& c) {
  a = ld3(V, F[3 * (int64_t)t]);
  b = ld3(V, F[3 * (int64_t)t + 1]);
  c = ld3(V, F[3 * (int64_t)t + 2]);
}

__global__ void k_udf_count(Grid g, const double* __restrict__ V, const int* __restrict__ F, int nf,
                            int* __restrict__ cnt, unsigned long long* total, int* err) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int n = 0;
  if (t < nf) {
    P3 a, b, c;
    tri_corners(V, F, t, a, b, c);
    if (!tri_tiles(g, a, b, c, [&](int64_t) { n++; })) atomicOr(err, PAMO_EBIT_TILES);
    cnt[t] = n;
  }
  // one atomic per wave for the 64-bit total (the int32 scan must not overflow)
  unsigned long long w = (unsigned long long)n;
  for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
  if ((threadIdx.x & 63) == 0 && w) atomicAdd(total, w);
}

__global__ void k_udf_emit(Grid g, const double* __restrict__ V, const int* __restrict__ F, int nf,
                           const int* __restrict__ off, uint32_t* __restrict__ tile, int* __restrict__ tri) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nf) return;
  P3 a, b, c;
  tri_corners(V, F, t, a, b, c);
  int o = off[t];
  tri_tiles(g, a, b, c, [&](int64_t id) {
    tile[o] = (uint32_t)id;
    tri[o] = t;
    o++;
  });
}

// the first pair of each tile's run in the sorted pair list
__global__ void k_udf_runs(const uint32_t* __restrict__ tile, int n, uint8_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = i == 0 || tile[i] != tile[i - 1];
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// one wave per tile with pairs: each lane one voxel, the tile's triangles
// staged 64 at a time with their bounding spheres.  A triangle whose sphere
// lies farther than the best distance so far (or than the band) by a margin
// far above rounding cannot lower the minimum and is skipped, so the result
// is the same as testing every triangle.
__global__ __launch_bounds__(64) void k_udf_tiles(Grid g, const double* __restrict__ V, const int* __restrict__ F,
                                                  const uint32_t* __restrict__ tile, const int* __restrict__ tri,
                                                  int npairs, const int* __restrict__ runs,
                                                  const int* __restrict__ nruns, double* __restrict__ udf) {
  __shared__ double tv[64][13];  // corners, centre, radius
  const int r = blockIdx.x;
  if (r >= *nruns) return;  // uniform over the block
  const int s = runs[r], e = r + 1 < *nruns ? runs[r + 1] : npairs;
  const int64_t id = tile[s];
  const int tz = (int)(id % g.nt), ty = (int)(id / g.nt % g.nt), tx = (int)(id / ((int64_t)g.nt * g.nt));
  const int l = threadIdx.x;
  const int i = UT * tx + l / (UT * UT), j = UT * ty + l / UT % UT, k = UT * tz + l % UT;
  const P3 p{centre(g, i), centre(g, j), centre(g, k)};
  const double margin = 1e-9 * (g.band + 1.0);
  double best = INFINITY;       // squared
  double cut = g.band + margin;  // skip spheres beyond this distance
  for (int c0 = s; c0 < e; c0 += 64) {
    if (c0 + l < e) {
      P3 a, b, c;
      tri_corners(V, F, tri[c0 + l], a, b, c);
      const double cx = (a.x + b.x + c.x) / 3.0, cy = (a.y + b.y + c.y) / 3.0, cz = (a.z + b.z + c.z) / 3.0;
      auto d2 = [&](P3 q) { return (q.x - cx) * (q.x - cx) + (q.y - cy) * (q.y - cy) + (q.z - cz) * (q.z - cz); };
      const double rad = sqrt(fmax(d2(a), fmax(d2(b), d2(c))));
      const double q[13] = {a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, cx, cy, cz, rad};
#pragma unroll
      for (int m = 0; m < 13; m++) tv[l][m] = q[m];
    }
    __syncthreads();
    const int n = e - c0 < 64 ? e - c0 : 64;
    for (int m = 0; m < n; m++) {
      const double* q = tv[m];
      const double dx = p.x - q[9], dy = p.y - q[10], dz = p.z - q[11];
      const double lim = q[12] + cut;
      if (dx * dx + dy * dy + dz * dz > lim * lim) continue;
      const double d = soup_dist2(p, P3{q[0], q[1], q[2]}, P3{q[3], q[4], q[5]}, P3{q[6], q[7], q[8]});
      if (d < best) {
        best = d;
        const double cd = sqrt(d) + margin;
        cut = cd < cut ? cd : cut;
      }
    }
    __syncthreads();
  }
  if (i < g.res && j < g.res && k < g.res) {
    const double d = sqrt(best);  // the square root is monotone: the smallest distance
    udf[((int64_t)i * g.res + j) * g.res + k] = d <= g.band ? d : INFINITY;
  }
}

}  // namespace

void udf_run(Workspace& ws, hipStream_t s, const double* V, const int* F, int nf, int res, double band, double* udf,
             int* err, const std::function<int64_t(const unsigned long long*)>& read_total) {
  Grid g;
  g.res = res;
  g.nt = (res + UT - 1) / UT;
  g.band = band;
  g.slack = 1e-9 * (band + 1.0);
  const int64_t nvox = (int64_t)res * res * res;
  hipLaunchKernelGGL(k_fill_f64, dim3(nblk(nvox)), dim3(256), 0, s, udf, nvox, (double)INFINITY);
  if (nf == 0) return;
  int* cnt = ws.get<int>("udf.cnt", nf + 1);
  int* off = ws.get<int>("udf.off", nf + 1);
  unsigned long long* total = ws.get<unsigned long long>("udf.total", 1);
  fill_i32(s, reinterpret_cast<int32_t*>(total), 2, 0);
  hipLaunchKernelGGL(k_udf_count, dim3(nblk(nf)), dim3(256), 0, s, g, V, F, nf, cnt, total, err);
  const int64_t np = read_total(total);  // also checks the error bits and the int32 range
  if (np == 0) return;
  scan_exclusive(ws, s, cnt, off, nf, nullptr);
  uint32_t* tile = ws.get<uint32_t>("udf.tile", np);
  int* tri = ws.get<int>("udf.tri", np);
  hipLaunchKernelGGL(k_udf_emit, dim3(nblk(nf)), dim3(256), 0, s, g, V, F, nf, (const int*)off, tile, tri);
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < (int64_t)g.nt * g.nt * g.nt) bits++;
  radix_sort_u32(ws, s, tile, tri, np, bits);  // stable; the order within a tile does not matter (a minimum)
  uint8_t* flag = ws.get<uint8_t>("udf.flag", np);
  int* runs = ws.get<int>("udf.runs", np);
  int* nruns = ws.get<int>("udf.nruns", 1);
  hipLaunchKernelGGL(k_udf_runs, dim3(nblk(np)), dim3(256), 0, s, (const uint32_t*)tile, (int)np, flag);
  compact_flags(ws, s, flag, np, runs, nruns);
  const int64_t ntiles = (int64_t)g.nt * g.nt * g.nt;
  const int64_t grid = np < ntiles ? np : ntiles;  // runs <= both; blocks past the count return
  hipLaunchKernelGGL(k_udf_tiles, dim3((unsigned)grid), dim3(64), 0, s, g, V, F, (const uint32_t*)tile,
                     (const int*)tri, (int)np, (const int*)runs, (const int*)nruns, udf);
  PAMO_HIP(hipGetLastError());
}

}  // namespace pamo
