// The learned proposal (an addition to the paper's method, which has no
// network): per-edge features, the network's inference on MFMA, its training
// (forward, backward, Adam), and the Hausdorff distance used to judge it.
//
// Network: 32 quantised features -> 64 -> 64 -> 1 logit, ReLU.  Weights of
// layer l are integers k (|k| <= 127) times 2^-e_l, biases integers times the
// same 2^-e_l; each hidden activation is scaled by 2^a_l and rounded to an
// integer in [0, 127].  Inputs are integers in [-127, 127].  Every product
// is then exact in float32 and every partial sum stays below 2^24 units of
// the layer's grid, so the MFMA float32 accumulation is exact in any order:
// the library and a float64 reference reach the same logits bit for bit.
#include <math.h>

#include "learn.hpp"
#include "mesh_dev.hpp"

namespace pamo {

namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

// ------------------------------------------------------------ features
// power-of-two scale of each feature before rounding to [-127, 127]
__constant__ int FEAT_SHIFT[LEARN_NF_USED] = {2, 3, 7, 7, 6, 6, 2, 2, 4, 0, 2};

__device__ __forceinline__ double plog2(double c) {
  if (!(c > 0.0)) return -64.0;
  if (isinf(c)) return 64.0;
  int e;
  double mant = frexp(c, &e);  // c = mant 2^e, mant in [0.5, 1)
  return (double)(e - 1) + (2.0 * mant - 1.0);
}

__device__ __forceinline__ float quantize_feature(double f, int shift) {
  double q = rint(ldexp(f, shift));
  if (q != q) return 0.0f;
  if (q > 127.0) q = 127.0;
  if (q < -127.0) q = -127.0;
  return (float)q;
}

__device__ __forceinline__ double seg_len(P3 p, P3 q) {
  double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
  return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ P3 face_normal(const double* __restrict__ V, const int* __restrict__ F, int f) {
  P3 p0 = ld3(V, F[3 * f]), p1 = ld3(V, F[3 * f + 1]), p2 = ld3(V, F[3 * f + 2]);
  double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  return P3{e1y * e2z - e1z * e2y, e1z * e2x - e1x * e2z, e1x * e2y - e1y * e2x};
}

__device__ __forceinline__ double normal_cos(P3 n0, P3 n1) {
  double d = n0.x * n1.x + n0.y * n1.y + n0.z * n1.z;
  double q = (n0.x * n0.x + n0.y * n0.y + n0.z * n0.z) * (n1.x * n1.x + n1.y * n1.y + n1.z * n1.z);
  if (!(q > 0.0)) return 1.0;
  return d / sqrt(q);
}

__device__ __forceinline__ double key_cost(uint64_t key) {
  uint32_t k = (uint32_t)(key >> 32);
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return (double)f;
}

constexpr int WALK_GUARD = 1 << 12;

// normal of a face given its corners starting at the corner of slot k
// (p = the corner in slot k, q = next, r = previous), in slot order 0, 1, 2 so
// that it matches face_normal bit for bit
__device__ __forceinline__ P3 rotated_normal(P3 p, P3 q, P3 r, int k) {
  const P3 p0 = k == 0 ? p : (k == 1 ? r : q);
  const P3 p1 = k == 0 ? q : (k == 1 ? p : r);
  const P3 p2 = k == 0 ? r : (k == 1 ? q : p);
  double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  return P3{e1y * e2z - e1z * e2y, e1z * e2x - e1x * e2z, e1x * e2y - e1y * e2x};
}

// The spokes and overlap counts of the faces of one stored star (n <= VSTAR
// half-edges g leaving v; faces holding `skip` add no overlap count): every
// edge (v, F[next g]) with the normals of its two faces g / 3 and twin[g] / 3.
// Every edge holding a or b is the out-edge of one of the two stars, so the
// spokes of both stars are exactly the spoke set of the walk below; lengths,
// cosines and overlap maxima are order-free and the overlap sum is an integer
// sum, so the features agree bit for bit.  Fills the star's targets in x[].
template <class Spoke, class Ovl>
__device__ __forceinline__ void stored_star(const MeshView& m, int v, int n, int skip, P3 pv, int* x, Spoke&& spoke,
                                            Ovl&& face_ovl) {
  const int* __restrict__ F = m.F;
  const int4* st4 = reinterpret_cast<const int4*>(m.vstar + (int64_t)VSTAR * v);
  int st[VSTAR];
#pragma unroll
  for (int q = 0; q < VSTAR / 4; q++) {
    const int4 w = st4[q];
    st[4 * q] = w.x;
    st[4 * q + 1] = w.y;
    st[4 * q + 2] = w.z;
    st[4 * q + 3] = w.w;
  }
#pragma unroll
  for (int i = 0; i < VSTAR; i++) {
    x[i] = -1;
    if (i < n) {
      const int g = st[i];
      const int xi = F[he_next(g)], yi = F[he_prev(g)];
      const int t = m.twin[g];  // >= 0: the quadrics kernel stored the star by walking twins
      const int zi = F[he_prev(t)];
      const P3 px = ld3(m.V, xi), py = ld3(m.V, yi), pz = ld3(m.V, zi);
      const P3 n0 = rotated_normal(pv, px, py, g % 3);
      const P3 n1 = rotated_normal(px, pv, pz, t % 3);  // twin face: x -> v -> z
      spoke(seg_len(pv, px), normal_cos(n0, n1));
      if (xi != skip && yi != skip) face_ovl(g / 3);
      x[i] = xi;
    }
  }
}

// Features of candidate edge h = (a, b); S = star(a) u star(b), spokes = the
// edges of S's faces that contain a or b:
//   0 plog2(cost)   1 plog2(length)   2 length / longest spoke   3 shortest spoke / length
//   4 cos between the normals of the edge's two faces   5 smallest such cos over the spokes
//   6 valence of a   7 valence of b   8 common neighbours   9 sum of ovl over S   10 largest ovl
__global__ __launch_bounds__(256) void k_features(MeshView m, const uint64_t* __restrict__ key,
                                                  const int* __restrict__ cand, const int* __restrict__ ncand,
                                                  const int* __restrict__ ovl, float* __restrict__ X, int* err,
                                                  const int* __restrict__ fmesh, const uint8_t* __restrict__ use_m) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= *ncand) return;
  const int h = cand[c];
  if (fmesh && use_m && !use_m[fmesh[h / 3]]) {  // its mesh does not consult the network this round
    float4* x = reinterpret_cast<float4*>(X + (int64_t)c * LEARN_NFEAT);
#pragma unroll
    for (int k = 0; k < LEARN_NFEAT / 4; k++) x[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const int* __restrict__ F = m.F;
  const int* __restrict__ tw = m.twin;
  const int a = F[h], b = F[he_next(h)];
  const double le = seg_len(ld3(m.V, a), ld3(m.V, b));
  double lmax = 0.0, lmin = INFINITY, cmin = INFINITY;
  int64_t osum = 0, omax = 0;
  const int hb = tw[h];
  int vala = 0, valb = 0, common = 0;
  bool stored = false;
  if (m.vstar) {
    vala = m.vdeg[a];
    valb = m.vdeg[b];
    stored = vala <= VSTAR && valb <= VSTAR;
  }
  if (stored) {
    auto spoke = [&](double l, double cs) {
      lmax = l > lmax ? l : lmax;
      lmin = l < lmin ? l : lmin;
      cmin = cs < cmin ? cs : cmin;
    };
    auto face_ovl = [&](int f) {
      int64_t o = ovl ? ovl[f] : 0;
      osum += o;
      omax = o > omax ? o : omax;
    };
    int xa[VSTAR], xb[VSTAR];
    const P3 pa = ld3(m.V, a), pb = ld3(m.V, b);
    stored_star(m, a, vala, -1, pa, xa, spoke, face_ovl);
    stored_star(m, b, valb, a, pb, xb, spoke, face_ovl);
#pragma unroll
    for (int j = 0; j < VSTAR; j++) {
      bool hit = false;
#pragma unroll
      for (int i = 0; i < VSTAR; i++) hit |= xa[i] == xb[j];
      common += xb[j] >= 0 && xb[j] != a && hit;
    }
  } else {
  auto spoke = [&](int hh) {
    double l = seg_len(ld3(m.V, F[hh]), ld3(m.V, F[he_next(hh)]));
    lmax = l > lmax ? l : lmax;
    lmin = l < lmin ? l : lmin;
    double cs = normal_cos(face_normal(m.V, F, hh / 3), face_normal(m.V, F, tw[hh] / 3));
    cmin = cs < cmin ? cs : cmin;
  };
  auto face_ovl = [&](int f) {
    int64_t o = ovl ? ovl[f] : 0;
    osum += o;
    omax = o > omax ? o : omax;
  };
  // star(a): every face once; all three edges of the two faces holding b
  vala = 0;
  int g = h, guard = 0;
  do {
    vala++;
    spoke(g);
    spoke(he_prev(g));
    int nx = he_next(g);
    if (F[nx] == b || F[he_next(nx)] == b) spoke(nx);
    face_ovl(g / 3);
    g = tw[he_prev(g)];
  } while (g != h && g >= 0 && ++guard < WALK_GUARD);
  // star(b) without those two faces
  valb = 0;
  g = hb;
  guard = 0;
  do {
    valb++;
    const int f = g / 3;
    if (F[3 * f] != a && F[3 * f + 1] != a && F[3 * f + 2] != a) {
      spoke(g);
      spoke(he_prev(g));
      face_ovl(f);
    }
    g = tw[he_prev(g)];
  } while (g != hb && g >= 0 && ++guard < WALK_GUARD);
  // common neighbours
  g = hb;
  guard = 0;
  do {
    const int y = F[he_next(g)];
    if (y != a) {
      int g2 = h, guard2 = 0;
      do {
        if (F[he_next(g2)] == y) {
          common++;
          break;
        }
        g2 = tw[he_prev(g2)];
      } while (g2 != h && g2 >= 0 && ++guard2 < WALK_GUARD);
    }
    g = tw[he_prev(g)];
  } while (g != hb && g >= 0 && ++guard < WALK_GUARD);
  if (guard >= WALK_GUARD || g < 0) atomicOr(err, PAMO_EBIT_RING);
  }
  double f[LEARN_NF_USED];
  f[0] = plog2(key_cost(key[h]));
  f[1] = plog2(le);
  f[2] = le / lmax;
  f[3] = lmin / le;
  f[4] = normal_cos(face_normal(m.V, F, h / 3), face_normal(m.V, F, hb / 3));
  f[5] = cmin;
  f[6] = (double)vala;
  f[7] = (double)valb;
  f[8] = (double)common;
  f[9] = (double)osum;
  f[10] = (double)omax;
  float* x = X + (int64_t)c * LEARN_NFEAT;
#pragma unroll
  for (int k = 0; k < LEARN_NFEAT; k++) x[k] = k < LEARN_NF_USED ? quantize_feature(f[k], FEAT_SHIFT[k]) : 0.0f;
}

// ------------------------------------------------------------ inference (MFMA)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float requant(float z, int a) {
  z = z > 0.0f ? z : 0.0f;
  float q = rintf(ldexpf(z, a));
  return q > 127.0f ? 127.0f : q;
}

// One wave per tile of 16 rows (grid-stride).  Layer 1 is one
// 16x16x32 MFMA per tile of 16 units; layer 2 two per tile; layer 3 a short
// dot product.  Lane l supplies row l % 16 of A and column l % 16 of B and
// receives rows 4 (l / 16) .. +3 of column l % 16 of D; the 8 k values a lane
// supplies only need to match between A and B, which they do by
// construction.  Hidden activations cross lanes through LDS.
// Modes: logits to `out` (may be null); set-aside: rows below the threshold
// get the largest key on both half-edges of cand[row], counted in *ndemote.
__global__ __launch_bounds__(256) void k_mlp(const float* __restrict__ X, const int* __restrict__ n_dev,
                                             const MlpDev* __restrict__ M, float* __restrict__ out,
                                             const int* __restrict__ cand, const int* __restrict__ twin,
                                             uint64_t* __restrict__ key, int* __restrict__ ndemote,
                                             const int* __restrict__ fmesh, int* __restrict__ ndemote_m,
                                             const uint8_t* __restrict__ use_m, int* __restrict__ dlist) {
  __shared__ __bf16 sh[4][16][64 + 8];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l & 15, kg = l >> 4;
  const int n = *n_dev;
  const int ntiles = (n + 15) / 16;
  if (blockIdx.x * 4 + w >= ntiles) return;  // whole wave idle
  bf16x8 B1[4], B2[4][2];
  float b1v[4], b2v[4];
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    const int u = 16 * nt + row;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      B1[nt][i] = M->w1[u * 32 + 8 * kg + i];
      B2[nt][0][i] = M->w2[u * 64 + 8 * kg + i];
      B2[nt][1][i] = M->w2[u * 64 + 32 + 8 * kg + i];
    }
    b1v[nt] = M->b1[u];
    b2v[nt] = M->b2[u];
  }
  float w3v[16];
#pragma unroll
  for (int i = 0; i < 16; i++) w3v[i] = M->w3[16 * kg + i];
  const int a1 = M->a1, a2 = M->a2;
  const float b3 = M->b3, thr = M->threshold;
  for (int t = blockIdx.x * 4 + w; t < ntiles; t += gridDim.x * 4) {
    const int rr = 16 * t + row;
    bf16x8 A;
#pragma unroll
    for (int i = 0; i < 8; i++) A[i] = (__bf16)(rr < n ? X[(int64_t)rr * LEARN_NFEAT + 8 * kg + i] : 0.0f);
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B1[nt], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; r++) sh[w][4 * kg + r][16 * nt + row] = (__bf16)requant(acc[r] + b1v[nt], a1);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    bf16x8 A2[2];
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
      for (int i = 0; i < 8; i++) A2[ks][i] = sh[w][row][32 * ks + 8 * kg + i];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[0], B2[nt][0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[1], B2[nt][1], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; r++) sh[w][4 * kg + r][16 * nt + row] = (__bf16)requant(acc[r] + b2v[nt], a2);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; i++) s += w3v[i] * (float)sh[w][row][16 * kg + i];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (kg == 0 && rr < n) {
      const float z = b3 + s;
      if (out) out[rr] = z;
      const int h = key ? cand[rr] : 0;
      if (key && z < thr && !(fmesh && use_m && !use_m[fmesh[h / 3]])) {
        key[h] = PAMO_KEY_MAX;
        key[twin[h]] = PAMO_KEY_MAX;
        const int slot = atomicAdd(ndemote, 1);
        if (dlist) dlist[slot] = h;
        if (fmesh) atomicAdd(&ndemote_m[fmesh[h / 3]], 1);
      }
    }
  }
}

// ------------------------------------------------------------ training
constexpr int TS = 32;  // samples per block (the block's working set stays under 64 KB of LDS)

__device__ __forceinline__ float qw(float w, int e) {
  float s = ldexpf(w, e);
  float k = rintf(s);
  k = k > 127.0f ? 127.0f : (k < -127.0f ? -127.0f : k);
  return ldexpf(k, -e);
}
__device__ __forceinline__ float qb(float b, int e) {
  float s = ldexpf(b, e);
  float k = rintf(s);
  const float M = 4194304.0f;  // 2^22
  k = k > M ? M : (k < -M ? -M : k);
  return ldexpf(k, -e);
}

// Forward and backward of one batch slice of TS samples per block; writes the
// block's summed parameter gradient (straight-through roundings, before the
// clamp masks of the weights) and summed loss.
__global__ __launch_bounds__(256) void k_train_grad(const float* __restrict__ P, MlpMeta meta,
                                                    const float* __restrict__ X, const uint8_t* __restrict__ Y,
                                                    const int* __restrict__ order, int64_t base, int nb,
                                                    int64_t nrows, float inv_b, float* __restrict__ part,
                                                    float* __restrict__ part_loss) {
  extern __shared__ float lds[];
  float* W = lds;                          // quantised parameters, flat layout
  float* x = W + LEARN_NPARAM + 3;         // [TS][32]
  float* h1 = x + TS * 32;                 // [TS][64]
  float* g1 = h1 + TS * 64;                // derivative, then d z1
  float* h2 = g1 + TS * 64;
  float* g2 = h2 + TS * 64;                // derivative, then d z2
  float* z3 = g2 + TS * 64;                // [TS]: logit, then d logit
  float* yv = z3 + TS;
  const int tid = threadIdx.x;
  for (int p = tid; p < LEARN_NPARAM; p += 256) {
    float v = P[p];
    int e = p < MLP_O_W2 ? meta.e1 : (p < MLP_O_W3 ? meta.e2 : meta.e3);
    bool bias = (p >= MLP_O_B1 && p < MLP_O_W2) || (p >= MLP_O_B2 && p < MLP_O_W3) || p == MLP_O_B3;
    W[p] = bias ? qb(v, e) : qw(v, e);
  }
  const int s0 = blockIdx.x * TS;
  // rows outside [0, nrows) count as absent samples
  for (int i = tid; i < TS * 32; i += 256) {
    int s = i / 32, k = i % 32;
    int gs = s0 + s;
    float v = 0.0f;
    if (gs < nb) {
      int64_t row = order ? order[base + gs] : base + gs;
      if (row >= 0 && row < nrows) v = X[row * LEARN_NFEAT + k];
    }
    x[i] = v;
  }
  if (tid < TS) {
    int gs = s0 + tid;
    float v = -1.0f;  // -1: absent
    if (gs < nb) {
      int64_t row = order ? order[base + gs] : base + gs;
      if (row >= 0 && row < nrows) v = (float)Y[row];
    }
    yv[tid] = v;
  }
  __syncthreads();
  const int s = tid >> 3, part8 = tid & 7;  // 8 lanes per sample
  const float sc1 = ldexpf(1.0f, meta.a1), sc2 = ldexpf(1.0f, meta.a2);
  // layer 1
  for (int jj = 0; jj < 8; jj++) {
    int j = 8 * part8 + jj;
    float z = W[MLP_O_B1 + j];
    for (int k = 0; k < 32; k++) z += W[MLP_O_W1 + j * 32 + k] * x[s * 32 + k];
    float sz = ldexpf(z > 0.0f ? z : 0.0f, meta.a1);
    float q = rintf(sz);
    h1[s * 64 + j] = q > 127.0f ? 127.0f : q;
    g1[s * 64 + j] = (z > 0.0f && sz <= 127.0f) ? sc1 : 0.0f;
  }
  __syncthreads();
  // layer 2
  for (int jj = 0; jj < 8; jj++) {
    int j = 8 * part8 + jj;
    float z = W[MLP_O_B2 + j];
    for (int k = 0; k < 64; k++) z += W[MLP_O_W2 + j * 64 + k] * h1[s * 64 + k];
    float sz = ldexpf(z > 0.0f ? z : 0.0f, meta.a2);
    float q = rintf(sz);
    h2[s * 64 + j] = q > 127.0f ? 127.0f : q;
    g2[s * 64 + j] = (z > 0.0f && sz <= 127.0f) ? sc2 : 0.0f;
  }
  __syncthreads();
  // layer 3 (8 lanes per sample)
  float acc = 0.0f;
  for (int kk = 0; kk < 8; kk++) {
    int k = 8 * part8 + kk;
    acc += W[MLP_O_W3 + k] * h2[s * 64 + k];
  }
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 4, 64);
  float lossv = 0.0f;
  if (part8 == 0) {
    float z = W[MLP_O_B3] + acc;
    float y = yv[s];
    bool valid = y >= 0.0f;
    float sig = 1.0f / (1.0f + expf(-z));
    z3[s] = valid ? (sig - y) * inv_b : 0.0f;
    lossv = valid ? (fmaxf(z, 0.0f) - y * z + log1pf(expf(-fabsf(z)))) : 0.0f;
  }
  __syncthreads();
  // d z2 = d logit * w3 * derivative
  for (int jj = 0; jj < 8; jj++) {
    int j = 8 * part8 + jj;
    g2[s * 64 + j] = z3[s] * W[MLP_O_W3 + j] * g2[s * 64 + j];
  }
  __syncthreads();
  // d z1 = (W2^T d z2) * derivative
  for (int kk = 0; kk < 8; kk++) {
    int k = 8 * part8 + kk;
    float d = 0.0f;
    for (int j = 0; j < 64; j++) d += W[MLP_O_W2 + j * 64 + k] * g2[s * 64 + j];
    g1[s * 64 + k] = d * g1[s * 64 + k];
  }
  __syncthreads();
  // parameter gradients summed over the block's samples
  float* out = part + (int64_t)blockIdx.x * LEARN_NPARAM;
  for (int p = tid; p < LEARN_NPARAM; p += 256) {
    float gsum = 0.0f;
    if (p < MLP_O_B1) {
      int j = p / 32, k = p % 32;
      for (int t = 0; t < TS; t++) gsum += g1[t * 64 + j] * x[t * 32 + k];
    } else if (p < MLP_O_W2) {
      int j = p - MLP_O_B1;
      for (int t = 0; t < TS; t++) gsum += g1[t * 64 + j];
    } else if (p < MLP_O_B2) {
      int q = p - MLP_O_W2, j = q / 64, k = q % 64;
      for (int t = 0; t < TS; t++) gsum += g2[t * 64 + j] * h1[t * 64 + k];
    } else if (p < MLP_O_W3) {
      int j = p - MLP_O_B2;
      for (int t = 0; t < TS; t++) gsum += g2[t * 64 + j];
    } else if (p < MLP_O_B3) {
      int k = p - MLP_O_W3;
      for (int t = 0; t < TS; t++) gsum += z3[t] * h2[t * 64 + k];
    } else {
      for (int t = 0; t < TS; t++) gsum += z3[t];
    }
    out[p] = gsum;
  }
  // block loss
  __shared__ float lsum[4];
  float ls = lossv;
  for (int d = 32; d >= 1; d >>= 1) ls += __shfl_xor(ls, d, 64);
  if ((tid & 63) == 0) lsum[tid >> 6] = ls;
  __syncthreads();
  if (tid == 0) part_loss[blockIdx.x] = lsum[0] + lsum[1] + lsum[2] + lsum[3];
}

// Sum the block gradients in block order, apply the straight-through clamp
// masks, then either store the gradient or take an Adam step (t >= 1).
__global__ __launch_bounds__(256) void k_train_reduce(const float* __restrict__ part,
                                                      const float* __restrict__ part_loss, int nblocks,
                                                      float inv_b, MlpMeta meta, float* __restrict__ P,
                                                      float* __restrict__ grad, float* __restrict__ am,
                                                      float* __restrict__ av, float lr, float bc1, float bc2,
                                                      float* __restrict__ loss_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss_out) {
    float l = 0.0f;
    for (int b = 0; b < nblocks; b++) l += part_loss[b];
    *loss_out = l * inv_b;
  }
  if (p >= LEARN_NPARAM) return;
  float g = 0.0f;
  for (int b = 0; b < nblocks; b++) g += part[(int64_t)b * LEARN_NPARAM + p];
  int e = p < MLP_O_W2 ? meta.e1 : (p < MLP_O_W3 ? meta.e2 : meta.e3);
  bool bias = (p >= MLP_O_B1 && p < MLP_O_W2) || (p >= MLP_O_B2 && p < MLP_O_W3) || p == MLP_O_B3;
  float s = fabsf(ldexpf(P[p], e));
  if (s > (bias ? 4194304.0f : 127.0f)) g = 0.0f;
  if (grad) grad[p] = g;
  if (am) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float m = b1 * am[p] + (1.0f - b1) * g;
    float v = b2 * av[p] + (1.0f - b2) * g * g;
    am[p] = m;
    av[p] = v;
    float mh = m / bc1, vh = v / bc2;
    P[p] = P[p] - lr * mh / (sqrtf(vh) + eps);
  }
}

// candidates of meshes whose learned round is run again take a reason that
// sets no flag (5)
__global__ void k_mark_retry(const int* __restrict__ cand, const int* __restrict__ ncand,
                             const int* __restrict__ fmesh, const int* __restrict__ demote_m,
                             const int* __restrict__ commits_m, uint8_t* __restrict__ reason,
                             const int* __restrict__ gate) {
  if (gate && *gate) return;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= *ncand) return;
  int m = fmesh[cand[c] / 3];
  if (demote_m[m] > 0 && commits_m[m] == 0) reason[c] = 5;
}

// ------------------------------------------------------------ training rows
__global__ void k_row_flags(const int* __restrict__ ncand, int bound, const uint8_t* __restrict__ reason,
                            uint8_t* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < bound) flag[c] = c < *ncand && reason[c] <= 3;
}

__global__ void k_row_copy(const int* __restrict__ idx, const int* __restrict__ nrows, const float* __restrict__ Xs,
                           const uint8_t* __restrict__ reason, float* __restrict__ X, uint8_t* __restrict__ y,
                           int64_t room) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= *nrows || i >= room) return;
  int c = idx[i];
#pragma unroll
  for (int k = 0; k < LEARN_NFEAT; k++) X[i * LEARN_NFEAT + k] = Xs[(int64_t)c * LEARN_NFEAT + k];
  y[i] = reason[c] == 0;
}

// ------------------------------------------------------------ Hausdorff
constexpr int HT = 256;

// distance of each point to the closest triangle: blocks of HT points sweep
// the triangles in tiles staged through LDS
__global__ __launch_bounds__(HT) void k_point_surface(const double* __restrict__ P, int np,
                                                      const double* __restrict__ V, const int* __restrict__ F,
                                                      int nf, double* __restrict__ dist, uint64_t* dmax_bits) {
  __shared__ double tri[HT][9];
  const int i = blockIdx.x * HT + threadIdx.x;
  P3 p = i < np ? ld3(P, i) : P3{0, 0, 0};
  double best = INFINITY;
  for (int t0 = 0; t0 < nf; t0 += HT) {
    int t = t0 + threadIdx.x;
    if (t < nf) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        P3 q = ld3(V, F[3 * t + c]);
        tri[threadIdx.x][3 * c] = q.x;
        tri[threadIdx.x][3 * c + 1] = q.y;
        tri[threadIdx.x][3 * c + 2] = q.z;
      }
    }
    __syncthreads();
    int cnt = nf - t0 < HT ? nf - t0 : HT;
    for (int j = 0; j < cnt; j++) {
      const double* q = tri[j];
      double d = tri_dist2(p, P3{q[0], q[1], q[2]}, P3{q[3], q[4], q[5]}, P3{q[6], q[7], q[8]});
      best = d < best ? d : best;
    }
    __syncthreads();
  }
  if (i < np) {
    double d = sqrt(best);
    if (dist) dist[i] = d;
    uint64_t bits;
    __builtin_memcpy(&bits, &d, 8);
    atomicMax((unsigned long long*)dmax_bits, (unsigned long long)bits);  // d >= 0: bit order = value order
  }
}

}  // namespace

// ============================================================ host wrappers
void launch_features(hipStream_t s, MeshView m, const uint64_t* key, const int* cand, const int* ncand, int bound,
                     const int* ovl, float* X, int* err, const int* fmesh, const uint8_t* use_m) {
  hipLaunchKernelGGL(k_features, dim3(nblk(bound)), dim3(256), 0, s, m, key, cand, ncand, ovl, X, err, fmesh, use_m);
  PAMO_HIP(hipGetLastError());
}

void launch_mlp(hipStream_t s, const float* X, const int* n_dev, int bound, const MlpDev* M, float* out,
                const int* cand, const int* twin, uint64_t* key, int* ndemote, const int* fmesh, int* ndemote_m,
                const uint8_t* use_m, int* dlist) {
  int64_t tiles = (bound + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp, dim3((unsigned)blocks), dim3(256), 0, s, X, n_dev, M, out, cand, twin, key, ndemote,
                     fmesh, ndemote_m, use_m, dlist);
  PAMO_HIP(hipGetLastError());
}

void launch_mark_retry(hipStream_t s, const int* cand, const int* ncand, int bound, const int* fmesh,
                       const int* demote_m, const int* commits_m, uint8_t* reason, const int* gate) {
  hipLaunchKernelGGL(k_mark_retry, dim3(nblk(bound)), dim3(256), 0, s, cand, ncand, fmesh, demote_m, commits_m, reason,
                     gate);
  PAMO_HIP(hipGetLastError());
}

void learn_reserve(Workspace& ws, int64_t bound) {
  ws.get<uint8_t>("log.flag", bound);
  ws.get<int>("log.idx", bound);
}

void launch_log_rows(Workspace& ws, hipStream_t s, const int* ncand, int bound, const uint8_t* reason, const float* Xs,
                     float* X, uint8_t* y, int64_t room, int* nrows) {
  uint8_t* flag = ws.get<uint8_t>("log.flag", bound);
  int* idx = ws.get<int>("log.idx", bound);
  hipLaunchKernelGGL(k_row_flags, dim3(nblk(bound)), dim3(256), 0, s, ncand, bound, reason, flag);
  compact_flags(ws, s, flag, bound, idx, nrows);
  hipLaunchKernelGGL(k_row_copy, dim3(nblk(bound)), dim3(256), 0, s, (const int*)idx, (const int*)nrows, Xs, reason, X,
                     y, room);
  PAMO_HIP(hipGetLastError());
}

size_t train_lds_bytes() { return sizeof(float) * (LEARN_NPARAM + 3 + TS * 32 + 4 * TS * 64 + 2 * TS); }

void launch_train_grad(hipStream_t s, const float* P, MlpMeta meta, const float* X, const uint8_t* Y,
                       const int* order, int64_t base, int nb, int64_t nrows, float* part, float* part_loss) {
  int blocks = (nb + TS - 1) / TS;
  hipLaunchKernelGGL(k_train_grad, dim3(blocks), dim3(256), train_lds_bytes(), s, P, meta, X, Y, order, base, nb,
                     nrows, 1.0f / (float)nb, part, part_loss);
  PAMO_HIP(hipGetLastError());
}

void launch_train_reduce(hipStream_t s, const float* part, const float* part_loss, int nb, MlpMeta meta, float* P,
                         float* grad, float* am, float* av, float lr, int64_t t, float* loss_out) {
  int blocks = (nb + TS - 1) / TS;
  float bc1 = t > 0 ? 1.0f - powf(0.9f, (float)t) : 1.0f;
  float bc2 = t > 0 ? 1.0f - powf(0.999f, (float)t) : 1.0f;
  hipLaunchKernelGGL(k_train_reduce, dim3(nblk(LEARN_NPARAM)), dim3(256), 0, s, part, part_loss, blocks,
                     1.0f / (float)nb, meta, P, grad, am, av, lr, bc1, bc2, loss_out);
  PAMO_HIP(hipGetLastError());
}

int train_blocks(int nb) { return (nb + TS - 1) / TS; }

void launch_point_surface(hipStream_t s, const double* P, int np, const double* V, const int* F, int nf,
                          double* dist, uint64_t* dmax_bits) {
  hipLaunchKernelGGL(k_point_surface, dim3(nblk(np, HT)), dim3(HT), 0, s, P, np, V, F, nf, dist, dmax_bits);
  PAMO_HIP(hipGetLastError());
}

}  // namespace pamo
