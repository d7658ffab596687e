// Linear BVH over triangle boxes and the queries of the check/undo loop
// (the paper's intersection check, Sec. 5.2, uses a Karras-style LBVH).
//
// Build: 30-bit Morton code of each box centre -> stable radix sort -> a
// balanced implicit binary tree over the sorted leaves (node k has children
// 2k+1, 2k+2; leaf j sits below node (2^H - 1 + j - 1) / 2).  Boxes are
// reduced level by level inside LDS, 11 levels per launch, so the build needs
// no atomics and no device-scope fences: on a chip whose L2 is split over 8
// XCDs those fences write back L2 and dominated the atomic bottom-up pass of a
// Karras tree.  Depth is ceil(log2 n), which bounds the traversal stack.
// Each node stores both child boxes (64 B, one load per visit).
//
// Query: one thread per query triangle walks the tree and only collects
// candidate pairs (wave-aggregated appends); a second kernel evaluates the
// filtered pair predicate one pair per thread; pairs the float filter cannot
// decide go to an exact pass.
#include "exact_dev.hpp"
#include "round.hpp"

namespace pamo {

namespace {

constexpr int LVL = 11;  // levels reduced per launch (2048 boxes in LDS)
constexpr int LVL_T = 256;
constexpr int STACK = 32;  // >= tree depth - 1; depth <= 30 for int32 face ids

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 10; i++) r |= ((v >> i) & 1u) << (3 * i);
  return r;
}

__global__ void k_morton(const float* __restrict__ box, int n, uint32_t* __restrict__ code, int* __restrict__ id) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const float* b = box + 6 * (int64_t)f;
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    float c = 0.5f * (b[k] + b[k + 3]);
    c = fminf(fmaxf(c, 0.0f), 1.0f);
    int x = (int)(c * 1024.0f);
    q[k] = (uint32_t)(x > 1023 ? 1023 : x);
  }
  code[f] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  id[f] = f;
}

// batches: key = (mesh, Morton code of the box centre moved back to [0,1]^3)
__global__ void k_morton_mesh(const float* __restrict__ box, int n, const int* __restrict__ fmesh,
                              uint64_t* __restrict__ code, int* __restrict__ id) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const float* b = box + 6 * (int64_t)f;
  int m = fmesh[f];
  double o[3];
  mesh_shift(m, o[0], o[1], o[2]);
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    float c = 0.5f * (b[k] + b[k + 3]) - (float)o[k];
    c = fminf(fmaxf(c, 0.0f), 1.0f);
    int x = (int)(c * 1024.0f);
    q[k] = (uint32_t)(x > 1023 ? 1023 : x);
  }
  code[f] = ((uint64_t)m << 30) | (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  id[f] = f;
}

struct Box {
  float lo[3], hi[3];
};

__device__ __forceinline__ Box empty_box() {
  Box b;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    b.lo[k] = INFINITY;
    b.hi[k] = -INFINITY;
  }
  return b;
}

__device__ __forceinline__ Box unite(const Box& a, const Box& b) {
  Box r;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    r.lo[k] = fminf(a.lo[k], b.lo[k]);
    r.hi[k] = fmaxf(a.hi[k], b.hi[k]);
  }
  return r;
}

__device__ __forceinline__ void write_node(BvhNode* nodes, int64_t k, const Box& L, const Box& R, int lf, int rf) {
  BvhNode n;
  n.a = make_float4(L.lo[0], L.lo[1], L.lo[2], L.hi[0]);
  n.b = make_float4(L.hi[1], L.hi[2], R.lo[0], R.lo[1]);
  n.c = make_float4(R.lo[2], R.hi[0], R.hi[1], R.hi[2]);
  n.d = make_int4(lf, rf, 0, 0);
  nodes[k] = n;
}

// One launch reduces `lv` levels above level l0.  Block b owns the 2^lv boxes
// [b 2^lv, (b+1) 2^lv) of level l0 (leaves when l0 == 0: box of face
// sorted[j], empty beyond n), writes the node records of levels l0+1..l0+lv
// and the box of its subtree root to top[b].
__global__ __launch_bounds__(LVL_T) void k_levels(const float* __restrict__ leafbox, const int* __restrict__ sorted,
                                                  int n, const Box* __restrict__ in, Box* __restrict__ top, int l0,
                                                  int lv, int H, BvhNode* __restrict__ nodes) {
  __shared__ Box sb[1 << LVL];
  __shared__ int sf[1 << LVL];
  const int M = 1 << lv;
  const int64_t base = (int64_t)blockIdx.x * M;
  for (int i = threadIdx.x; i < M; i += LVL_T) {
    int64_t j = base + i;
    Box b = empty_box();
    int f = -1;
    if (l0 == 0) {
      if (j < n) {
        f = sorted[j];
        const float* p = leafbox + 6 * (int64_t)f;
        b = Box{{p[0], p[1], p[2]}, {p[3], p[4], p[5]}};
      }
    } else {
      b = in[j];
    }
    sb[i] = b;
    sf[i] = f;
  }
  __syncthreads();
  const int64_t N0 = (int64_t)1 << H;
  for (int k = 1; k <= lv; k++) {
    int cnt = M >> k;
    int level = l0 + k;
    Box u[(1 << LVL) / 2 / LVL_T];
    int nu = 0;
    for (int t = threadIdx.x; t < cnt; t += LVL_T) {
      Box L = sb[2 * t], R = sb[2 * t + 1];
      int lf = level == 1 ? sf[2 * t] : -1, rf = level == 1 ? sf[2 * t + 1] : -1;
      int64_t j = (base >> k) + t;
      write_node(nodes, (N0 >> level) - 1 + j, L, R, lf, rf);
      u[nu++] = unite(L, R);
    }
    __syncthreads();
    nu = 0;
    for (int t = threadIdx.x; t < cnt; t += LVL_T) sb[t] = u[nu++];
    __syncthreads();
  }
  if (threadIdx.x == 0) top[blockIdx.x] = sb[0];
}

// ------------------------------------------------------------ queries
struct Tri {
  P3 p[3];
  int id[3];
  double lo[3], hi[3];
};

__device__ __forceinline__ void load_tri(const double* __restrict__ V, const int* __restrict__ F, int f, Tri& T) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    T.id[k] = F[3 * f + k];
    T.p[k] = ld3(V, T.id[k]);
  }
  T.lo[0] = fmin(fmin(T.p[0].x, T.p[1].x), T.p[2].x);
  T.lo[1] = fmin(fmin(T.p[0].y, T.p[1].y), T.p[2].y);
  T.lo[2] = fmin(fmin(T.p[0].z, T.p[1].z), T.p[2].z);
  T.hi[0] = fmax(fmax(T.p[0].x, T.p[1].x), T.p[2].x);
  T.hi[1] = fmax(fmax(T.p[0].y, T.p[1].y), T.p[2].y);
  T.hi[2] = fmax(fmax(T.p[0].z, T.p[1].z), T.p[2].z);
}

__device__ __forceinline__ bool share_vertex(const Tri& A, const Tri& B) {
  bool r = false;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) r |= A.id[i] == B.id[j];
  return r;
}

__device__ __forceinline__ bool tri_box_overlap(const Tri& A, const Tri& B) {
#pragma unroll
  for (int k = 0; k < 3; k++)
    if (A.hi[k] < B.lo[k] || B.hi[k] < A.lo[k]) return false;
  return true;
}

template <int MODE>
__device__ __forceinline__ void mark(const QueryArgs& a, int t, int u) {
  if (MODE == QUERY_ALL_PAIRS) {
    int k = atomicAdd(a.npairs, 1);
    if (k < a.pairs_cap) a.pairs[k] = make_int2(t, u);
    return;
  }
  if (MODE == QUERY_CHANGED) {
    int ot = a.owner[t];
    if (atomicCAS(&a.undone[ot], 0, a.iter) == 0) atomicAdd(a.nundo, 1);
  }
  int ou = a.owner[u];
  if (ou >= 0 && atomicCAS(&a.undone[ou], 0, a.iter) == 0) atomicAdd(a.nundo, 1);
}

// pair filters that need no geometry
template <int MODE>
__device__ __forceinline__ bool leaf_candidate(const QueryArgs& a, int t, int u) {
  if (u == t) return false;
  if (a.falive && !a.falive[u]) return false;
  if (a.fmesh && a.fmesh[u] != a.fmesh[t]) return false;  // batches: meshes never meet
  if (MODE == QUERY_ALL_PAIRS) return u > t;
  int ou = a.owner[u];
  if (MODE == QUERY_CHANGED) {
    // both changed: the query of the smaller face takes the pair
    if (ou >= 0 && u < t) return false;
    return true;
  }
  // QUERY_RESTORED: t is restored (pre-round geometry); only currently
  // changed faces can meet it
  if (ou < 0) return false;
  int st = a.undone[ou];
  if (st != 0 && st < a.iter) return false;
  return true;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

constexpr int WPB = 4;     // waves per block in the packet traversal
constexpr int SEG = 256;   // staged pairs per wave before a flush

// Per-wave staging of candidate pairs in LDS: lanes append without atomics
// (ballot prefix); the wave flushes to the global buffer with one atomic per
// ~200 pairs.  `fill` is wave-uniform.
struct Stage {
  int2* buf;  // this wave's LDS segment
  int fill;
};

__device__ __forceinline__ void stage_flush(Stage& st, int2* gbuf, int* gcnt, int cap) {
  if (st.fill == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  int lane = lane_id();
  int base = 0;
  if (lane == 0) base = atomicAdd(gcnt, st.fill);
  base = __shfl(base, 0, 64);
  for (int j = lane; j < st.fill; j += 64)
    if (base + j < cap) gbuf[base + j] = st.buf[j];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  st.fill = 0;
}

__device__ __forceinline__ void stage_append(Stage& st, bool has, int t, int u, int2* gbuf, int* gcnt, int cap) {
  unsigned long long m = __ballot(has);
  if (m == 0) return;
  int lane = lane_id();
  if (has) {
    unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    st.buf[st.fill + __popcll(m & lt)] = make_int2(t, u);
  }
  st.fill += __popcll(m);
  if (st.fill > SEG - 64) stage_flush(st, gbuf, gcnt, cap);
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fminf(x, __shfl_xor(x, d, 64));
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, 64));
  return x;
}

__device__ __forceinline__ bool box_hit(const float* tb, float lx, float ly, float lz, float hx, float hy, float hz) {
  return tb[0] <= hx && lx <= tb[3] && tb[1] <= hy && ly <= tb[4] && tb[2] <= hz && lz <= tb[5];
}

// min/max over the G lanes of a packet (G a power of two <= 64)
template <int G>
__device__ __forceinline__ float group_min(float x) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) x = fminf(x, __shfl_xor(x, d, 64));
  return x;
}
template <int G>
__device__ __forceinline__ float group_max(float x) {
#pragma unroll
  for (int d = G / 2; d >= 1; d >>= 1) x = fmaxf(x, __shfl_xor(x, d, 64));
  return x;
}

// float32 box of query face t, rounded outward, in its mesh's cell
__device__ __forceinline__ void query_box(const QueryArgs& a, int t, float* tb) {
  Tri T;
  load_tri(a.V, a.F, t, T);
  double o[3] = {0, 0, 0};
  if (a.fmesh) mesh_shift(a.fmesh[t], o[0], o[1], o[2]);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    double dl = T.lo[k] + o[k], dh = T.hi[k] + o[k];
    float lo = (float)dl, hi = (float)dh;
    if ((double)lo > dl) lo = nextafterf(lo, -INFINITY);
    if ((double)hi < dh) hi = nextafterf(hi, INFINITY);
    tb[k] = lo;
    tb[k + 3] = hi;
  }
}

// Wave-cooperative traversal in packets of G lanes.  The query list is in
// Morton order, so the G queries of a packet are neighbours; each packet walks
// the tree once (its lanes load the same node: one coalesced request), entering
// a child when any of its lanes' own boxes meets it (the packet's union box is
// a cheap uniform pre-test).  The 64/G packets of a wave advance in lockstep,
// each with its own stack in LDS.  At a node whose children are leaves every
// lane tests its own box; hits are staged per wave in LDS and flushed with one
// atomic per ~200 pairs.  The traversal does no data-dependent loads besides
// the nodes: the state filters run in the pair kernel.
template <int MODE, int G>
__global__ __launch_bounds__(64 * WPB) void k_collect(const BvhNode* __restrict__ nodes, int H, int n,
                                                      const int* __restrict__ qlist, const int* __restrict__ nq,
                                                      QueryArgs a) {
  constexpr int NG = 64 / G;
  __shared__ int2 sbuf[WPB][SEG];
  __shared__ int sstack[WPB][NG][STACK];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int grp = lane / G;
  const unsigned long long gmask = (G == 64 ? ~0ull : (((1ull << G) - 1) << (grp * G)));
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nqv = *nq;
  if (blockIdx.x * blockDim.x + w * 64 >= nqv || n < 2) return;  // whole wave idle
  const bool active = i < nqv;
  const int t = active ? qlist[i] : -1;
  float tb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  if (active) query_box(a, t, tb);
  float ub[6];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    ub[k] = group_min<G>(tb[k]);
    ub[k + 3] = group_max<G>(tb[k + 3]);
  }
  Stage st{sbuf[w], 0};
  int* stk = sstack[w][grp];
  const int64_t leaf0 = ((int64_t)1 << H) - 1;  // heap index of the first leaf
  // a packet with no active lane has an empty union box: it is done at once
  bool done = !(ub[0] <= ub[3]);
  int sp = 0;
  int node = 0;
  while (__ballot(!done)) {
    bool hl = false, hr = false;
    int lf = 0, rf = 0;
    if (!done) {
      const BvhNode nd = nodes[node];
      const bool uL = box_hit(ub, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y);
      const bool uR = box_hit(ub, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w);
      const bool oL = uL && box_hit(tb, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y);
      const bool oR = uR && box_hit(tb, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w);
      const int cl = 2 * node + 1;
      int next = -1;
      if (cl >= leaf0) {  // both children are leaves
        lf = nd.d.x;
        rf = nd.d.y;
        hl = oL && lf >= 0 && lf != t;
        hr = oR && rf >= 0 && rf != t;
      } else {
        const bool anyL = (__ballot(oL) & gmask) != 0, anyR = (__ballot(oR) & gmask) != 0;
        if (anyL) {
          next = cl;
          if (anyR) stk[sp++] = cl + 1;  // depth <= H < STACK; every lane of the packet writes the same value
        } else if (anyR) {
          next = cl + 1;
        }
      }
      if (next < 0) {
        if (sp == 0)
          done = true;
        else
          next = stk[--sp];
      }
      node = next;
    }
    stage_append(st, hl, t, lf, a.cand, a.ncand, a.cand_cap);
    stage_append(st, hr, t, rf, a.cand, a.ncand, a.cand_cap);
  }
  stage_flush(st, a.cand, a.ncand, a.cand_cap);
}

// Cooperative traversal: G lanes share ONE query.  The group keeps a stack of
// pending nodes in LDS; each step its lanes pop up to G nodes (one each), load
// them in parallel, test both children against the query box, push the
// internal children that meet it and stage the leaf hits.  A query costs
// about max(depth, visited nodes / G) dependent loads instead of one per
// visited node, which matters when few queries are left (late rounds) and the
// walk is bound by load latency rather than throughput.  Popping the top G
// entries leaves at most G entries behind per level descended, so the stack
// holds at most G (H + 2) entries.
constexpr int COOP_HMAX = 24;

template <int MODE, int G>
__global__ __launch_bounds__(64 * WPB) void k_collect_coop(const BvhNode* __restrict__ nodes, int H, int n,
                                                           const int* __restrict__ qlist, const int* __restrict__ nq,
                                                           QueryArgs a) {
  constexpr int NG = 64 / G;
  constexpr int CST = G * (COOP_HMAX + 2);
  __shared__ int2 sbuf[WPB][SEG];
  __shared__ int sstack[WPB][NG][CST];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int grp = lane / G, gl = lane % G;
  const unsigned long long gmask = (G == 64 ? ~0ull : (((1ull << G) - 1) << (grp * G)));
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int wave_q0 = (blockIdx.x * WPB + w) * NG;
  const int nqv = *nq;
  if (wave_q0 >= nqv || n < 2) return;  // whole wave idle
  const int q = wave_q0 + grp;
  const bool active = q < nqv;
  const int t = active ? qlist[q] : -1;
  float tb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  if (active) query_box(a, t, tb);
  Stage st{sbuf[w], 0};
  int* stk = sstack[w][grp];
  const int64_t leaf0 = ((int64_t)1 << H) - 1;
  if (active && gl == 0) stk[0] = 0;
  int sp = active ? 1 : 0;  // uniform over the group
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  while (__ballot(sp > 0)) {
    const int take = sp < G ? sp : G;
    const int node = gl < take ? stk[sp - take + gl] : -1;
    sp -= take;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // pops read before pushes overwrite
    bool hl = false, hr = false, pl = false, pr = false;
    int lf = 0, rf = 0;
    const int cl = 2 * node + 1;
    if (node >= 0) {
      const BvhNode nd = nodes[node];
      const bool oL = box_hit(tb, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y);
      const bool oR = box_hit(tb, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w);
      if (cl >= leaf0) {
        lf = nd.d.x;
        rf = nd.d.y;
        hl = oL && lf >= 0 && lf != t;
        hr = oR && rf >= 0 && rf != t;
      } else {
        pl = oL;
        pr = oR;
      }
    }
    const unsigned long long bl = __ballot(pl) & gmask, br = __ballot(pr) & gmask;
    int pos = sp + __popcll(bl & below) + __popcll(br & below);
    if (pl) {
      if (pos < CST) stk[pos] = cl;
      pos++;
    }
    if (pr && pos < CST) stk[pos] = cl + 1;
    sp += __popcll(bl) + __popcll(br);
    if (sp > CST) {  // cannot happen for H <= COOP_HMAX; report instead of losing pairs
      if (gl == 0) atomicOr(a.err, PAMO_EBIT_STACK);
      sp = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    stage_append(st, hl, t, lf, a.cand, a.ncand, a.cand_cap);
    stage_append(st, hr, t, rf, a.cand, a.ncand, a.cand_cap);
  }
  stage_flush(st, a.cand, a.ncand, a.cand_cap);
}

// evaluate the collected pairs: exact float64 box test, filtered predicate,
// mark the owners of intersecting pairs, defer the undecided ones
template <int MODE>
__global__ __launch_bounds__(256, 5) void k_pairs(QueryArgs a) {
  int n = *a.ncand;
  if (n > a.cand_cap) n = a.cand_cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int2 pr = a.cand[i];
    // the triangles are loaded alongside the state filter rather than after
    // it: one dependent load fewer on the path of every pair
    Tri T, U;
    load_tri(a.V, a.F, pr.x, T);
    load_tri(a.V, a.F, pr.y, U);
    if (a.ovl_cnt && (!a.falive || a.falive[pr.y]) && (!a.fmesh || a.fmesh[pr.y] == a.fmesh[pr.x]) &&
        !share_vertex(T, U) && tri_box_overlap(T, U))
      atomicAdd(&a.ovl_cnt[pr.x], 1);
    if (!leaf_candidate<MODE>(a, pr.x, pr.y)) continue;
    if (!tri_box_overlap(T, U)) continue;
    int r = tri_pair<false>(T.p, T.id, U.p, U.id);
    if (r == 1) {
      mark<MODE>(a, pr.x, pr.y);
    } else if (r == UNK) {
      int k = atomicAdd(a.ndefer, 1);
      if (k < a.defer_cap)
        a.defer[k] = pr;
      else
        atomicOr(a.err, PAMO_EBIT_DEFER);
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(64) void k_resolve(QueryArgs a) {
  int n = *a.ndefer;
  if (n > a.defer_cap) n = a.defer_cap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int2 pr = a.defer[i];
    Tri T, U;
    load_tri(a.V, a.F, pr.x, T);
    load_tri(a.V, a.F, pr.y, U);
    if (tri_pair<true>(T.p, T.id, U.p, U.id) == 1) mark<MODE>(a, pr.x, pr.y);
  }
}

}  // namespace

Bvh build_bvh(Workspace& ws, hipStream_t s, const float* box, int nf, const int* order, const int* fmesh,
              int nmesh) {
  Bvh b;
  b.n = nf;
  int H = 1;
  while (((int64_t)1 << H) < nf) H++;
  b.H = H;
  int64_t N0 = (int64_t)1 << H;
  b.nodes = ws.get<BvhNode>("bvh.nodes", N0 - 1);
  b.sorted = nullptr;
  if (nf < 2) return b;
  const int* id = order;
  if (!order && !fmesh) {
    uint32_t* code = ws.get<uint32_t>("bvh.code", nf);
    int* ids = ws.get<int>("bvh.id", nf);
    hipLaunchKernelGGL(k_morton, dim3(nblk(nf)), dim3(256), 0, s, box, nf, code, ids);
    radix_sort_u32(ws, s, code, ids, nf, 30);
    id = ids;
  } else if (!order) {
    uint64_t* code = ws.get<uint64_t>("bvh.code64", nf);
    int* ids = ws.get<int>("bvh.id", nf);
    int mbits = 1;
    while ((1 << mbits) < nmesh) mbits++;
    hipLaunchKernelGGL(k_morton_mesh, dim3(nblk(nf)), dim3(256), 0, s, box, nf, fmesh, code, ids);
    radix_sort_u64(ws, s, code, ids, nf, 30 + mbits);
    id = ids;
  }
  b.sorted = id;
  Box* ta = ws.get<Box>("bvh.topA", (N0 >> LVL) + 1);
  Box* tb = ws.get<Box>("bvh.topB", (N0 >> LVL) + 1);
  int l0 = 0;
  const Box* in = nullptr;
  Box* out = ta;
  while (l0 < H) {
    int lv = H - l0 < LVL ? H - l0 : LVL;
    int64_t blocks = N0 >> (l0 + lv);
    hipLaunchKernelGGL(k_levels, dim3((unsigned)blocks), dim3(LVL_T), 0, s, box, id, nf, in, out, l0,
                       lv, H, b.nodes);
    in = out;
    out = out == ta ? tb : ta;
    l0 += lv;
  }
  PAMO_HIP(hipGetLastError());
  return b;
}

template <int G>
void launch_collect_g(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, dim3 g,
                      const QueryArgs& a) {
  dim3 t(64 * WPB);
  const BvhNode* nodes = bvh.nodes;
  if (mode == QUERY_CHANGED)
    hipLaunchKernelGGL((k_collect<QUERY_CHANGED, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL((k_collect<QUERY_RESTORED, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
  else
    hipLaunchKernelGGL((k_collect<QUERY_ALL_PAIRS, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
}

template <int G>
void launch_coop_g(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, int nq_bound,
                   const QueryArgs& a) {
  dim3 g(nblk((int64_t)nq_bound * G, 64 * WPB)), t(64 * WPB);
  const BvhNode* nodes = bvh.nodes;
  if (mode == QUERY_CHANGED)
    hipLaunchKernelGGL((k_collect_coop<QUERY_CHANGED, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL((k_collect_coop<QUERY_RESTORED, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
  else
    hipLaunchKernelGGL((k_collect_coop<QUERY_ALL_PAIRS, G>), g, t, 0, s, nodes, bvh.H, bvh.n, qlist, nq, a);
}

void launch_query(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, int nq_bound,
                  const QueryArgs& a, int packet, int coop) {
  if (nq_bound <= 0 || bvh.n < 2) return;
  if (bvh.H - 1 > STACK) throw std::runtime_error("BVH deeper than the traversal stack");
  if (coop > 1 && bvh.H <= COOP_HMAX) {
    switch (coop) {
      case 2: launch_coop_g<2>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      case 4: launch_coop_g<4>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      case 16: launch_coop_g<16>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      default: launch_coop_g<8>(s, bvh, mode, qlist, nq, nq_bound, a); break;
    }
    PAMO_HIP(hipGetLastError());
    return;
  }
  dim3 g(nblk(nq_bound, 64 * WPB));
  switch (packet) {
    case 2: launch_collect_g<2>(s, bvh, mode, qlist, nq, g, a); break;
    case 4: launch_collect_g<4>(s, bvh, mode, qlist, nq, g, a); break;
    case 8: launch_collect_g<8>(s, bvh, mode, qlist, nq, g, a); break;
    case 16: launch_collect_g<16>(s, bvh, mode, qlist, nq, g, a); break;
    case 32: launch_collect_g<32>(s, bvh, mode, qlist, nq, g, a); break;
    case 64: launch_collect_g<64>(s, bvh, mode, qlist, nq, g, a); break;
    default: launch_collect_g<1>(s, bvh, mode, qlist, nq, g, a); break;
  }
  PAMO_HIP(hipGetLastError());
}

void launch_pairs(hipStream_t s, QueryMode mode, const QueryArgs& a, int64_t pairs_est) {
  int64_t b = (pairs_est + 255) / 256;
  dim3 g((unsigned)(b < 64 ? 64 : b > 2048 ? 2048 : b)), t(256);
  if (mode == QUERY_CHANGED)
    hipLaunchKernelGGL(k_pairs<QUERY_CHANGED>, g, t, 0, s, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL(k_pairs<QUERY_RESTORED>, g, t, 0, s, a);
  else
    hipLaunchKernelGGL(k_pairs<QUERY_ALL_PAIRS>, g, t, 0, s, a);
  PAMO_HIP(hipGetLastError());
}

void launch_resolve(hipStream_t s, QueryMode mode, const QueryArgs& a) {
  dim3 g(256), t(64);
  if (mode == QUERY_CHANGED)
    hipLaunchKernelGGL(k_resolve<QUERY_CHANGED>, g, t, 0, s, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL(k_resolve<QUERY_RESTORED>, g, t, 0, s, a);
  else
    hipLaunchKernelGGL(k_resolve<QUERY_ALL_PAIRS>, g, t, 0, s, a);
  PAMO_HIP(hipGetLastError());
}

}  // namespace pamo
