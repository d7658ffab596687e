// Linear BVH over triangle boxes and the queries of the check/undo loop
// (the paper's intersection check, Sec. 5.2, uses a Karras-style LBVH).
//
// Build: 30-bit Hilbert index of each box centre -> stable radix sort -> a
// balanced implicit 4-ary tree over the sorted leaves (node k has children
// 4k+1 .. 4k+4).  The tree groups runs of consecutive leaves, so the curve
// matters: the Hilbert curve never jumps, a Morton curve does, and a node
// whose leaves straddle a jump gets a large box; with Hilbert order the
// headline's check queries take 15% less time than with Morton order (same
// pairs).  Boxes are reduced level by level inside LDS, five levels per
// launch, so the build needs no atomics and no device-scope fences: on a chip
// whose L2 is split over 8 XCDs those fences write back L2 and dominated the
// atomic bottom-up pass of a Karras tree.  A node holds the boxes of its four
// children (128 B, fetched together): a query walks half as many levels as in
// a binary tree.
//
// Query: one thread per query triangle walks the tree and only collects
// candidate pairs (wave-aggregated appends); a second kernel evaluates the
// filtered pair predicate one pair per thread; pairs the float filter cannot
// decide go to an exact pass.
#include "exact_dev.hpp"
#include "round.hpp"

namespace pamo {

namespace {

constexpr int LVL = 5;  // levels reduced per launch (4^5 = 1024 boxes in LDS)
constexpr int LVL_T = 256;
constexpr int STACK = 14;  // >= BVH_DMAX: one entry per level above the current node

// level of internal node k: (4^l - 1)/3 <= k < (4^(l+1) - 1)/3, i.e. 4^l <= 3k+1
__device__ __forceinline__ int node_level(int k) { return (31 - __clz(3 * k + 1)) >> 1; }
// index of the first node of level l
__device__ __forceinline__ int level_first(int l) { return (int)(((1u << (2 * l)) - 1u) / 3u); }

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }
// grids for xcd_item: a multiple of 8 blocks
inline unsigned nblk8(int64_t n, int t = 256) { return (nblk(n, t) + 7u) & ~7u; }

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 10; i++) r |= ((v >> i) & 1u) << (3 * i);
  return r;
}

// Hilbert index of a cell of the 1024^3 grid: the coordinates turned into the
// curve's "transpose" form (Skilling, Programming the Hilbert curve, 2004:
// undo the excess inversions and exchanges level by level, then Gray-code),
// whose bits interleaved give the index.  Consecutive indices are face
// neighbours.
__device__ __forceinline__ uint32_t hilbert30(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x, y, z};
  for (uint32_t Q = 512; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = 512; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  return (spread10(X[0] ^ t) << 2) | (spread10(X[1] ^ t) << 1) | spread10(X[2] ^ t);
}

__global__ void k_curve_codes(const float* __restrict__ box, int n, uint32_t* __restrict__ code,
                              int* __restrict__ id) {
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
  code[f] = hilbert30(q[0], q[1], q[2]);
  id[f] = f;
}

// batches: key = (mesh, Hilbert index of the box centre moved back to [0,1]^3)
__global__ void k_curve_codes_mesh(const float* __restrict__ box, int n, const int* __restrict__ fmesh,
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
  code[f] = ((uint64_t)m << 30) | hilbert30(q[0], q[1], q[2]);
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

__device__ __forceinline__ BvhNode make_node(const Box* c, int4 leaf) {
  BvhNode nd;
  nd.lx = make_float4(c[0].lo[0], c[1].lo[0], c[2].lo[0], c[3].lo[0]);
  nd.ly = make_float4(c[0].lo[1], c[1].lo[1], c[2].lo[1], c[3].lo[1]);
  nd.lz = make_float4(c[0].lo[2], c[1].lo[2], c[2].lo[2], c[3].lo[2]);
  nd.hx = make_float4(c[0].hi[0], c[1].hi[0], c[2].hi[0], c[3].hi[0]);
  nd.hy = make_float4(c[0].hi[1], c[1].hi[1], c[2].hi[1], c[3].hi[1]);
  nd.hz = make_float4(c[0].hi[2], c[1].hi[2], c[2].hi[2], c[3].hi[2]);
  nd.leaf = leaf;
  nd.pad = make_int4(0, 0, 0, 0);
  return nd;
}

// One launch reduces `lv` levels above height h0 (h0 = 0: the leaves).  Block
// b owns the 4^lv boxes [b 4^lv, (b+1) 4^lv) of height h0 (leaves: box of face
// sorted[j], empty beyond n; above: in[j], empty beyond cnt), writes the node
// records of heights h0+1 .. h0+lv and the box of its subtree root to top[b].
__global__ __launch_bounds__(LVL_T) void k_levels(const float* __restrict__ leafbox, const int* __restrict__ sorted,
                                                  int n, const Box* __restrict__ in, int cnt, Box* __restrict__ top,
                                                  int h0, int lv, int D, BvhNode* __restrict__ nodes,
                                                  const int* __restrict__ owner, const uint8_t* __restrict__ falive) {
  __shared__ Box sb[1 << (2 * LVL)];
  __shared__ int sf[1 << (2 * LVL)];
  const int M = 1 << (2 * lv);
  const int64_t base = (int64_t)blockIdx.x * M;
  for (int i = threadIdx.x; i < M; i += LVL_T) {
    int64_t j = base + i;
    Box b = empty_box();
    int f = -1;
    if (h0 == 0) {
      if (j < n) {
        f = sorted[j];
        const float* p = leafbox + 6 * (int64_t)f;
        b = Box{{p[0], p[1], p[2]}, {p[3], p[4], p[5]}};
        const bool chg = owner && owner[f] >= 0, dead = falive && !falive[f];
        f |= (chg ? LEAF_CHANGED : 0) | (dead ? LEAF_DEAD : 0);
      }
    } else if (j < cnt) {
      b = in[j];
    }
    sb[i] = b;
    sf[i] = f;
  }
  __syncthreads();
  for (int k = 1; k <= lv; k++) {
    const int cntk = M >> (2 * k);
    const int level = D - (h0 + k);
    const int64_t first = ((((int64_t)1) << (2 * level)) - 1) / 3;  // heap index of the level's first node
    static_assert((1 << (2 * LVL)) / 4 <= LVL_T, "one node per thread and level");
    Box u = empty_box();
    const int t = threadIdx.x;
    if (t < cntk) {
      const Box c[4] = {sb[4 * t], sb[4 * t + 1], sb[4 * t + 2], sb[4 * t + 3]};
      const int4 lf = h0 + k == 1 ? make_int4(sf[4 * t], sf[4 * t + 1], sf[4 * t + 2], sf[4 * t + 3])
                                  : make_int4(-1, -1, -1, -1);
      nodes[first + (base >> (2 * k)) + t] = make_node(c, lf);
      u = unite(unite(c[0], c[1]), unite(c[2], c[3]));
    }
    __syncthreads();
    if (t < cntk) sb[t] = u;
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
    if (k < a.pairs_cap) a.pairs[k] = t < u ? make_int2(t, u) : make_int2(u, t);
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
  if (MODE == QUERY_ALL_PAIRS) return true;  // staged once per pair (later_children)
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
// staged pairs per wave (one-lane walk, cooperative walk).  Every flush takes
// one atomic on the single global pair counter, and those atomics contend:
// the one-lane walk of the early rounds, which emits most pairs, runs 20%
// faster with 768 slots than with 256.
constexpr int SEG = 768;
constexpr int SEG_COOP = 256;

// Per-wave staging of candidate pairs in LDS: lanes append without atomics
// (ballot prefix); the wave flushes to the global buffer with one atomic per
// ~200 pairs.  `fill` is wave-uniform.
struct Stage {
  int2* buf;  // this wave's LDS segment
  int fill;
  int limit;  // flush beyond this fill (segment size - 64: room for one more append)
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
  if (st.fill > st.limit) stage_flush(st, gbuf, gcnt, cap);
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

// overlap mask of the four child boxes of nd with box b (bit c: child c)
__device__ __forceinline__ int child_hits(const BvhNode& nd, const float* b) {
  const float lx[4] = {nd.lx.x, nd.lx.y, nd.lx.z, nd.lx.w}, ly[4] = {nd.ly.x, nd.ly.y, nd.ly.z, nd.ly.w};
  const float lz[4] = {nd.lz.x, nd.lz.y, nd.lz.z, nd.lz.w}, hx[4] = {nd.hx.x, nd.hx.y, nd.hx.z, nd.hx.w};
  const float hy[4] = {nd.hy.x, nd.hy.y, nd.hy.z, nd.hy.w}, hz[4] = {nd.hz.x, nd.hz.y, nd.hz.z, nd.hz.w};
  int m = 0;
#pragma unroll
  for (int c = 0; c < 4; c++)
    m |= (lx[c] <= b[3] && b[0] <= hx[c] && ly[c] <= b[4] && b[1] <= hy[c] && lz[c] <= b[5] && b[2] <= hz[c]) << c;
  return m;
}

// Whole-mesh check: the query list is the leaf order, so query i is leaf i.
// Each pair is found by the query of its earlier leaf: the children of node
// (level L, in-level index k) whose leaves all come at or before leaf i are
// skipped (child c holds leaves [(4k + c) 4^(D-L-1), (4k + c + 1) 4^(D-L-1))).
template <int MODE>
__device__ __forceinline__ int later_children(int node, int D, int64_t i) {
  if (MODE != QUERY_ALL_PAIRS) return 15;
  const int L = node_level(node);
  const int64_t k = node - ((((int64_t)1) << (2 * L)) - 1) / 3;
  const int sh = 2 * (D - L - 1);
  int m = 0;
#pragma unroll
  for (int c = 0; c < 4; c++) m |= (((4 * k + c + 1) << sh) > i + 1) << c;
  return m;
}

// A leaf hit of query t (a changed face in the first pass, any face in the
// whole-mesh check): its face id, and whether to stage it.  In the first pass
// a deleted face meets nothing, and two changed faces meet in both their
// queries: the query of the smaller one takes the pair; in the whole-mesh
// check the query of the earlier leaf takes it (later_children).  The pair
// kernel then counts the overlap for both faces when the learned proposal's
// overlap counts are kept.  Later passes (faces restored) use the state
// arrays in the pair kernel only.
template <int MODE>
__device__ __forceinline__ bool leaf_take(const QueryArgs& a, int hit, int v, int t, int& u) {
  u = v & LEAF_ID;
  if (!hit || v < 0 || u == t) return false;
  if (MODE == QUERY_CHANGED && (v & LEAF_DEAD)) return false;
  if (MODE == QUERY_CHANGED && (v & LEAF_CHANGED) && u < t) return false;
  return true;
}

// Wave-cooperative traversal in packets of G lanes.  The query list is in
// Hilbert order, so the G queries of a packet are neighbours; each packet walks
// the tree once (its lanes load the same node: one coalesced request),
// entering a child when any of its lanes' own boxes meets it (the packet's
// union box is a cheap uniform pre-test).  The walk needs no stack in memory:
// in the implicit tree the path to the current node follows from its index,
// so the only state is, per level, the mask of children still to visit, four
// bits per level in one 64-bit register (14 levels at most); backtracking
// goes to the deepest level with a bit left, whose node is the current node's
// ancestor at that level.  At a node of the last internal level every lane
// tests its own box against the four leaves; hits are staged per wave in LDS
// and flushed with one atomic per ~200 pairs.  The traversal does no
// data-dependent loads besides the nodes: the state filters run in the pair
// kernel, except the one the leaf records carry (leaf_take).
template <int MODE, int G>
__global__ __launch_bounds__(64 * WPB) void k_collect(const BvhNode* __restrict__ nodes, int D, int n,
                                                      const int* __restrict__ qlist, const int* __restrict__ nq,
                                                      QueryArgs a) {
  __shared__ int2 sbuf[WPB][SEG];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int grp = lane / G;
  const unsigned long long gmask = (G == 64 ? ~0ull : (((1ull << G) - 1) << (grp * G)));
  // XCD-contiguous ranges of the query list: it is in leaf (Hilbert) order, so
  // each XCD walks one region of the tree and keeps its nodes in its own L2
  const int nqv = *nq;
  int64_t end;
  const int64_t i = xcd_item(nqv, blockDim.x, threadIdx.x, &end);
  if (i - lane >= end || n < 2) return;  // whole wave idle
  const bool active = i < end;
  const int t = active ? qlist[i] : -1;
  float tb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  if (active) query_box(a, t, tb);
  float ub[6];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    ub[k] = group_min<G>(tb[k]);
    ub[k + 3] = group_max<G>(tb[k + 3]);
  }
  Stage st{sbuf[w], 0, SEG - 64};
  // a packet with no active lane has an empty union box: it is done at once
  bool done = !(ub[0] <= ub[3]);
  uint64_t pend = 0;  // bits 4l .. 4l+3: children of the path's level-l node still to visit
  int node = 0, lvl = 0;
  while (__ballot(!done)) {
    int hit = 0;
    int4 lf = make_int4(-1, -1, -1, -1);
    if (!done) {
      const BvhNode nd = nodes[node];
      const int later = later_children<MODE>(node, D, i);
      int pm = 0;
      if (lvl == D - 1) {  // the children are leaves
        hit = child_hits(nd, tb) & later;
        lf = nd.leaf;
      } else if (G == 1) {
        pm = child_hits(nd, tb) & later;
      } else {
        const int um = child_hits(nd, ub);  // uniform over the packet
        const int own = um ? child_hits(nd, tb) & later : 0;
#pragma unroll
        for (int c = 0; c < 4; c++) pm |= ((__ballot((own >> c) & 1) & gmask) != 0) << c;
      }
      if (pm) {  // descend into the first child met, remember the others
        const int c = __builtin_ctz(pm);
        pend |= (uint64_t)(pm & (pm - 1)) << (4 * lvl);
        node = 4 * node + 1 + c;
        lvl++;
      } else if (pend == 0) {
        done = true;
      } else {  // next child of the deepest path node with children left
        const int L = (63 - __clzll(pend)) >> 2;
        const int c = __builtin_ctz((int)(pend >> (4 * L)) & 15);
        pend &= ~(1ull << (4 * L + c));
        const int anc = level_first(L) + ((node - level_first(lvl)) >> (2 * (lvl - L)));
        node = 4 * anc + 1 + c;
        lvl = L + 1;
      }
    }
    {
      int u0, u1, u2, u3;
      const bool k0 = leaf_take<MODE>(a, hit & 1, lf.x, t, u0), k1 = leaf_take<MODE>(a, hit & 2, lf.y, t, u1);
      const bool k2 = leaf_take<MODE>(a, hit & 4, lf.z, t, u2), k3 = leaf_take<MODE>(a, hit & 8, lf.w, t, u3);
      stage_append(st, k0, t, u0, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k1, t, u1, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k2, t, u2, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k3, t, u3, a.cand, a.ncand, a.cand_cap);
    }
  }
  stage_flush(st, a.cand, a.ncand, a.cand_cap);
}

// Cooperative traversal: G lanes share ONE query.  The group keeps a stack of
// pending nodes in LDS; each step its lanes pop up to G nodes (one each), load
// them in parallel, test the four children against the query box, push the
// internal children that meet it and stage the leaf hits.  A query costs
// about max(depth, visited nodes / G) dependent loads instead of one per
// visited node, which matters when few queries are left (late rounds) and the
// walk is bound by load latency rather than throughput.  A step pushes at
// most 4 G entries and the next pops G of them, so at most 3 G entries are
// left behind per level: the stack holds at most G (3 D + 4).
constexpr int COOP_DMAX = 12;

template <int MODE, int G>
__global__ __launch_bounds__(64 * WPB) void k_collect_coop(const BvhNode* __restrict__ nodes, int D, int n,
                                                           const int* __restrict__ qlist, const int* __restrict__ nq,
                                                           QueryArgs a) {
  constexpr int NG = 64 / G;
  constexpr int CST = G * (3 * COOP_DMAX + 4);
  __shared__ int2 sbuf[WPB][SEG_COOP];
  __shared__ int sstack[WPB][NG][CST];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int grp = lane / G, gl = lane % G;
  const unsigned long long gmask = (G == 64 ? ~0ull : (((1ull << G) - 1) << (grp * G)));
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int nqv = *nq;
  int64_t end;  // XCD-contiguous ranges, as in k_collect
  const int64_t wave_q0 = xcd_item(nqv, WPB * NG, w * NG, &end);
  if (wave_q0 >= end || n < 2) return;  // whole wave idle
  const int64_t q = wave_q0 + grp;
  const bool active = q < end;
  const int t = active ? qlist[q] : -1;
  float tb[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  if (active) query_box(a, t, tb);
  Stage st{sbuf[w], 0, SEG_COOP - 64};
  int* stk = sstack[w][grp];
  if (active && gl == 0) stk[0] = 0;
  int sp = active ? 1 : 0;  // uniform over the group
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  while (__ballot(sp > 0)) {
    const int take = sp < G ? sp : G;
    const int node = gl < take ? stk[sp - take + gl] : -1;
    sp -= take;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // pops read before pushes overwrite
    int hit = 0, push = 0;
    int4 lf = make_int4(-1, -1, -1, -1);
    if (node >= 0) {
      const BvhNode nd = nodes[node];
      const int m = child_hits(nd, tb) & later_children<MODE>(node, D, q);
      if (node_level(node) == D - 1) {
        hit = m;
        lf = nd.leaf;
      } else {
        push = m;
      }
    }
    // group-wide offsets of this lane's pushes: lanes below it push first
    const int np = __popc(push);
    int before = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) before += __popcll(__ballot((push >> c) & 1) & gmask & below);
    int total = 0;
#pragma unroll
    for (int c = 0; c < 4; c++) total += __popcll(__ballot((push >> c) & 1) & gmask);
    int pos = sp + before;
#pragma unroll
    for (int c = 0; c < 4; c++)
      if ((push >> c) & 1) {
        if (pos < CST) stk[pos] = 4 * node + 1 + c;
        pos++;
      }
    (void)np;
    sp += total;
    if (sp > CST) {  // cannot happen for D <= COOP_DMAX; report instead of losing pairs
      if (gl == 0) atomicOr(a.err, PAMO_EBIT_STACK);
      sp = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    {
      int u0, u1, u2, u3;
      const bool k0 = leaf_take<MODE>(a, hit & 1, lf.x, t, u0), k1 = leaf_take<MODE>(a, hit & 2, lf.y, t, u1);
      const bool k2 = leaf_take<MODE>(a, hit & 4, lf.z, t, u2), k3 = leaf_take<MODE>(a, hit & 8, lf.w, t, u3);
      stage_append(st, k0, t, u0, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k1, t, u1, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k2, t, u2, a.cand, a.ncand, a.cand_cap);
      stage_append(st, k3, t, u3, a.cand, a.ncand, a.cand_cap);
    }
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
        !share_vertex(T, U) && tri_box_overlap(T, U)) {
      atomicAdd(&a.ovl_cnt[pr.x], 1);
      // a partner whose own query left this pair to the smaller face (a changed
      // face; any face in the whole-mesh check) counts here too (the overlap
      // test is symmetric)
      if ((MODE == QUERY_CHANGED && a.owner[pr.y] >= 0) || MODE == QUERY_ALL_PAIRS) atomicAdd(&a.ovl_cnt[pr.y], 1);
    }
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

void bvh_reserve(Workspace& ws, int64_t nf, bool mesh_codes) {
  int D = 1;
  while (((int64_t)1 << (2 * D)) < nf) D++;
  ws.get<BvhNode>("bvh.nodes", ((((int64_t)1) << (2 * D)) - 1) / 3);
  ws.get<uint32_t>("bvh.code", nf);
  if (mesh_codes) ws.get<uint64_t>("bvh.code64", nf);
  ws.get<int>("bvh.id", nf);
  const int64_t top_cap = (nf + (1 << (2 * LVL)) - 1) >> (2 * LVL);
  ws.get<Box>("bvh.topA", top_cap + 1);
  ws.get<Box>("bvh.topB", top_cap + 1);
}

Bvh build_bvh(Workspace& ws, hipStream_t s, const float* box, int nf, const int* order, const int* fmesh,
              int nmesh, const int* owner, const uint8_t* falive) {
  Bvh b;
  b.n = nf;
  int D = 1;
  while (((int64_t)1 << (2 * D)) < nf) D++;
  if (D > BVH_DMAX) throw std::runtime_error("mesh too large for the BVH (more than 4^14 faces)");
  b.D = D;
  b.nodes = ws.get<BvhNode>("bvh.nodes", ((((int64_t)1) << (2 * D)) - 1) / 3);
  b.sorted = nullptr;
  if (nf < 2) return b;
  const int* id = order;
  if (!order && !fmesh) {
    uint32_t* code = ws.get<uint32_t>("bvh.code", nf);
    int* ids = ws.get<int>("bvh.id", nf);
    hipLaunchKernelGGL(k_curve_codes, dim3(nblk(nf)), dim3(256), 0, s, box, nf, code, ids);
    radix_sort_u32(ws, s, code, ids, nf, 30);
    id = ids;
  } else if (!order) {
    uint64_t* code = ws.get<uint64_t>("bvh.code64", nf);
    int* ids = ws.get<int>("bvh.id", nf);
    int mbits = 1;
    while ((1 << mbits) < nmesh) mbits++;
    hipLaunchKernelGGL(k_curve_codes_mesh, dim3(nblk(nf)), dim3(256), 0, s, box, nf, fmesh, code, ids);
    radix_sort_u64(ws, s, code, ids, nf, 30 + mbits);
    id = ids;
  }
  b.sorted = id;
  const int64_t top_cap = ((int64_t)nf + (1 << (2 * LVL)) - 1) >> (2 * LVL);
  Box* ta = ws.get<Box>("bvh.topA", top_cap + 1);
  Box* tb = ws.get<Box>("bvh.topB", top_cap + 1);
  int h0 = 0;
  int64_t cnt = nf;  // boxes of height h0 that may be non-empty
  const Box* in = nullptr;
  Box* out = ta;
  while (h0 < D) {
    const int lv = D - h0 < LVL ? D - h0 : LVL;
    const int64_t blocks = (cnt + (1ll << (2 * lv)) - 1) >> (2 * lv);
    hipLaunchKernelGGL(k_levels, dim3((unsigned)blocks), dim3(LVL_T), 0, s, box, id, nf, in, (int)cnt, out, h0, lv, D,
                       b.nodes, owner, falive);
    in = out;
    out = out == ta ? tb : ta;
    cnt = blocks;
    h0 += lv;
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
    hipLaunchKernelGGL((k_collect<QUERY_CHANGED, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL((k_collect<QUERY_RESTORED, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
  else
    hipLaunchKernelGGL((k_collect<QUERY_ALL_PAIRS, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
}

template <int G>
void launch_coop_g(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, int nq_bound,
                   const QueryArgs& a) {
  dim3 g(nblk8((int64_t)nq_bound * G, 64 * WPB)), t(64 * WPB);
  const BvhNode* nodes = bvh.nodes;
  if (mode == QUERY_CHANGED)
    hipLaunchKernelGGL((k_collect_coop<QUERY_CHANGED, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
  else if (mode == QUERY_RESTORED)
    hipLaunchKernelGGL((k_collect_coop<QUERY_RESTORED, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
  else
    hipLaunchKernelGGL((k_collect_coop<QUERY_ALL_PAIRS, G>), g, t, 0, s, nodes, bvh.D, bvh.n, qlist, nq, a);
}

void launch_query(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, int nq_bound,
                  const QueryArgs& a, int packet, int coop) {
  if (nq_bound <= 0 || bvh.n < 2) return;
  if (bvh.D > STACK) throw std::runtime_error("BVH deeper than the traversal stack");
  if (coop > 1 && bvh.D <= COOP_DMAX) {
    switch (coop) {
      case 2: launch_coop_g<2>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      case 4: launch_coop_g<4>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      case 16: launch_coop_g<16>(s, bvh, mode, qlist, nq, nq_bound, a); break;
      default: launch_coop_g<8>(s, bvh, mode, qlist, nq, nq_bound, a); break;
    }
    PAMO_HIP(hipGetLastError());
    return;
  }
  dim3 g(nblk8(nq_bound, 64 * WPB));
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
  dim3 g((unsigned)(b < 64 ? 64 : b > 8192 ? 8192 : b)), t(256);
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
