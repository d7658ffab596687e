// Device-wide primitives: prefix sums, stream compaction and a stable LSD
// radix sort, written for 64-lane wavefronts (ballot / popcount ranking).
#include <algorithm>

#include "internal.hpp"

namespace pamo {

namespace {

constexpr int T = 256;       // threads per block (4 waves)
constexpr int ITEMS = 16;    // items per thread in scans
constexpr int TILE = T * ITEMS;
constexpr int TOP_T = 1024;  // single-block scan of tile sums
constexpr int TOP_ITEMS = 16;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_incl_scan(int x) {
  int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// exclusive scan over the block; *total gets the block sum (all threads)
template <int NT>
__device__ __forceinline__ int block_excl_scan(int x, int& total) {
  constexpr int NW = NT / 64;
  __shared__ int wsum[NW + 1];
  int lane = lane_id(), w = threadIdx.x >> 6;
  int inc = wave_incl_scan(x);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    int v = lane < NW ? wsum[lane] : 0;
    int vi = wave_incl_scan(v);
    if (lane < NW) wsum[lane] = vi - v;
    if (lane == NW - 1) wsum[NW] = vi;
  }
  __syncthreads();
  int r = wsum[w] + inc - x;
  total = wsum[NW];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ int block_sum(int x) {
  int t;
  block_excl_scan<NT>(x, t);
  return t;
}

// Item loaders.  load16 reads the 16 consecutive items of one thread (i a
// multiple of 16, zero past n) with vector loads where the run is aligned and
// complete, so a thread has all of its items in flight at once.
struct FlagLoad {
  const uint8_t* f;
  __device__ int load(int64_t i) const { return f[i] != 0; }
  __device__ void load16(int64_t i, int64_t n, int* v) const {
    if (i + 16 <= n && (reinterpret_cast<uintptr_t>(f + i) & 15) == 0) {
      const uint4 x = *reinterpret_cast<const uint4*>(f + i);
      const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int k = 0; k < 16; k++) v[k] = ((w[k >> 2] >> (8 * (k & 3))) & 0xffu) != 0;
    } else {
#pragma unroll
      for (int k = 0; k < 16; k++) v[k] = i + k < n ? load(i + k) : 0;
    }
  }
};
struct IntLoad {
  const int32_t* a;
  __device__ int load(int64_t i) const { return a[i]; }
  __device__ void load16(int64_t i, int64_t n, int* v) const {
    if (i + 16 <= n && (reinterpret_cast<uintptr_t>(a + i) & 15) == 0) {
      const int4* p = reinterpret_cast<const int4*>(a + i);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int4 x = p[q];
        v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; k++) v[k] = i + k < n ? load(i + k) : 0;
    }
  }
};
static_assert(ITEMS == 16 && TOP_ITEMS == 16, "loaders read 16 items per thread");

// tile sums; thread t of a tile holds items [16 t, 16 t + 16) of it
template <class Op>
__global__ __launch_bounds__(T) void k_tile_reduce(Op op, int64_t n, int32_t* tile_sum) {
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * ITEMS;
  int v[ITEMS];
  op.load16(base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) s += v[i];
  s = block_sum<T>(s);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// exclusive scan of a[0..n) in place (n <= TOP_T*TOP_ITEMS); total -> *total
__global__ __launch_bounds__(TOP_T) void k_top_scan(int32_t* a, int n, int32_t* total) {
  int base = threadIdx.x * TOP_ITEMS;
  int v[TOP_ITEMS];
  int s = 0;
#pragma unroll
  for (int i = 0; i < TOP_ITEMS; i++) {
    v[i] = base + i < n ? a[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_excl_scan<TOP_T>(s, tot);
#pragma unroll
  for (int i = 0; i < TOP_ITEMS; i++) {
    if (base + i < n) a[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

struct CompactStore {
  int32_t* out;
  __device__ void store(int64_t i, int prefix, int v) const {
    if (v) out[prefix] = (int32_t)i;
  }
};
struct CompactMapStore {
  int32_t* out;
  const int32_t* map;
  __device__ void store(int64_t i, int prefix, int v) const {
    if (v) out[prefix] = map[i];
  }
};
struct RankStore {
  int32_t* map;
  __device__ void store(int64_t i, int prefix, int v) const { map[i] = v ? prefix : -1; }
};
struct ScanStore {
  int32_t* out;
  __device__ void store(int64_t i, int prefix, int) const { out[i] = prefix; }
};

// Scan pass over tiles.  tile_off: exclusive offsets of the tiles (three-pass
// form), or null, in which case each block adds up the sums of the tiles
// before it itself (two-pass form, for up to LOCAL_TILES tiles); the last
// block then writes the total.
constexpr int64_t LOCAL_TILES = 1024;

template <class Op, class St>
__global__ __launch_bounds__(T) void k_tile_scan(Op op, St st, int64_t n, const int32_t* tile_off,
                                                 const int32_t* tile_sum, int32_t* total) {
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * ITEMS;
  int v[ITEMS];
  op.load16(base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) s += v[i];
  int off;
  if (tile_off) {
    off = tile_off[blockIdx.x];
  } else {
    int pre = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += T) pre += tile_sum[t];
    off = block_sum<T>(pre);
  }
  int tot;
  int ex = block_excl_scan<T>(s, tot) + off;
  if (!tile_off && total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    if (base + i < n) st.store(base + i, ex, v[i]);
    ex += v[i];
  }
}

// Small inputs: the whole scan in one block and one launch (a carry walks the
// chunks of TOP_T * TOP_ITEMS items in order).  Late rounds run on small
// meshes, where three launches per scan cost more than the work (one block
// over more than one chunk measured no faster than two launches).
constexpr int64_t SINGLE_MAX = (int64_t)TOP_T * TOP_ITEMS;

template <class Op, class St>
__global__ __launch_bounds__(TOP_T) void k_scan_single(Op op, St st, int64_t n, int32_t* total) {
  int carry = 0;
  for (int64_t base0 = 0; base0 < n; base0 += (int64_t)TOP_T * TOP_ITEMS) {
    int64_t base = base0 + (int64_t)threadIdx.x * TOP_ITEMS;
    int v[TOP_ITEMS];
    op.load16(base, n, v);
    int s = 0;
#pragma unroll
    for (int i = 0; i < TOP_ITEMS; i++) s += v[i];
    int tot;
    int ex = block_excl_scan<TOP_T>(s, tot) + carry;
#pragma unroll
    for (int i = 0; i < TOP_ITEMS; i++) {
      if (base + i < n) st.store(base + i, ex, v[i]);
      ex += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class Op, class St>
void run_scan(Workspace& ws, hipStream_t s, Op op, St st, int64_t n, int32_t* total) {
  if (n > 0 && n <= SINGLE_MAX) {
    hipLaunchKernelGGL((k_scan_single<Op, St>), dim3(1), dim3(TOP_T), 0, s, op, st, n, total);
    PAMO_HIP(hipGetLastError());
    return;
  }
  int64_t ntiles = (n + TILE - 1) / TILE;
  if (ntiles > (int64_t)TOP_T * TOP_ITEMS) throw std::runtime_error("scan: input too large");
  if (ntiles == 0) {
    if (total) fill_i32(s, total, 1, 0);
    return;
  }
  int32_t* tiles = ws.get<int32_t>("prim.tiles", ntiles);
  hipLaunchKernelGGL(k_tile_reduce<Op>, dim3((unsigned)ntiles), dim3(T), 0, s, op, n, tiles);
  if (ntiles <= LOCAL_TILES) {
    hipLaunchKernelGGL((k_tile_scan<Op, St>), dim3((unsigned)ntiles), dim3(T), 0, s, op, st, n, nullptr,
                       (const int32_t*)tiles, total);
  } else {
    hipLaunchKernelGGL(k_top_scan, dim3(1), dim3(TOP_T), 0, s, tiles, (int)ntiles, total);
    hipLaunchKernelGGL((k_tile_scan<Op, St>), dim3((unsigned)ntiles), dim3(T), 0, s, op, st, n,
                       (const int32_t*)tiles, nullptr, nullptr);
  }
  PAMO_HIP(hipGetLastError());
}

// ------------------------------------------------------------ segmented ranks
// Up to three independent flag scans in one launch (or one pair): the
// segments lie end to end, each padded to whole tiles, so that a tile belongs
// to one segment and its offset is the sum of the segment's earlier tiles.
// Segment k: item i is flagged when flag[k][i] (or flag[k][gather[k][i]] when
// gather[k] is set) is nonzero; rank[k][i] gets its rank or -1, list[k][rank]
// gets i (or gather[k][i]); total[k] the count.  Absent arrays are skipped.
struct Seg3 {
  const uint8_t* flag[3];
  const int32_t* gather[3];
  int32_t* rank[3];
  int32_t* list[3];
  int32_t* excl[3];
  int32_t* total[3];
  int64_t n[3];
  int64_t tile0[4];  // first tile of each segment; tile0[3]: all tiles
};

__device__ __forceinline__ int seg_of(const Seg3& g, int64_t tile) { return tile >= g.tile0[2] ? 2 : tile >= g.tile0[1]; }

__device__ __forceinline__ void seg_load16(const Seg3& g, int k, int64_t i, int* v) {
  const int64_t n = g.n[k];
  if (g.gather[k]) {
#pragma unroll
    for (int j = 0; j < 16; j++) v[j] = i + j < n ? g.flag[k][g.gather[k][i + j]] != 0 : 0;
  } else {
    FlagLoad{g.flag[k]}.load16(i, n, v);
  }
}

__device__ __forceinline__ void seg_store(const Seg3& g, int k, int64_t i, int prefix, int v) {
  if (g.excl[k]) g.excl[k][i] = prefix;
  if (g.rank[k]) g.rank[k][i] = v ? prefix : -1;
  if (v && g.list[k]) g.list[k][prefix] = g.gather[k] ? g.gather[k][i] : (int32_t)i;
}

__global__ __launch_bounds__(T) void k_seg_reduce(Seg3 g, int32_t* tile_sum) {
  const int64_t b = blockIdx.x;
  const int k = seg_of(g, b);
  const int64_t base = (b - g.tile0[k]) * TILE + (int64_t)threadIdx.x * ITEMS;
  int v[ITEMS];
  seg_load16(g, k, base, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) s += v[i];
  s = block_sum<T>(s);
  if (threadIdx.x == 0) tile_sum[b] = s;
}

__global__ __launch_bounds__(T) void k_seg_scan(Seg3 g, const int32_t* tile_sum) {
  const int64_t b = blockIdx.x;
  const int k = seg_of(g, b);
  const int64_t base = (b - g.tile0[k]) * TILE + (int64_t)threadIdx.x * ITEMS;
  int v[ITEMS];
  seg_load16(g, k, base, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) s += v[i];
  int pre = 0;
  for (int64_t t = g.tile0[k] + threadIdx.x; t < b; t += T) pre += tile_sum[t];
  const int off = block_sum<T>(pre);
  int tot;
  int ex = block_excl_scan<T>(s, tot) + off;
  if (g.total[k] && b == g.tile0[k + 1] - 1 && threadIdx.x == 0) *g.total[k] = off + tot;
#pragma unroll
  for (int i = 0; i < ITEMS; i++) {
    if (base + i < g.n[k]) seg_store(g, k, base + i, ex, v[i]);
    ex += v[i];
  }
}

// small inputs: the segments one after the other in a single block
__global__ __launch_bounds__(TOP_T) void k_seg_single(Seg3 g) {
  for (int k = 0; k < 3; k++) {
    if (!g.flag[k]) continue;
    int carry = 0;
    for (int64_t base0 = 0; base0 < g.n[k]; base0 += (int64_t)TOP_T * TOP_ITEMS) {
      const int64_t base = base0 + (int64_t)threadIdx.x * TOP_ITEMS;
      int v[TOP_ITEMS];
      seg_load16(g, k, base, v);
      int s = 0;
#pragma unroll
      for (int i = 0; i < TOP_ITEMS; i++) s += v[i];
      int tot;
      int ex = block_excl_scan<TOP_T>(s, tot) + carry;
#pragma unroll
      for (int i = 0; i < TOP_ITEMS; i++) {
        if (base + i < g.n[k]) seg_store(g, k, base + i, ex, v[i]);
        ex += v[i];
      }
      carry += tot;
    }
    if (threadIdx.x == 0 && g.total[k]) *g.total[k] = carry;
  }
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid_for(int64_t n, int t = 256) {
  int64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

// ------------------------------------------------------------ radix sort
constexpr int RS_T = 256;
constexpr int RS_CHUNKS = 16;
constexpr int RS_TILE = RS_T * RS_CHUNKS;

template <class K>
__global__ __launch_bounds__(RS_T) void k_radix_hist(const K* keys, int64_t n, int shift, int32_t* ghist,
                                                      int nblocks) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = threadIdx.x; i < RS_TILE; i += RS_T) {
    int64_t g = base + i;
    if (g < n) atomicAdd(&hist[(int)((keys[g] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  ghist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

template <class K>
__global__ __launch_bounds__(RS_T) void k_radix_scatter(const K* kin, const int32_t* vin, K* kout, int32_t* vout,
                                                         int64_t n, int shift, const int32_t* ghist,
                                                         int nblocks) {
  __shared__ int running[256];
  __shared__ int wcount[RS_T / 64][256];
  int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
  running[tid] = ghist[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
  for (int k = 0; k < RS_T / 64; k++) wcount[k][tid] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int c = 0; c < RS_CHUNKS; c++) {
    int64_t g = base + (int64_t)c * RS_T + tid;
    bool valid = g < n;
    K key = valid ? kin[g] : (K)0;
    int32_t val = valid ? vin[g] : 0;
    int d = (int)((key >> shift) & 0xFF);
    unsigned long long mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      unsigned long long bb = __ballot((d >> b) & 1);
      mask &= ((d >> b) & 1) ? bb : ~bb;
    }
    unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = __popcll(mask & lt);
    if (valid && rank == 0) wcount[w][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int off = running[d] + rank;
      for (int k = 0; k < w; k++) off += wcount[k][d];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int k = 0; k < RS_T / 64; k++) {
      add += wcount[k][tid];
      wcount[k][tid] = 0;
    }
    running[tid] += add;
    __syncthreads();
  }
}

template <class K>
void radix_sort_impl(Workspace& ws, hipStream_t s, K* keys, int32_t* vals, int64_t n, int bits, const char* tag) {
  if (n <= 1) return;
  int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
  int passes = (bits + 7) / 8;
  std::string t(tag);
  K* k2 = ws.get<K>(t + ".k2", n);
  int32_t* v2 = ws.get<int32_t>(t + ".v2", n);
  int32_t* hist = ws.get<int32_t>(t + ".hist", (size_t)256 * nblocks);
  K *ki = keys, *ko = k2;
  int32_t *vi = vals, *vo = v2;
  for (int p = 0; p < passes; p++) {
    int shift = 8 * p;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(nblocks), dim3(RS_T), 0, s, (const K*)ki, n, shift, hist, nblocks);
    scan_exclusive(ws, s, hist, hist, (int64_t)256 * nblocks, nullptr);
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nblocks), dim3(RS_T), 0, s, (const K*)ki, (const int32_t*)vi, ko, vo,
                       n, shift, (const int32_t*)hist, nblocks);
    PAMO_HIP(hipGetLastError());
    K* tk = ki; ki = ko; ko = tk;
    int32_t* tv = vi; vi = vo; vo = tv;
  }
  if (ki != keys) {
    PAMO_HIP(hipMemcpyAsync(keys, ki, n * sizeof(K), hipMemcpyDeviceToDevice, s));
    PAMO_HIP(hipMemcpyAsync(vals, vi, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace

void fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

void compact_flags(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* out, int32_t* count) {
  run_scan(ws, s, FlagLoad{flags}, CompactStore{out}, n, count);
}
void compact_flags_map(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, const int32_t* map,
                       int32_t* out, int32_t* count) {
  run_scan(ws, s, FlagLoad{flags}, CompactMapStore{out, map}, n, count);
}
void rank_segments(Workspace& ws, hipStream_t s, const FlagSegment* seg, int nseg) {
  if (nseg < 1 || nseg > 3) throw std::runtime_error("rank_segments: 1 to 3 segments");
  Seg3 g{};
  int64_t tiles = 0, items = 0;
  for (int k = 0; k < 3; k++) {
    g.tile0[k] = tiles;
    if (k < nseg && seg[k].n > 0) {
      g.flag[k] = seg[k].flag;
      g.gather[k] = seg[k].gather;
      g.rank[k] = seg[k].rank;
      g.list[k] = seg[k].list;
      g.excl[k] = seg[k].excl;
      g.total[k] = seg[k].total;
      g.n[k] = seg[k].n;
      tiles += (seg[k].n + TILE - 1) / TILE;
      items += seg[k].n;
    } else if (k < nseg && seg[k].total) {
      fill_i32(s, seg[k].total, 1, 0);
    }
  }
  g.tile0[3] = tiles;
  if (tiles == 0) return;
  if (items <= SINGLE_MAX) {
    hipLaunchKernelGGL(k_seg_single, dim3(1), dim3(TOP_T), 0, s, g);
  } else if (tiles <= LOCAL_TILES) {
    int32_t* ts = ws.get<int32_t>("prim.segtiles", tiles);
    hipLaunchKernelGGL(k_seg_reduce, dim3((unsigned)tiles), dim3(T), 0, s, g, ts);
    hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)tiles), dim3(T), 0, s, g, (const int32_t*)ts);
  } else {  // large: one scan per segment
    for (int k = 0; k < nseg; k++) {
      if (seg[k].n <= 0) continue;
      Seg3 one{};
      one.flag[0] = g.flag[k];
      one.gather[0] = g.gather[k];
      one.rank[0] = g.rank[k];
      one.list[0] = g.list[k];
      one.excl[0] = g.excl[k];
      one.total[0] = g.total[k];
      one.n[0] = g.n[k];
      const int64_t t = (g.n[k] + TILE - 1) / TILE;
      one.tile0[1] = one.tile0[2] = one.tile0[3] = t;
      if (t > LOCAL_TILES) {
        // beyond the two-pass form: the plain three-pass scans
        if (one.gather[0] || one.list[0]) throw std::runtime_error("rank_segments: list segment too large");
        if (one.rank[0]) rank_flags(ws, s, one.flag[0], one.n[0], one.rank[0], one.total[0]);
        if (one.excl[0]) run_flag_scan(ws, s, one.flag[0], one.n[0], one.excl[0], one.rank[0] ? nullptr : one.total[0]);
        continue;
      }
      int32_t* ts = ws.get<int32_t>("prim.segtiles", t);
      hipLaunchKernelGGL(k_seg_reduce, dim3((unsigned)t), dim3(T), 0, s, one, ts);
      hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)t), dim3(T), 0, s, one, (const int32_t*)ts);
    }
  }
  PAMO_HIP(hipGetLastError());
}

void rank_flags(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* map, int32_t* count) {
  run_scan(ws, s, FlagLoad{flags}, RankStore{map}, n, count);
}
void run_flag_scan(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* out, int32_t* total) {
  run_scan(ws, s, FlagLoad{flags}, ScanStore{out}, n, total);
}
void scan_exclusive(Workspace& ws, hipStream_t s, const int32_t* in, int32_t* out, int64_t n, int32_t* total) {
  // the tile pass reads all of a tile before writing it, so in == out is fine
  run_scan(ws, s, IntLoad{in}, ScanStore{out}, n, total);
}
void prim_reserve(Workspace& ws, int64_t scan_n, int64_t sort32_n, int64_t sort64_n, int64_t seg_n) {
  auto hist_items = [](int64_t n) { return (int64_t)256 * ((n + RS_TILE - 1) / RS_TILE); };
  int64_t scan = scan_n;
  if (sort32_n > 1) {
    ws.get<uint32_t>("rs32.k2", sort32_n);
    ws.get<int32_t>("rs32.v2", sort32_n);
    ws.get<int32_t>("rs32.hist", hist_items(sort32_n));
    scan = std::max(scan, hist_items(sort32_n));
  }
  if (sort64_n > 1) {
    ws.get<uint64_t>("rs64.k2", sort64_n);
    ws.get<int32_t>("rs64.v2", sort64_n);
    ws.get<int32_t>("rs64.hist", hist_items(sort64_n));
    scan = std::max(scan, hist_items(sort64_n));
  }
  ws.get<int32_t>("prim.tiles", (scan + TILE - 1) / TILE);
  ws.get<int32_t>("prim.segtiles", (seg_n + TILE - 1) / TILE + 3);
}

void radix_sort_u32(Workspace& ws, hipStream_t s, uint32_t* keys, int32_t* vals, int64_t n, int bits) {
  radix_sort_impl<uint32_t>(ws, s, keys, vals, n, bits, "rs32");
}
void radix_sort_u64(Workspace& ws, hipStream_t s, uint64_t* keys, int32_t* vals, int64_t n, int bits) {
  radix_sort_impl<uint64_t>(ws, s, keys, vals, n, bits, "rs64");
}

}  // namespace pamo
