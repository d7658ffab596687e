// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <stdexcept>
#include <string>

#include "../../include/pamo.h"

namespace pamo {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define PAMO_HIP(x)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess)                                                                        \
      throw ::pamo::HipError(std::string(#x) + ": " + hipGetErrorString(e_) + " at " __FILE__ ":" + \
                             std::to_string(__LINE__));                                          \
  } while (0)

// A request for workspace that a caller-owned arena cannot hold.
struct WorkspaceFull : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Device workspace: named buffers that live as long as the context.  Every
// kernel of a context runs on its one stream.  Three modes:
//   own      (default) buffers are hipMalloc'd on demand and grow to fit the
//            largest mesh seen;
//   arena    buffers are carved, 256-byte aligned, from caller-owned device
//            memory (pamo_set_workspace, or the library's static scratch);
//            every call starts carving afresh at the arena's start, nothing
//            is allocated, and a request the arena cannot hold throws
//            WorkspaceFull;
//   counting nothing is allocated or touched: requests only add up the bytes
//            the arena mode would carve (the size query).
// The mesh entry points first reserve every buffer their path can request at
// its largest size (reserve_mesh in api.hip), so in arena mode no later
// request grows a buffer and the size query is the exact sum.
struct Workspace {
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  size_t total = 0;  // bytes held (own) or carved so far in this call (arena, counting)
  char* arena = nullptr;
  size_t arena_bytes = 0;
  bool counting = false;
  static size_t align(size_t b) { return (b + 255) & ~(size_t)255; }
  template <class T>
  T* get(const std::string& name, size_t count) {
    size_t need = count * sizeof(T);
    if (need == 0) need = sizeof(T);
    Buf& b = bufs[name];
    if (b.bytes >= need) return static_cast<T*>(b.p);
    if (counting) {  // a stand-in address that is never dereferenced
      total += align(need);
      b.bytes = align(need);
      b.p = reinterpret_cast<void*>((uintptr_t)256);
      return static_cast<T*>(b.p);
    }
    if (arena) {
      const size_t a = align(need);
      if (total + a > arena_bytes)
        throw WorkspaceFull("workspace of " + std::to_string(arena_bytes) + " bytes too small: buffer '" + name +
                            "' needs " + std::to_string(a) + " more bytes at offset " + std::to_string(total));
      b.p = arena + total;  // a buffer that grows leaves its old block behind
      b.bytes = a;
      total += a;
      return static_cast<T*>(b.p);
    }
    if (b.p) PAMO_HIP(hipFree(b.p));
    b.p = nullptr;
    size_t want = need + need / 8;  // headroom so slightly larger meshes reuse it
    PAMO_HIP(hipMalloc(&b.p, want));
    total += want - b.bytes;
    b.bytes = want;
    return static_cast<T*>(b.p);
  }
  // start of an entry point: an arena is carved afresh (nothing in the
  // workspace outlives a call)
  void begin_call() {
    if (arena || counting) {
      bufs.clear();
      total = 0;
    }
  }
  // caller-owned memory from now on (p = null: back to own allocations)
  void set_arena(void* p, size_t bytes) {
    release();
    arena = static_cast<char*>(p);
    arena_bytes = p ? bytes : 0;
  }
  void release() {
    if (!arena && !counting)
      for (auto& kv : bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    bufs.clear();
    total = 0;
  }
};

// ------------------------------------------------------------- primitives
// All asynchronous on `s`.  Counts written to device memory.
void fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v);
void fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
// out[i] = index of the i-th nonzero flag, ascending; *count = number of them
void compact_flags(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* out, int32_t* count);
// out[k] = map[i] for the k-th nonzero flag i
void compact_flags_map(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, const int32_t* map,
                       int32_t* out, int32_t* count);
// map[i] = rank of i among nonzero flags, -1 where zero; *count = total
void rank_flags(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* map, int32_t* count);
// Up to three independent flag scans in one launch pair.  Item i of a segment
// is flagged when flag[i] (flag[gather[i]] with gather) is nonzero; rank[i]
// (optional) gets its rank or -1, excl[i] (optional) the number of flagged
// items before it, list[rank] (optional) gets i (gather[i]), *total
// (optional) the count.  A segment with a list and more than 1,024 tiles of
// 4,096 items is refused.
struct FlagSegment {
  const uint8_t* flag = nullptr;
  const int32_t* gather = nullptr;
  int64_t n = 0;
  int32_t* rank = nullptr;
  int32_t* list = nullptr;
  int32_t* excl = nullptr;
  int32_t* total = nullptr;
};
void rank_segments(Workspace& ws, hipStream_t s, const FlagSegment* seg, int nseg);
// exclusive prefix count of nonzero flags; *total optional
void run_flag_scan(Workspace& ws, hipStream_t s, const uint8_t* flags, int64_t n, int32_t* out, int32_t* total);
// exclusive prefix sum of int32, in place allowed; *total optional
void scan_exclusive(Workspace& ws, hipStream_t s, const int32_t* in, int32_t* out, int64_t n, int32_t* total);
// stable LSD radix sort of (key, value) pairs on the low `bits` bits; the
// sorted data ends in keys/vals (the arrays passed in)
void radix_sort_u32(Workspace& ws, hipStream_t s, uint32_t* keys, int32_t* vals, int64_t n, int bits);
// reserve the primitives' buffers for scans of up to scan_n items, radix sorts
// of up to sort32_n / sort64_n pairs and segmented ranks over up to seg_n
// items in all (see Workspace)
void prim_reserve(Workspace& ws, int64_t scan_n, int64_t sort32_n, int64_t sort64_n, int64_t seg_n);
void radix_sort_u64(Workspace& ws, hipStream_t s, uint64_t* keys, int32_t* vals, int64_t n, int bits);

}  // namespace pamo
