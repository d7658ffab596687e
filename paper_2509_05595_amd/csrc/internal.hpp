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

// Device workspace: named buffers that grow on demand and live as long as the
// context.  Every kernel of a context runs on its one stream.
struct Workspace {
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  size_t total = 0;
  template <class T>
  T* get(const std::string& name, size_t count) {
    size_t need = count * sizeof(T);
    if (need == 0) need = sizeof(T);
    Buf& b = bufs[name];
    if (b.bytes < need) {
      if (b.p) PAMO_HIP(hipFree(b.p));
      size_t want = need + need / 8;  // headroom so slightly larger meshes reuse it
      PAMO_HIP(hipMalloc(&b.p, want));
      total += want - b.bytes;
      b.bytes = want;
    }
    return static_cast<T*>(b.p);
  }
  void release() {
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
void radix_sort_u64(Workspace& ws, hipStream_t s, uint64_t* keys, int32_t* vals, int64_t n, int bits);

}  // namespace pamo
