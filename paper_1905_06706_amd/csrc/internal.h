// internal.h -- host-side declarations shared by the library's translation
// units (scratch arena, primitives, sampler stages).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <vector>

#include "device_common.h"

namespace hg {

// Bump allocator over device chunks.  Allocations never move; reset() returns
// everything above a mark; chunks are kept (cached) until release().
class Arena {
 public:
  struct Mark {
    size_t chunk;
    size_t used;
  };
  ~Arena() { release(); }

  // a fixed device buffer instead of chunks of its own: the arena then never
  // calls hipMalloc or hipFree, and an allocation beyond the buffer fails
  void attach(char* base, size_t size) {
    ext_base_ = base;
    ext_size_ = size;
    ext_used_ = 0;
  }
  bool attached() const { return ext_base_ != nullptr; }

  Mark mark() const {
    if (ext_base_) return Mark{0, ext_used_};
    return Mark{cur_, chunks_.empty() ? 0 : chunks_[cur_].used};
  }
  void reset(Mark m) {
    if (ext_base_) {
      ext_used_ = m.used;
      return;
    }
    for (size_t c = m.chunk + 1; c < chunks_.size(); ++c) chunks_[c].used = 0;
    cur_ = m.chunk;
    if (!chunks_.empty()) chunks_[cur_].used = m.used;
  }
  void reset_all() {
    ext_used_ = 0;
    for (auto& c : chunks_) c.used = 0;
    cur_ = 0;
  }
  template <typename T>
  T* get(uint64_t count) {
    void* p = raw(count * sizeof(T));
    return static_cast<T*>(p);
  }
  void* raw(size_t bytes);  // nullptr on allocation failure (sets failed())
  bool failed() const { return failed_; }
  void clear_failure() { failed_ = false; }
  void release();

 private:
  struct Chunk {
    char* base;
    size_t size;
    size_t used;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
  bool failed_ = false;
  char* ext_base_ = nullptr;
  size_t ext_size_ = 0, ext_used_ = 0;
};

hipError_t scan_u32(Arena& ar, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                    hipStream_t st);
hipError_t scan_u64(Arena& ar, const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* total,
                    hipStream_t st);
// out6 (device): sums of terms mode0..mode0+nterms-1, then min, max of w;
// with fi0 >= 0 only over the w with ilogb(w / fw0) < fi0 (the layers below fi0)
hipError_t reduce_terms(Arena& ar, const double* w, uint64_t n, int nterms, int mode0, double W,
                        double invT, double* out6, hipStream_t st, double fw0 = 1.0, int fi0 = -1);
// bit patterns of the weights with ilogb(w / w0) >= i0 into out (any order;
// *cnt, zeroed by the caller, counts them; at most cap are stored)
hipError_t launch_tail_collect(const double* w, uint64_t n, double w0, int i0, uint64_t* out,
                               unsigned int* cnt, uint32_t cap, hipStream_t st);
// in-place exclusive scans of up to four u64 arrays by one workgroup; the
// running sum carries from array k - 1 into array k unless bit k of `reset`
// is set (array 0 always starts at zero).  Arrays with n = 0 may be null.
struct SegScan {
  uint64_t* p[4];
  uint64_t n[4];
  uint32_t reset;
};
hipError_t seg_scan_u64(Arena& ar, const SegScan& s, hipStream_t st);
hipError_t launch_iota(uint32_t* p, uint64_t n, hipStream_t st);
// out[i] = x_i^e, x_i positive doubles given as bit patterns (u64)
hipError_t launch_pow_bits(const uint64_t* xb, double* out, uint64_t n, double e, hipStream_t st);
// stable sort of (keys, vals) by key; keys below 2^bits, vals distinct
// indices below n (every caller passes 0 .. n - 1)
hipError_t radix_sort(Arena& ar, uint64_t* keys, uint32_t* vals, uint64_t n, int bits,
                      hipStream_t st);

}  // namespace hg
