// log2_probe.hip -- exhaustive error of the FP32 logarithms that the sampler's
// filters rely on, measured on the GPU against FP64 on every float of the
// ranges they see.  Built beside the library (tests/probes.py) and run by
// tests/test_gpu_log2.py.
//
// which = 0: log2_1m_series_f32(t) for every float t in [2^-53, 1/16), against
//            log1p(-t) / ln 2: max |error| / |exact|.
// which = 1: __log2f(x) for every float x in [2^-53, 0.9375]: max relative error.
// which = 2: __log2f(x) for every positive normal float x:
//            max |error| / (1 + |log2 x|).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "device_common.h"

namespace {

__global__ void k_log2_err(uint32_t lo_bits, uint32_t count, int which,
                           unsigned long long* __restrict__ out) {
  double m = 0.0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const float x = __uint_as_float(lo_bits + i);
    double e;
    if (which == 0) {
      const double ex = log1p(-(double)x) * 1.4426950408889634;
      e = fabs((double)hg::log2_1m_series_f32(x) - ex) / fabs(ex);
    } else {
      const double ex = log2((double)x);
      const double err = fabs((double)__log2f(x) - ex);
      e = which == 1 ? err / fabs(ex) : err / (1.0 + fabs(ex));
    }
    m = e > m ? e : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_down(m, o, 64);
    m = t > m ? t : m;
  }
  // non-negative doubles order like their bit patterns
  if ((threadIdx.x & 63) == 0) atomicMax(&out[which], (unsigned long long)__double_as_longlong(m));
}

uint32_t bits_of(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

}  // namespace

// Fills out[0..2] (host memory) with the three maxima above; returns the
// first HIP error code, 0 on success.  Allocates 24 bytes of device memory.
extern "C" int log2_probe(double* out) {
  unsigned long long* d = nullptr;
  hipError_t e = hipMalloc(&d, 3 * sizeof(unsigned long long));
  if (e != hipSuccess) return (int)e;
  e = hipMemset(d, 0, 3 * sizeof(unsigned long long));
  const uint32_t lo = bits_of(0x1p-53f);
  const uint32_t ranges[3][2] = {
      {lo, bits_of(0.0625f) - lo},                // [2^-53, 1/16)
      {lo, bits_of(0.9375f) + 1 - lo},            // [2^-53, 0.9375]
      {bits_of(0x1p-126f), bits_of(0x1.fffffep127f) + 1 - bits_of(0x1p-126f)}};
  for (int w = 0; w < 3 && e == hipSuccess; ++w) {
    k_log2_err<<<2048, 256>>>(ranges[w][0], ranges[w][1], w, d);
    e = hipGetLastError();
  }
  unsigned long long h[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
  hipFree(d);
  for (int w = 0; w < 3; ++w) memcpy(&out[w], &h[w], 8);
  return (int)e;
}
