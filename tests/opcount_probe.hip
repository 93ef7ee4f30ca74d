// One unit of each decision of the sampling kernels, written with the
// library's own device functions, so that the VALU instructions of the unit's
// arithmetic can be counted in the gfx950 assembly (tests/test_opcount.py).
// Each unit kernel has an io_* twin with the same loads and stores and no
// arithmetic; the difference of the two counts is the unit's work.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "fastpow.h"

using namespace hg;

struct G {
  double c, W, invT, ilg, pbar, kappa;
  uint32_t k0, k1;
};

__device__ __forceinline__ double torus3(const double4& a, const double4& b) {
  const double xa[3] = {a.y, a.z, a.w}, xb[3] = {b.y, b.z, b.w};
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double df = fabs(xa[k] - xb[k]);
    const double m = df < 1.0 - df ? df : 1.0 - df;
    r = m > r ? m : r;
  }
  return r;
}

// binomial pair decision (d = 3) given its coin U: distance, p_uv of Eq. (1), compare
extern "C" __global__ void u_prob(const double4* rec, G g, const double* U, int* out) {
  const int t = threadIdx.x;
  const double4 a = rec[2 * t], b = rec[2 * t + 1];
  const double r = torus3(a, b);
  double p = 1.0;
  if (r != 0.0) {
    p = g.c * pow_pos((a.x * b.x) / (g.W * (r * r * r)), g.invT);
    p = p < 1.0 ? p : 1.0;
  }
  out[t] = U[t] < p;
}
extern "C" __global__ void io_prob(const double4* rec, G g, const double* U, int* out) {
  const int t = threadIdx.x;
  const double4 a = rec[2 * t], b = rec[2 * t + 1];
  out[t] = (a.x + b.x + a.y + b.y + a.z + b.z + a.w + b.w) < U[t];
}

// one Philox4x32-10 block and its two 53-bit uniforms (two type-I coins)
extern "C" __global__ void u_philox(const uint4* ctr, G g, double2* out) {
  const int t = threadIdx.x;
  const uint4 c = ctr[t];
  const U4 o = philox(c.x, c.y, c.z, c.w, g.k0, g.k1);
  out[t] = make_double2(u53(o.x, o.y), u53(o.z, o.w));
}
extern "C" __global__ void io_philox(const uint4* ctr, G g, double2* out) {
  const int t = threadIdx.x;
  const uint4 c = ctr[t];
  out[t] = make_double2((double)(c.x ^ c.y), (double)(c.z ^ c.w));
}

// one geometric draw: block, S, ln S / ln(1 - pbar), end test, skip, Acc pbar
extern "C" __global__ void u_draw(const uint4* ctr, G g, const uint64_t* rem, uint64_t* out,
                                  double* apb) {
  const int t = threadIdx.x;
  const uint4 c = ctr[t];
  const U4 o = philox(c.x, c.y, c.z, c.w, g.k0, g.k1);
  const uint64_t vv = (((uint64_t)o.y << 32) | o.x) >> 11;
  const double S = (double)(vv + 1) * 0x1p-53;
  const double ls = log_pos(S);
  const double q = ls == 0.0 ? 0.0 : ls * g.ilg;
  out[t] = q >= (double)rem[t] ? ~0ull : (uint64_t)q;
  apb[t] = u53(o.z, o.w) * g.pbar;
}
extern "C" __global__ void io_draw(const uint4* ctr, G g, const uint64_t* rem, uint64_t* out,
                                   double* apb) {
  const int t = threadIdx.x;
  const uint4 c = ctr[t];
  out[t] = rem[t] ^ c.x ^ c.y;
  apb[t] = (double)(c.z ^ c.w);
}

// threshold pair decision (d = 3): r^d W <= kappa w_u w_v
extern "C" __global__ void u_thresh(const double4* rec, G g, int* out) {
  const int t = threadIdx.x;
  const double4 a = rec[2 * t], b = rec[2 * t + 1];
  const double r = torus3(a, b);
  out[t] = r * r * r * g.W <= g.kappa * a.x * b.x;
}
extern "C" __global__ void io_thresh(const double4* rec, G g, int* out) {
  const int t = threadIdx.x;
  const double4 a = rec[2 * t], b = rec[2 * t + 1];
  out[t] = (a.x + b.x + a.y + b.y + a.z + b.z + a.w + b.w) < 0.0;
}
