// device_common.h -- device primitives of the gfx950 GIRG/HRG sampler:
// Philox4x32-10, 53-bit uniforms, Morton codes, wave64 append helpers and the
// per-graph description shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int kMaxLayers = 64;
constexpr int kMaxLevels = 33;  // levels 0..32
constexpr int kHrgTab = 100;    // HRG distance filter: grid points of p_T
constexpr int kWave = 64;
constexpr int kSegExp = 5;       // type-II segment: about 2^5..2^6 expected candidates
constexpr int kSegMaxBits = 12;  // at most 2^12 segments per item

enum Kind : uint32_t { kKindType1 = 0, kKindType2 = 1, kKindPoints = 2, kKindSeq = 3 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
// as 1, 2, 3", SC 2011).  Round: (c0,c1,c2,c3) <- (hi(M1 c2) ^ c1 ^ k0,
// lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); key += (W0, W1) between rounds.
// The key is wave-uniform (the seed), so the bumped keys live in SGPRs.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Counter word 3: level | i << 6 | j << 12 | kind << 18 | high << 20.
__device__ __forceinline__ uint32_t ctr_word3(uint32_t level, uint32_t i, uint32_t j, uint32_t kind,
                                              uint32_t high) {
  return level | (i << 6) | (j << 12) | (kind << 18) | (high << 20);
}

// Uniform in [0,1): the top 53 bits of hi:lo times 2^-53 (exact).
__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi) {
  const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
  return (double)v * 0x1p-53;
}
// Uniform in (0,1].
__device__ __forceinline__ double u53_open(uint32_t lo, uint32_t hi) {
  const uint64_t v = ((((uint64_t)hi << 32) | lo) >> 11) + 1;
  return (double)v * 0x1p-53;
}

// ---------------------------------------------------------------------------
// FP32 logarithm of the type-II skip filter.  A skip is
// floor(log2 S / log2(1 - pbar)) for S = (vv + 1) 2^-53 in (0, 1].
// * 1 - S = om 2^-53 is exact.  Below 1/16 the series
//   -(t + t^2/2 + ... + t^5/5) / ln 2 of log2(1 - t) is taken in t = fl32(1 - S)
//   (truncation below t^5 / (6 (1 - t)) < 2^-22.5 relative, t's rounding
//   2^-24 relative).
// * Otherwise v_log_f32 of fl32(S).  There |log2 S| >= 0.093, so the rounding
//   of S moves the result by less than 2^-20 relative.
// tests/log2_probe.hip measures both pieces on every float of their ranges
// (series and v_log_f32 each below 2^-21 relative), so the result is within
// 2^-19.4 of log2 S, relative; with the rounding of 1 / log2(1 - pbar) and of
// the product the FP32 quotient is within 2^-19.3 of the exact one, and the
// filter decides only outside kSkipRel (relative) of it.
// ---------------------------------------------------------------------------
constexpr double kSkipRel = 0x1p-17;

__device__ __forceinline__ float log2_1m_series_f32(float t) {
  return -t * (1.0f + t * (0.5f + t * (0.33333334f + t * (0.25f + t * 0.2f)))) * 1.44269504f;
}

__device__ __forceinline__ float log2_unit_f32(uint64_t vv) {
  const uint64_t om = (1ull << 53) - 1 - vv;
  if (!om) return 0.0f;
  const float t = (float)om * 0x1p-53f;
  if (t < 0.0625f) return log2_1m_series_f32(t);
  return __log2f((float)((double)(vv + 1) * 0x1p-53));
}

// ---------------------------------------------------------------------------
// Morton codes (Sec. 3.4 / App. B.3): coordinate bits interleaved, dimension 0
// most significant in every group.  Shift-and-mask spreading for fixed d.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread2(uint32_t v) {  // 16 -> 32 bits, one gap
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__device__ __forceinline__ uint32_t compact2(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}
__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 -> 30 bits, two gaps
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x3FFu;
  return v;
}
__device__ __forceinline__ uint32_t spread4(uint32_t v) {  // 8 -> 32 bits, three gaps
  v &= 0xFFu;
  v = (v | (v << 12)) & 0x000F000Fu;
  v = (v | (v << 6)) & 0x03030303u;
  v = (v | (v << 3)) & 0x11111111u;
  return v;
}
__device__ __forceinline__ uint32_t compact4(uint32_t v) {
  v &= 0x11111111u;
  v = (v | (v >> 3)) & 0x03030303u;
  v = (v | (v >> 6)) & 0x000F000Fu;
  v = (v | (v >> 12)) & 0xFFu;
  return v;
}

template <int D>
__device__ __forceinline__ uint32_t morton_encode(const uint32_t* q) {
  if constexpr (D == 1) {
    return q[0];
  } else if constexpr (D == 2) {
    return (spread2(q[0]) << 1) | spread2(q[1]);
  } else if constexpr (D == 3) {
    return (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  } else {
    return (spread4(q[0]) << 3) | (spread4(q[1]) << 2) | (spread4(q[2]) << 1) | spread4(q[3]);
  }
}
template <int D>
__device__ __forceinline__ void morton_decode(uint32_t m, uint32_t* q) {
  if constexpr (D == 1) {
    q[0] = m;
  } else if constexpr (D == 2) {
    q[0] = compact2(m >> 1);
    q[1] = compact2(m);
  } else if constexpr (D == 3) {
    q[0] = compact3(m >> 2);
    q[1] = compact3(m >> 1);
    q[2] = compact3(m);
  } else {
    q[0] = compact4(m >> 3);
    q[1] = compact4(m >> 2);
    q[2] = compact4(m >> 1);
    q[3] = compact4(m);
  }
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// cells
// ---------------------------------------------------------------------------
// Morton code of the cell at level lvl of a code at level Dmax (bits wide)
__device__ __forceinline__ uint32_t cell_at(uint32_t m, int lvl, int d, int bits) {
  return lvl == 0 ? 0u : (m >> (bits - d * lvl));
}

__device__ __forceinline__ int bitlen64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

template <int D>
struct Offs {
  static constexpr int n1 = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;      // neighbour offsets
  static constexpr int n2 = D == 1 ? 6 : D == 2 ? 36 : D == 3 ? 216 : 1296;  // parent-neighbour children
  // longest row of the distant-offset table (one orientation of each pair)
  static constexpr int nd = D == 1 ? 2 : D == 2 ? 17 : D == 3 ? 116 : 737;
};

// ---------------------------------------------------------------------------
// Per-graph description, built on the device by the table kernel and read by
// every sampling kernel.
// ---------------------------------------------------------------------------
struct Pbar {
  double pbar;  // upper bound of the edge probability for (i, j, level, gap)
  double ilg;   // 1 / log1p(-pbar): a skip is ln(S) * ilg
  int32_t e;    // segment exponent 5 - ilogb(pbar)
  float qscale; // 1 / log2(1 - pbar): a skip is log2(S) * qscale (FP32 filter)
};

struct Graph {
  // sizes and model
  uint32_t n;
  int32_t d, model, L, D, Dmax, bits;  // bits = d * Dmax (Morton width)
  int32_t cl_bias, max_depth, precision;
  double T, c, W, w0, R, coshR, kappa, inv_T, alpha;
  // mixed precision: log2 p = C32 + invT32 (log2 w_u + log2 w_v - d log2 r)
  float C32, invT32;
  uint32_t seed_lo, seed_hi;
  // tables (filled by the table kernel)
  int32_t count[kMaxLayers];
  double ext[kMaxLayers];          // GIRG: max weight; HRG: min radius
  uint32_t lstart[kMaxLayers + 1];
  int8_t CL[kMaxLayers][kMaxLayers];
  int8_t I[kMaxLayers];
  uint64_t pbase[kMaxLayers];       // offset of layer i's prefix sums
  uint64_t jI[kMaxLayers][kMaxLevels];   // j with CL(i,j) == level
  uint64_t jII[kMaxLayers][kMaxLevels];  // j with CL(i,j) >= level
  uint64_t cells;                   // total prefix-sum entries
  // per-cell layer sets: entry moff[l] + A at level l (levels up to
  // max_i I(i)), bit j set iff V_j^A is nonempty
  uint64_t moff[kMaxLevels + 1];
  // HRG binomial distance filter (App. B.4): hct[m] = cosh of the distance at
  // which p_T equals m / (kHrgTab - 1) (+inf at m = 0, 0 where that distance
  // is not positive)
  double hct[kHrgTab];
};

// Per sorted vertex, everything a pair decision reads, in one aligned record
// of rec_stride(d, model) doubles: GIRG (w, x_0 .. x_{d-1}), padded to 2, 4 or
// 8 doubles; HRG (x, e^r, e^-r, sinh r).
__host__ __device__ constexpr int rec_stride(int d, int model) {
  return model == 1 ? 4 : (d == 1 ? 2 : (d <= 3 ? 4 : 8));
}

// Sorted vertex arrays.
struct Verts {
  const double* rec;    // [n][rec_stride] records
  const uint32_t* id;   // original id
  const uint32_t* mort; // Morton code at level Dmax
  const uint8_t* layer;
  // FP32 filter records of the mixed path (GIRG, d <= 3; null otherwise):
  // (log2 w as FP32 bits, floor(x_k 2^32) for k < d, zero after)
  const uint4* frec;
};

// Per cell and level (index moff[l] + cell): the layers with vertices there
// and the index of the first of their (first sorted position, count) records,
// which follow in layer order.
struct CellL {
  uint64_t mask;
  uint32_t base;
  uint32_t pad;
};

}  // namespace hg
