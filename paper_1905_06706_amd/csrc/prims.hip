// prims.hip -- deterministic parallel primitives for gfx950 (wave64):
// exclusive scans, double-double sum and min/max reductions, and a stable LSD
// radix sort of 64-bit keys with 32-bit payloads (LDS-ranked, 8-bit digits).
#include "internal.h"

namespace hg {

// ---------------------------------------------------------------------------
// exclusive scan (u32 / u64), tiles of 256 threads x 8 items
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// block-wide exclusive scan of one value per thread; returns the block total
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* total) {
  __shared__ T wsum[kScanThreads / 64];
  const int w = threadIdx.x / 64, lane = lane_id();
  T inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const T* __restrict__ in,
                                                             T* __restrict__ out,
                                                             T* __restrict__ sums, uint64_t n) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    v[k] = i < n ? in[i] : (T)0;
    acc += v[k];
  }
  T total;
  T run = block_excl_scan(acc, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(T* __restrict__ out,
                                                           const T* __restrict__ offs, uint64_t n) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  const T o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    if (i < n) out[i] += o;
  }
}

// Exclusive scan of n elements (in may equal out).  Returns the total through
// `total_dev` (device pointer, may be null).  Scratch comes from the arena.
template <typename T>
static hipError_t scan_impl(Arena& ar, const T* in, T* out, uint64_t n, T* total_dev, hipStream_t st) {
  if (n == 0) {
    if (total_dev) return hipMemsetAsync(total_dev, 0, sizeof(T), st);
    return hipSuccess;
  }
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  T* sums = ar.get<T>(tiles + 1);
  hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, out, sums, n);
  if (tiles == 1) {
    if (total_dev) return hipMemcpyAsync(total_dev, sums, sizeof(T), hipMemcpyDeviceToDevice, st);
    return hipGetLastError();
  }
  // sums[tiles] <- total of the block sums (exclusive scan writes offsets in place)
  hipError_t e = scan_impl<T>(ar, sums, sums, tiles, total_dev, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, out, sums, n);
  return hipGetLastError();
}

hipError_t scan_u32(Arena& ar, const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total,
                    hipStream_t st) {
  Arena::Mark m = ar.mark();
  hipError_t e = scan_impl<uint32_t>(ar, in, out, n, total, st);
  ar.reset(m);
  return e;
}
hipError_t scan_u64(Arena& ar, const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* total,
                    hipStream_t st) {
  Arena::Mark m = ar.mark();
  hipError_t e = scan_impl<uint64_t>(ar, in, out, n, total, st);
  ar.reset(m);
  return e;
}

// one workgroup, 1024 threads x 8 items per tile, the carry in a register:
// for the short per-chunk count arrays, where one launch beats several
constexpr int kSegThreads = 1024;
constexpr int kSegItems = 8;

__global__ __launch_bounds__(kSegThreads) void k_seg_scan(SegScan s) {
  __shared__ uint64_t wsum[kSegThreads / 64];
  const int w = threadIdx.x / 64, lane = lane_id();
  uint64_t carry = 0;
  for (int k = 0; k < 4; ++k) {
    if ((s.reset >> k) & 1u) carry = 0;
    uint64_t* p = s.p[k];
    const uint64_t n = s.n[k];
    for (uint64_t t0 = 0; t0 < n; t0 += (uint64_t)kSegThreads * kSegItems) {
      const uint64_t b = t0 + (uint64_t)threadIdx.x * kSegItems;
      uint64_t v[kSegItems];
      uint64_t acc = 0;
#pragma unroll
      for (int j = 0; j < kSegItems; ++j) {
        v[j] = b + j < n ? p[b + j] : 0ull;
        acc += v[j];
      }
      const uint64_t inc = wave_incl_scan(acc);
      if (lane == 63) wsum[w] = inc;
      __syncthreads();
      uint64_t base = carry, tot = 0;
#pragma unroll
      for (int q = 0; q < kSegThreads / 64; ++q) {
        if (q < w) base += wsum[q];
        tot += wsum[q];
      }
      __syncthreads();
      uint64_t run = base + inc - acc;
#pragma unroll
      for (int j = 0; j < kSegItems; ++j) {
        if (b + j < n) p[b + j] = run;
        run += v[j];
      }
      carry += tot;
    }
  }
}

// long arrays: tiles of kScanTile scanned locally (tiles never straddle two
// arrays), the tile sums scanned by k_seg_scan with the same resets, then
// added back
__global__ __launch_bounds__(kScanThreads) void k_seg_tiles(SegScan s, uint4 tstart,
                                                            uint64_t* __restrict__ sums) {
  const uint32_t b = blockIdx.x;
  const uint32_t ts[4] = {tstart.x, tstart.y, tstart.z, tstart.w};
  int k = 0;
  while (k < 3 && b >= ts[k + 1]) ++k;
  uint64_t* p = s.p[k];
  const uint64_t n = s.n[k];
  const uint64_t base = (uint64_t)(b - ts[k]) * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? p[base + j] : 0ull;
    acc += v[j];
  }
  uint64_t total;
  uint64_t run = block_excl_scan(acc, &total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) p[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) sums[b] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_seg_add(SegScan s, uint4 tstart,
                                                          const uint64_t* __restrict__ sums) {
  const uint32_t b = blockIdx.x;
  const uint32_t ts[4] = {tstart.x, tstart.y, tstart.z, tstart.w};
  int k = 0;
  while (k < 3 && b >= ts[k + 1]) ++k;
  uint64_t* p = s.p[k];
  const uint64_t n = s.n[k];
  const uint64_t base = (uint64_t)(b - ts[k]) * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  const uint64_t o = sums[b];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) p[base + j] += o;
}

hipError_t seg_scan_u64(Arena& ar, const SegScan& s, hipStream_t st) {
  const uint64_t tot = s.n[0] + s.n[1] + s.n[2] + s.n[3];
  if (tot == 0) return hipSuccess;
  if (tot <= (uint64_t)kSegThreads * kSegItems) {
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(kSegThreads), 0, st, s);
    return hipGetLastError();
  }
  uint64_t tiles[4], start[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) {
    tiles[k] = (s.n[k] + kScanTile - 1) / kScanTile;
    start[k + 1] = start[k] + tiles[k];
  }
  if (start[4] >= (1ull << 31)) return hipErrorInvalidValue;
  Arena::Mark m = ar.mark();
  uint64_t* sums = ar.get<uint64_t>(start[4]);
  if (!sums) {
    ar.reset(m);
    return hipErrorOutOfMemory;
  }
  const uint4 ts = make_uint4((uint32_t)start[0], (uint32_t)start[1], (uint32_t)start[2], (uint32_t)start[3]);
  hipLaunchKernelGGL(k_seg_tiles, dim3((uint32_t)start[4]), dim3(kScanThreads), 0, st, s, ts, sums);
  SegScan ss{{sums + start[0], sums + start[1], sums + start[2], sums + start[3]},
             {tiles[0], tiles[1], tiles[2], tiles[3]}, s.reset};
  hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(kSegThreads), 0, st, ss);
  hipLaunchKernelGGL(k_seg_add, dim3((uint32_t)start[4]), dim3(kScanThreads), 0, st, s, ts, sums);
  const hipError_t e = hipGetLastError();
  ar.reset(m);
  return e;
}

// ---------------------------------------------------------------------------
// reductions: fixed grid, fixed order => bitwise reproducible
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 2048;
constexpr int kRedThreads = 256;

// error-free transformation (Knuth TwoSum)
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dd_add(double& hi, double& lo, double x) {
  double s, e;
  two_sum(hi, x, s, e);
  hi = s;
  lo += e;
}
__device__ __forceinline__ void dd_merge(double& hi, double& lo, double h2, double l2) {
  double s, e;
  two_sum(hi, h2, s, e);
  hi = s;
  lo = lo + l2 + e;
}

// mode: per-vertex terms.  0 = w; 1 = w^2 / W; 2 = w^(1/T); 3 = (w^2 / W)^(1/T),
// the last two from one power p = w^(1/T) and WT = W^(-1/T): 3 = p^2 WT
__device__ __forceinline__ double red_term(int mode, double w, double W, double p, double WT) {
  switch (mode) {
    case 0: return w;
    case 1: return w * w / W;
    case 2: return p;
    default: return p * p * WT;
  }
}

// out layout per block: [hi, lo] for each of nterms sums, then min, max
// fi0 >= 0: only the weights of the layers below fi0 (ilogb(w / fw0) < fi0)
__global__ __launch_bounds__(kRedThreads) void k_reduce_partials(const double* __restrict__ w,
                                                                 uint64_t n, int nterms,
                                                                 int mode0, double W, double invT,
                                                                 double WT, double fw0, int fi0,
                                                                 double* __restrict__ part) {
  __shared__ double shi[4][kRedThreads], slo[4][kRedThreads], smin[kRedThreads], smax[kRedThreads];
  const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = per * blockIdx.x, b1 = b0 + per < n ? b0 + per : n;
  double hi[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
  double mn = __builtin_inf(), mx = -__builtin_inf();
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    const double v = w[i];
    if (fi0 >= 0 && ilogb(v / fw0) >= fi0) continue;
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    const double p = mode0 + nterms > 2 ? pow(v, invT) : 0.0;
    for (int t = 0; t < nterms; ++t) dd_add(hi[t], lo[t], red_term(mode0 + t, v, W, p, WT));
  }
  for (int t = 0; t < nterms; ++t) {
    shi[t][threadIdx.x] = hi[t];
    slo[t][threadIdx.x] = lo[t];
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int t = 0; t < nterms; ++t) {
        double h = shi[t][threadIdx.x], l = slo[t][threadIdx.x];
        dd_merge(h, l, shi[t][threadIdx.x + s], slo[t][threadIdx.x + s]);
        shi[t][threadIdx.x] = h;
        slo[t][threadIdx.x] = l;
      }
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + (uint64_t)blockIdx.x * 10;
    for (int t = 0; t < 4; ++t) {
      o[2 * t] = t < nterms ? shi[t][0] : 0.0;
      o[2 * t + 1] = t < nterms ? slo[t][0] : 0.0;
    }
    o[8] = smin[0];
    o[9] = smax[0];
  }
}

// one thread folds the block partials in order: out = [sum_0..sum_3, min, max]
// one wave: lane t merges partials t, t + 64, ... in order, then a fixed
// pairwise tree over the lanes (deterministic)
__global__ __launch_bounds__(64) void k_reduce_final(const double* __restrict__ part, int nblocks,
                                                     double* __restrict__ out) {
  __shared__ double shi[4][64], slo[4][64], smin[64], smax[64];
  const int t = threadIdx.x;
  double hi[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
  double mn = __builtin_inf(), mx = -__builtin_inf();
  for (int b = t; b < nblocks; b += 64) {
    const double* o = part + (uint64_t)b * 10;
    for (int k = 0; k < 4; ++k) dd_merge(hi[k], lo[k], o[2 * k], o[2 * k + 1]);
    mn = fmin(mn, o[8]);
    mx = fmax(mx, o[9]);
  }
  for (int k = 0; k < 4; ++k) {
    shi[k][t] = hi[k];
    slo[k][t] = lo[k];
  }
  smin[t] = mn;
  smax[t] = mx;
  __syncthreads();
  for (int s = 32; s > 0; s >>= 1) {
    if (t < s) {
      for (int k = 0; k < 4; ++k) {
        double h = shi[k][t], l = slo[k][t];
        dd_merge(h, l, shi[k][t + s], slo[k][t + s]);
        shi[k][t] = h;
        slo[k][t] = l;
      }
      smin[t] = fmin(smin[t], smin[t + s]);
      smax[t] = fmax(smax[t], smax[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int k = 0; k < 4; ++k) out[k] = shi[k][0] + slo[k][0];
    out[4] = smin[0];
    out[5] = smax[0];
  }
}

hipError_t reduce_terms(Arena& ar, const double* w, uint64_t n, int nterms, int mode0, double W,
                        double invT, double* out6, hipStream_t st, double fw0, int fi0) {
  Arena::Mark m = ar.mark();
  double* part = ar.get<double>((uint64_t)kRedBlocks * 10);
  if (!part) {
    ar.reset(m);
    return hipErrorOutOfMemory;
  }
  const double WT = mode0 + nterms > 3 ? std::pow(W, -invT) : 0.0;
  hipLaunchKernelGGL(k_reduce_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, st, w, n, nterms,
                     mode0, W, invT, WT, fw0, fi0, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, st, part, kRedBlocks, out6);
  ar.reset(m);
  return hipGetLastError();
}

// the weights of the layers from i0 up (ilogb(w / w0) >= i0, as the layer
// keys), as bit patterns, in any order.  A workgroup takes 16 x 256 weights,
// counts its tail ones, reserves their slots with one atomic and writes them:
// one atomic per wave had serialised on the counter when the tail is long
// (n = 10^7: about 8 10^4 waves with a tail weight, 0.95 ms).
constexpr int kTailRounds = 16;
__global__ __launch_bounds__(256) void k_tail_collect(const double* __restrict__ w, uint64_t n,
                                                      double w0, int i0, uint64_t* __restrict__ out,
                                                      unsigned int* __restrict__ cnt, uint32_t cap) {
  __shared__ unsigned int wtot[4];
  __shared__ unsigned int sbase;
  const uint32_t t = threadIdx.x, lane = lane_id(), wv = t / 64;
  const uint64_t base = (uint64_t)blockIdx.x * (256u * kTailRounds);
  uint32_t sel = 0;  // bit r: weight base + 256 r + t is in the tail
#pragma unroll
  for (int r = 0; r < kTailRounds; ++r) {
    const uint64_t u = base + (uint64_t)r * 256u + t;
    if (u < n && ilogb(w[u] / w0) >= i0) sel |= 1u << r;
  }
  // this thread's first slot: a scan over the wave, then over the waves
  const uint32_t c = (uint32_t)__popc(sel);
  uint32_t incl = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += y;
  }
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (uint32_t q = 0; q < 4; ++q) {
    before += q < wv ? wtot[q] : 0u;
    total += wtot[q];
  }
  if (t == 0) sbase = total ? atomicAdd(cnt, total) : 0u;
  __syncthreads();
  if (!sel) return;
  uint32_t pos = sbase + before + incl - c;
  for (int r = 0; r < kTailRounds; ++r) {
    if (sel >> r & 1u) {
      const uint64_t u = base + (uint64_t)r * 256u + t;
      if (pos < cap) out[pos] = (uint64_t)__double_as_longlong(w[u]);
      ++pos;
    }
  }
}

hipError_t launch_tail_collect(const double* w, uint64_t n, double w0, int i0, uint64_t* out,
                               unsigned int* cnt, uint32_t cap, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t per = 256u * kTailRounds;
  hipLaunchKernelGGL(k_tail_collect, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, st, w, n, w0,
                     i0, out, cnt, cap);
  return hipGetLastError();
}

// out[i] = x_i^e for positive doubles x_i stored as their bit patterns
__global__ void k_pow_bits(const uint64_t* __restrict__ xb, double* __restrict__ out, uint64_t n,
                           double e) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = pow(__longlong_as_double((long long)xb[i]), e);
}

hipError_t launch_pow_bits(const uint64_t* xb, double* out, uint64_t n, double e, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pow_bits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xb, out, n, e);
  return hipGetLastError();
}

__global__ void k_iota(uint32_t* __restrict__ p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

hipError_t launch_iota(uint32_t* p, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, tiles of 256 threads x 16 keys
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;

__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint64_t* __restrict__ keys,
                                                          uint64_t n, int shift, uint32_t ntiles,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// The tile's keys are ranked stably by digit (ballots per round, as they
// arrive in tile order) into LDS, grouped by digit, and then written out in
// that order: a digit's keys from one tile go to consecutive positions, so the
// stores are coalesced runs instead of one cache line per key.
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, uint64_t n, int shift, uint32_t ntiles,
    const uint32_t* __restrict__ offs) {
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  __shared__ uint32_t gofs[256];  // output position of the tile's first key of each digit
  __shared__ uint32_t lofs[256];  // the digit's first slot in the tile's LDS copy
  __shared__ uint32_t run[256];   // next free slot per digit
  __shared__ uint32_t wc[kSortThreads / 64][256];
  const int t = threadIdx.x, w = t / 64;
  // digit t of this tile: [offs[t ntiles + b], the next entry of the scanned
  // histogram) holds its keys (the next entry is the same digit's next tile,
  // or the next digit's first tile, or the end)
  const uint64_t fi = (uint64_t)t * ntiles + blockIdx.x;
  const uint32_t g0 = offs[fi];
  const uint32_t g1 = fi + 1 < (uint64_t)256 * ntiles ? offs[fi + 1] : (uint32_t)n;
  gofs[t] = g0;
  lofs[t] = g1 - g0;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive scan of the tile's digit counts
    const uint32_t v = t >= o ? lofs[t - o] : 0u;
    __syncthreads();
    lofs[t] += v;
    __syncthreads();
  }
  lofs[t] -= g1 - g0;
  run[t] = lofs[t];
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    for (int q = 0; q < kSortThreads / 64; ++q) wc[q][t] = 0;
    __syncthreads();
    const uint64_t i = base + (uint64_t)r * kSortThreads + t;
    const bool valid = i < n;
    const uint64_t key = valid ? kin[i] : 0;
    const uint32_t val = valid ? vin[i] : 0;
    const uint32_t dig = (uint32_t)(key >> shift) & 255u;
    // lanes of this wave holding the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((dig >> b) & 1u);
      same &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = lanes_below(same);
    if (valid && rank == 0) wc[w][dig] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int q = 0; q < w; ++q) pos += wc[q][dig];
      sk[pos] = key;
      sv[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < kSortThreads / 64; ++q) add += wc[q][t];
    run[t] += add;
    __syncthreads();
  }
  const uint32_t tn = n - base < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
  for (uint32_t e = t; e < tn; e += kSortThreads) {
    const uint64_t key = sk[e];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    const uint32_t gp = gofs[d] + (e - lofs[d]);
    kout[gp] = key;
    vout[gp] = sv[e];
  }
}

// Sorts (keys, vals) by the low `bits` bits of the key, stably.  Results end
// in (keys, vals); tmp buffers come from the arena.
// one workgroup, bitonic network in LDS over (key, value) pairs ordered
// lexicographically (padding sorts last).  With distinct values (indices in
// ascending order, as every caller passes) this is the stable sort by key.
constexpr int kSmallSort = 4096;
__global__ __launch_bounds__(1024) void k_small_sort(uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals, uint32_t n,
                                                     uint32_t np) {
  __shared__ uint64_t sk[kSmallSort];
  __shared__ uint32_t sv[kSmallSort];
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) {
    sk[i] = i < n ? keys[i] : ~0ull;
    sv[i] = i < n ? vals[i] : ~0u;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= np; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < np / 2; t += blockDim.x) {
        const uint32_t i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
        const bool up = (i & size) == 0;
        const uint64_t ki = sk[i], kj = sk[j];
        const uint32_t vi = sv[i], vj = sv[j];
        const bool gt = ki > kj || (ki == kj && vi > vj);
        if (gt == up) {
          sk[i] = kj; sk[j] = ki;
          sv[i] = vj; sv[j] = vi;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    keys[i] = sk[i];
    vals[i] = sv[i];
  }
}

// up to 16384 pairs whose key and value fit one word together (key below
// 2^bits, value below 2^vbits, bits + vbits <= 63): the word key << vbits |
// value, sorted by a bitonic network in LDS in one workgroup.  With distinct
// values (the callers' indices) the words are distinct, and this is the
// stable sort by key.
constexpr int kSmallSortPacked = 16384;
__global__ __launch_bounds__(1024) void k_small_sort_packed(uint64_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals, uint32_t n,
                                                            uint32_t np, int vbits) {
  __shared__ uint64_t s[kSmallSortPacked];
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x)
    s[i] = i < n ? (keys[i] << vbits) | (uint64_t)vals[i] : ~0ull;
  __syncthreads();
  for (uint32_t size = 2; size <= np; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < np / 2; t += blockDim.x) {
        const uint32_t i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
        const bool up = (i & size) == 0;
        const uint64_t a = s[i], b = s[j];
        if ((a > b) == up) {
          s[i] = b;
          s[j] = a;
        }
      }
      __syncthreads();
    }
  }
  const uint64_t vm = (1ull << vbits) - 1ull;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    keys[i] = s[i] >> vbits;
    vals[i] = (uint32_t)(s[i] & vm);
  }
}

hipError_t radix_sort(Arena& ar, uint64_t* keys, uint32_t* vals, uint64_t n, int bits,
                      hipStream_t st) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  // the values are indices below n (every caller's): bitlen(n - 1) bits
  int vbits = 0;
  while ((1ull << vbits) < n) ++vbits;
  if (n <= (uint64_t)kSmallSortPacked && bits + vbits <= 63) {
    uint32_t np = 2;
    while (np < n) np <<= 1;
    hipLaunchKernelGGL(k_small_sort_packed, dim3(1), dim3(1024), 0, st, keys, vals, (uint32_t)n, np,
                       vbits);
    return hipGetLastError();
  }
  if (n <= (uint64_t)kSmallSort) {
    uint32_t np = 2;
    while (np < n) np <<= 1;
    hipLaunchKernelGGL(k_small_sort, dim3(1), dim3(1024), 0, st, keys, vals, (uint32_t)n, np);
    return hipGetLastError();
  }
  Arena::Mark m = ar.mark();
  const uint32_t ntiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
  uint64_t* k2 = ar.get<uint64_t>(n);
  uint32_t* v2 = ar.get<uint32_t>(n);
  uint32_t* hist = ar.get<uint32_t>((uint64_t)ntiles * 256);
  uint64_t* ka = keys;
  uint32_t* va = vals;
  uint64_t* kb = k2;
  uint32_t* vb = v2;
  const int passes = (bits + 7) / 8;
  hipError_t e = hipSuccess;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(kSortThreads), 0, st, ka, n, 8 * p, ntiles, hist);
    e = scan_u32(ar, hist, hist, (uint64_t)ntiles * 256, nullptr, st);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(kSortThreads), 0, st, ka, va, kb, vb, n,
                       8 * p, ntiles, hist);
    uint64_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  if (e == hipSuccess && ka != keys) {
    e = hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  }
  ar.reset(m);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace hg
