// sampler.hip -- gfx950 kernels of the GIRG / HRG sampler (Sec. 3 of
// arXiv:1905.06706): points, weight layers and Morton keys, the level tables
// (CL, I, pbar), prefix sums per layer, run sources, and the fused cell-pair
// enumeration + sampling kernels for type-I (every pair tested) and type-II
// (geometric jumps under pbar, then rejection) cell pairs.
//
// Work decomposition: every sampling kernel runs on a fixed grid of waves;
// wave w owns a contiguous range of work units and its lanes take interleaved
// units.  Each lane runs a small state machine (fetch the next non-empty item,
// then one test / one draw per step) inside a loop that is converged across
// the wave, so every step ends with a wave ballot that appends the accepted
// edges in a fixed order.  A count pass records the number of edges per wave;
// a scan gives each wave its output offset; the write pass repeats the work
// and stores the edges.  The edge array is therefore a pure function of the
// inputs and the seed.
#include "sampler.h"

namespace hg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_at(uint32_t m, int lvl, int d, int bits) {
  return lvl == 0 ? 0u : (m >> (bits - d * lvl));
}

__device__ __forceinline__ int bitlen64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

template <int D>
struct Offs {
  static constexpr int n1 = D == 1 ? 3 : D == 2 ? 9 : D == 3 ? 27 : 81;      // neighbour offsets
  static constexpr int n2 = D == 1 ? 6 : D == 2 ? 36 : D == 3 ? 216 : 1296;  // parent-neighbour children
};

// ---------------------------------------------------------------------------
// points (Sec. 2.1 / Sec. 2.2)
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_points_girg(uint64_t n, double expo, uint32_t k0,
                                                     uint32_t k1, double* __restrict__ w,
                                                     double* __restrict__ x) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const uint32_t w3 = ctr_word3(0, 0, 0, kKindPoints, 0);
  U4 o = philox((uint32_t)u, 0u, 0u, w3, k0, k1);
  w[u] = pow(u53_open(o.x, o.y), expo);
#pragma unroll
  for (int k = 0; k < D; k += 2) {
    o = philox((uint32_t)u, (uint32_t)(1 + k / 2), 0u, w3, k0, k1);
    x[(uint64_t)k * n + u] = u53(o.x, o.y);
    if (k + 1 < D) x[(uint64_t)(k + 1) * n + u] = u53(o.z, o.w);
  }
}

__global__ __launch_bounds__(256) void k_points_hrg(uint64_t n, double alpha, double R, double cm1,
                                                    uint32_t k0, uint32_t k1,
                                                    double* __restrict__ r, double* __restrict__ x) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const uint32_t w3 = ctr_word3(0, 0, 0, kKindPoints, 0);
  U4 o = philox((uint32_t)u, 0u, 0u, w3, k0, k1);
  const double ru = acosh(1.0 + u53(o.x, o.y) * cm1) / alpha;
  r[u] = ru < R ? ru : R;
  o = philox((uint32_t)u, 1u, 0u, w3, k0, k1);
  x[u] = u53(o.x, o.y);
}

hipError_t launch_points(const Graph& g, double beta, double* w, double* x, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  if (g.model == 1) {
    hipLaunchKernelGGL(k_points_hrg, dim3(blocks), dim3(256), 0, st, (uint64_t)g.n, g.alpha, g.R,
                       cosh(g.alpha * g.R) - 1.0, g.seed_lo, g.seed_hi, w, x);
  } else {
    const double expo = -1.0 / (beta - 1.0);
    switch (g.d) {
      case 1: hipLaunchKernelGGL(k_points_girg<1>, dim3(blocks), dim3(256), 0, st, (uint64_t)g.n, expo, g.seed_lo, g.seed_hi, w, x); break;
      case 2: hipLaunchKernelGGL(k_points_girg<2>, dim3(blocks), dim3(256), 0, st, (uint64_t)g.n, expo, g.seed_lo, g.seed_hi, w, x); break;
      case 3: hipLaunchKernelGGL(k_points_girg<3>, dim3(blocks), dim3(256), 0, st, (uint64_t)g.n, expo, g.seed_lo, g.seed_hi, w, x); break;
      default: hipLaunchKernelGGL(k_points_girg<4>, dim3(blocks), dim3(256), 0, st, (uint64_t)g.n, expo, g.seed_lo, g.seed_hi, w, x); break;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight layers (Sec. 3.1) and Morton keys (Sec. 3.4)
// key = layer << bits | Morton code of the cell at level Dmax
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_layer_key(Graph* __restrict__ g,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ x,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ ids,
                                                   uint32_t* __restrict__ flag) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = g->n;
  if (u >= n) return;
  const double wu = w[u];
  int layer;
  if (g->model == 0) {
    if (!(wu > 0.0) || !(wu < __builtin_inf())) { atomicOr(flag, 1u); return; }
    layer = ilogb(wu / g->w0);
  } else {
    if (!(wu >= 0.0 && wu <= g->R)) { atomicOr(flag, 1u); return; }
    layer = (int)floor((g->R - wu) / (2.0 * 0.6931471805599453));
  }
  if (layer < 0 || layer >= kMaxLayers) { atomicOr(flag, 2u); return; }
  uint32_t q[D];
  const double scale = ldexp(1.0, g->Dmax);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double xk = x[(uint64_t)k * n + u];
    if (!(xk >= 0.0 && xk < 1.0)) { atomicOr(flag, 4u); return; }
    q[k] = (uint32_t)(xk * scale);
  }
  const uint32_t m = morton_encode<D>(q);
  keys[u] = ((uint64_t)layer << g->bits) | m;
  ids[u] = (uint32_t)u;
  atomicAdd(&g->count[layer], 1);
  const unsigned long long bitsw = (unsigned long long)__double_as_longlong(wu);
  if (g->model == 0)
    atomicMax((unsigned long long*)&g->ext[layer], bitsw);  // positive doubles order as integers
  else
    atomicMin((unsigned long long*)&g->ext[layer], bitsw);
}

hipError_t launch_layer_key(const Graph& g, Graph* gd, const double* w, const double* x,
                            uint64_t* keys, uint32_t* ids, uint32_t* flag, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  switch (g.d) {
    case 1: hipLaunchKernelGGL(k_layer_key<1>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, flag); break;
    case 2: hipLaunchKernelGGL(k_layer_key<2>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, flag); break;
    case 3: hipLaunchKernelGGL(k_layer_key<3>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, flag); break;
    default: hipLaunchKernelGGL(k_layer_key<4>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, flag); break;
  }
  return hipGetLastError();
}

// sorted structure-of-arrays copy
__global__ __launch_bounds__(256) void k_gather(const Graph* __restrict__ g,
                                                const uint64_t* __restrict__ keys,
                                                const uint32_t* __restrict__ ids,
                                                const double* __restrict__ w,
                                                const double* __restrict__ x, double* __restrict__ sw,
                                                double* __restrict__ sx, uint32_t* __restrict__ smort,
                                                uint8_t* __restrict__ slayer,
                                                double* __restrict__ aux) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = g->n;
  if (s >= n) return;
  const uint32_t u = ids[s];
  const uint64_t key = keys[s];
  const double wu = w[u];
  sw[s] = wu;
  for (int k = 0; k < g->d; ++k) sx[(uint64_t)k * n + s] = x[(uint64_t)k * n + u];
  smort[s] = g->bits == 32 ? (uint32_t)key : (uint32_t)(key & ((1ull << g->bits) - 1));
  slayer[s] = (uint8_t)(key >> g->bits);
  if (g->model == 1) {
    aux[s] = exp(wu);
    aux[(uint64_t)n + s] = exp(-wu);
    aux[2 * (uint64_t)n + s] = sinh(wu);
  }
}

hipError_t launch_gather(const Graph& g, const Graph* gd, const uint64_t* keys, const uint32_t* ids,
                         const double* w, const double* x, double* sw, double* sx, uint32_t* smort,
                         uint8_t* slayer, double* aux, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, gd, keys, ids, w,
                     x, sw, sx, smort, slayer, aux);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// level tables: comparison level CL(i,j) (Sec. 3.1; HRG by search over
// levels, Sec. 4.3), insertion level I(i), deepest level D, the masks of
// layer pairs served by neighbouring (CL == level) and distant (CL >= level)
// cell pairs (loop swap, Sec. 3.3), and the type-II bounds pbar.
// One block; the sizes are tiny (<= 64 x 64 layer pairs).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tables(Graph* __restrict__ g, int Dcap,
                                                Pbar* __restrict__ pb) {
  __shared__ int dmax;
  const int L = g->L, d = g->d;
  if (threadIdx.x == 0) dmax = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < kMaxLayers * kMaxLayers; p += blockDim.x) {
    const int i = p / kMaxLayers, j = p % kMaxLayers;
    int l = -1;
    if (i < L && j < L && g->count[i] > 0 && g->count[j] > 0) {
      l = 0;
      const double ei = g->ext[i], ej = g->ext[j];
      if (g->model == 0 && g->T == 0.0) {
        const double tmax = g->c * pow(ei * ej / g->W, 1.0 / d);
        while (l < Dcap && ldexp(1.0, -(l + 1)) >= tmax) ++l;
      } else if (g->model == 0) {
        const double V = g->kappa * ei * ej / g->W;
        while (l < Dcap && ldexp(1.0, -(l + 1) * d) >= V) ++l;
      } else {
        const double shh = 2.0 * sinh(ei) * sinh(ej);
        while (l < Dcap) {
          const int nl = l + 1;
          if (nl >= 2) {
            const double s = sin(3.141592653589793 * ldexp(1.0, -nl));
            if (!(1.0 + shh * s * s >= g->coshR)) break;
          }
          l = nl;
        }
      }
      l += g->cl_bias;
      if (l < 0) l = 0;
      if (l > Dcap) l = Dcap;
      if (g->max_depth >= 0 && l > g->max_depth) l = g->max_depth;
      atomicMax(&dmax, l);
    }
    g->CL[i][j] = (int8_t)l;
  }
  __syncthreads();
  if (threadIdx.x == 0) g->D = dmax;
  for (int i = threadIdx.x; i < kMaxLayers; i += blockDim.x) {
    int I = -1;
    for (int j = 0; j < kMaxLayers; ++j) I = g->CL[i][j] > I ? g->CL[i][j] : I;
    g->I[i] = (int8_t)I;
    for (int l = 0; l < kMaxLevels; ++l) {
      uint64_t m1 = 0, m2 = 0;
      for (int j = 0; j < kMaxLayers; ++j) {
        const int cl = g->CL[i][j];
        if (cl < 0) continue;
        if (cl == l) m1 |= 1ull << j;
        if (cl >= l && l >= 2) m2 |= 1ull << j;  // distant pairs exist from level 2
      }
      g->jI[i][l] = m1;
      g->jII[i][l] = g->T > 0.0 ? m2 : 0ull;  // threshold: distant cells hold no edges
    }
  }
  if (!(g->T > 0.0) || pb == nullptr) return;
  // pbar for (i, j, level, gap): largest weights, smallest distance gap 2^-level
  const int nl = Dcap + 1;
  for (int p = threadIdx.x; p < L * L * nl * 2; p += blockDim.x) {
    const int gi = p & 1, l = (p >> 1) % nl, ij = (p >> 1) / nl, i = ij / L, j = ij % L;
    const int cl = (i < L && j < L) ? g->CL[i][j] : -1;
    Pbar e{0.0, 0.0, 0, 0};
    if (cl >= l && l >= 2) {
      const double dist = ldexp((double)(gi + 1), -l);
      double pbar;
      if (g->model == 0) {
        double dd = dist;
        for (int k = 1; k < d; ++k) dd *= dist;
        pbar = g->c * pow((g->ext[i] * g->ext[j] / g->W) / dd, g->inv_T);
        pbar = pbar < 1.0 ? pbar : 1.0;
      } else {
        const double s = sin(3.141592653589793 * dist);
        const double ch = 1.0 + 2.0 * sinh(g->ext[i]) * sinh(g->ext[j]) * s * s;
        pbar = 1.0 / (exp((acosh(ch) - g->R) / (2.0 * g->T)) + 1.0);
      }
      e.pbar = pbar;
      e.lg = log1p(-pbar);
      e.e = pbar > 0.0 ? kSegExp - ilogb(pbar) : 1 << 20;
    }
    pb[p] = e;
  }
}

hipError_t launch_tables(Graph* gd, int Dcap, Pbar* pb, hipStream_t st) {
  hipLaunchKernelGGL(k_tables, dim3(1), dim3(256), 0, st, gd, Dcap, pb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// prefix sums per layer at its insertion level (Lemma 1): counts, then one
// exclusive scan over the concatenated layers gives absolute sorted positions
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cell_count(const Graph* __restrict__ g,
                                                    const uint32_t* __restrict__ smort,
                                                    const uint8_t* __restrict__ slayer,
                                                    uint32_t* __restrict__ cnt) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g->n) return;
  const int i = slayer[s];
  const uint32_t c = cell_at(smort[s], g->I[i], g->d, g->bits);
  atomicAdd(&cnt[g->pbase[i] + c], 1u);
}

hipError_t launch_cell_count(const Graph& g, const Graph* gd, const uint32_t* smort,
                             const uint8_t* slayer, uint32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_count, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, gd, smort,
                     slayer, cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// run sources: sorted vertex s starts the run of its layer's cell at every
// level l in [h(s), I(layer)], where h(s) is the first level at which its cell
// differs from that of s-1 (0 at the start of a layer).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int head_level(const Graph* __restrict__ g,
                                          const uint32_t* __restrict__ smort,
                                          const uint8_t* __restrict__ slayer, uint32_t s) {
  const int i = slayer[s];
  if (s == g->lstart[i]) return 0;
  const uint32_t x = smort[s] ^ smort[s - 1];
  if (x == 0) return 1 << 20;
  const int p = 31 - __clz((int)x);
  return (g->bits - p + g->d - 1) / g->d;
}

__global__ __launch_bounds__(256) void k_src_count(const Graph* __restrict__ g,
                                                   const uint32_t* __restrict__ smort,
                                                   const uint8_t* __restrict__ slayer,
                                                   uint32_t* __restrict__ cnt) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g->n) return;
  const int h = head_level(g, smort, slayer, (uint32_t)s);
  const int I = g->I[slayer[s]];
  cnt[s] = I >= h ? (uint32_t)(I - h + 1) : 0u;
}

__global__ __launch_bounds__(256) void k_src_fill(const Graph* __restrict__ g,
                                                  const uint32_t* __restrict__ smort,
                                                  const uint8_t* __restrict__ slayer,
                                                  const uint32_t* __restrict__ off,
                                                  uint64_t* __restrict__ src) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g->n) return;
  const int h = head_level(g, smort, slayer, (uint32_t)s);
  const int I = g->I[slayer[s]];
  uint64_t o = off[s];
  for (int l = h; l <= I; ++l) src[o++] = ((uint64_t)l << 32) | s;
}

hipError_t launch_sources(const Graph& g, const Graph* gd, const uint32_t* smort,
                          const uint8_t* slayer, uint32_t* cnt, const uint32_t* off, uint64_t* src,
                          bool fill, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  if (!fill)
    hipLaunchKernelGGL(k_src_count, dim3(blocks), dim3(256), 0, st, gd, smort, slayer, cnt);
  else
    hipLaunchKernelGGL(k_src_fill, dim3(blocks), dim3(256), 0, st, gd, smort, slayer, off, src);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// edge decisions (FP64)
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double torus_r(const double* __restrict__ x, uint32_t n, uint32_t su,
                                          uint32_t sv) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double df = fabs(x[(uint64_t)k * n + su] - x[(uint64_t)k * n + sv]);
    const double m = df < 1.0 - df ? df : 1.0 - df;
    r = m > r ? m : r;
  }
  return r;
}

template <int D>
__device__ __forceinline__ double pow_d(double r) {
  double rd = r;
#pragma unroll
  for (int k = 1; k < D; ++k) rd *= r;
  return rd;
}

// GIRG binomial probability of Eq. (1)
template <int D>
__device__ __forceinline__ double girg_prob(const Graph* __restrict__ g, double wu, double wv,
                                           double r) {
  if (r == 0.0) return 1.0;
  const double p = g->c * pow((wu * wv / g->W) / pow_d<D>(r), g->inv_T);
  return p < 1.0 ? p : 1.0;
}

// HRG: cosh of the hyperbolic distance, cosh(ru - rv) + 2 sinh ru sinh rv
// sin^2(pi dx), with cosh(ru - rv) from per-vertex e^r, e^-r.
__device__ __forceinline__ double hrg_coshd(const Verts& v, uint32_t n, uint32_t su, uint32_t sv,
                                            double dx) {
  const double* e = v.aux;
  const double* ei = v.aux + n;
  const double* sh = v.aux + 2 * (uint64_t)n;
  const double ch = 0.5 * (e[su] * ei[sv] + e[sv] * ei[su]);
  const double s = sinpi(dx);
  return ch + 2.0 * sh[su] * sh[sv] * s * s;
}

__device__ __forceinline__ double hrg_prob(const Graph* __restrict__ g, double coshd) {
  return 1.0 / (exp((acosh(coshd) - g->R) * (0.5 * g->inv_T)) + 1.0);
}

// probability (binomial variants) of the pair of sorted vertices (su, sv)
template <int D, int MODEL>
__device__ __forceinline__ double pair_prob(const Graph* __restrict__ g, const Verts& v,
                                            uint32_t su, uint32_t sv) {
  const uint32_t n = g->n;
  const double r = torus_r<D>(v.x, n, su, sv);
  if constexpr (MODEL == 0) {
    return girg_prob<D>(g, v.w[su], v.w[sv], r);
  } else {
    return hrg_prob(g, hrg_coshd(v, n, su, sv, r));
  }
}

// threshold variants
template <int D, int MODEL>
__device__ __forceinline__ bool pair_thresh(const Graph* __restrict__ g, const Verts& v,
                                            uint32_t su, uint32_t sv) {
  const uint32_t n = g->n;
  const double r = torus_r<D>(v.x, n, su, sv);
  if constexpr (MODEL == 0) {
    // ||x_u - x_v|| <= c (w_u w_v / W)^{1/d}  <=>  r^d W <= c^d w_u w_v
    return pow_d<D>(r) * g->W <= g->kappa * v.w[su] * v.w[sv];
  } else {
    return hrg_coshd(v, n, su, sv, r) < g->coshR;
  }
}

// ---------------------------------------------------------------------------
// unit decoding: source (l, s) x neighbour / distant offset -> cell pair
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ bool neighbour_cell(uint32_t A, int lvl, uint32_t off, uint32_t* B) {
  uint32_t q[D], b[D];
  morton_decode<D>(A, q);
  const uint64_t side = 1ull << lvl;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t jk = off % 3;
    off /= 3;
    if (jk >= side) return false;  // wraps onto an offset already listed
    b[k] = (uint32_t)((q[k] + side - 1 + jk) % side);
  }
  *B = morton_encode<D>(b);
  return true;
}

// children of the parent's neighbours that are not neighbours themselves;
// gap g = max_k (torus difference - 1)
template <int D>
__device__ __forceinline__ bool distant_cell(uint32_t A, int lvl, uint32_t off, uint32_t* B,
                                             int* gap) {
  uint32_t q[D], b[D];
  morton_decode<D>(A, q);
  const uint64_t side = 1ull << lvl;
  int dm = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t jk = off % 6;
    off /= 6;
    if (jk >= side) return false;
    b[k] = (uint32_t)((2ull * (q[k] >> 1) + side - 2 + jk) % side);
    const uint64_t df = q[k] > b[k] ? q[k] - b[k] : b[k] - q[k];
    const uint64_t dt = df < side - df ? df : side - df;
    dm = (int)dt > dm ? (int)dt : dm;
  }
  if (dm <= 1) return false;  // neighbours
  *B = morton_encode<D>(b);
  *gap = dm - 1;
  return true;
}

__device__ __forceinline__ void cell_range(const Graph* __restrict__ g, const uint32_t* __restrict__ P,
                                           int j, int lvl, uint32_t B, uint32_t* b0,
                                           uint32_t* nb) {
  const int sh = g->d * (g->I[j] - lvl);
  const uint32_t* Pj = P + g->pbase[j];
  const uint32_t lo = Pj[(uint64_t)B << sh];
  *b0 = lo;
  *nb = Pj[((uint64_t)B + 1) << sh] - lo;
}

// ---------------------------------------------------------------------------
// type-I: neighbouring cell pairs at level CL(i,j); every pair of
// V_i^A x V_j^B gets its own coin (Sec. 3.2).  Pair index k = a*|V_j^B| + b;
// for A = B and i = j only a < b with k = b(b-1)/2 + a (App. B.1).  Two tests
// share one Philox block (words 0-1 for even k, 2-3 for odd k).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_range(uint64_t nunits, uint64_t* ub, uint64_t* ue,
                                           uint64_t* wave) {
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  *wave = w;
  *ub = nunits * w / nw;
  *ue = nunits * (w + 1) / nw;
}

template <int D, int MODEL, bool T0, bool WRITE>
__global__ __launch_bounds__(256) void k_type1(const Graph* __restrict__ g, Verts v,
                                               const uint32_t* __restrict__ P,
                                               const uint64_t* __restrict__ src, uint64_t nunits,
                                               WaveOut wo) {
  constexpr int NOFF = Offs<D>::n1;
  uint64_t ub, ue, wave;
  wave_range(nunits, &ub, &ue, &wave);
  const uint32_t lane = lane_id();
  const uint32_t k0 = g->seed_lo, k1 = g->seed_hi;
  const int bits = g->bits;
  uint64_t u = ub + lane;
  // unit state
  uint64_t jm = 0;
  uint32_t A = 0, B = 0, a0 = 0, na = 0, lvl = 0, li = 0;
  bool same = false;
  // item state
  bool act = false, tri = false;
  uint32_t lj = 0, b0 = 0, nb = 0, a = 0, b = 0;
  uint64_t k = 0, tot = 0;
  uint64_t running = WRITE ? wo.base[wave] : 0;
  uint64_t ntests = 0;
  for (;;) {
    while (!act) {
      if (jm == 0) {
        if (u >= ue) break;
        const uint64_t sidx = u / NOFF;
        const uint32_t off = (uint32_t)(u - sidx * NOFF);
        u += kWave;
        const uint64_t sv = src[sidx];
        const uint32_t s = (uint32_t)sv;
        lvl = (uint32_t)(sv >> 32);
        li = v.layer[s];
        jm = g->jI[li][lvl];
        if (!jm) continue;
        A = cell_at(v.mort[s], lvl, D, bits);
        if (!neighbour_cell<D>(A, lvl, off, &B) || B < A) { jm = 0; continue; }
        same = (B == A);
        if (same) jm &= ~((1ull << li) - 1ull);  // j >= i when A = B
        a0 = s;
        const int sh = D * (g->I[li] - (int)lvl);
        na = P[g->pbase[li] + (((uint64_t)A + 1) << sh)] - s;
        continue;
      }
      lj = (uint32_t)__ffsll((long long)jm) - 1;
      jm &= jm - 1;
      cell_range(g, P, lj, lvl, B, &b0, &nb);
      if (!nb) continue;
      tri = same && lj == li;
      if (tri) {
        if (na < 2) continue;
        tot = (uint64_t)na * (na - 1) / 2;
        a = 0; b = 1;
      } else {
        tot = (uint64_t)na * nb;
        a = 0; b = 0;
      }
      k = 0;
      act = true;
    }
    if (!__any(act)) break;
    bool e0 = false, e1 = false;
    uint2 p0 = make_uint2(0, 0), p1 = make_uint2(0, 0);
    if (act) {
      U4 o;
      if constexpr (!T0)
        o = philox((uint32_t)(k >> 1), A, B, ctr_word3(lvl, li, lj, kKindType1, (uint32_t)(k >> 33)), k0, k1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (k < tot) {
          const uint32_t su = a0 + a, sv = (tri ? a0 : b0) + b;
          bool e;
          if constexpr (T0) {
            e = pair_thresh<D, MODEL>(g, v, su, sv);
          } else {
            const double U = h == 0 ? u53(o.x, o.y) : u53(o.z, o.w);
            e = U < pair_prob<D, MODEL>(g, v, su, sv);
          }
          if (WRITE && e) {
            if (h == 0) p0 = make_uint2(v.id[su], v.id[sv]);
            else p1 = make_uint2(v.id[su], v.id[sv]);
          }
          if (h == 0) e0 = e; else e1 = e;
          ++ntests;
          ++k;
          if (tri) {
            if (++a == b) { a = 0; ++b; }
          } else {
            if (++b == nb) { b = 0; ++a; }
          }
        }
      }
      if (k >= tot) act = false;
    }
    const uint64_t m0 = __ballot(e0), m1 = __ballot(e1);
    if (WRITE) {
      if (e0) wo.edges[running + lanes_below(m0)] = p0;
      if (e1) wo.edges[running + __popcll(m0) + lanes_below(m1)] = p1;
    }
    running += __popcll(m0) + __popcll(m1);
  }
  if (!WRITE) {
    if (lane == 0) wo.count[wave] = (uint32_t)running;
    // statistics: tests
    for (int o = 32; o > 0; o >>= 1) ntests += __shfl_down(ntests, o, 64);
    if (lane == 0) atomicAdd(&wo.stats[0], (unsigned long long)ntests);
  }
}

// ---------------------------------------------------------------------------
// type-II: distant cell pairs (neighbouring parents) at levels l <= CL(i,j).
// Candidates of V_i^A x V_j^B are drawn by geometric jumps under pbar and
// accepted with p_uv / pbar (Sec. 3.2).  The candidate range is cut into
// segments of G = 2^e (e = 5 - ilogb(pbar), raised to keep <= 2^12
// segments); segment s draws from counter (t, A, B, l|i|j|kind=1|s).  Items
// with one segment are sampled here; items with more are deferred to the
// segment-parallel kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void segment_size(uint64_t N, int e, uint64_t* G, uint64_t* nseg) {
  const int emin = bitlen64(N - 1) - kSegMaxBits;
  if (e < emin) e = emin;
  *G = (e >= 63 || (1ull << e) >= N) ? N : (1ull << e);
  *nseg = (N + *G - 1) / *G;
}

// one geometric draw of an item / segment; returns true when an edge is accepted
template <int D, int MODEL>
__device__ __forceinline__ bool type2_draw(const Graph* __restrict__ g, const Verts& v,
                                           uint32_t A, uint32_t B, uint32_t w3, uint32_t t,
                                           double pb, double lg, uint32_t a0, uint32_t b0,
                                           uint32_t nb, uint64_t& k, uint64_t kend, bool& done,
                                           uint32_t& su, uint32_t& sv, uint64_t& ncand) {
  const U4 o = philox(t, A, B, w3, g->seed_lo, g->seed_hi);
  const double S = u53_open(o.x, o.y);
  const double q = pb >= 1.0 ? 0.0 : log(S) / lg;
  if (q >= (double)(kend - k)) {
    done = true;
    return false;
  }
  k += (uint64_t)q;
  uint64_t aa, bb;
  if (k < 0xFFFFFFFFull) {
    const uint32_t k32 = (uint32_t)k;
    aa = k32 / nb;
    bb = k32 - (uint32_t)aa * nb;
  } else {
    aa = k / nb;
    bb = k - aa * nb;
  }
  su = a0 + (uint32_t)aa;
  sv = b0 + (uint32_t)bb;
  ++ncand;
  const double p = pair_prob<D, MODEL>(g, v, su, sv);
  const bool e = u53(o.z, o.w) * pb < p;
  ++k;
  done = k >= kend;
  return e;
}

template <int D, int MODEL, bool WRITE>
__global__ __launch_bounds__(256) void k_type2(const Graph* __restrict__ g, Verts v,
                                               const uint32_t* __restrict__ P,
                                               const uint64_t* __restrict__ src, uint64_t nunits,
                                               const Pbar* __restrict__ pbt, int nlev, WaveOut wo,
                                               HeavyOut ho) {
  constexpr int NOFF = Offs<D>::n2;
  uint64_t ub, ue, wave;
  wave_range(nunits, &ub, &ue, &wave);
  const uint32_t lane = lane_id();
  const int bits = g->bits, L = g->L;
  uint64_t u = ub + lane;
  uint64_t jm = 0;
  uint32_t A = 0, B = 0, a0 = 0, na = 0, lvl = 0, li = 0;
  int gap = 1;
  bool act = false, hv = false;
  uint32_t lj = 0, b0 = 0, nb = 0, t = 0, w3 = 0;
  uint64_t k = 0, N = 0;
  double pb = 0.0, lg = 0.0;
  HeavyRec hr{};
  uint64_t running = WRITE ? wo.base[wave] : 0;
  uint32_t hseq = 0;
  uint64_t ndraws = 0, ncand = 0;
  for (;;) {
    while (!act && !hv) {
      if (jm == 0) {
        if (u >= ue) break;
        const uint64_t sidx = u / NOFF;
        const uint32_t off = (uint32_t)(u - sidx * NOFF);
        u += kWave;
        const uint64_t sv = src[sidx];
        const uint32_t s = (uint32_t)sv;
        lvl = (uint32_t)(sv >> 32);
        li = v.layer[s];
        jm = g->jII[li][lvl];
        if (!jm) continue;
        A = cell_at(v.mort[s], lvl, D, bits);
        if (!distant_cell<D>(A, lvl, off, &B, &gap) || B < A) { jm = 0; continue; }
        a0 = s;
        const int sh = D * (g->I[li] - (int)lvl);
        na = P[g->pbase[li] + (((uint64_t)A + 1) << sh)] - s;
        continue;
      }
      lj = (uint32_t)__ffsll((long long)jm) - 1;
      jm &= jm - 1;
      cell_range(g, P, lj, lvl, B, &b0, &nb);
      if (!nb) continue;
      const Pbar pe = pbt[(((uint64_t)li * L + lj) * nlev + lvl) * 2 + (gap - 1)];
      if (!(pe.pbar > 0.0)) continue;
      N = (uint64_t)na * nb;
      uint64_t G, nseg;
      segment_size(N, pe.e, &G, &nseg);
      if (nseg > 1) {
        hr = HeavyRec{a0, na, b0, nb, A, B, lvl | (li << 8) | (lj << 16) | ((uint32_t)gap << 24),
                      (uint32_t)pe.e};
        hv = true;
        continue;
      }
      pb = pe.pbar;
      lg = pe.lg;
      w3 = ctr_word3(lvl, li, lj, kKindType2, 0);
      k = 0;
      t = 0;
      act = true;
    }
    const bool any_h = __any(hv);
    if (!any_h && !__any(act)) break;
    if (any_h) {
      const uint64_t mh = __ballot(hv);
      if (!WRITE && hv) {
        const unsigned int slot = atomicAdd(ho.count, 1u);
        if (slot < ho.cap) {
          ho.rec[slot] = hr;
          ho.key[slot] = (wave << 24) | (hseq + lanes_below(mh));
        }
      }
      hseq += __popcll(mh);
      hv = false;
    }
    bool e0 = false;
    uint2 p0 = make_uint2(0, 0);
    if (act) {
      uint32_t su, sv;
      bool done;
      e0 = type2_draw<D, MODEL>(g, v, A, B, w3, t, pb, lg, a0, b0, nb, k, N, done, su, sv, ncand);
      ++t;
      ++ndraws;
      if (WRITE && e0) p0 = make_uint2(v.id[su], v.id[sv]);
      if (done) act = false;
    }
    const uint64_t m0 = __ballot(e0);
    if (WRITE && e0) wo.edges[running + lanes_below(m0)] = p0;
    running += __popcll(m0);
  }
  if (!WRITE) {
    if (lane == 0) wo.count[wave] = (uint32_t)running;
    for (int o = 32; o > 0; o >>= 1) {
      ndraws += __shfl_down(ndraws, o, 64);
      ncand += __shfl_down(ncand, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&wo.stats[1], (unsigned long long)ndraws);
      atomicAdd(&wo.stats[2], (unsigned long long)ncand);
    }
  }
}

// number of segments of each heavy item
__global__ __launch_bounds__(256) void k_heavy_nseg(const HeavyRec* __restrict__ rec, uint32_t nh,
                                                    uint64_t* __restrict__ nseg) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  uint64_t G, ns;
  segment_size((uint64_t)rec[h].na * rec[h].nb, (int)rec[h].e, &G, &ns);
  nseg[h] = ns;
}

// heavy items, one segment per unit
template <int D, int MODEL, bool WRITE>
__global__ __launch_bounds__(256) void k_heavy(const Graph* __restrict__ g, Verts v,
                                               const HeavyRec* __restrict__ rec,
                                               const uint64_t* __restrict__ segoff, uint32_t nh,
                                               uint64_t nunits, const Pbar* __restrict__ pbt,
                                               int nlev, WaveOut wo) {
  uint64_t ub, ue, wave;
  wave_range(nunits, &ub, &ue, &wave);
  const uint32_t lane = lane_id();
  const int L = g->L;
  uint64_t u = ub + lane;
  bool act = false;
  uint32_t A = 0, B = 0, a0 = 0, b0 = 0, nb = 0, t = 0, w3 = 0;
  uint64_t k = 0, kend = 0;
  double pb = 0.0, lg = 0.0;
  uint64_t running = WRITE ? wo.base[wave] : 0;
  uint64_t ndraws = 0, ncand = 0;
  for (;;) {
    if (!act && u < ue) {
      // heavy item holding segment u: last h with segoff[h] <= u
      uint32_t lo = 0, hi = nh;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (segoff[mid] <= u) lo = mid; else hi = mid;
      }
      const HeavyRec r = rec[lo];
      const uint64_t s = u - segoff[lo];
      u += kWave;
      const uint32_t lvl = r.meta & 255u, li = (r.meta >> 8) & 255u, lj = (r.meta >> 16) & 255u,
                     gp = r.meta >> 24;
      const Pbar pe = pbt[(((uint64_t)li * L + lj) * nlev + lvl) * 2 + (gp - 1)];
      const uint64_t N = (uint64_t)r.na * r.nb;
      uint64_t G, ns;
      segment_size(N, (int)r.e, &G, &ns);
      A = r.A; B = r.B; a0 = r.a0; b0 = r.b0; nb = r.nb;
      pb = pe.pbar; lg = pe.lg;
      w3 = ctr_word3(lvl, li, lj, kKindType2, (uint32_t)s);
      k = s * G;
      kend = (s + 1) * G < N ? (s + 1) * G : N;
      t = 0;
      act = true;
    }
    if (!__any(act)) break;
    bool e0 = false;
    uint2 p0 = make_uint2(0, 0);
    if (act) {
      uint32_t su, sv;
      bool done;
      e0 = type2_draw<D, MODEL>(g, v, A, B, w3, t, pb, lg, a0, b0, nb, k, kend, done, su, sv, ncand);
      ++t;
      ++ndraws;
      if (WRITE && e0) p0 = make_uint2(v.id[su], v.id[sv]);
      if (done) act = false;
    }
    const uint64_t m0 = __ballot(e0);
    if (WRITE && e0) wo.edges[running + lanes_below(m0)] = p0;
    running += __popcll(m0);
  }
  if (!WRITE) {
    if (lane == 0) wo.count[wave] = (uint32_t)running;
    for (int o = 32; o > 0; o >>= 1) {
      ndraws += __shfl_down(ndraws, o, 64);
      ncand += __shfl_down(ncand, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&wo.stats[1], (unsigned long long)ndraws);
      atomicAdd(&wo.stats[2], (unsigned long long)ncand);
    }
  }
}

__global__ __launch_bounds__(256) void k_heavy_gather(const HeavyRec* __restrict__ in,
                                                      const uint32_t* __restrict__ perm,
                                                      uint32_t nh, HeavyRec* __restrict__ out) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < nh) out[h] = in[perm[h]];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int D, int MODEL>
static void launch_t1_d(bool t0, bool write, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nunits, const WaveOut& wo, hipStream_t st) {
  const dim3 grid(kSampleBlocks), block(256);
  if (t0) {
    if (write) hipLaunchKernelGGL((k_type1<D, MODEL, true, true>), grid, block, 0, st, gd, v, P, src, nunits, wo);
    else hipLaunchKernelGGL((k_type1<D, MODEL, true, false>), grid, block, 0, st, gd, v, P, src, nunits, wo);
  } else {
    if (write) hipLaunchKernelGGL((k_type1<D, MODEL, false, true>), grid, block, 0, st, gd, v, P, src, nunits, wo);
    else hipLaunchKernelGGL((k_type1<D, MODEL, false, false>), grid, block, 0, st, gd, v, P, src, nunits, wo);
  }
}

hipError_t launch_type1(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nsrc, bool write, const WaveOut& wo,
                        hipStream_t st) {
  const bool t0 = !(g.T > 0.0);
  if (g.model == 1) {
    launch_t1_d<1, 1>(t0, write, gd, v, P, src, nsrc * Offs<1>::n1, wo, st);
  } else {
    switch (g.d) {
      case 1: launch_t1_d<1, 0>(t0, write, gd, v, P, src, nsrc * Offs<1>::n1, wo, st); break;
      case 2: launch_t1_d<2, 0>(t0, write, gd, v, P, src, nsrc * Offs<2>::n1, wo, st); break;
      case 3: launch_t1_d<3, 0>(t0, write, gd, v, P, src, nsrc * Offs<3>::n1, wo, st); break;
      default: launch_t1_d<4, 0>(t0, write, gd, v, P, src, nsrc * Offs<4>::n1, wo, st); break;
    }
  }
  return hipGetLastError();
}

template <int D, int MODEL>
static void launch_t2_d(bool write, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nunits, const Pbar* pbt, int nlev,
                        const WaveOut& wo, const HeavyOut& ho, hipStream_t st) {
  const dim3 grid(kSampleBlocks), block(256);
  if (write) hipLaunchKernelGGL((k_type2<D, MODEL, true>), grid, block, 0, st, gd, v, P, src, nunits, pbt, nlev, wo, ho);
  else hipLaunchKernelGGL((k_type2<D, MODEL, false>), grid, block, 0, st, gd, v, P, src, nunits, pbt, nlev, wo, ho);
}

hipError_t launch_type2(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nsrc, const Pbar* pbt, int nlev, bool write,
                        const WaveOut& wo, const HeavyOut& ho, hipStream_t st) {
  if (g.model == 1) {
    launch_t2_d<1, 1>(write, gd, v, P, src, nsrc * Offs<1>::n2, pbt, nlev, wo, ho, st);
  } else {
    switch (g.d) {
      case 1: launch_t2_d<1, 0>(write, gd, v, P, src, nsrc * Offs<1>::n2, pbt, nlev, wo, ho, st); break;
      case 2: launch_t2_d<2, 0>(write, gd, v, P, src, nsrc * Offs<2>::n2, pbt, nlev, wo, ho, st); break;
      case 3: launch_t2_d<3, 0>(write, gd, v, P, src, nsrc * Offs<3>::n2, pbt, nlev, wo, ho, st); break;
      default: launch_t2_d<4, 0>(write, gd, v, P, src, nsrc * Offs<4>::n2, pbt, nlev, wo, ho, st); break;
    }
  }
  return hipGetLastError();
}

template <int D, int MODEL>
static void launch_h_d(bool write, const Graph* gd, const Verts& v, const HeavyRec* rec,
                       const uint64_t* segoff, uint32_t nh, uint64_t nseg, const Pbar* pbt,
                       int nlev, const WaveOut& wo, hipStream_t st) {
  const dim3 grid(kSampleBlocks), block(256);
  if (write) hipLaunchKernelGGL((k_heavy<D, MODEL, true>), grid, block, 0, st, gd, v, rec, segoff, nh, nseg, pbt, nlev, wo);
  else hipLaunchKernelGGL((k_heavy<D, MODEL, false>), grid, block, 0, st, gd, v, rec, segoff, nh, nseg, pbt, nlev, wo);
}

hipError_t launch_heavy(const Graph& g, const Graph* gd, const Verts& v, const void* rec,
                        const uint64_t* segoff, uint32_t nh, uint64_t nseg, const Pbar* pbt,
                        int nlev, bool write, const WaveOut& wo, hipStream_t st) {
  const HeavyRec* r = static_cast<const HeavyRec*>(rec);
  if (g.model == 1) {
    launch_h_d<1, 1>(write, gd, v, r, segoff, nh, nseg, pbt, nlev, wo, st);
  } else {
    switch (g.d) {
      case 1: launch_h_d<1, 0>(write, gd, v, r, segoff, nh, nseg, pbt, nlev, wo, st); break;
      case 2: launch_h_d<2, 0>(write, gd, v, r, segoff, nh, nseg, pbt, nlev, wo, st); break;
      case 3: launch_h_d<3, 0>(write, gd, v, r, segoff, nh, nseg, pbt, nlev, wo, st); break;
      default: launch_h_d<4, 0>(write, gd, v, r, segoff, nh, nseg, pbt, nlev, wo, st); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_heavy_prep(const void* rec, uint32_t nh, uint64_t* nseg, hipStream_t st) {
  hipLaunchKernelGGL(k_heavy_nseg, dim3((nh + 255) / 256), dim3(256), 0, st,
                     static_cast<const HeavyRec*>(rec), nh, nseg);
  return hipGetLastError();
}

hipError_t launch_heavy_gather(const void* in, const uint32_t* perm, uint32_t nh, void* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_heavy_gather, dim3((nh + 255) / 256), dim3(256), 0, st,
                     static_cast<const HeavyRec*>(in), perm, nh, static_cast<HeavyRec*>(out));
  return hipGetLastError();
}

size_t heavy_rec_size() { return sizeof(HeavyRec); }

}  // namespace hg
