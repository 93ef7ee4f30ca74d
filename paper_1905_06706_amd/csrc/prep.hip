// prep.hip -- gfx950 preprocessing kernels of the GIRG / HRG sampler
// (arXiv:1905.06706): points (Sec. 2), weight layers and Morton keys (Sec. 3.1,
// Sec. 3.4), the level tables CL, I and pbar (Sec. 3.1-3.3, Sec. 4.3), prefix
// sums per layer (Lemma 1) and the run sources that seed the sampling passes.
#include "sampler.h"

namespace hg {

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
                                                   double* __restrict__ pts,
                                                   uint32_t* __restrict__ flag) {
  // per-block layer sizes and extreme weights, merged once per block
  __shared__ int scount[kMaxLayers];
  __shared__ unsigned long long sext[kMaxLayers];
  const int model = g->model;
  if (threadIdx.x < kMaxLayers) {
    scount[threadIdx.x] = 0;
    sext[threadIdx.x] = model == 0 ? 0ull : ~0ull;
  }
  __syncthreads();
  const uint32_t n = g->n;
  const double scale = ldexp(1.0, g->Dmax);
  // grid-stride over the vertices: few workgroups, so few global atomics on
  // the same layer counters at the end
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t u_end = ((uint64_t)n + blockDim.x - 1) / blockDim.x * blockDim.x;  // whole waves
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < u_end; u += stride) {
    uint32_t bad = 0;
    int layer = 0;
    double wu = 0.0;
    if (u < n) {
      wu = w[u];
      if (model == 0) {
        if (!(wu > 0.0) || !(wu < __builtin_inf())) bad |= 1u;
        else layer = ilogb(wu / g->w0);
      } else {
        if (!(wu >= 0.0 && wu <= g->R)) bad |= 1u;
        else layer = (int)floor((g->R - wu) / (2.0 * 0.6931471805599453));
      }
      if (!bad && (layer < 0 || layer >= kMaxLayers)) bad |= 2u;
      uint32_t q[D];
      // the point packed for the gather (one record load per vertex there)
      const int P = pts_stride(D, model);
      double* pu = pts + (uint64_t)u * P;
      pu[0] = wu;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double xk = x[(uint64_t)k * n + u];
        if (!(xk >= 0.0 && xk < 1.0)) bad |= 4u;
        q[k] = bad ? 0u : (uint32_t)(xk * scale);
        if (model == 0 || k == 0) pu[1 + k] = xk;
      }
      if (model == 0)
        for (int k = 1 + D; k < P; ++k) pu[k] = 0.0;
      if (bad) {
        atomicOr(flag, bad);
      } else {
        const uint32_t m = morton_encode<D>(q);
        keys[u] = ((uint64_t)layer << g->bits) | m;
        ids[u] = (uint32_t)u;
      }
    }
    // one LDS update per distinct layer of the wave: most lanes share a layer,
    // and same-address LDS atomics serialise
    const bool ok = u < n && !bad;
    const int lay = ok ? layer : -1;
    const unsigned long long bw = ok ? (unsigned long long)__double_as_longlong(wu) : 0ull;
    uint64_t pending = __ballot(ok);
    while (pending) {
      const int L0 = __shfl(lay, __ffsll((unsigned long long)pending) - 1, 64);
      const bool mine = lay == L0;
      const uint64_t same = __ballot(mine);
      // extreme weight of the layer over the wave (positive doubles order as integers)
      unsigned long long v = mine ? bw : (model == 0 ? 0ull : ~0ull);
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(v, o, 64);
        v = model == 0 ? (t > v ? t : v) : (t < v ? t : v);
      }
      if ((int)lane_id() == __ffsll((unsigned long long)same) - 1) {
        atomicAdd(&scount[L0], (int)__popcll(same));
        if (model == 0) atomicMax(&sext[L0], v);
        else atomicMin(&sext[L0], v);
      }
      pending &= ~same;
    }
  }
  __syncthreads();
  if (threadIdx.x < kMaxLayers && scount[threadIdx.x] > 0) {
    atomicAdd(&g->count[threadIdx.x], scount[threadIdx.x]);
    if (model == 0) atomicMax((unsigned long long*)&g->ext[threadIdx.x], sext[threadIdx.x]);
    else atomicMin((unsigned long long*)&g->ext[threadIdx.x], sext[threadIdx.x]);
  }
}

hipError_t launch_layer_key(const Graph& g, Graph* gd, const double* w, const double* x,
                            uint64_t* keys, uint32_t* ids, double* pts, uint32_t* flag, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<uint64_t>((g.n + 255) / 256, 512);
  switch (g.d) {
    case 1: hipLaunchKernelGGL(k_layer_key<1>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, pts, flag); break;
    case 2: hipLaunchKernelGGL(k_layer_key<2>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, pts, flag); break;
    case 3: hipLaunchKernelGGL(k_layer_key<3>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, pts, flag); break;
    default: hipLaunchKernelGGL(k_layer_key<4>, dim3(blocks), dim3(256), 0, st, gd, w, x, keys, ids, pts, flag); break;
  }
  return hipGetLastError();
}

// W = sum of the weights and w0 = the smallest, from the reduction's results
// (red[0], red[4]), into the device Graph before the layer keys need w0
__global__ void k_set_weight_sums(Graph* __restrict__ g, const double* __restrict__ red) {
  if (threadIdx.x == 0) {
    g->W = red[0];
    g->w0 = red[4];
  }
}

hipError_t launch_set_weight_sums(Graph* gd, const double* red, hipStream_t st) {
  hipLaunchKernelGGL(k_set_weight_sums, dim3(1), dim3(64), 0, st, gd, red);
  return hipGetLastError();
}

// sorted structure-of-arrays copy
// sorted arrays from the packed points: one scattered record load per vertex
// (the point of sorted position s is pts[ids[s]])
__global__ __launch_bounds__(256) void k_gather(const Graph* __restrict__ g,
                                                const uint64_t* __restrict__ keys,
                                                const uint32_t* __restrict__ ids,
                                                const double* __restrict__ pts, double* __restrict__ sw,
                                                double* __restrict__ rec, uint32_t* __restrict__ smort,
                                                uint8_t* __restrict__ slayer, uint4* __restrict__ frec) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = g->n;
  if (s >= n) return;
  const uint32_t u = ids[s];
  const uint64_t key = keys[s];
  smort[s] = g->bits == 32 ? (uint32_t)key : (uint32_t)(key & ((1ull << g->bits) - 1));
  slayer[s] = (uint8_t)(key >> g->bits);
  const int S = rec_stride(g->d, g->model);
  double* r = rec + s * (uint64_t)S;
  if (g->model == 1) {
    const double wu = pts[2 * (uint64_t)u], xu = pts[2 * (uint64_t)u + 1];
    sw[s] = wu;
    r[0] = xu;
    r[1] = exp(wu);
    r[2] = exp(-wu);
    r[3] = sinh(wu);
  } else {
    // the GIRG record is the packed point itself (same stride)
    const double2* p2 = reinterpret_cast<const double2*>(pts + (uint64_t)u * S);
    double2* r2 = reinterpret_cast<double2*>(r);
    for (int k = 0; k < S / 2; ++k) r2[k] = p2[k];
    sw[s] = r[0];
    if (frec) {
      // the mixed path's FP32 filter record: log2 w, coordinates in 32-bit
      // fixed point (x in [0, 1), so x 2^32 < 2^32 and its floor is exact)
      const int d = g->d;
      uint4 f;
      f.x = __float_as_uint((float)log2(r[0]));
      f.y = (uint32_t)(uint64_t)(r[1] * 0x1p32);
      f.z = d > 1 ? (uint32_t)(uint64_t)(r[2] * 0x1p32) : 0u;
      f.w = d > 2 ? (uint32_t)(uint64_t)(r[3] * 0x1p32) : 0u;
      frec[s] = f;
    }
  }
}

hipError_t launch_gather(const Graph& g, const Graph* gd, const uint64_t* keys, const uint32_t* ids,
                         const double* pts, double* sw, double* rec, uint32_t* smort,
                         uint8_t* slayer, uint4* frec, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, gd, keys, ids, pts,
                     sw, rec, smort, slayer, frec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// level tables: comparison level CL(i,j) (Sec. 3.1; HRG by search over
// levels, Sec. 4.3), insertion level I(i), deepest level D, the masks of
// layer pairs served by neighbouring (CL == level) and distant (CL >= level)
// cell pairs (loop swap, Sec. 3.3), and the type-II bounds pbar.  The
// tables are tiny (<= 64 x 64 layer pairs) and the host needs I(i) to size
// the cell arrays: they are computed on the host and uploaded with the
// Graph, which saves a readback; pbar runs on the device over a grid.
// ---------------------------------------------------------------------------
void tables_host(Graph& g, int Dcap) {
  const int L = g.L, d = g.d;
  int dmax = 0;
  for (int i = 0; i < kMaxLayers; ++i) {
    for (int j = 0; j < kMaxLayers; ++j) {
      int l = -1;
      if (i < L && j < L && g.count[i] > 0 && g.count[j] > 0) {
        l = 0;
        const double ei = g.ext[i], ej = g.ext[j];
        if (g.model == 0 && g.T == 0.0) {
          const double tmax = g.c * std::pow(ei * ej / g.W, 1.0 / d);
          while (l < Dcap && std::ldexp(1.0, -(l + 1)) >= tmax) ++l;
        } else if (g.model == 0) {
          const double V = g.kappa * ei * ej / g.W;
          while (l < Dcap && std::ldexp(1.0, -(l + 1) * d) >= V) ++l;
        } else {
          const double shh = 2.0 * std::sinh(ei) * std::sinh(ej);
          while (l < Dcap) {
            const int nl = l + 1;
            if (nl >= 2) {
              const double s = std::sin(3.141592653589793 * std::ldexp(1.0, -nl));
              if (!(1.0 + shh * s * s >= g.coshR)) break;
            }
            l = nl;
          }
        }
        l += g.cl_bias;
        if (l < 0) l = 0;
        if (l > Dcap) l = Dcap;
        if (g.max_depth >= 0 && l > g.max_depth) l = g.max_depth;
        dmax = std::max(dmax, l);
      }
      g.CL[i][j] = (int8_t)l;
    }
  }
  g.D = dmax;
  for (int i = 0; i < kMaxLayers; ++i) {
    int I = -1;
    for (int j = 0; j < kMaxLayers; ++j) I = std::max<int>(I, g.CL[i][j]);
    g.I[i] = (int8_t)I;
  }
  for (int i = 0; i < kMaxLayers; ++i) {
    for (int l = 0; l < kMaxLevels; ++l) {
      uint64_t m1 = 0, m2 = 0;
      for (int j = 0; j < (i < L ? L : 0); ++j) {  // CL is -1 outside the L x L block
        const int cl = g.CL[i][j];
        if (cl < 0) continue;
        if (cl == l) m1 |= 1ull << j;
        if (cl >= l && l >= 2) m2 |= 1ull << j;  // distant pairs exist from level 2
      }
      g.jI[i][l] = m1;
      g.jII[i][l] = g.T > 0.0 ? m2 : 0ull;  // threshold: distant cells hold no edges
    }
  }
}

// pbar for (i, j, level, gap): largest weights, smallest distance gap
// 2^-level; one entry per thread over the whole grid (CL from tables_host).
// Entry ((i (Dcap + 1) + level) L + j) 2 + gap - 1: the row of one source
// layer and level is contiguous.
__global__ __launch_bounds__(256) void k_pbar(const Graph* __restrict__ g, int Dcap,
                                              Pbar* __restrict__ pb, int total) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int L = g->L, d = g->d;
  const int nl = Dcap + 1;
  {
    const int gi = p & 1, j = (p >> 1) % L, il = (p >> 1) / L, l = il % nl, i = il / nl;
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
      e.ilg = 1.0 / log1p(-pbar);
      e.e = pbar > 0.0 ? kSegExp - ilogb(pbar) : 1 << 20;
      e.qscale = pbar > 0.0 && pbar < 1.0 ? (float)(0.6931471805599453 * e.ilg) : 0.0f;
    }
    pb[p] = e;
  }
}

hipError_t launch_pbar(const Graph* gd, int L, int Dcap, Pbar* pb, hipStream_t st) {
  if (pb && L > 0) {
    const int total = L * L * (Dcap + 1) * 2;
    hipLaunchKernelGGL(k_pbar, dim3((total + 255) / 256), dim3(256), 0, st, gd, Dcap, pb, total);
  }
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
                                                  const uint32_t* __restrict__ P,
                                                  const uint32_t* __restrict__ off,
                                                  Src* __restrict__ src,
                                                  CellL* __restrict__ cl) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g->n) return;
  const int h = head_level(g, smort, slayer, (uint32_t)s);
  const int i = slayer[s];
  const int I = g->I[i];
  const uint32_t m = smort[s];
  const uint32_t* Pi = P + g->pbase[i];
  uint64_t o = off[s];
  for (int l = h; l <= I; ++l) {
    const uint32_t A = cell_at(m, l, g->d, g->bits);
    const int sh = g->d * (I - l);
    const uint32_t end = Pi[((uint64_t)A + 1) << sh];
    src[o++] = Src{(uint32_t)s, A, end - (uint32_t)s, (uint32_t)l | ((uint32_t)i << 8)};
    atomicOr(reinterpret_cast<unsigned long long*>(&cl[g->moff[l] + A].mask), 1ull << i);
  }
}

// layer counts of every (level, cell) entry, for the scan that gives `base`
__global__ __launch_bounds__(256) void k_cell_popc(const CellL* __restrict__ cl, uint64_t ne,
                                                   uint32_t* __restrict__ cnt) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) cnt[e] = (uint32_t)__popcll(cl[e].mask);
}

__global__ __launch_bounds__(256) void k_cell_base(CellL* __restrict__ cl, uint64_t ne,
                                                   const uint32_t* __restrict__ off) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) cl[e].base = off[e];
}

// every source's (first sorted position, count) at its rank among the layers
// of its cell
__global__ __launch_bounds__(256) void k_src_rank(const Graph* __restrict__ g,
                                                  const Src* __restrict__ src, uint64_t nsrc,
                                                  const CellL* __restrict__ cl,
                                                  uint2* __restrict__ crec) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nsrc) return;
  const Src sr = src[q];
  const uint32_t l = sr.meta & 255u, i = sr.meta >> 8;
  const CellL c = cl[g->moff[l] + sr.A];
  crec[c.base + (uint32_t)__popcll(c.mask & ((1ull << i) - 1ull))] = make_uint2(sr.s, sr.na);
}

hipError_t launch_sources(const Graph& g, const Graph* gd, const uint32_t* smort,
                          const uint8_t* slayer, const uint32_t* P, uint32_t* cnt,
                          const uint32_t* off, Src* src, CellL* cl, bool fill, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.n + 255) / 256);
  if (!fill)
    hipLaunchKernelGGL(k_src_count, dim3(blocks), dim3(256), 0, st, gd, smort, slayer, cnt);
  else
    hipLaunchKernelGGL(k_src_fill, dim3(blocks), dim3(256), 0, st, gd, smort, slayer, P, off, src, cl);
  return hipGetLastError();
}

hipError_t launch_cell_layers(const Graph* gd, CellL* cl, uint64_t ne, uint32_t* cnt,
                              const Src* src, uint64_t nsrc, uint2* crec, bool ranks,
                              hipStream_t st) {
  if (!ranks) {
    if (ne)
      hipLaunchKernelGGL(k_cell_popc, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, cl, ne, cnt);
  } else {
    if (ne)
      hipLaunchKernelGGL(k_cell_base, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, cl, ne, cnt);
    if (nsrc)
      hipLaunchKernelGGL(k_src_rank, dim3((unsigned)((nsrc + 255) / 256)), dim3(256), 0, st, gd, src,
                         nsrc, cl, crec);
  }
  return hipGetLastError();
}

}  // namespace hg
