// sample.hip -- gfx950 sampling kernels of the GIRG / HRG sampler
// (arXiv:1905.06706, Sec. 3): fused cell-pair enumeration and sampling for
// type-I (neighbouring cells, every pair tested) and type-II (distant cells,
// geometric jumps under pbar, then rejection) cell pairs, plus the kernels for
// items deferred because they are large.
//
// Work decomposition.  The unit of work is (run source, cell offset).  Waves
// take chunks of consecutive units by atomic ticket (persistent grid); inside
// a chunk the 64 lanes take interleaved units and each runs a small state
// machine: fetch the next non-empty item (layer pair x cell pair), then one
// test (type-I: two per Philox block) or one geometric draw (type-II) per
// step.  The step loop is converged across the wave, so each step ends in a
// ballot that appends the accepted edges in a fixed order.  A count pass
// stores the edge count of every chunk; a scan gives each chunk its offset;
// the write pass repeats the work and stores the edges.  The edge array is a
// pure function of the inputs and the seed, whatever wave ran which chunk.
#include "sampler.h"

namespace hg {

__device__ __forceinline__ uint32_t next_chunk(unsigned int* next) {
  uint32_t c = 0;
  if (lane_id() == 0) c = atomicAdd(next, 1u);
  return __builtin_amdgcn_readfirstlane(c);
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


// ---------------------------------------------------------------------------
// type-I step: up to two tests of the current item sharing one Philox block.
// Pair index k = a * |V_j^B| + b, or for A = B and i = j (only a < b)
// k = b (b - 1) / 2 + a (App. B.1); tests k and k + 1 use words 0-1 and 2-3
// of block k / 2 (k is even at every step).
// ---------------------------------------------------------------------------
template <int D, int MODEL, bool T0, bool WRITE>
__device__ __forceinline__ void type1_step(const Graph* __restrict__ g, const Verts& v, uint32_t A,
                                           uint32_t B, uint32_t w3base, uint32_t a0, uint32_t b0,
                                           uint32_t nb, bool tri, uint32_t& a, uint32_t& b,
                                           uint64_t& k, uint64_t kend, bool& e0, bool& e1,
                                           uint2& p0, uint2& p1, uint64_t& ntests) {
  U4 o{0, 0, 0, 0};
  if constexpr (!T0)
    o = philox((uint32_t)(k >> 1), A, B, w3base | ((uint32_t)(k >> 33) << 20), g->seed_lo, g->seed_hi);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (k < kend) {
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
}

__device__ __forceinline__ void append2(bool WRITE, bool e0, bool e1, uint2 p0, uint2 p1,
                                        uint2* __restrict__ edges, uint64_t& running) {
  const uint64_t m0 = __ballot(e0), m1 = __ballot(e1);
  if (WRITE) {
    if (e0) edges[running + lanes_below(m0)] = p0;
    if (e1) edges[running + __popcll(m0) + lanes_below(m1)] = p1;
  }
  running += __popcll(m0) + __popcll(m1);
}

__device__ __forceinline__ void defer_item(bool WRITE, bool pending, const ItemRec& rec,
                                           uint32_t chunk, uint32_t& seq, const DeferOut& dfo) {
  const uint64_t mb = __ballot(pending);
  if (!WRITE && pending) {
    const unsigned int slot = atomicAdd(dfo.count, 1u);
    if (slot < dfo.cap) {
      dfo.rec[slot] = rec;
      dfo.key[slot] = ((uint64_t)chunk << 24) | (seq + lanes_below(mb));
    }
  }
  seq += __popcll(mb);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return x;
}

// ---------------------------------------------------------------------------
// type-I pass: neighbouring cell pairs at level CL(i,j) (loop swap, Sec. 3.3)
// ---------------------------------------------------------------------------
template <int D, int MODEL, bool T0, bool WRITE>
__global__ __launch_bounds__(256) void k_type1(const Graph* __restrict__ g, Verts v,
                                               const uint32_t* __restrict__ P,
                                               const Src* __restrict__ src, Sched sc, PassOut po,
                                               DeferOut dfo) {
  constexpr int NOFF = Offs<D>::n1;
  const uint32_t lane = lane_id();
  uint64_t ntests = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    uint64_t u = ub + lane;
    uint64_t jm = 0;
    uint32_t A = 0, B = 0, a0 = 0, na = 0, lvl = 0, li = 0;
    bool same = false, act = false, tri = false, big = false;
    uint32_t b0 = 0, nb = 0, a = 0, b = 0, w3 = 0;
    uint64_t k = 0, tot = 0;
    ItemRec rec{};
    uint64_t running = WRITE ? po.add + po.base[c] : 0;
    uint32_t dseq = 0;
    for (;;) {
      while (!act && !big) {
        if (jm == 0) {
          if (u >= ue) break;
          const uint64_t sidx = u / NOFF;
          const uint32_t off = (uint32_t)(u - sidx * NOFF);
          u += kWave;
          const Src sr = src[sidx];
          lvl = sr.meta & 255u;
          li = sr.meta >> 8;
          jm = g->jI[li][lvl];
          if (!jm) continue;
          A = sr.A;
          if (!neighbour_cell<D>(A, lvl, off, &B) || B < A) { jm = 0; continue; }
          same = (B == A);
          if (same) jm &= ~((1ull << li) - 1ull);  // j >= i when A = B
          a0 = sr.s;
          na = sr.na;
          continue;
        }
        const uint32_t lj = (uint32_t)__ffsll((long long)jm) - 1;
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
        w3 = ctr_word3(lvl, li, lj, kKindType1, 0);
        if (tot > kBigTests) {
          rec = ItemRec{a0, na, b0, nb, A, B, lvl | (li << 8) | (lj << 16) | (tri ? 1u << 31 : 0u), 0u};
          big = true;
          continue;
        }
        k = 0;
        act = true;
      }
      const bool anyb = __any(big);
      if (!anyb && !__any(act)) break;
      if (anyb) {
        defer_item(WRITE, big, rec, c, dseq, dfo);
        big = false;
      }
      bool e0 = false, e1 = false;
      uint2 p0 = make_uint2(0, 0), p1 = make_uint2(0, 0);
      if (act) {
        type1_step<D, MODEL, T0, WRITE>(g, v, A, B, w3, a0, b0, nb, tri, a, b, k, tot, e0, e1, p0, p1, ntests);
        if (k >= tot) act = false;
      }
      append2(WRITE, e0, e1, p0, p1, po.edges, running);
    }
    if (!WRITE && lane == 0) po.count[c] = running;
  }
  if (!WRITE) {
    ntests = wave_sum(ntests);
    if (lane == 0) atomicAdd(&po.stats[0], (unsigned long long)ntests);
  }
}

// split type-I items: units of kTestChunk consecutive tests
template <int D, int MODEL, bool T0, bool WRITE>
__global__ __launch_bounds__(256) void k_big1(const Graph* __restrict__ g, Verts v,
                                              const ItemRec* __restrict__ rec,
                                              const uint64_t* __restrict__ uoff, uint32_t nrec,
                                              Sched sc, PassOut po) {
  const uint32_t lane = lane_id();
  uint64_t ntests = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    uint64_t u = ub + lane;
    bool act = false, tri = false;
    uint32_t A = 0, B = 0, a0 = 0, b0 = 0, nb = 0, a = 0, b = 0, w3 = 0;
    uint64_t k = 0, kend = 0;
    uint64_t running = WRITE ? po.add + po.base[c] : 0;
    for (;;) {
      if (!act && u < ue) {
        uint32_t lo = 0, hi = nrec;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (uoff[mid] <= u) lo = mid; else hi = mid;
        }
        const ItemRec r = rec[lo];
        tri = (r.meta >> 31) != 0;
        const uint64_t tot = tri ? (uint64_t)r.na * (r.na - 1) / 2 : (uint64_t)r.na * r.nb;
        k = (u - uoff[lo]) * kTestChunk;
        kend = k + kTestChunk < tot ? k + kTestChunk : tot;
        A = r.A; B = r.B; a0 = r.a0; b0 = r.b0; nb = r.nb;
        w3 = ctr_word3(r.meta & 255u, (r.meta >> 8) & 255u, (r.meta >> 16) & 255u, kKindType1, 0);
        if (tri) {
          // b = largest with b (b - 1) / 2 <= k
          uint64_t bb = (uint64_t)floor(0.5 * (1.0 + sqrt(1.0 + 8.0 * (double)k)));
          while (bb * (bb - 1) / 2 > k) --bb;
          while ((bb + 1) * bb / 2 <= k) ++bb;
          b = (uint32_t)bb;
          a = (uint32_t)(k - bb * (bb - 1) / 2);
        } else {
          a = (uint32_t)(k / nb);
          b = (uint32_t)(k - (uint64_t)a * nb);
        }
        u += kWave;
        act = true;
      }
      if (!__any(act)) break;
      bool e0 = false, e1 = false;
      uint2 p0 = make_uint2(0, 0), p1 = make_uint2(0, 0);
      if (act) {
        type1_step<D, MODEL, T0, WRITE>(g, v, A, B, w3, a0, b0, nb, tri, a, b, k, kend, e0, e1, p0, p1, ntests);
        if (k >= kend) act = false;
      }
      append2(WRITE, e0, e1, p0, p1, po.edges, running);
    }
    if (!WRITE && lane == 0) po.count[c] = running;
  }
  if (!WRITE) {
    ntests = wave_sum(ntests);
    if (lane == 0) atomicAdd(&po.stats[0], (unsigned long long)ntests);
  }
}

// ---------------------------------------------------------------------------
// type-II pass: distant cell pairs with neighbouring parents at levels
// l <= CL(i,j).  Candidates of V_i^A x V_j^B are drawn by geometric jumps
// under pbar and accepted with p_uv / pbar (Sec. 3.2).  The candidate range is
// cut into segments of G = 2^e (e = 5 - ilogb(pbar), raised to keep at most
// 2^12 segments); segment s draws from counter (t, A, B, l|i|j|1|s).  Items
// with one segment are sampled here, the others are deferred.
// ---------------------------------------------------------------------------
template <int D, int MODEL, bool WRITE>
__global__ __launch_bounds__(256) void k_type2(const Graph* __restrict__ g, Verts v,
                                               const uint32_t* __restrict__ P,
                                               const Src* __restrict__ src, Sched sc,
                                               const Pbar* __restrict__ pbt, int nlev, PassOut po,
                                               DeferOut dfo) {
  constexpr int NOFF = Offs<D>::n2;
  const uint32_t lane = lane_id();
  const int L = g->L;
  uint64_t ndraws = 0, ncand = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    uint64_t u = ub + lane;
    uint64_t jm = 0;
    uint32_t A = 0, B = 0, a0 = 0, na = 0, lvl = 0, li = 0;
    int gap = 1;
    bool act = false, hv = false;
    uint32_t b0 = 0, nb = 0, t = 0, w3 = 0;
    uint64_t k = 0, N = 0;
    double pb = 0.0, lg = 0.0;
    ItemRec rec{};
    uint64_t running = WRITE ? po.add + po.base[c] : 0;
    uint32_t dseq = 0;
    for (;;) {
      while (!act && !hv) {
        if (jm == 0) {
          if (u >= ue) break;
          const uint64_t sidx = u / NOFF;
          const uint32_t off = (uint32_t)(u - sidx * NOFF);
          u += kWave;
          const Src sr = src[sidx];
          lvl = sr.meta & 255u;
          li = sr.meta >> 8;
          jm = g->jII[li][lvl];
          if (!jm) continue;
          A = sr.A;
          if (!distant_cell<D>(A, lvl, off, &B, &gap) || B < A) { jm = 0; continue; }
          a0 = sr.s;
          na = sr.na;
          continue;
        }
        const uint32_t lj = (uint32_t)__ffsll((long long)jm) - 1;
        jm &= jm - 1;
        cell_range(g, P, lj, lvl, B, &b0, &nb);
        if (!nb) continue;
        const Pbar pe = pbt[(((uint64_t)li * L + lj) * nlev + lvl) * 2 + (gap - 1)];
        if (!(pe.pbar > 0.0)) continue;
        N = (uint64_t)na * nb;
        uint64_t G, nseg;
        segment_size(N, pe.e, &G, &nseg);
        if (nseg > 1) {
          rec = ItemRec{a0, na, b0, nb, A, B, lvl | (li << 8) | (lj << 16) | ((uint32_t)gap << 24),
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
      const bool anyh = __any(hv);
      if (!anyh && !__any(act)) break;
      if (anyh) {
        defer_item(WRITE, hv, rec, c, dseq, dfo);
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
      append2(WRITE, e0, false, p0, p0, po.edges, running);
    }
    if (!WRITE && lane == 0) po.count[c] = running;
  }
  if (!WRITE) {
    ndraws = wave_sum(ndraws);
    ncand = wave_sum(ncand);
    if (lane == 0) {
      atomicAdd(&po.stats[1], (unsigned long long)ndraws);
      atomicAdd(&po.stats[2], (unsigned long long)ncand);
    }
  }
}

// deferred type-II items: one segment per unit
template <int D, int MODEL, bool WRITE>
__global__ __launch_bounds__(256) void k_heavy2(const Graph* __restrict__ g, Verts v,
                                                const ItemRec* __restrict__ rec,
                                                const uint64_t* __restrict__ uoff, uint32_t nrec,
                                                Sched sc, const Pbar* __restrict__ pbt, int nlev,
                                                PassOut po) {
  const uint32_t lane = lane_id();
  const int L = g->L;
  uint64_t ndraws = 0, ncand = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    uint64_t u = ub + lane;
    bool act = false;
    uint32_t A = 0, B = 0, a0 = 0, b0 = 0, nb = 0, t = 0, w3 = 0;
    uint64_t k = 0, kend = 0;
    double pb = 0.0, lg = 0.0;
    uint64_t running = WRITE ? po.add + po.base[c] : 0;
    for (;;) {
      if (!act && u < ue) {
        uint32_t lo = 0, hi = nrec;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (uoff[mid] <= u) lo = mid; else hi = mid;
        }
        const ItemRec r = rec[lo];
        const uint64_t s = u - uoff[lo];
        const uint32_t lvl = r.meta & 255u, li = (r.meta >> 8) & 255u, lj = (r.meta >> 16) & 255u,
                       gp = (r.meta >> 24) & 127u;
        const Pbar pe = pbt[(((uint64_t)li * L + lj) * nlev + lvl) * 2 + (gp - 1)];
        const uint64_t N = (uint64_t)r.na * r.nb;
        uint64_t G, ns;
        segment_size(N, (int)r.e, &G, &ns);
        A = r.A; B = r.B; a0 = r.a0; b0 = r.b0; nb = r.nb;
        pb = pe.pbar;
        lg = pe.lg;
        w3 = ctr_word3(lvl, li, lj, kKindType2, (uint32_t)s);
        k = s * G;
        kend = (s + 1) * G < N ? (s + 1) * G : N;
        t = 0;
        u += kWave;
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
      append2(WRITE, e0, false, p0, p0, po.edges, running);
    }
    if (!WRITE && lane == 0) po.count[c] = running;
  }
  if (!WRITE) {
    ndraws = wave_sum(ndraws);
    ncand = wave_sum(ncand);
    if (lane == 0) {
      atomicAdd(&po.stats[1], (unsigned long long)ndraws);
      atomicAdd(&po.stats[2], (unsigned long long)ncand);
    }
  }
}

__global__ __launch_bounds__(256) void k_rec_units(const ItemRec* __restrict__ rec, uint32_t nrec,
                                                   int kind, uint64_t* __restrict__ units) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nrec) return;
  const ItemRec r = rec[h];
  if (kind == 1) {
    const bool tri = (r.meta >> 31) != 0;
    const uint64_t tot = tri ? (uint64_t)r.na * (r.na - 1) / 2 : (uint64_t)r.na * r.nb;
    units[h] = (tot + kTestChunk - 1) / kTestChunk;
  } else {
    uint64_t G, ns;
    segment_size((uint64_t)r.na * r.nb, (int)r.e, &G, &ns);
    units[h] = ns;
  }
}

__global__ __launch_bounds__(256) void k_rec_gather(const ItemRec* __restrict__ in,
                                                    const uint32_t* __restrict__ perm, uint32_t nrec,
                                                    ItemRec* __restrict__ out) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < nrec) out[h] = in[perm[h]];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define HG_DISPATCH_D(MODELV, ...)                                              \
  do {                                                                          \
    if (g.model == 1) { constexpr int DD = 1; constexpr int MM = 1; __VA_ARGS__; } \
    else switch (g.d) {                                                         \
      case 1: { constexpr int DD = 1; constexpr int MM = 0; __VA_ARGS__; } break; \
      case 2: { constexpr int DD = 2; constexpr int MM = 0; __VA_ARGS__; } break; \
      case 3: { constexpr int DD = 3; constexpr int MM = 0; __VA_ARGS__; } break; \
      default: { constexpr int DD = 4; constexpr int MM = 0; __VA_ARGS__; } break; \
    }                                                                           \
  } while (0)

hipError_t launch_type1(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const Src* src, const Sched& sc, bool write, const PassOut& po,
                        const DeferOut& dfo, hipStream_t st) {
  const bool t0 = !(g.T > 0.0);
  const dim3 grid(kPersistBlocks), block(256);
  HG_DISPATCH_D(0, {
    if (t0) {
      if (write) hipLaunchKernelGGL((k_type1<DD, MM, true, true>), grid, block, 0, st, gd, v, P, src, sc, po, dfo);
      else hipLaunchKernelGGL((k_type1<DD, MM, true, false>), grid, block, 0, st, gd, v, P, src, sc, po, dfo);
    } else {
      if (write) hipLaunchKernelGGL((k_type1<DD, MM, false, true>), grid, block, 0, st, gd, v, P, src, sc, po, dfo);
      else hipLaunchKernelGGL((k_type1<DD, MM, false, false>), grid, block, 0, st, gd, v, P, src, sc, po, dfo);
    }
  });
  return hipGetLastError();
}

hipError_t launch_big1(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                       const uint64_t* uoff, uint32_t nrec, const Sched& sc, bool write,
                       const PassOut& po, hipStream_t st) {
  const bool t0 = !(g.T > 0.0);
  const dim3 grid(kPersistBlocks), block(256);
  HG_DISPATCH_D(0, {
    if (t0) {
      if (write) hipLaunchKernelGGL((k_big1<DD, MM, true, true>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, po);
      else hipLaunchKernelGGL((k_big1<DD, MM, true, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, po);
    } else {
      if (write) hipLaunchKernelGGL((k_big1<DD, MM, false, true>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, po);
      else hipLaunchKernelGGL((k_big1<DD, MM, false, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, po);
    }
  });
  return hipGetLastError();
}

hipError_t launch_type2(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const Src* src, const Sched& sc, const Pbar* pbt, int nlev, bool write,
                        const PassOut& po, const DeferOut& dfo, hipStream_t st) {
  const dim3 grid(kPersistBlocks), block(256);
  HG_DISPATCH_D(0, {
    if (write) hipLaunchKernelGGL((k_type2<DD, MM, true>), grid, block, 0, st, gd, v, P, src, sc, pbt, nlev, po, dfo);
    else hipLaunchKernelGGL((k_type2<DD, MM, false>), grid, block, 0, st, gd, v, P, src, sc, pbt, nlev, po, dfo);
  });
  return hipGetLastError();
}

hipError_t launch_heavy2(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                         const uint64_t* uoff, uint32_t nrec, const Sched& sc, const Pbar* pbt,
                         int nlev, bool write, const PassOut& po, hipStream_t st) {
  const dim3 grid(kPersistBlocks), block(256);
  HG_DISPATCH_D(0, {
    if (write) hipLaunchKernelGGL((k_heavy2<DD, MM, true>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, pbt, nlev, po);
    else hipLaunchKernelGGL((k_heavy2<DD, MM, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, pbt, nlev, po);
  });
  return hipGetLastError();
}

hipError_t launch_rec_units(const ItemRec* rec, uint32_t nrec, int kind, uint64_t* units,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rec_units, dim3((nrec + 255) / 256), dim3(256), 0, st, rec, nrec, kind, units);
  return hipGetLastError();
}

hipError_t launch_rec_gather(const ItemRec* in, const uint32_t* perm, uint32_t nrec, ItemRec* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_rec_gather, dim3((nrec + 255) / 256), dim3(256), 0, st, in, perm, nrec, out);
  return hipGetLastError();
}

}  // namespace hg
