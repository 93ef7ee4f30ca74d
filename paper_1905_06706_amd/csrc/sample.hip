// sample.hip -- gfx950 sampling kernels of the GIRG / HRG sampler
// (arXiv:1905.06706, Sec. 3): fused cell-pair enumeration and sampling for
// type-I (neighbouring cells, every pair tested) and type-II (distant cells,
// geometric jumps under pbar, then rejection) cell pairs, plus the kernels for
// items split because they are large.
//
// Work decomposition.  The unit of work is a run source (layer i, level l,
// cell X).  Waves take chunks of consecutive sources by atomic ticket
// (persistent grid) and run converged phases over small per-wave LDS buffers:
//   A  lanes take 64 sources and count their candidate cells; a wave prefix
//      sum spreads the (source, cell Y) pairs over the lanes, which read the
//      layer set of Y at level l (one 16-byte entry) and append one entry per
//      nonempty item to an LDS list;
//   B  lanes take 64 items, read the (first, count) record of V_j^Y, orient
//      the pair (smaller cell = A side) and queue it (large ones go to a
//      deferred list);
//   C  type-I: 64 Philox blocks (two tests each) per step, flat across the
//      queued items; type-II: each item makes its first draw at once, items
//      with draws left are queued, one draw per lane and step, and candidates
//      go to a ring that is evaluated 64 at a time.
// Pair decisions read one packed record (w, x) per vertex.
// Accepted edges are appended (wave ballots) to an LDS buffer that is flushed
// in blocks of at least 128 edges to a staging array at an atomically reserved
// position, with a record of its chunk and of the chunk's edges flushed
// before it.  A chunk's wave also stores the chunk's edge total; a scan of the
// totals in (pass, chunk) order places every block, so the edge array is a
// pure function of the inputs and the seed, whatever wave ran which chunk, in
// one sampling pass.
#include "sampler.h"
#include "fastpow.h"

namespace hg {

__device__ __forceinline__ uint32_t next_chunk(unsigned int* next) {
  uint32_t c = 0;
  if (lane_id() == 0) c = atomicAdd(next, 1u);
  return __builtin_amdgcn_readfirstlane(c);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return x;
}

// statistics slots of the decisions that lie inside the parity margins (rare,
// so each is counted by one atomic): coins within 1e-12 of the probability
// they are compared with (threshold variants: distance within 1e-12, relative,
// of the threshold), and type-II draws whose skip quotient lies within 1e-12
// (relative) of an integer that can still decide a candidate or the end
constexpr int kStatNear = 12, kStatTie = 13;
__device__ __forceinline__ void count_stat(unsigned long long* st, int slot) {
  atomicAdd(&st[slot], 1ull);
}
// list a type-II candidate with |apb - p_uv| < 1e-12 for the test against the
// band 1e-12 pbar after the passes (k_near2)
__device__ __forceinline__ void list_near2(uint4* nbuf, unsigned int* ncnt, uint32_t ncap,
                                           uint32_t su, uint32_t sv, double apb) {
  const unsigned int slot = atomicAdd(ncnt, 1u);
  const uint64_t bits = (uint64_t)__double_as_longlong(apb);
  if (slot < ncap) nbuf[slot] = make_uint4(su, sv, (uint32_t)bits, (uint32_t)(bits >> 32));
}

// ---------------------------------------------------------------------------
// edge decisions (FP64)
// ---------------------------------------------------------------------------
// the record of sorted vertex s, loaded 16 bytes at a time
template <int D, int MODEL>
struct Rec {
  static constexpr int S = rec_stride(D, MODEL);
  double v[S];
};

template <int D, int MODEL>
__device__ __forceinline__ Rec<D, MODEL> load_rec(const double* __restrict__ rec, uint32_t s) {
  constexpr int S = rec_stride(D, MODEL);
  Rec<D, MODEL> r;
  const double2* p = reinterpret_cast<const double2*>(rec + (uint64_t)s * S);
#pragma unroll
  for (int q = 0; q < S / 2; ++q) {
    const double2 t = p[q];
    r.v[2 * q] = t.x;
    r.v[2 * q + 1] = t.y;
  }
  return r;
}

// the records of both vertices of a pair in one round trip to memory: the
// first slot is needed last (after the distance), and without the empty asm
// the compiler loads it only then, and each record after the other
template <int D, int MODEL>
struct RecPair {
  Rec<D, MODEL> a, b;
};
template <int D, int MODEL>
__device__ __forceinline__ RecPair<D, MODEL> load_recs(const double* __restrict__ rec, uint32_t su,
                                                      uint32_t sv) {
  RecPair<D, MODEL> p{load_rec<D, MODEL>(rec, su), load_rec<D, MODEL>(rec, sv)};
  asm volatile("" ::"v"(p.a.v[0]), "v"(p.b.v[0]));
  return p;
}

// L-infinity torus distance of two records (GIRG: coordinates from slot 1,
// HRG: the angle / 2 pi in slot 0)
template <int D, int MODEL>
__device__ __forceinline__ double torus_r(const Rec<D, MODEL>& a, const Rec<D, MODEL>& b) {
  constexpr int X0 = MODEL == 1 ? 0 : 1;
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double df = fabs(a.v[X0 + k] - b.v[X0 + k]);
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

// GIRG binomial probability of Eq. (1); the power 1/T by pow_pos (relative
// error a few 2^-52, see fastpow.h)
template <int D>
__device__ __forceinline__ double girg_prob(const Graph* __restrict__ g, double wu, double wv,
                                           double r) {
  if (r == 0.0) return 1.0;
  const double p = g->c * pow_pos((wu * wv) / (g->W * pow_d<D>(r)), g->inv_T);
  return p < 1.0 ? p : 1.0;
}

// HRG: cosh of the hyperbolic distance, cosh(ru - rv) + 2 sinh ru sinh rv
// sin^2(pi dx), with cosh(ru - rv) from per-vertex e^r, e^-r.
template <int D>
__device__ __forceinline__ double hrg_coshd(const Rec<D, 1>& a, const Rec<D, 1>& b, double dx) {
  const double ch = 0.5 * (a.v[1] * b.v[2] + b.v[1] * a.v[2]);
  const double s = sinpi(dx);
  return ch + 2.0 * a.v[3] * b.v[3] * s * s;
}

// (out of line: the distance filter below decides most pairs without it, and
// inlined at every call site it made the type-II kernel spill registers)
__device__ __noinline__ double hrg_prob(const Graph* __restrict__ g, double coshd) {
  return 1.0 / (exp((acosh(coshd) - g->R) * (0.5 * g->inv_T)) + 1.0);
}

// binomial HRG decision U < p_T(d) with the distance filter of App. B.4: for
// U in [x_m, x_{m+1}) on the grid x = m / (kHrgTab - 1), d below the distance
// where p_T = x_{m+1} means an edge and d above the one where p_T = x_m means
// none (p_T decreases in d), compared as cosh d against the table.  Only
// pairs outside a 1e-12 relative margin of both entries, and U outside 1e-9
// of a grid point, are decided by the table; the rest evaluate p_T, so the
// result is that of the direct FP64 comparison.
// A pair the table decides lies more than 1e-11 from p_T; nr is set when the
// direct comparison finds |U - p_T| < 1e-12.
template <int D>
__device__ __forceinline__ bool hrg_below(const Graph* __restrict__ g, const Rec<D, 1>& a,
                                          const Rec<D, 1>& b, double U, bool& nr) {
  const double ch = hrg_coshd<D>(a, b, torus_r<D, 1>(a, b));
  const double t = U * (double)(kHrgTab - 1);
  const int m = (int)t;
  if (m < kHrgTab - 1 && t - (double)m > 1e-9 && (double)(m + 1) - t > 1e-9) {
    if (ch < g->hct[m + 1] * (1.0 - 1e-12)) return true;
    if (ch > g->hct[m] * (1.0 + 1e-12)) return false;
  }
  const double p = hrg_prob(g, ch);
  nr = fabs(U - p) < 1e-12;
  return U < p;
}

// probability (binomial variants) of the pair of sorted vertices (su, sv)
template <int D, int MODEL>
__device__ __forceinline__ double pair_prob(const Graph* __restrict__ g, const Verts& v,
                                            uint32_t su, uint32_t sv) {
  const RecPair<D, MODEL> ab = load_recs<D, MODEL>(v.rec, su, sv);
  const Rec<D, MODEL>& a = ab.a;
  const Rec<D, MODEL>& b = ab.b;
  const double r = torus_r<D, MODEL>(a, b);
  if constexpr (MODEL == 0) {
    return girg_prob<D>(g, a.v[0], b.v[0], r);
  } else {
    return hrg_prob(g, hrg_coshd<D>(a, b, r));
  }
}

// threshold variants
// (nr: the distance lies within 1e-12, relative, of the threshold; for GIRGs
// (r / t)^d within d 1e-12 of 1)
template <int D, int MODEL>
__device__ __forceinline__ bool pair_thresh(const Graph* __restrict__ g, const Verts& v,
                                            uint32_t su, uint32_t sv, bool& nr) {
  const RecPair<D, MODEL> ab = load_recs<D, MODEL>(v.rec, su, sv);
  const Rec<D, MODEL>& a = ab.a;
  const Rec<D, MODEL>& b = ab.b;
  const double r = torus_r<D, MODEL>(a, b);
  if constexpr (MODEL == 0) {
    // ||x_u - x_v|| <= c (w_u w_v / W)^{1/d}  <=>  r^d W <= c^d w_u w_v
    const double lhs = pow_d<D>(r) * g->W, rhs = g->kappa * a.v[0] * b.v[0];
    nr = fabs(lhs - rhs) <= (1e-12 * D) * rhs;
    return lhs <= rhs;
  } else {
    const double ch = hrg_coshd<D>(a, b, r);
    nr = fabs(ch - g->coshR) <= 1e-12 * g->coshR;
    return ch < g->coshR;
  }
}

// ---------------------------------------------------------------------------
// mixed precision (GIRG, T > 0).  log2 min(p_uv, 1) is evaluated in FP32 as
// C + (1/T)(log2 w_u + log2 w_v - d log2 r) with C = log2 c - (1/T) log2 W
// (here, for d = 4: w and r exact in FP64, rounded to FP32, then __log2f).
// Every term carries a relative error of a few 2^-24, and __log2f one below
// 2^-23 (1 + |log2 x|) (tests/log2_probe.hip, on every positive float), so
// |L32 - log2 p| < 2^-20 (1 + |C| + (1/T)(|log2 w_u| + |log2 w_v| + d |log2 r|));
// the filter decides only outside 2^-13 times that sum (a factor 128 of
// slack) and re-decides every other pair with the FP64 formula, so the result
// is the FP64 path's decision.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ bool mixed_logp(const Graph* __restrict__ g, double wu, double wv,
                                           double r, float& Lc, float& err) {
  if (!(r >= 0x1p-100)) return false;  // r = 0 (p = 1) or below FP32 range: FP64
  const float lr = __log2f((float)r);
  const float a = __log2f((float)wu), b = __log2f((float)wv);
  const float L = g->C32 + g->invT32 * (a + b - (float)D * lr);
  err = 0x1p-13f * (1.0f + fabsf(g->C32) + g->invT32 * (fabsf(a) + fabsf(b) + (float)D * fabsf(lr)));
  Lc = fminf(L, 0.0f);
  return true;
}

// The same filter from the 16-byte records of Verts::frec (d <= 3): log2 w
// in FP32 (rounded from the FP64 log2: 2^-24 relative) and each coordinate as
// floor(x 2^32).  Per dimension the torus difference of two such coordinates
// is exact in 32-bit unsigned arithmetic, and it lies within 2^-32 of that of
// the points (it is 1-Lipschitz in each coordinate), so the L-infinity
// distance R 2^-32 is within 2^-32 of r.  For R >= 2^12 that moves log2 r by
// less than 1.5 / R, which the margin takes as (1/T) d 2 / R; closer pairs are
// decided in FP64.  log2 r = __log2f(fl32(R) 2^-32) keeps the error budget
// above, since |log2 r| >= 1 (r <= 1/2).
template <int D>
__device__ __forceinline__ bool mixed_logp_f(const Graph* __restrict__ g,
                                             const uint4* __restrict__ frec, uint32_t su,
                                             uint32_t sv, float& Lc, float& err) {
  const uint4 a = frec[su], b = frec[sv];
  asm volatile("" ::"v"(a.x), "v"(b.x));  // log2 w with the coordinates, in one load
  const uint32_t ax[3] = {a.y, a.z, a.w}, bx[3] = {b.y, b.z, b.w};
  uint32_t R = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const uint32_t df = ax[k] - bx[k];
    const uint32_t m = df < 0u - df ? df : 0u - df;
    R = m > R ? m : R;
  }
  if (R < 4096u) return false;
  const float fr = (float)R;
  const float lr = __log2f(fr * 0x1p-32f);
  const float la = __uint_as_float(a.x), lb = __uint_as_float(b.x);
  const float L = g->C32 + g->invT32 * (la + lb - (float)D * lr);
  err = 0x1p-13f * (1.0f + fabsf(g->C32) + g->invT32 * (fabsf(la) + fabsf(lb) + (float)D * fabsf(lr))) +
        g->invT32 * (float)(2 * D) * __builtin_amdgcn_rcpf(fr);
  Lc = fminf(L, 0.0f);
  return true;
}

// the FP64 decision of the mixed path's rechecks
template <int D>
__device__ __forceinline__ double mixed_prob64(const Graph* __restrict__ g, const Verts& v,
                                               uint32_t su, uint32_t sv) {
  const RecPair<D, 0> ab = load_recs<D, 0>(v.rec, su, sv);
  const Rec<D, 0>& a = ab.a;
  const Rec<D, 0>& b = ab.b;
  return girg_prob<D>(g, a.v[0], b.v[0], torus_r<D, 0>(a, b));
}

// type-I test: edge iff U < p_uv (nr: |U - p_uv| < 1e-12)
template <int D>
__device__ __forceinline__ bool mixed_test(const Graph* __restrict__ g, const Verts& v, uint32_t su,
                                           uint32_t sv, double U, uint32_t& nre, bool& nr) {
  if constexpr (D <= 3) {
    float Lc, err;
    if (U > 0.0 && mixed_logp_f<D>(g, v.frec, su, sv, Lc, err)) {
      const float lu = __log2f((float)U);
      if (lu < Lc - err) return true;
      if (lu > Lc + err) return false;
    }
    ++nre;
    const double p = mixed_prob64<D>(g, v, su, sv);
    nr = fabs(U - p) < 1e-12;
    return U < p;
  } else {
    const RecPair<D, 0> ab = load_recs<D, 0>(v.rec, su, sv);
    const Rec<D, 0>& a = ab.a;
    const Rec<D, 0>& b = ab.b;
    const double r = torus_r<D, 0>(a, b);
    float Lc, err;
    if (U > 0.0 && mixed_logp<D>(g, a.v[0], b.v[0], r, Lc, err)) {
      const float lu = __log2f((float)U);
      if (lu < Lc - err) return true;
      if (lu > Lc + err) return false;
    }
    ++nre;
    const double p = girg_prob<D>(g, a.v[0], b.v[0], r);
    nr = fabs(U - p) < 1e-12;
    return U < p;
  }
}

// type-II candidate: accepted iff Acc * pbar < p_uv (apb = Acc * pbar in FP64;
// a recheck with |apb - p_uv| < 1e-12 is listed for k_near2)
template <int D>
__device__ __forceinline__ bool mixed_cand(const Graph* __restrict__ g, const Verts& v, uint32_t su,
                                           uint32_t sv, double apb, uint32_t& nre, const Stage& sg) {
  double p;
  if constexpr (D <= 3) {
    float Lc, err;
    if (apb >= 0x1p-120 && mixed_logp_f<D>(g, v.frec, su, sv, Lc, err)) {
      const float la = __log2f((float)apb);
      const float e2 = err + 0x1p-13f * (1.0f + fabsf(la));
      if (la < Lc - e2) return true;
      if (la > Lc + e2) return false;
    }
    ++nre;
    p = mixed_prob64<D>(g, v, su, sv);
  } else {
    const RecPair<D, 0> ab = load_recs<D, 0>(v.rec, su, sv);
    const Rec<D, 0>& a = ab.a;
    const Rec<D, 0>& b = ab.b;
    const double r = torus_r<D, 0>(a, b);
    float Lc, err;
    if (apb >= 0x1p-120 && mixed_logp<D>(g, a.v[0], b.v[0], r, Lc, err)) {
      const float la = __log2f((float)apb);
      const float e2 = err + 0x1p-13f * (1.0f + fabsf(la));
      if (la < Lc - e2) return true;
      if (la > Lc + e2) return false;
    }
    ++nre;
    p = girg_prob<D>(g, a.v[0], b.v[0], r);
  }
  if (fabs(apb - p) < 1e-12) list_near2(sg.nbuf, sg.ncnt, sg.ncap, su, sv, apb);
  return apb < p;
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

__device__ __forceinline__ void segment_size(uint64_t N, int e, uint64_t* G, uint64_t* nseg) {
  const int emin = bitlen64(N - 1) - kSegMaxBits;
  if (e < emin) e = emin;
  *G = (e >= 63 || (1ull << e) >= N) ? N : (1ull << e);
  *nseg = (N + *G - 1) / *G;
}

// whether an item of N >= 1 candidates has more than one segment, without
// segment_size's division: raising e to emin keeps 2^e < N (2^emin < N for
// every N >= 2), so the test on the pbar exponent e (>= 5) decides alone
__device__ __forceinline__ bool multi_segment(uint64_t N, int e) {
  return e < 63 && N > (1ull << e);
}

// ---------------------------------------------------------------------------
// per-wave edge buffer and its flushes to the staging array
// ---------------------------------------------------------------------------
constexpr uint32_t kEdgeBuf = 256;   // LDS edges per wave; flushed above 128
constexpr uint32_t kEdgeBuf2 = 192;  // the same for waves that emit at most one edge per lane

struct Out {
  uint2* lb;           // LDS buffer of this wave: sorted positions of the edges
  uint32_t bn;         // edges in it
  uint64_t off;        // edges of the current chunk flushed so far
  uint64_t tag;        // pass << 32 | chunk
  const uint32_t* id;  // original ids of the sorted positions (applied at the flush)
};

__device__ __forceinline__ void flush(const Stage& sg, Out& o) {
  if (o.bn == 0) return;
  const uint32_t lane = lane_id();
  unsigned long long pos = 0;
  if (lane == 0) pos = atomicAdd(sg.cursor, (unsigned long long)o.bn);
  pos = __shfl(pos, 0, 64);
  for (uint32_t i = lane; i < o.bn; i += kWave)
    if (pos + i < sg.cap) {
      const uint2 e = o.lb[i];
      sg.buf[pos + i] = make_uint2(o.id[e.x], o.id[e.y]);
    }
  if (lane == 0) {
    const unsigned int slot = atomicAdd(sg.nrec, 1u);
    if (slot < sg.rcap) {
      sg.rtag[slot] = o.tag;
      sg.roff[slot] = o.off;
      sg.rpos[slot] = pos;
      sg.rcnt[slot] = o.bn;
    }
  }
  o.off += o.bn;
  o.bn = 0;
}

// the last flush of chunk c, then its totals: edges, and items deferred
__device__ __forceinline__ void end_chunk(const Stage& sg, Out& o, const Sched& sc, uint32_t c,
                                          uint32_t ndef) {
  flush(sg, o);
  if (lane_id() == 0) {
    sc.ctot[c] = o.off;
    if (sc.dtot) sc.dtot[c] = ndef;
  }
}

// append up to two edges per lane (order: all first edges, then all second)
__device__ __forceinline__ void emit(bool e0, bool e1, uint2 p0, uint2 p1, const Stage& sg,
                                     Out& o) {
  const uint64_t m0 = __ballot(e0), m1 = __ballot(e1);
  if (e0) o.lb[o.bn + lanes_below(m0)] = p0;
  if (e1) o.lb[o.bn + __popcll(m0) + lanes_below(m1)] = p1;
  o.bn += (uint32_t)(__popcll(m0) + __popcll(m1));
  if (o.bn > kEdgeBuf - 128) flush(sg, o);
}

__device__ __forceinline__ void defer_item(bool pending, const ItemRec& rec, uint32_t chunk,
                                           uint32_t& seq, const DeferOut& dfo) {
  const uint64_t mb = __ballot(pending);
  if (pending) {
    const unsigned int slot = atomicAdd(dfo.count, 1u);
    if (slot < dfo.cap) {
      dfo.rec[slot] = rec;
      dfo.key[slot] = ((uint64_t)chunk << 24) | (seq + lanes_below(mb));
    }
  }
  seq += (uint32_t)__popcll(mb);
}

// ---------------------------------------------------------------------------
// per-wave LDS buffers: item lists, item rings, candidate ring
// ---------------------------------------------------------------------------
constexpr int kQCap = 128;  // item ring (power of two, >= 2 x 64)
constexpr int kCCap = 128;  // candidate ring (power of two, >= 2 x 64)
constexpr int kICap = 128;  // item lists (>= 2 x 64)

// type-I item (or a piece of a split one): Philox blocks [kb, kb + nbk) of
// the item; cs = index of its first block in the wave's stream of blocks
struct QItem1 {
  uint32_t A, B, w3, a0, b0, nb, na, tri, cs, kb, nbk, pad;
};

// type-II item (or one segment of a segmented one): candidates [k, N)
struct QItem2 {
  uint32_t A, B, w3, a0, b0, nb, t;
  uint32_t pidx;  // entry of the pbar table
  uint64_t k, N;
};

// the pbar-table values an item's draws use, held in registers by the lane
// that owns the item
struct PB {
  double pbar, ilg;
  float qs;  // 1 / log2(1 - pbar)
};
// entry of (i, j, level, gap) in the pbar table, laid out [i][level][j][gap]:
// the items of one source (i, level) read one contiguous row of L x 2 entries
__device__ __forceinline__ uint32_t pbar_index(uint32_t i, uint32_t j, uint32_t lvl, uint32_t gap,
                                               uint32_t L, uint32_t nlev) {
  return ((i * nlev + lvl) * L + j) * 2u + (gap - 1u);
}
__device__ __forceinline__ PB load_pb(const Pbar* __restrict__ pbt, uint32_t pidx) {
  const Pbar e = pbt[pidx];
  return PB{e.pbar, e.ilg, e.qscale};
}

// type-II candidate: sorted indices and Acc * pbar
struct Cand {
  uint32_t su, sv;
  double apb;
};

// ---------------------------------------------------------------------------
// type-I tests.  Pair index k = a * |V_j^B| + b, or for A = B and i = j (only
// a < b) k = b (b - 1) / 2 + a (App. B.1); tests k and k + 1 use words 0-1 and
// 2-3 of Philox block k / 2.
// ---------------------------------------------------------------------------
struct Ring1 {
  uint32_t qh, qt;  // items [qh, qt) are queued (logical indices)
  uint32_t bc, bt;  // next Philox block to process / end of the queued blocks
};

template <int D, int MODEL, bool T0, bool MX>
__device__ __forceinline__ void test_block(const Graph* __restrict__ g, const Verts& v,
                                           const QItem1& it, uint64_t k, uint64_t kend, bool& e0,
                                           bool& e1, uint2& p0, uint2& p1, uint32_t& ntests,
                                           uint32_t& nre, unsigned long long* st) {
  const bool tri = it.tri != 0;
  uint32_t a, b;
  if (tri) {
    uint32_t bb = (uint32_t)(0.5 * (1.0 + sqrt(1.0 + 8.0 * (double)k)));
    while ((uint64_t)bb * (bb - 1) / 2 > k) --bb;
    while ((uint64_t)(bb + 1) * bb / 2 <= k) ++bb;
    b = bb;
    a = (uint32_t)(k - (uint64_t)bb * (bb - 1) / 2);
  } else if (k < 0xFFFFFFFFull) {
    a = (uint32_t)k / it.nb;
    b = (uint32_t)k - a * it.nb;
  } else {
    a = (uint32_t)(k / it.nb);
    b = (uint32_t)(k - (uint64_t)a * it.nb);
  }
  U4 o{0, 0, 0, 0};
  if constexpr (!T0)
    o = philox((uint32_t)(k >> 1), it.A, it.B, it.w3 | ((uint32_t)(k >> 33) << 20), g->seed_lo,
               g->seed_hi);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (k < kend) {
      const uint32_t su = it.a0 + a, sv = (tri ? it.a0 : it.b0) + b;
      bool e, nr = false;
      if constexpr (T0) {
        e = pair_thresh<D, MODEL>(g, v, su, sv, nr);
      } else {
        const double U = h == 0 ? u53(o.x, o.y) : u53(o.z, o.w);
        if constexpr (MX) e = mixed_test<D>(g, v, su, sv, U, nre, nr);
        else if constexpr (MODEL == 1)
          {
            const RecPair<D, 1> ab = load_recs<D, 1>(v.rec, su, sv);
            e = hrg_below<D>(g, ab.a, ab.b, U, nr);
          }
        else {
          const double p = pair_prob<D, MODEL>(g, v, su, sv);
          nr = fabs(U - p) < 1e-12;
          e = U < p;
        }
      }
      if (nr) count_stat(st, kStatNear);
      if (e) {
        if (h == 0) p0 = make_uint2(su, sv);
        else p1 = make_uint2(su, sv);
      }
      if (h == 0) e0 = e; else e1 = e;
      ++ntests;
      ++k;
      if (tri) {
        if (++a == b) { a = 0; ++b; }
      } else {
        if (++b == it.nb) { b = 0; ++a; }
      }
    }
  }
}

// one converged step over up to 64 queued Philox blocks
// Lane l takes block bc + l.  The items whose blocks all lie below bc are
// retired, so item qh holds block bc and every later item starts above it.
// Items qh + 1 .. qh + 63 that start inside the window mark their first lane
// (mk, one word per lane); a lane's item is the last mark at or below it.
template <int D, int MODEL, bool T0, bool MX>
__device__ __forceinline__ void step1(const Graph* __restrict__ g, const Verts& v,
                                      const QItem1* __restrict__ q, uint32_t* __restrict__ mk,
                                      Ring1& r, const Stage& sg, Out& out, uint32_t& ntests,
                                      uint32_t& nre) {
  const uint32_t lane = lane_id();
  const uint32_t avail = r.bt - r.bc;
  const uint32_t take = avail < 64 ? avail : 64;
  mk[lane] = 0u;
  if (lane + 1 < r.qt - r.qh) {
    const uint32_t off = q[(r.qh + lane + 1) & (kQCap - 1)].cs - r.bc;  // >= 1
    if (off < take) mk[off] = lane + 1;
  }
  // the other lanes' marks: without the fence the compiler may return this
  // lane's own zero from a register instead of reading the word back
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const uint32_t mv = mk[lane];
  const uint64_t below = __ballot(mv != 0u) & (~0ull >> (63u - lane));
  const uint32_t rel = __shfl(mv, below ? 63u - (uint32_t)__clzll((long long)below) : lane, 64);
  bool e0 = false, e1 = false;
  uint2 p0 = make_uint2(0, 0), p1 = make_uint2(0, 0);
  if (lane < take) {
    const uint32_t gb = r.bc + lane;
    const QItem1 it = q[(r.qh + rel) & (kQCap - 1)];
    const uint64_t tot = it.tri ? (uint64_t)it.na * (it.na - 1) / 2 : (uint64_t)it.na * it.nb;
    const uint64_t kb = (uint64_t)it.kb + (gb - it.cs);
    const uint64_t kend = 2ull * ((uint64_t)it.kb + it.nbk) < tot ? 2ull * ((uint64_t)it.kb + it.nbk) : tot;
    test_block<D, MODEL, T0, MX>(g, v, it, 2ull * kb, kend, e0, e1, p0, p1, ntests, nre, sg.stats);
  }
  emit(e0, e1, p0, p1, sg, out);
  r.bc += take;
  // retire the items whose blocks are all done
  while (r.qh < r.qt) {
    const uint32_t nxt = r.qh + 1 < r.qt ? q[(r.qh + 1) & (kQCap - 1)].cs : r.bt;
    if (nxt > r.bc) break;
    ++r.qh;
  }
}

// enqueue one item per lane (enq) with its first-block index from a wave
// prefix sum of the block counts
__device__ __forceinline__ void enqueue1(bool enq, QItem1& it, QItem1* __restrict__ q, Ring1& r) {
  const uint32_t lane = lane_id();
  const uint64_t me = __ballot(enq);
  uint32_t pre = enq ? it.nbk : 0u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(pre, o, 64);
    if ((int)lane >= o) pre += t;
  }
  const uint32_t total = __shfl(pre, 63, 64);
  if (enq) {
    it.cs = r.bt + pre - it.nbk;
    q[(r.qt + lanes_below(me)) & (kQCap - 1)] = it;
  }
  r.qt += (uint32_t)__popcll(me);
  r.bt += total;
}

// per-wave source batch: 64 sources, their candidate-cell counts and the
// inclusive prefix of the counts (load-balanced expansion over the lanes)
struct SrcSlot {
  uint32_t sidx;  // source index
  uint32_t A;     // its cell
  uint32_t info;  // level | kind << 8 | layer << 16 (kind: table row, 255 = all offsets)
  uint32_t incl;  // inclusive prefix of the counts
};

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

// type-I pass: neighbouring cell pairs at level CL(i,j) (loop swap, Sec. 3.3).
// Waves take batches of 64 sources (layer i, level l, cell X); the
// (source, neighbour) pairs are spread over the lanes.  At levels >= 2 the
// neighbours are X itself (layers j >= i) and the offsets in {-1,0,1}^d whose
// first nonzero component is positive (index o > (3^d - 1) / 2 in balanced
// ternary, dimension 0 most significant); the other orientation of each pair
// is listed at the other cell.  At levels <= 1 all 3^d offsets are decoded,
// deduplicated, with Y >= X.  The layer mask of Y restricted to
// {j : CL(i,j) == l} lists the nonempty items; they are oriented with the
// smaller cell as their A side and queued for the flat test steps.
struct IEnt1 {
  uint32_t sidx;  // source of the X side
  uint32_t Y;     // the other cell
  uint32_t ridx;  // record (first, count) of V_j^Y
  uint32_t j;     // layer of the Y side
};

template <int D, int MODEL, bool T0, bool MX>
__device__ __forceinline__ void take_items1(const Graph* __restrict__ g, const Verts& v,
                                            const uint2* __restrict__ crec,
                                            const Src* __restrict__ src, IEnt1* ib, uint32_t& in,
                                            QItem1* __restrict__ q, uint32_t* __restrict__ mk,
                                            Ring1& r, uint32_t chunk,
                                            uint32_t& dseq, const DeferOut& dfo, const Stage& sg,
                                            Out& out, uint32_t& ntests, uint32_t& nre) {
  const uint32_t lane = lane_id();
  const uint32_t take = in < 64 ? in : 64;
  const bool have = lane < take;
  IEnt1 e{0, 0, 0, 0};
  if (have) e = ib[lane];
  const uint32_t rest = in - take;
  IEnt1 tmp{0, 0, 0, 0};
  if (lane < rest) tmp = ib[take + lane];
  if (lane < rest) ib[lane] = tmp;
  in = rest;
  // room for 64 more items; consume blocks when there are several steps of them
  while (r.qt - r.qh > (uint32_t)(kQCap - 64) || r.bt - r.bc >= 256)
    step1<D, MODEL, T0, MX>(g, v, q, mk, r, sg, out, ntests, nre);
  bool enq = false, big = false;
  QItem1 it{};
  ItemRec rec{};
  if (have) {
    const Src sr = src[e.sidx];
    const uint2 cr = crec[e.ridx];
    asm volatile("" ::"v"(sr.s), "v"(sr.A), "v"(sr.na), "v"(sr.meta), "v"(cr.x), "v"(cr.y));
    const uint32_t lvl = sr.meta & 255u, li = sr.meta >> 8, lj = e.j;
    const uint32_t b0 = cr.x, nb = cr.y;
    // orientation: the smaller cell is the A side
    const bool fwd = e.Y >= sr.A;
    const uint32_t cA = fwd ? sr.A : e.Y, cB = fwd ? e.Y : sr.A;
    const uint32_t ci = fwd ? li : lj, cj = fwd ? lj : li;
    const uint32_t ca0 = fwd ? sr.s : b0, cna = fwd ? sr.na : nb;
    const uint32_t cb0 = fwd ? b0 : sr.s, cnb = fwd ? nb : sr.na;
    const bool tri = cA == cB && ci == cj;
    const uint64_t tot = tri ? (uint64_t)cna * (cna - 1) / 2 : (uint64_t)cna * cnb;
    if (nb && tot) {
      if (tot > dfo.big) {
        rec = ItemRec{ca0, cna, cb0, cnb, cA, cB,
                      lvl | (ci << 8) | (cj << 16) | (tri ? 1u << 31 : 0u), 0u};
        big = true;
      } else {
        it = QItem1{cA, cB, ctr_word3(lvl, ci, cj, kKindType1, 0), ca0, cb0, cnb, cna,
                    tri ? 1u : 0u, 0u, 0u, (uint32_t)((tot + 1) / 2), 0u};
        enq = true;
      }
    }
  }
  if (__any(big)) defer_item(big, rec, chunk, dseq, dfo);
  enqueue1(enq, it, q, r);
}

template <int D, int MODEL, bool T0, bool MX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_type1(const Graph* __restrict__ g, Verts v,
                                               const CellL* __restrict__ cl,
                                               const uint2* __restrict__ crec,
                                               const Src* __restrict__ src, Sched sc, Stage sg,
                                               DeferOut dfo) {
  __shared__ IEnt1 ibs[4][kICap];
  __shared__ QItem1 qs[4][kQCap];
  __shared__ uint32_t mks[4][kWave];
  __shared__ uint2 ebs[4][kEdgeBuf];
  __shared__ SrcSlot sss[4][kWave];
  constexpr uint32_t NOFF = Offs<D>::n1;
  constexpr uint32_t HALF = (Offs<D>::n1 - 1) / 2;
  const uint32_t wv = threadIdx.x / kWave;
  IEnt1* ib = ibs[wv];
  QItem1* q = qs[wv];
  uint32_t* mk = mks[wv];
  SrcSlot* ss = sss[wv];
  const uint32_t lane = lane_id();
  uint32_t ntests = 0, nre = 0;
  uint64_t nedge = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t sb = (uint64_t)c * sc.chunk;
    const uint64_t se = sb + sc.chunk < sc.nunits ? sb + sc.chunk : sc.nunits;
    uint32_t in = 0, dseq = 0;
    Ring1 r{0, 0, 0, 0};
    Out out{ebs[wv], 0, 0, ((uint64_t)sc.pass << 32) | c, v.id};
    for (uint64_t base = sb; base < se; base += kWave) {
      // one source per lane: its neighbour cells
      const uint64_t si = base + lane;
      uint32_t cnt = 0;
      SrcSlot mine{(uint32_t)si, 0u, 0u, 0u};
      if (si < se) {
        const Src sr = src[si];
        const uint32_t lvl = sr.meta & 255u, li = sr.meta >> 8;
        mine.A = sr.A;
        // info: level | table flag << 8 | layer << 16
        if (g->jI[li][lvl]) {
          const bool tab = lvl >= 2;
          cnt = tab ? HALF + 1 : NOFF;
          mine.info = lvl | (tab ? 0u : 255u << 8) | (li << 16);
        }
      }
      mine.incl = wave_incl_scan(cnt);
      ss[lane] = mine;
      const uint32_t total = __shfl(mine.incl, 63, 64);
      for (uint32_t k0 = 0; k0 < total; k0 += kWave) {
        const uint32_t k = k0 + lane;
        uint64_t m = 0, fm = 0;
        uint32_t Y = 0, sidx = 0, base = 0;
        if (k < total) {
          uint32_t lo = 0, hi = 64;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ss[mid].incl <= k) lo = mid + 1;
            else hi = mid;
          }
          const SrcSlot sl = ss[lo];
          const uint32_t t = k - (lo ? ss[lo - 1].incl : 0u);  // offset within the source
          const uint32_t lvl = sl.info & 255u, li = sl.info >> 16;
          sidx = sl.sidx;
          // loaded while the cell is computed (left alone, the compiler loads
          // them after it, one more round trip before the cell's layer set)
          const uint64_t mo = g->moff[lvl], jm = g->jI[li][lvl];
          bool ok;
          if (((sl.info >> 8) & 255u) == 0u) {
            // balanced-ternary offset o = HALF + t: t = 0 is X itself
            uint32_t qa[D], b[D];
            morton_decode<D>(sl.A, qa);
            const uint32_t cm = (uint32_t)((1ull << lvl) - 1);
            uint32_t o = HALF + t;
#pragma unroll
            for (int kk = D - 1; kk >= 0; --kk) {
              b[kk] = (qa[kk] + (o % 3u) - 1u) & cm;
              o /= 3u;
            }
            Y = morton_encode<D>(b);
            ok = true;
          } else {
            ok = neighbour_cell<D>(sl.A, (int)lvl, t, &Y) && Y >= sl.A;
          }
          asm volatile("" ::"v"(mo), "v"(jm));
          if (ok) {
            const CellL ce = cl[mo + Y];
            fm = ce.mask;
            base = ce.base;
            m = fm & jm;
            if (Y == sl.A) m &= ~((1ull << li) - 1ull);  // j >= i when X = Y
          }
        }
        // expand the items of the lane's cell into the list; take 64 when full
        while (__any(m != 0)) {
          const bool has = m != 0;
          uint32_t j = 0;
          if (has) {
            j = (uint32_t)__ffsll((long long)m) - 1;
            m &= m - 1;
          }
          const uint64_t mb = __ballot(has);
          if (has)
            ib[in + lanes_below(mb)] =
                IEnt1{sidx, Y, base + (uint32_t)__popcll(fm & ((1ull << j) - 1ull)), j};
          in += (uint32_t)__popcll(mb);
          if (in >= 64)
            take_items1<D, MODEL, T0, MX>(g, v, crec, src, ib, in, q, mk, r, c, dseq, dfo, sg, out, ntests,
                                          nre);
        }
      }
    }
    while (in)
      take_items1<D, MODEL, T0, MX>(g, v, crec, src, ib, in, q, mk, r, c, dseq, dfo, sg, out, ntests, nre);
    while (r.bc < r.bt) step1<D, MODEL, T0, MX>(g, v, q, mk, r, sg, out, ntests, nre);
    end_chunk(sg, out, sc, c, dseq);
    nedge += out.off;
  }
  // per-lane counts are 32-bit (a lane's share of one launch); the wave's sums 64-bit
  const uint64_t stests = wave_sum((uint64_t)ntests), sre = wave_sum((uint64_t)nre);
  if (lane == 0) {
    if (nedge) atomicAdd(&sg.stats[8 + sc.pass], (unsigned long long)nedge);  // edges of the pass
    atomicAdd(&sg.stats[sc.pass], (unsigned long long)stests);  // tests of pass 0 / 1
    if (sre) atomicAdd(&sg.stats[6], (unsigned long long)sre);
  }
}

// split type-I items: pieces of kTestChunk tests (kTestChunk / 2 blocks)
template <int D, int MODEL, bool T0, bool MX>
__global__ __launch_bounds__(256) void k_big1(const Graph* __restrict__ g, Verts v,
                                              const ItemRec* __restrict__ rec,
                                              const uint64_t* __restrict__ uoff, uint32_t nrec,
                                              Sched sc, Stage sg) {
  __shared__ QItem1 qs[4][kQCap];
  __shared__ uint32_t mks[4][kWave];
  __shared__ uint2 ebs[4][kEdgeBuf];
  const uint32_t wv = threadIdx.x / kWave;
  QItem1* q = qs[wv];
  uint32_t* mk = mks[wv];
  const uint32_t lane = lane_id();
  uint32_t ntests = 0, nre = 0;
  uint64_t nedge = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    Ring1 r{0, 0, 0, 0};
    Out out{ebs[wv], 0, 0, ((uint64_t)sc.pass << 32) | c, v.id};
    for (uint64_t u0 = ub; u0 < ue; u0 += kWave) {
      while (r.qt - r.qh > (uint32_t)(kQCap - 64) || r.bt - r.bc >= 256)
        step1<D, MODEL, T0, MX>(g, v, q, mk, r, sg, out, ntests, nre);
      const uint64_t u = u0 + lane;
      bool enq = false;
      QItem1 it{};
      if (u < ue) {
        uint32_t lo = 0, hi = nrec;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (uoff[mid] <= u) lo = mid; else hi = mid;
        }
        const ItemRec rr = rec[lo];
        const bool tri = (rr.meta >> 31) != 0;
        const uint64_t tot = tri ? (uint64_t)rr.na * (rr.na - 1) / 2 : (uint64_t)rr.na * rr.nb;
        const uint64_t nbt = (tot + 1) / 2;  // blocks of the item
        const uint64_t kb = (u - uoff[lo]) * (kTestChunk / 2);
        const uint64_t nbk = kb + kTestChunk / 2 < nbt ? kTestChunk / 2 : nbt - kb;
        it = QItem1{rr.A, rr.B,
                    ctr_word3(rr.meta & 255u, (rr.meta >> 8) & 255u, (rr.meta >> 16) & 255u, kKindType1, 0),
                    rr.a0, rr.b0, rr.nb, rr.na, tri ? 1u : 0u, 0u, (uint32_t)kb, (uint32_t)nbk, 0u};
        enq = true;
      }
      enqueue1(enq, it, q, r);
    }
    while (r.bc < r.bt) step1<D, MODEL, T0, MX>(g, v, q, mk, r, sg, out, ntests, nre);
    end_chunk(sg, out, sc, c, 0);
    nedge += out.off;
  }
  // per-lane counts are 32-bit (a lane's share of one launch); the wave's sums 64-bit
  const uint64_t stests = wave_sum((uint64_t)ntests), sre = wave_sum((uint64_t)nre);
  if (lane == 0) {
    if (nedge) atomicAdd(&sg.stats[8 + sc.pass], (unsigned long long)nedge);  // edges of the pass
    atomicAdd(&sg.stats[sc.pass], (unsigned long long)stests);  // tests of pass 0 / 1
    if (sre) atomicAdd(&sg.stats[6], (unsigned long long)sre);
  }
}

// ---------------------------------------------------------------------------
// type-II draws.  Candidates of V_i^A x V_j^B are drawn by geometric jumps
// under pbar and accepted with p_uv / pbar (Sec. 3.2).  The candidate range is
// cut into segments of G = 2^e (e = 5 - ilogb(pbar), raised to keep at most
// 2^12 segments); draw t of segment s uses counter (t, A, B, l|i|j|1|s).
// ---------------------------------------------------------------------------
struct Ring2 {
  uint32_t qh, qt;  // queued items
  uint32_t ch, ct;  // queued candidates
};

// one geometric draw without the candidate test: X ~ Geom_0(pbar) candidates
// are skipped (X = floor(ln S / ln(1 - pbar))); returns true with the
// candidate's sorted indices when it lies in the range.  Mixed precision:
// log2 S in FP32 (log2_unit_f32), times 1 / log2(1 - pbar); X and the end
// test are taken from it only when both ends of its kSkipRel relative interval
// agree, otherwise from the FP64 quotient.
template <bool MX>
__device__ __forceinline__ bool geo_draw(uint32_t k0s, uint32_t k1s, QItem2& it, const PB& pe,
                                         bool& done, Cand& cd, uint32_t& nre,
                                         unsigned long long* st) {
  const U4 o = philox(it.t, it.A, it.B, it.w3, k0s, k1s);
  ++it.t;
  const uint64_t vv = (((uint64_t)o.y << 32) | o.x) >> 11;
  const double S = (double)(vv + 1) * 0x1p-53;
  const uint64_t rem = it.N - it.k;
  uint64_t skip = 0;
  bool end = false, decided = false;
  if (pe.pbar >= 1.0) {
    decided = true;  // every candidate is drawn
  } else if (MX) {
    const double q32 = (double)(log2_unit_f32(vv) * pe.qs);
    const double qe = kSkipRel * q32;
    const double qlo = q32 - qe > 0.0 ? q32 - qe : 0.0, qhi = q32 + qe;
    if (qlo >= (double)rem) {
      end = true;
      decided = true;
    } else if (qhi < (double)rem && floor(qlo) == floor(qhi)) {
      skip = (uint64_t)qhi;
      decided = true;
    }
  }
  if (!decided) {
    if (MX) ++nre;
    // ln S * (1 / ln(1 - pbar)); S = 1 skips nothing (also where the
    // reciprocal overflows to -inf)
    const double ls = log_pos(S);
    const double q = ls == 0.0 ? 0.0 : ls * pe.ilg;
    // a quotient within 1e-12 (relative) of an integer >= 1 that can decide
    // a candidate or the end (the FP32 filter never decides those)
    if (pe.pbar < 1.0 && q >= 0.5 && q < (double)rem + 1.0) {
      const double fl = rint(q);
      if (fabs(q - fl) < 1e-12 * q) count_stat(st, kStatTie);
    }
    if (q >= (double)rem) end = true;
    else skip = (uint64_t)q;
  }
  if (end) {
    done = true;
    return false;
  }
  it.k += skip;
  uint32_t aa, bb;
  if (it.k < 0xFFFFFFFFull) {
    aa = (uint32_t)it.k / it.nb;
    bb = (uint32_t)it.k - aa * it.nb;
  } else {
    aa = (uint32_t)(it.k / it.nb);
    bb = (uint32_t)(it.k - (uint64_t)aa * it.nb);
  }
  cd.su = it.a0 + aa;
  cd.sv = it.b0 + bb;
  cd.apb = u53(o.z, o.w) * pe.pbar;
  ++it.k;
  done = it.k >= it.N;
  return true;
}

// Whether a type-II candidate's coin lies within 1e-12 of its acceptance
// probability, |Acc - p_uv / pbar| < 1e-12, i.e. |apb - p_uv| < 1e-12 pbar.
// The sampling kernels list the candidates with |apb - p_uv| < 1e-12 (rare);
// k_near2 applies this test to them afterwards.  pbar is that of the item:
// its level is the first at which the cells of the two vertices are not
// neighbours (their parents are), with gap max_k(torus difference - 1) there.
template <int D, int MODEL>
__device__ __forceinline__ bool t2_near(const Graph* __restrict__ g, const Verts& v,
                                     const Pbar* __restrict__ pbt, int nlev, uint32_t su,
                                     uint32_t sv, double apb) {
  uint32_t qa[D], qb[D];
  morton_decode<D>(v.mort[su], qa);
  morton_decode<D>(v.mort[sv], qb);
  int lvl = -1, gap = 0;
  for (int l = 1; l < nlev && lvl < 0; ++l) {
    const int sh = g->Dmax - l;
    const uint64_t side = 1ull << l;
    int dm = 0;
    for (int k = 0; k < D; ++k) {
      const uint64_t a = qa[k] >> sh, b = qb[k] >> sh;
      const uint64_t df = a > b ? a - b : b - a;
      const uint64_t dt = df < side - df ? df : side - df;
      dm = (int)dt > dm ? (int)dt : dm;
    }
    if (dm > 1) {
      lvl = l;
      gap = dm - 1;
    }
  }
  if (lvl < 0) return false;
  const uint32_t pidx = pbar_index(v.layer[su], v.layer[sv], (uint32_t)lvl, (uint32_t)gap, (uint32_t)g->L,
                                   (uint32_t)nlev);
  const double pbar = pbt[pidx].pbar;
  return fabs(apb - pair_prob<D, MODEL>(g, v, su, sv)) < 1e-12 * pbar;
}

// evaluate up to 64 queued candidates (accept iff Acc * pbar < p_uv)
template <int D, int MODEL, bool MX>
__device__ __forceinline__ void eval_cands(const Graph* __restrict__ g, const Verts& v,
                                           const Pbar* __restrict__ pbt, int nlev,
                                           const Cand* __restrict__ cq, Ring2& r, const Stage& sg,
                                           Out& out, uint32_t& nre) {
  const uint32_t lane = lane_id();
  const uint32_t avail = r.ct - r.ch;
  const uint32_t take = avail < 64 ? avail : 64;
  bool e0 = false;
  uint2 p0 = make_uint2(0, 0);
  if (lane < take) {
    const Cand cd = cq[(r.ch + lane) & (kCCap - 1)];
    bool nr = false;
    if constexpr (MX) e0 = mixed_cand<D>(g, v, cd.su, cd.sv, cd.apb, nre, sg);
    else if constexpr (MODEL == 1)
    {
      const RecPair<D, 1> ab = load_recs<D, 1>(v.rec, cd.su, cd.sv);
      e0 = hrg_below<D>(g, ab.a, ab.b, cd.apb, nr);
    }
    else {
      const double p = pair_prob<D, MODEL>(g, v, cd.su, cd.sv);
      nr = fabs(cd.apb - p) < 1e-12;
      e0 = cd.apb < p;
    }
    // |apb - p_uv| < 1e-12 (rare): the band 1e-12 pbar is checked after the passes
    if (nr) list_near2(sg.nbuf, sg.ncnt, sg.ncap, cd.su, cd.sv, cd.apb);
    if (e0) p0 = make_uint2(cd.su, cd.sv);
  }
  emit(e0, false, p0, p0, sg, out);
  r.ch += take;
}

// draw steps: lanes own items (dequeued from the ring), one draw per step;
// runs while at least `need` items are queued or held (to the end if 0)
template <int D, int MODEL, bool MX>
__device__ __forceinline__ void draws2(const Graph* __restrict__ g, const Verts& v,
                                       const Pbar* __restrict__ pbt, int nlev,
                                       const QItem2* __restrict__ q, Cand* __restrict__ cq,
                                       Ring2& r, bool& act, QItem2& it, PB& pe, uint32_t need,
                                       const Stage& sg, Out& out, uint32_t& ndraws,
                                       uint32_t& ncand, uint32_t& nre) {
  const uint32_t k0s = g->seed_lo, k1s = g->seed_hi;
  for (;;) {
    const uint64_t mi = __ballot(!act);
    const uint32_t avail = r.qt - r.qh;
    const uint32_t held = 64u - (uint32_t)__popcll(mi);
    if (need && held + avail < need) break;
    if (!act) {
      const uint32_t rk = lanes_below(mi);
      if (rk < avail) {
        it = q[(r.qh + rk) & (kQCap - 1)];
        pe = load_pb(pbt, it.pidx);
        act = true;
      }
    }
    const uint32_t got = (uint32_t)__popcll(mi);
    r.qh += got < avail ? got : avail;
    if (!__any(act)) break;
    bool hc = false;
    Cand cd{0, 0, 0.0};
    if (act) {
      bool done = false;
      hc = geo_draw<MX>(k0s, k1s, it, pe, done, cd, nre, sg.stats);
      ++ndraws;
      if (done) act = false;
    }
    const uint64_t mc = __ballot(hc);
    if (hc) cq[(r.ct + lanes_below(mc)) & (kCCap - 1)] = cd;
    r.ct += (uint32_t)__popcll(mc);
    ncand += hc ? 1 : 0;
    if (r.ct - r.ch >= 64) eval_cands<D, MODEL, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
  }
}

__device__ __forceinline__ void enqueue2(bool enq, const QItem2& it, QItem2* __restrict__ q,
                                         Ring2& r) {
  const uint64_t me = __ballot(enq);
  if (enq) q[(r.qt + lanes_below(me)) & (kQCap - 1)] = it;
  r.qt += (uint32_t)__popcll(me);
}

// type-II pass.  A wave walks whole sources (layer i, level l, cell X) of
// its chunk.  Lanes take the cells Y distant from X whose parents neighbour
// X's parent: at levels >= 3 from the table of offsets with a positive first
// nonzero component (each unordered pair once), at levels <= 2 from all
// 6^d children, deduplicated, with Y > X.  The layer mask of Y restricted to
// {j : CL(i,j) >= l} lists the nonempty items; they are expanded into an
// LDS list and taken 64 at a time.  An item is oriented with the smaller cell
// as its A side (App. B.1), makes its first draw at once, and is queued for
// more draws only if its range is not exhausted.
struct IEnt {
  uint32_t sidx;  // source of the X side
  uint32_t Y;     // the other cell
  uint32_t ridx;  // record (first, count) of V_j^Y
  uint32_t jg;    // layer j of the Y side | gap << 8 | layer i of X << 16 | level << 24
};

template <int D, int MODEL, bool MX>
__device__ __forceinline__ void take_items2(const Graph* __restrict__ g, const Verts& v,
                                            const uint2* __restrict__ crec,
                                            const Src* __restrict__ src,
                                            const Pbar* __restrict__ pbt, int nlev, IEnt* ib,
                                            uint32_t& in, QItem2* __restrict__ q,
                                            Cand* __restrict__ cq, Ring2& r, bool& act,
                                            QItem2& cur, PB& cpe, uint32_t chunk, uint32_t& dseq,
                                            const DeferOut& dfo, const Stage& sg, Out& out,
                                            uint32_t& ndraws, uint32_t& ncand, uint32_t& nre) {
  const uint32_t lane = lane_id();
  const uint32_t take = in < 64 ? in : 64;
  const bool have = lane < take;
  IEnt e{0, 0, 0, 0};
  if (have) e = ib[lane];
  const uint32_t rest = in - take;
  IEnt tmp{0, 0, 0, 0};
  if (lane < rest) tmp = ib[take + lane];
  if (lane < rest) ib[lane] = tmp;
  in = rest;

  bool fresh = false, hv = false;
  QItem2 it{};
  PB pe{0.0, 0.0, 0.0f};
  ItemRec rec{};
  if (have) {
    const uint32_t lj = e.jg & 255u, gp = (e.jg >> 8) & 255u, li = (e.jg >> 16) & 255u,
                   lvl = e.jg >> 24;
    // three independent loads; the pbar table is symmetric in the layer pair
    // (it depends on w_i w_j only), so it is indexed before the orientation
    const uint32_t pidx = pbar_index(li, lj, lvl, gp, (uint32_t)g->L, (uint32_t)nlev);
    const Pbar pv = pbt[pidx];
    const Src sr = src[e.sidx];
    const uint2 cr = crec[e.ridx];
    // wait for all three here, at once: left alone, the compiler sinks the
    // source and the second half of the pbar entry into the branch below,
    // which costs two more round trips to memory per item
    asm volatile("" ::"v"(pv.pbar), "v"(pv.ilg), "v"(pv.e), "v"(pv.qscale), "v"(sr.s), "v"(sr.A),
                 "v"(sr.na), "v"(cr.x), "v"(cr.y));
    const uint32_t b0 = cr.x, nb = cr.y;
    // orientation: the smaller cell is the A side
    const bool fwd = e.Y > sr.A;
    const uint32_t cA = fwd ? sr.A : e.Y, cB = fwd ? e.Y : sr.A;
    const uint32_t ci = fwd ? li : lj, cj = fwd ? lj : li;
    const uint32_t ca0 = fwd ? sr.s : b0, cna = fwd ? sr.na : nb;
    const uint32_t cb0 = fwd ? b0 : sr.s, cnb = fwd ? nb : sr.na;
    if (pv.pbar > 0.0 && nb > 0) {
      const uint64_t N = (uint64_t)cna * cnb;
      if (multi_segment(N, pv.e)) {
        rec = ItemRec{ca0, cna, cb0, cnb, cA, cB, lvl | (ci << 8) | (cj << 16) | (gp << 24),
                      (uint32_t)pv.e};
        hv = true;
      } else {
        it = QItem2{cA, cB, ctr_word3(lvl, ci, cj, kKindType2, 0), ca0, cb0, cnb, 0u, pidx, 0ull, N};
        pe = PB{pv.pbar, pv.ilg, pv.qscale};
        fresh = true;
      }
    }
  }
  if (__any(hv)) defer_item(hv, rec, chunk, dseq, dfo);
  // first draw of every new item
  bool hc = false, cont = false;
  Cand cd{0, 0, 0.0};
  if (fresh) {
    bool done = false;
    hc = geo_draw<MX>(g->seed_lo, g->seed_hi, it, pe, done, cd, nre, sg.stats);
    ++ndraws;
    cont = !done;
  }
  const uint64_t mc = __ballot(hc);
  if (hc) cq[(r.ct + lanes_below(mc)) & (kCCap - 1)] = cd;
  r.ct += (uint32_t)__popcll(mc);
  ncand += hc ? 1 : 0;
  if (r.ct - r.ch >= 64) eval_cands<D, MODEL, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
  if (__any(cont)) {
    if (r.qt - r.qh > (uint32_t)(kQCap - 64))
      draws2<D, MODEL, MX>(g, v, pbt, nlev, q, cq, r, act, cur, cpe, 64, sg, out, ndraws, ncand, nre);
    enqueue2(cont, it, q, r);
  }
}

// append the items of mask m (lane's cell Y, gap) to the list; take 64 when full
template <int D, int MODEL, bool MX>
__device__ __forceinline__ void push_items2(uint64_t m, uint64_t fm, uint32_t base, uint32_t sidx,
                                            uint32_t Y, uint32_t tag,
                                            const Graph* __restrict__ g, const Verts& v,
                                            const uint2* __restrict__ crec,
                                            const Src* __restrict__ src,
                                            const Pbar* __restrict__ pbt, int nlev, IEnt* ib,
                                            uint32_t& in, QItem2* __restrict__ q,
                                            Cand* __restrict__ cq, Ring2& r, bool& act,
                                            QItem2& cur, PB& cpe, uint32_t chunk, uint32_t& dseq,
                                            const DeferOut& dfo, const Stage& sg, Out& out,
                                            uint32_t& ndraws, uint32_t& ncand, uint32_t& nre) {
  while (__any(m != 0)) {
    const bool has = m != 0;
    uint32_t j = 0;
    if (has) {
      j = (uint32_t)__ffsll((long long)m) - 1;
      m &= m - 1;
    }
    const uint64_t mb = __ballot(has);
    if (has)
      ib[in + lanes_below(mb)] =
          IEnt{sidx, Y, base + (uint32_t)__popcll(fm & ((1ull << j) - 1ull)), j | (tag << 8)};
    in += (uint32_t)__popcll(mb);
    if (in >= 64)
      take_items2<D, MODEL, MX>(g, v, crec, src, pbt, nlev, ib, in, q, cq, r, act, cur, cpe, chunk,
                                dseq, dfo, sg, out, ndraws, ncand, nre);
  }
}

template <int D, int MODEL, bool MX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_type2(const Graph* __restrict__ g, Verts v,
                                               const CellL* __restrict__ cl,
                                               const uint2* __restrict__ crec,
                                               const Src* __restrict__ src, Sched sc,
                                               const Pbar* __restrict__ pbt, int nlev,
                                               const uint32_t* __restrict__ dtab, Stage sg,
                                               DeferOut dfo, uint32_t lvl_skip) {
  __shared__ IEnt ibs[4][kICap];
  __shared__ QItem2 qs[4][kQCap];
  __shared__ Cand cqs[4][kCCap];
  __shared__ uint2 ebs[4][kEdgeBuf2];
  __shared__ SrcSlot sss[D < 3 ? 4 : 1][kWave];  // (d >= 3 finds sources without it)
  constexpr uint32_t NOFF = Offs<D>::n2;
  const uint32_t wv = threadIdx.x / kWave;
  IEnt* ib = ibs[wv];
  QItem2* q = qs[wv];
  Cand* cq = cqs[wv];
  SrcSlot* ss = sss[D < 3 ? wv : 0];
  const uint32_t lane = lane_id();
  const uint32_t dstride = dtab[0];
  // d <= 3: the distant-offset table in LDS (at most 3.8 KB)
  constexpr uint32_t TL = D <= 3 ? kDistHead + (1u << D) * Offs<D>::nd : 1u;
  __shared__ uint32_t ltab[TL];
  if constexpr (D <= 3) {
    const uint32_t tn = kDistHead + (1u << D) * dstride;
    for (uint32_t i = threadIdx.x; i < (tn < TL ? tn : TL); i += blockDim.x) ltab[i] = dtab[i];
    __syncthreads();
  }
  const uint32_t* __restrict__ tab = D <= 3 ? ltab : dtab;
  uint32_t ndraws = 0, ncand = 0, nre = 0;
  uint64_t nedge = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t sb = (uint64_t)c * sc.chunk;
    const uint64_t se = sb + sc.chunk < sc.nunits ? sb + sc.chunk : sc.nunits;
    uint32_t in = 0, dseq = 0;
    Ring2 r{0, 0, 0, 0};
    bool act = false;
    QItem2 cur{};
    PB cpe{0.0, 0.0, 0.0f};
    Out out{ebs[wv], 0, 0, ((uint64_t)sc.pass << 32) | c, v.id};
    for (uint64_t base = sb; base < se; base += kWave) {
      // one source per lane: its candidate cells
      const uint64_t si = base + lane;
      uint32_t cnt = 0;
      SrcSlot mine{(uint32_t)si, 0u, 0u, 0u};
      if (si < se) {
        const Src sr = src[si];
        const uint32_t lvl = sr.meta & 255u, li = sr.meta >> 8;
        mine.A = sr.A;
        // (levels >= lvl_skip: the batched sequences of k_type2s)
        if (lvl < lvl_skip && g->jII[li][lvl]) {
          if (lvl >= 3) {
            uint32_t qa[D];
            morton_decode<D>(sr.A, qa);
            uint32_t par = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) par |= (qa[k] & 1u) << k;
            cnt = tab[1 + par];
            mine.info = lvl | (par << 8) | (li << 16);
          } else {
            cnt = NOFF;
            mine.info = lvl | (255u << 8) | (li << 16);
          }
        }
      }
      mine.incl = wave_incl_scan(cnt);
      if constexpr (D < 3) ss[lane] = mine;
      const uint32_t total = __shfl(mine.incl, 63, 64);
      const uint32_t mstart = mine.incl - cnt;
      // (source, offset) pairs spread over the lanes
      for (uint32_t k0 = 0; k0 < total; k0 += kWave) {
        const uint32_t k = k0 + lane;
        // d >= 3: a source with work has at least 64 candidate cells (the
        // table rows hold 73 to 116 offsets at d = 3, and levels below 3 take
        // all 6^d; the host checks this), so the window of 64 pairs spans at
        // most two sources: s0, which holds pair k0, and the next one with
        // work, s1.  Their fields come from their lanes, without a search.
        SrcSlot w0{}, w1{};
        uint32_t i0 = 0, st0 = 0, st1 = 0;
        if constexpr (D >= 3) {
          auto rl = [](uint32_t x, uint32_t l) {
            return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
          };
          const uint32_t s0 = (uint32_t)__popcll(__ballot(mine.incl <= k0));
          i0 = rl(mine.incl, s0);
          const uint32_t s1 = (uint32_t)__popcll(__ballot(mine.incl <= i0));
          w0 = SrcSlot{(uint32_t)base + s0, rl(mine.A, s0), rl(mine.info, s0), i0};
          st0 = rl(mstart, s0);
          if (s1 < 64) {
            w1 = SrcSlot{(uint32_t)base + s1, rl(mine.A, s1), rl(mine.info, s1), rl(mine.incl, s1)};
            st1 = i0;
          }
        }
        uint64_t m = 0, fm = 0;
        uint32_t Y = 0, gap = 0, sidx = 0, base = 0, tli = 0, tlvl = 0;
        bool in_window = k < total;
        SrcSlot sl{};
        uint32_t t = 0;
        if constexpr (D >= 3) {
          const bool second = k >= i0;
          sl = second ? w1 : w0;
          t = k - (second ? st1 : st0);
          in_window = in_window && k < sl.incl;
        }
        if (in_window) {
          if constexpr (D < 3) {
            // slot = number of inclusive prefixes <= k
            uint32_t lo = 0, hi = 64;
            while (lo < hi) {
              const uint32_t mid = (lo + hi) >> 1;
              if (ss[mid].incl <= k) lo = mid + 1;
              else hi = mid;
            }
            sl = ss[lo];
            t = k - (lo ? ss[lo - 1].incl : 0u);  // offset within the source
          }
          const uint32_t lvl = sl.info & 255u, par = (sl.info >> 8) & 255u, li = sl.info >> 16;
          sidx = sl.sidx;
          tli = li;
          tlvl = lvl;
          // the level's cell offset and layer mask load beside the offset
          // table entry, not after it (one round trip to memory instead of two)
          const uint64_t mo = g->moff[lvl], jm = g->jII[li][lvl];
          bool ok;
          if (par != 255u) {
            const uint32_t en = tab[kDistHead + par * dstride + t];
            asm volatile("" ::"v"(en), "v"(mo), "v"(jm));
            if constexpr (D == 3) {
              // add the dilated displacement per dimension in Morton space:
              // the other dimensions' bits set to 1 carry through, and the
              // code is taken mod 2^(3 lvl) (the torus wrap)
              uint32_t y = 0;
#pragma unroll
              for (int kk = 0; kk < 3; ++kk) {
                const uint32_t M = 0x24924924u >> kk;
                y |= ((sl.A | ~M) + (en & M)) & M;
              }
              Y = y & (uint32_t)((1ull << (3 * lvl)) - 1);
              gap = en >> 30;
            } else {
              uint32_t qa[D], b[D];
              morton_decode<D>(sl.A, qa);
              const uint32_t cm = (uint32_t)((1ull << lvl) - 1);
#pragma unroll
              for (int kk = 0; kk < D; ++kk) b[kk] = (qa[kk] + ((en >> (3 * kk)) & 7u) - 3u) & cm;
              Y = morton_encode<D>(b);
              gap = en >> 28;
            }
            ok = true;
          } else {
            int gp = 0;
            ok = distant_cell<D>(sl.A, (int)lvl, t, &Y, &gp) && Y > sl.A;
            gap = (uint32_t)gp;
          }
          if (ok) {
            const CellL ce = cl[mo + Y];
            fm = ce.mask;
            base = ce.base;
            m = fm & jm;
          }
        }
        push_items2<D, MODEL, MX>(m, fm, base, sidx, Y, gap | (tli << 8) | (tlvl << 16), g, v, crec,
                                  src, pbt, nlev, ib, in, q, cq, r, act, cur, cpe, c, dseq, dfo, sg,
                                  out, ndraws, ncand, nre);
      }
    }
    while (in)
      take_items2<D, MODEL, MX>(g, v, crec, src, pbt, nlev, ib, in, q, cq, r, act, cur, cpe, c, dseq,
                                dfo, sg, out, ndraws, ncand, nre);
    draws2<D, MODEL, MX>(g, v, pbt, nlev, q, cq, r, act, cur, cpe, 0, sg, out, ndraws, ncand, nre);
    while (r.ct != r.ch) eval_cands<D, MODEL, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
    end_chunk(sg, out, sc, c, dseq);
    nedge += out.off;
  }
  // per-lane counts are 32-bit (a lane's share of one launch); the wave's sums 64-bit
  const uint64_t sdraws = wave_sum((uint64_t)ndraws), scand = wave_sum((uint64_t)ncand),
                 sre = wave_sum((uint64_t)nre);
  if (lane == 0) {
    if (nedge) atomicAdd(&sg.stats[8 + sc.pass], (unsigned long long)nedge);  // edges of the pass
    const int sl = sc.pass == 3 ? 1 : 0;  // draws / candidates of pass 2 / 3
    atomicAdd(&sg.stats[2 + sl], (unsigned long long)sdraws);
    atomicAdd(&sg.stats[4 + sl], (unsigned long long)scand);
    if (sre) atomicAdd(&sg.stats[6], (unsigned long long)sre);
  }
}

// segmented type-II items: one segment per unit
template <int D, int MODEL, bool MX>
__global__ __launch_bounds__(256) void k_heavy2(const Graph* __restrict__ g, Verts v,
                                                const ItemRec* __restrict__ rec,
                                                const uint64_t* __restrict__ uoff, uint32_t nrec,
                                                Sched sc, const Pbar* __restrict__ pbt, int nlev,
                                                Stage sg) {
  __shared__ QItem2 qs[4][kQCap];
  __shared__ Cand cqs[4][kCCap];
  __shared__ uint2 ebs[4][kEdgeBuf2];
  const uint32_t wv = threadIdx.x / kWave;
  QItem2* q = qs[wv];
  Cand* cq = cqs[wv];
  const uint32_t lane = lane_id();
  const int L = g->L;
  uint32_t ndraws = 0, ncand = 0, nre = 0;
  uint64_t nedge = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint64_t ub = (uint64_t)c * sc.chunk;
    const uint64_t ue = ub + sc.chunk < sc.nunits ? ub + sc.chunk : sc.nunits;
    Ring2 r{0, 0, 0, 0};
    bool act = false;
    QItem2 cur{};
    PB cpe{0.0, 0.0, 0.0f};
    Out out{ebs[wv], 0, 0, ((uint64_t)sc.pass << 32) | c, v.id};
    for (uint64_t u0 = ub; u0 < ue; u0 += kWave) {
      if (r.qt - r.qh > (uint32_t)(kQCap - 64))
        draws2<D, MODEL, MX>(g, v, pbt, nlev, q, cq, r, act, cur, cpe, 64, sg, out, ndraws, ncand, nre);
      const uint64_t u = u0 + lane;
      bool enq = false;
      QItem2 it{};
      if (u < ue) {
        uint32_t lo = 0, hi = nrec;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (uoff[mid] <= u) lo = mid; else hi = mid;
        }
        const ItemRec rr = rec[lo];
        const uint64_t s = u - uoff[lo];
        const uint32_t lvl = rr.meta & 255u, li = (rr.meta >> 8) & 255u, lj = (rr.meta >> 16) & 255u,
                       gp = (rr.meta >> 24) & 127u;
        const uint32_t pidx = pbar_index(li, lj, lvl, gp, (uint32_t)L, (uint32_t)nlev);
        const uint64_t N = (uint64_t)rr.na * rr.nb;
        uint64_t G, ns;
        segment_size(N, (int)rr.e, &G, &ns);
        const uint64_t k0 = s * G, kend = (s + 1) * G < N ? (s + 1) * G : N;
        it = QItem2{rr.A, rr.B, ctr_word3(lvl, li, lj, kKindType2, (uint32_t)s), rr.a0, rr.b0, rr.nb,
                    0u, pidx, k0, kend};
        enq = true;
      }
      enqueue2(enq, it, q, r);
    }
    draws2<D, MODEL, MX>(g, v, pbt, nlev, q, cq, r, act, cur, cpe, 0, sg, out, ndraws, ncand, nre);
    while (r.ct != r.ch) eval_cands<D, MODEL, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
    end_chunk(sg, out, sc, c, 0);
    nedge += out.off;
  }
  // per-lane counts are 32-bit (a lane's share of one launch); the wave's sums 64-bit
  const uint64_t sdraws = wave_sum((uint64_t)ndraws), scand = wave_sum((uint64_t)ncand),
                 sre = wave_sum((uint64_t)nre);
  if (lane == 0) {
    if (nedge) atomicAdd(&sg.stats[8 + sc.pass], (unsigned long long)nedge);  // edges of the pass
    const int sl = sc.pass == 3 ? 1 : 0;  // draws / candidates of pass 2 / 3
    atomicAdd(&sg.stats[2 + sl], (unsigned long long)sdraws);
    atomicAdd(&sg.stats[4 + sl], (unsigned long long)scand);
    if (sre) atomicAdd(&sg.stats[6], (unsigned long long)sre);
  }
}


// ---------------------------------------------------------------------------
// batched type-II jump sequences (GIRG, d = 2 or 3, levels >= 3).  The
// candidates of the distant cell pairs of one source that share pbar are
// independent Bernoulli(pbar) trials, so one jump sequence runs over their
// concatenation (Sec. 3.2 applied across cell pairs): for source (layer i,
// level l, cell X), layer j with CL(i,j) >= l and gap g, the distant cells Y
// of X's parity table with gap g, in table order, whose V_j^Y is nonempty
// and whose candidates fit one segment; candidate x |V_j^Y| + y of a pair,
// the pairs one after another.  Draw t of the sequence uses the counter
// (t, X, g, l | i << 6 | j << 12 | 3 << 18).  Pairs of more than one segment
// are deferred to the segmented pass, as in k_type2.
//
// A wave keeps rings of staged sources and of their kept cells in LDS.  A
// source is staged by the whole wave (lanes over its table offsets, one cell
// record load each; the cells with some layer j of the source are kept in
// table order, gap 1 first) whenever fewer than 64 sequences wait and the
// rings have room.  Each lane runs one sequence at a time and takes the next
// waiting one as soon as its own ends, so the lanes stay busy across
// sources.  A round walks every lane to the pair holding its next candidate
// (cell records from the ring, the (first, count) record of V_j^Y from
// global memory), then takes every lane's candidate and next draw at once;
// candidates go to the candidate ring, evaluated 64 at a time.  A source's
// cells are released when its last sequence ends and all older sources are
// released.  Layers j < 32: a kept cell stores the low 32 bits of its layer
// mask, which give the rank of V_j^Y among the cell's records.  Pairs of more
// than 2^(e - 4) candidates (e = 5 - ilogb(pbar)) are not part of a sequence:
// the walk queues them as items with their own streams, drawn as in k_type2
// (draws2) whenever 64 are queued, so that no lane holds a long sequence.
// ---------------------------------------------------------------------------
constexpr int kSeqWaves = 2;    // waves per workgroup
constexpr int kSeqEnt = 768;    // kept cells per wave (ring)
constexpr int kSeqRing = 32;    // staged sources per wave (ring, power of two)
constexpr int kSeqOff = 120;    // >= the largest parity table (116 offsets at d = 3)

struct SSrc {
  uint32_t s0, na, X, info;  // info = level | layer << 8 | parity << 16
  uint32_t e0;               // ring position of its first kept cell
  uint32_t n1, n;            // kept cells of gap 1; kept cells
  uint32_t cs;               // sequences of the chunk's sources up to this one
  uint32_t U1, U2;           // layers among its kept cells of gap 1 / gap 2
  uint32_t left;             // its sequences not yet ended
  uint32_t pad;
};

__device__ __forceinline__ uint32_t wave_or32(uint32_t x) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

// one draw of a sequence: the skip floor(ln S / ln(1 - pbar)) (clamped at
// 2^62) and the acceptance uniform Acc; tie: the quotient lies within 1e-12
// (relative) of an integer >= 1 (decided by the walk: it counts when the skip
// lands in the sequence or ends exactly at its end).  Mixed precision: the
// FP32 quotient when both ends of its kSkipRel interval have the same floor.
template <bool MX>
__device__ __forceinline__ uint64_t seq_draw(uint32_t k0s, uint32_t k1s, uint32_t X, uint32_t g,
                                             uint32_t w3, uint32_t t, const PB& pe, double& acc,
                                             bool& tie, uint32_t& nre) {
  const U4 o = philox(t, X, g, w3, k0s, k1s);
  const uint64_t vv = (((uint64_t)o.y << 32) | o.x) >> 11;
  acc = u53(o.z, o.w);
  tie = false;
  if (pe.pbar >= 1.0) return 0;  // every candidate is drawn
  if (MX) {
    const double q32 = (double)(log2_unit_f32(vv) * pe.qs);
    const double qe = kSkipRel * q32;
    const double qlo = q32 - qe > 0.0 ? q32 - qe : 0.0, qhi = q32 + qe;
    if (qhi < 0x1p62 && floor(qlo) == floor(qhi)) return (uint64_t)qhi;
    ++nre;
  }
  const double S = (double)(vv + 1) * 0x1p-53;
  const double ls = log_pos(S);
  const double q = ls == 0.0 ? 0.0 : ls * pe.ilg;
  if (q >= 0.5) {
    const double fl = rint(q);
    tie = fabs(q - fl) < 1e-12 * q;
  }
  return q >= 0x1p62 ? (1ull << 62) : (uint64_t)q;
}

// the cell at table offset en of cell X (coordinates qa) at level lvl
template <int D>
__device__ __forceinline__ uint32_t offset_cell(const uint32_t* qa, uint32_t en, uint32_t lvl) {
  const uint32_t cm = (uint32_t)((1ull << lvl) - 1);
  uint32_t b[D];
#pragma unroll
  for (int k = 0; k < D; ++k) b[k] = (qa[k] + ((en >> (3 * k)) & 7u) - 3u) & cm;
  return morton_encode<D>(b);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D, bool MX>
__global__ __launch_bounds__(kSeqWaves * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_type2s(
    const Graph* __restrict__ g, Verts v, const CellL* __restrict__ cl, const uint2* __restrict__ crec,
    const Src* __restrict__ src, Sched sc, const Pbar* __restrict__ pbt, int nlev,
    const uint32_t* __restrict__ dtab2, Stage sg, DeferOut dfo, uint32_t coff) {
  __shared__ uint32_t ltab[kDistHead + (1 << D) * kSeqOff];
  __shared__ uint32_t ems[kSeqWaves][kSeqEnt];
  __shared__ uint32_t ebs_[kSeqWaves][kSeqEnt];
  __shared__ uint8_t eas[kSeqWaves][kSeqEnt];
  __shared__ SSrc sss[kSeqWaves][kSeqRing];
  __shared__ Cand cqs[kSeqWaves][kCCap];
  __shared__ QItem2 iqs[kSeqWaves][kQCap];
  __shared__ uint2 obs[kSeqWaves][kEdgeBuf2];
  // the parity tables (offsets of each parity, gap 1 first), once per workgroup
  {
    const uint32_t tsz = kDistHead + (1u << D) * dtab2[0];
    for (uint32_t k = threadIdx.x; k < tsz; k += blockDim.x) ltab[k] = dtab2[k];
    __syncthreads();
  }
  const uint32_t wv = threadIdx.x / kWave;
  uint32_t* em = ems[wv];   // kept cells: low 32 bits of the layer mask
  uint32_t* eb = ebs_[wv];  // kept cells: index of the first (first, count) record
  uint8_t* ea = eas[wv];    // kept cells: table offset | (X < Y) << 7
  SSrc* ss = sss[wv];
  Cand* cq = cqs[wv];
  QItem2* iq = iqs[wv];
  const uint32_t lane = lane_id();
  const uint32_t dstride = ltab[0];
  const uint32_t k0s = g->seed_lo, k1s = g->seed_hi;
  const int L = g->L;
  constexpr uint32_t QM = kSeqRing - 1;
  uint32_t ndraws = 0, ncand = 0, nre = 0;
  uint64_t nedge = 0;
  for (;;) {
    const uint32_t c = next_chunk(sc.next);
    if (c >= sc.nchunks) break;
    const uint32_t cc = coff + c;  // the chunk's index among the pass's chunks
    const uint64_t sb = (uint64_t)c * sc.chunk;
    const uint64_t se = sb + sc.chunk < sc.nunits ? sb + sc.chunk : sc.nunits;
    uint32_t dseq = 0;
    Ring2 r{0, 0, 0, 0};
    Out out{obs[wv], 0, 0, ((uint64_t)sc.pass << 32) | cc, v.id};
    // the source window: lane k holds source wb - 64 + k; wm = its eligible
    // sources not yet staged
    uint64_t wb = sb, wm = 0;
    Src wsr{0, 0, 0, 0};
    bool srcs = sb < se;
    // rings (positions count from the chunk's start): sources [qt, qh), kept
    // cells [et, eh); sequences [0, zs) staged, [0, za) taken by lanes
    uint32_t qt = 0, qh = 0, et = 0, eh = 0, zs = 0, za = 0;
    // the lane's queued item (draws2)
    bool iact = false;
    QItem2 icur{};
    PB ipe{0.0, 0.0, 0.0f};
    // the lane's sequence: its source's ring position, gap, layer j, kept
    // cells [ecur, eend) still ahead; walk state: the current cell pair
    // (b0, nb, N, orientation xa); rem = the position, from the pair's start,
    // of the next candidate (once drawn) or of the next draw's start (need);
    // the last draw's acc and tie; the draw counter td
    bool act = false, have = false, need = true, tie = false, xa = false;
    uint32_t slot = 0, gp = 1, j = 0, ecur = 0, eend = 0, s0 = 0, na = 0, X = 0, lvl = 0, li = 0,
             par = 0, w3 = 0, b0 = 0, nb = 0, td = 0, pidx = 0;
    PB pe{0.0, 0.0, 0.0f};
    int pexp = 0;
    uint64_t rem = 0, N = 0;
    double acc = 0.0;
    for (;;) {
      // --- stage sources while fewer than 64 sequences wait and the rings have room
      while (srcs && zs - za < (uint32_t)kWave) {
        if (wm == 0) {
          if (wb >= se) {
            srcs = false;
            break;
          }
          const uint64_t sj = wb + lane;
          bool elig = false;
          if (sj < se) {
            wsr = src[sj];
            const uint32_t lv = wsr.meta & 255u, lj = wsr.meta >> 8;
            elig = lv >= 3 && g->jII[lj][lv] != 0;
          }
          wm = __ballot(elig);
          wb += kWave;
          continue;
        }
        const int f = __ffsll((long long)wm) - 1;
        const uint32_t fX = __shfl(wsr.A, f, 64), fmeta = __shfl(wsr.meta, f, 64);
        const uint32_t flv = fmeta & 255u, fli = fmeta >> 8;
        uint32_t qa[D], fpar = 0;
        morton_decode<D>(fX, qa);
#pragma unroll
        for (int k = 0; k < D; ++k) fpar |= (qa[k] & 1u) << k;
        const uint32_t c1 = ltab[1 + 2 * fpar], cn = c1 + ltab[2 + 2 * fpar];
        if (eh - et + cn > (uint32_t)kSeqEnt || qh - qt >= (uint32_t)kSeqRing) break;  // no room yet
        const uint32_t fs0 = __shfl(wsr.s, f, 64), fna = __shfl(wsr.na, f, 64);
        wm &= wm - 1;
        const uint64_t J = g->jII[fli][flv];
        const uint32_t mo = g->moff[flv];
        uint32_t nk = 0, nk1 = 0, u1 = 0, u2 = 0;
        for (uint32_t k0 = 0; k0 < cn; k0 += kWave) {
          const uint32_t k = k0 + lane;
          bool keep = false;
          const bool g1 = k < c1;
          uint32_t m = 0, bs = 0, ax = 0;
          if (k < cn) {
            const uint32_t Yc = offset_cell<D>(qa, ltab[kDistHead + fpar * dstride + k], flv);
            const CellL ce = cl[mo + Yc];
            keep = (ce.mask & J) != 0;
            m = (uint32_t)ce.mask;
            bs = ce.base;
            ax = k | (fX < Yc ? 0x80u : 0u);
          }
          const uint64_t mk = __ballot(keep);
          if (keep) {
            const uint32_t p = (eh + nk + lanes_below(mk)) % (uint32_t)kSeqEnt;
            em[p] = m;
            eb[p] = bs;
            ea[p] = (uint8_t)ax;
            if (g1) u1 |= m & (uint32_t)J;
            else u2 |= m & (uint32_t)J;
          }
          nk += (uint32_t)__popcll(mk);
          nk1 += (uint32_t)__popcll(__ballot(keep && g1));
        }
        u1 = wave_or32(u1);
        u2 = wave_or32(u2);
        if (nk) {
          const uint32_t ns = (uint32_t)(__popc(u1) + __popc(u2));
          if (lane == 0)
            ss[qh & QM] = SSrc{fs0, fna, fX, flv | (fli << 8) | (fpar << 16), eh, nk1, nk, zs + ns,
                               u1, u2, ns, 0u};
          eh += nk;
          zs += ns;
          qh += 1;
        }
        wave_sync_lds();
      }
      // --- idle lanes take the next waiting sequences
      {
        const uint64_t mi = __ballot(!act);
        const uint32_t z = za + lanes_below(mi);
        if (!act && z < zs) {
          // the source: the first ring position a with cs(a) > z
          uint32_t lo = qt, hi = qh;
          while (lo != hi) {
            const uint32_t mid = lo + ((hi - lo) >> 1);
            if (ss[mid & QM].cs <= z) lo = mid + 1;
            else hi = mid;
          }
          const SSrc sv = ss[lo & QM];
          slot = lo;
          const uint32_t n1s = (uint32_t)__popc(sv.U1), ns = n1s + (uint32_t)__popc(sv.U2);
          uint32_t h = z - (sv.cs - ns);
          uint32_t mm = sv.U1;
          gp = 1;
          if (h >= n1s) {
            h -= n1s;
            mm = sv.U2;
            gp = 2;
          }
          for (; h > 0; --h) mm &= mm - 1;
          j = (uint32_t)__ffs(mm) - 1;
          s0 = sv.s0;
          na = sv.na;
          X = sv.X;
          lvl = sv.info & 255u;
          li = (sv.info >> 8) & 255u;
          par = sv.info >> 16;
          ecur = gp == 1 ? sv.e0 : sv.e0 + sv.n1;
          eend = gp == 1 ? sv.e0 + sv.n1 : sv.e0 + sv.n;
          pidx = pbar_index(li, j, lvl, gp, (uint32_t)L, (uint32_t)nlev);
          const Pbar pv = pbt[pidx];
          pe = PB{pv.pbar, pv.ilg, pv.qscale};
          pexp = pv.e;
          w3 = ctr_word3(lvl, li, j, kKindSeq, 0);
          have = false;
          need = true;
          tie = false;
          rem = 0;
          N = 0;
          td = 0;
          act = pv.pbar > 0.0;
          if (!act) atomicSub(&ss[slot & QM].left, 1u);  // no candidates: ends at once
        }
        const uint32_t nid = (uint32_t)__popcll(mi);
        za = zs - za < nid ? zs : za + nid;
      }
      // the chunk's sequences have all ended: its queued items follow
      const bool fin = !srcs && za == zs && !__any(act);
      if (!fin) {
        // --- walk: move every lane past the pairs that rem passes (a lane
        // that meets a pair of many candidates queues it as an item; the
        // walk pauses while the item queue lacks room for 64)
        bool mv = act && (!have || rem >= N);
        while (__any(mv) && r.qt - r.qh <= (uint32_t)(kQCap - 64)) {
          bool hv = false, dn = false;
          ItemRec rec{};
          QItem2 dq{};
          if (mv) {
            if (have) {
              rem -= N;
              have = false;
            }
            bool found = false;
            uint32_t m = 0, p = 0;
            while (ecur != eend && !found) {
              p = ecur % (uint32_t)kSeqEnt;
              m = em[p];
              ++ecur;
              found = ((m >> j) & 1u) != 0;
            }
            if (found) {
              const uint32_t ax = ea[p];
              const uint2 cr = crec[eb[p] + (uint32_t)__popc(m & ((1u << j) - 1u))];
              b0 = cr.x;
              nb = cr.y;
              xa = (ax >> 7) != 0;
              N = (uint64_t)na * nb;
              const bool heavy = multi_segment(N, pexp), dense = multi_segment(N, pexp - 4);
              if (heavy || dense) {
                uint32_t qa[D];
                morton_decode<D>(X, qa);
                const uint32_t Yc = offset_cell<D>(qa, ltab[kDistHead + par * dstride + (ax & 127u)], lvl);
                const uint32_t cA = xa ? X : Yc, cB = xa ? Yc : X, ci = xa ? li : j, cj = xa ? j : li;
                if (heavy) {
                  // more than one segment: the segmented pass, with the pair's own streams
                  rec = ItemRec{xa ? s0 : b0, xa ? na : nb, xa ? b0 : s0, xa ? nb : na, cA, cB,
                                lvl | (ci << 8) | (cj << 16) | (gp << 24), (uint32_t)pexp};
                  hv = true;
                } else {
                  // one segment of many candidates: an item with its own stream, as in k_type2
                  dq = QItem2{cA, cB, ctr_word3(lvl, ci, cj, kKindType2, 0), xa ? s0 : b0, xa ? b0 : s0,
                              xa ? nb : na, 0u, pidx, 0ull, N};
                  dn = true;
                }
              } else {
                have = true;
              }
            } else {
              // the sequence ends (no draw after a candidate at its very
              // end); a tie of its last draw counts when that draw's skip
              // ends exactly at the end of the sequence
              if (!need && tie && rem == 0) count_stat(sg.stats, kStatTie);
              act = false;
              atomicSub(&ss[slot & QM].left, 1u);
            }
          }
          if (__any(hv)) defer_item(hv, rec, cc, dseq, dfo);
          enqueue2(dn, dq, iq, r);
          mv = act && (!have || rem >= N);
        }
        // --- the lanes whose rem lies inside their pair: the candidate there
        // (unless a draw is due first), then the next draw while the
        // position stays inside the pair
        bool hc = false;
        Cand cd{0, 0, 0.0};
        if (act && have && rem < N) {
          if (!need) {
            // the candidate at rem: x rem / nb of V_i^X, y rem % nb of V_j^Y
            const uint64_t xi = rem / nb, yi = rem - xi * nb;
            const uint32_t sx = s0 + (uint32_t)xi, sy = b0 + (uint32_t)yi;
            cd = Cand{xa ? sx : sy, xa ? sy : sx, acc * pe.pbar};
            hc = true;
            if (tie) count_stat(sg.stats, kStatTie);
            rem += 1;
            need = true;
          }
          if (need && rem < N) {
            rem += seq_draw<MX>(k0s, k1s, X, gp, w3, td, pe, acc, tie, nre);
            ++td;
            ++ndraws;
            need = false;
          }
        }
        const uint64_t mc = __ballot(hc);
        if (hc) cq[(r.ct + lanes_below(mc)) & (kCCap - 1)] = cd;
        r.ct += (uint32_t)__popcll(mc);
        ncand += hc ? 1 : 0;
        if (r.ct - r.ch >= 64) eval_cands<D, 0, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
      }
      // --- the queued items: while 64 are queued or held; at the end all
      if (fin || r.qt - r.qh >= 64)
        draws2<D, 0, MX>(g, v, pbt, nlev, iq, cq, r, iact, icur, ipe, fin ? 0u : 64u, sg, out, ndraws,
                         ncand, nre);
      if (fin) break;
      // --- release the oldest sources whose sequences have all ended
      wave_sync_lds();
      while (qt != qh && ss[qt & QM].left == 0) {
        ++qt;
        et = qt != qh ? ss[qt & QM].e0 : eh;
      }
    }
    while (r.ct != r.ch) eval_cands<D, 0, MX>(g, v, pbt, nlev, cq, r, sg, out, nre);
    end_chunk(sg, out, sc, c, dseq);
    nedge += out.off;
  }
  const uint64_t sdraws = wave_sum((uint64_t)ndraws), scand = wave_sum((uint64_t)ncand),
                 sre = wave_sum((uint64_t)nre);
  if (lane == 0) {
    if (nedge) atomicAdd(&sg.stats[8 + sc.pass], (unsigned long long)nedge);
    atomicAdd(&sg.stats[2], (unsigned long long)sdraws);
    atomicAdd(&sg.stats[4], (unsigned long long)scand);
    if (sre) atomicAdd(&sg.stats[6], (unsigned long long)sre);
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

// deferred items to their (chunk, sequence) order; dbase = exclusive scan of
// the per-chunk deferred counts
__global__ __launch_bounds__(256) void k_defer_place(const ItemRec* __restrict__ rec,
                                                     const uint64_t* __restrict__ key, uint32_t n,
                                                     const uint64_t* __restrict__ dbase,
                                                     ItemRec* __restrict__ out) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n) return;
  const uint64_t k = key[h];
  const uint64_t dst = dbase[k >> 24] + (k & 0xFFFFFFull);
  if (dst < n) out[dst] = rec[h];
}

// staged blocks -> final order (one wave per record): chunk start + the
// edges of the chunk flushed before the block
__global__ __launch_bounds__(256) void k_stage_copy(const uint2* __restrict__ stage,
                                                    const uint64_t* __restrict__ rtag,
                                                    const uint64_t* __restrict__ roff,
                                                    const uint64_t* __restrict__ rpos,
                                                    const uint32_t* __restrict__ rcnt, uint32_t nrec,
                                                    ChunkBases cb, uint64_t m,
                                                    uint2* __restrict__ out) {
  const uint32_t lane = lane_id();
  const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t w = (uint64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; w < nrec; w += nw) {
    const uint64_t t = rtag[w];
    const uint64_t dst = cb.base[t >> 32][(uint32_t)t] + roff[w];
    const uint64_t src = rpos[w];
    const uint32_t cnt = rcnt[w];
    for (uint32_t i = lane; i < cnt; i += kWave)
      if (dst + i < m) out[dst + i] = stage[src + i];
  }
}

// the type-II candidates listed as within 1e-12 of their probability: count
// those inside the band 1e-12 pbar; a list that overflowed counts the rest
// (an upper bound)
template <int D, int MODEL>
__global__ __launch_bounds__(256) void k_near2(const Graph* __restrict__ g, Verts v,
                                               const Pbar* __restrict__ pbt, int nlev,
                                               const uint4* __restrict__ nbuf,
                                               const unsigned int* __restrict__ ncnt, uint32_t ncap,
                                               unsigned long long* __restrict__ stats) {
  const uint32_t cnt = *ncnt;
  const uint32_t nl = cnt < ncap ? cnt : ncap;
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h == 0 && cnt > ncap) atomicAdd(&stats[kStatNear], (unsigned long long)(cnt - ncap));
  for (uint32_t e = h; e < nl; e += gridDim.x * blockDim.x) {
    const uint4 t = nbuf[e];
    const double apb = __longlong_as_double((long long)(((uint64_t)t.w << 32) | t.z));
    if (t2_near<D, MODEL>(g, v, pbt, nlev, t.x, t.y, apb)) atomicAdd(&stats[kStatNear], 1ull);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define HG_DISPATCH_D(...)                                                         \
  do {                                                                             \
    if (g.model == 1) { constexpr int DD = 1; constexpr int MM = 1; __VA_ARGS__; } \
    else switch (g.d) {                                                            \
      case 1: { constexpr int DD = 1; constexpr int MM = 0; __VA_ARGS__; } break;  \
      case 2: { constexpr int DD = 2; constexpr int MM = 0; __VA_ARGS__; } break;  \
      case 3: { constexpr int DD = 3; constexpr int MM = 0; __VA_ARGS__; } break;  \
      default: { constexpr int DD = 4; constexpr int MM = 0; __VA_ARGS__; } break; \
    }                                                                              \
  } while (0)

// mixed precision applies to the binomial GIRG only
static bool use_mixed(const Graph& g) { return g.precision == 1 && g.model == 0 && g.T > 0.0; }

hipError_t launch_type1(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                        const uint2* crec, const Src* src, const Sched& sc, const Stage& sg,
                        const DeferOut& dfo, hipStream_t st) {
  const dim3 grid(sc.blocks), block(kWavesPerBlock * kWave);
  const bool t0 = !(g.T > 0.0), mx = use_mixed(g);
  HG_DISPATCH_D({
    if (t0) hipLaunchKernelGGL((k_type1<DD, MM, true, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, sg, dfo);
    else if constexpr (MM == 0) {
      if (mx) hipLaunchKernelGGL((k_type1<DD, 0, false, true>), grid, block, 0, st, gd, v, cl, crec, src, sc, sg, dfo);
      else hipLaunchKernelGGL((k_type1<DD, 0, false, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, sg, dfo);
    } else hipLaunchKernelGGL((k_type1<DD, MM, false, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, sg, dfo);
  });
  return hipGetLastError();
}

hipError_t launch_big1(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                       const uint64_t* uoff, uint32_t nrec, const Sched& sc, const Stage& sg,
                       hipStream_t st) {
  const dim3 grid(sc.blocks), block(kWavesPerBlock * kWave);
  const bool t0 = !(g.T > 0.0), mx = use_mixed(g);
  HG_DISPATCH_D({
    if (t0) hipLaunchKernelGGL((k_big1<DD, MM, true, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, sg);
    else if constexpr (MM == 0) {
      if (mx) hipLaunchKernelGGL((k_big1<DD, 0, false, true>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, sg);
      else hipLaunchKernelGGL((k_big1<DD, 0, false, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, sg);
    } else hipLaunchKernelGGL((k_big1<DD, MM, false, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, sg);
  });
  return hipGetLastError();
}

hipError_t launch_type2(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                        const uint2* crec, const Src* src, const Sched& sc, const Pbar* pbt,
                        int nlev, const uint32_t* dtab, const Stage& sg, const DeferOut& dfo,
                        uint32_t lvl_skip, hipStream_t st) {
  const dim3 grid(sc.blocks), block(kWavesPerBlock * kWave);
  const bool mx = use_mixed(g);
  HG_DISPATCH_D({
    if constexpr (MM == 0) {
      if (mx) hipLaunchKernelGGL((k_type2<DD, 0, true>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab, sg, dfo, lvl_skip);
      else hipLaunchKernelGGL((k_type2<DD, 0, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab, sg, dfo, lvl_skip);
    } else hipLaunchKernelGGL((k_type2<DD, MM, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab, sg, dfo, lvl_skip);
  });
  return hipGetLastError();
}

hipError_t launch_type2s(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                         const uint2* crec, const Src* src, const Sched& sc, const Pbar* pbt,
                         int nlev, const uint32_t* dtab2, const Stage& sg, const DeferOut& dfo,
                         uint32_t coff, hipStream_t st) {
  // workgroups of kSeqWaves waves, as many waves as sc.blocks workgroups hold
  const dim3 grid(sc.blocks * (kWavesPerBlock / kSeqWaves)), block(kSeqWaves * kWave);
  const bool mx = use_mixed(g);
  if (g.model != 0 || g.d < 2 || g.d > 3 || g.L > 32) return hipErrorInvalidValue;
  if (g.d == 2) {
    if (mx) hipLaunchKernelGGL((k_type2s<2, true>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab2, sg, dfo, coff);
    else hipLaunchKernelGGL((k_type2s<2, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab2, sg, dfo, coff);
  } else {
    if (mx) hipLaunchKernelGGL((k_type2s<3, true>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab2, sg, dfo, coff);
    else hipLaunchKernelGGL((k_type2s<3, false>), grid, block, 0, st, gd, v, cl, crec, src, sc, pbt, nlev, dtab2, sg, dfo, coff);
  }
  return hipGetLastError();
}



// the distant offsets of a parity pattern: children of the parent's
// neighbours (offset delta_k = jk - 2 - parity_k) that are not neighbours,
// listed once per unordered pair (first nonzero delta positive).  Calls f(t,
// entry) for the t-th entry; returns the count.
template <typename F>
static uint32_t distant_offsets(int d, int par, F&& f) {
  int noff = 1;
  for (int k = 0; k < d; ++k) noff *= 6;
  uint32_t t = 0;
  for (int o = 0; o < noff; ++o) {
    int rem = o, dm = 0, first = 0;
    uint32_t en = 0;
    for (int k = 0; k < d; ++k) {
      const int jk = rem % 6;
      rem /= 6;
      const int delta = jk - 2 - ((par >> k) & 1);  // child of a parent-neighbour
      const int ad = delta < 0 ? -delta : delta;
      dm = ad > dm ? ad : dm;
      if (first == 0) first = delta;
      en |= (uint32_t)(delta + 3) << (3 * k);
    }
    if (dm < 2 || first < 0) continue;  // a neighbour, or listed at the other cell
    f(t++, en | ((uint32_t)(dm - 1) << 28));
  }
  return t;
}

size_t distant_table_fill(int d, uint32_t* out, size_t cap) {
  const int npar = 1 << d;
  uint32_t stride = 1, least = ~0u;
  for (int par = 0; par < npar; ++par) {
    const uint32_t c = distant_offsets(d, par, [](uint32_t, uint32_t) {});
    stride = c > stride ? c : stride;
    least = c < least ? c : least;
  }
  // k_type2 at d >= 3 relies on every row holding at least 64 offsets, and
  // at d <= 3 holds the table in LDS sized by the longest row
  if (d >= 3 && least < (uint32_t)kWave) return 0;
  const int nd = d == 1 ? Offs<1>::nd : d == 2 ? Offs<2>::nd : d == 3 ? Offs<3>::nd : Offs<4>::nd;
  if (stride > (uint32_t)nd) return 0;
  const size_t size = (size_t)kDistHead + (size_t)npar * stride;
  if (!out || cap < size) return size;
  for (size_t k = 0; k < size; ++k) out[k] = 0u;
  out[0] = stride;
  // d = 3: each entry as the Morton displacement itself, delta_k mod 2^10
  // spread into dimension k's bits (dimension 0 most significant), with the
  // gap in bits 30-31; k_type2 adds it to a cell's code per dimension
  auto spread3h = [](uint32_t v) {
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
  };
  for (int par = 0; par < npar; ++par)
    out[1 + par] = distant_offsets(d, par, [&](uint32_t t, uint32_t en) {
      if (d == 3) {
        uint32_t dil = 0;
        for (int k = 0; k < 3; ++k) {
          const uint32_t dk = (((en >> (3 * k)) & 7u) - 3u) & 1023u;  // delta_k mod 2^10
          dil |= spread3h(dk) << (2 - k);
        }
        en = dil | ((en >> 28) << 30);
      }
      out[kDistHead + (size_t)par * stride + t] = en;
    });
  return size;
}

std::vector<uint32_t> distant_table(int d) {
  std::vector<uint32_t> tab(distant_table_fill(d, nullptr, 0), 0u);
  distant_table_fill(d, tab.data(), tab.size());
  return tab;
}

// the distant offsets of each parity split by gap: head[1 + 2p] = gap-1
// count, head[2 + 2p] = gap-2 count; row p holds the gap-1 entries, then the
// gap-2 entries, each in the table order of distant_offsets
size_t seq_table_fill(int d, uint32_t* out, size_t cap) {
  const int npar = 1 << d;
  uint32_t stride = 1;
  for (int par = 0; par < npar; ++par) {
    const uint32_t c = distant_offsets(d, par, [](uint32_t, uint32_t) {});
    stride = c > stride ? c : stride;
  }
  if (stride > (uint32_t)kSeqOff) return 0;  // (k_type2s holds kSeqOff offsets per parity)
  const size_t size = (size_t)kDistHead + (size_t)npar * stride;
  if (!out || cap < size) return size;
  for (size_t k = 0; k < size; ++k) out[k] = 0u;
  out[0] = stride;
  for (int par = 0; par < npar; ++par) {
    uint32_t t = 0;
    for (uint32_t gp = 1; gp <= 2; ++gp) {
      uint32_t cnt = 0;
      distant_offsets(d, par, [&](uint32_t, uint32_t en) {
        if ((en >> 28) == gp) {
          out[kDistHead + (size_t)par * stride + t++] = en;
          ++cnt;
        }
      });
      out[gp == 1 ? 1 + 2 * par : 2 + 2 * par] = cnt;
    }
  }
  return size;
}

hipError_t launch_heavy2(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                         const uint64_t* uoff, uint32_t nrec, const Sched& sc, const Pbar* pbt,
                         int nlev, const Stage& sg, hipStream_t st) {
  const dim3 grid(sc.blocks), block(kWavesPerBlock * kWave);
  const bool mx = use_mixed(g);
  HG_DISPATCH_D({
    if constexpr (MM == 0) {
      if (mx) hipLaunchKernelGGL((k_heavy2<DD, 0, true>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, pbt, nlev, sg);
      else hipLaunchKernelGGL((k_heavy2<DD, 0, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, pbt, nlev, sg);
    } else hipLaunchKernelGGL((k_heavy2<DD, MM, false>), grid, block, 0, st, gd, v, rec, uoff, nrec, sc, pbt, nlev, sg);
  });
  return hipGetLastError();
}

hipError_t launch_near2(const Graph& g, const Graph* gd, const Verts& v, const Pbar* pbt, int nlev,
                        const Stage& sg, hipStream_t st) {
  HG_DISPATCH_D({
    hipLaunchKernelGGL((k_near2<DD, MM>), dim3(16), dim3(256), 0, st, gd, v, pbt, nlev, sg.nbuf, sg.ncnt,
                       sg.ncap, sg.stats);
  });
  return hipGetLastError();
}

hipError_t launch_rec_units(const ItemRec* rec, uint32_t nrec, int kind, uint64_t* units,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rec_units, dim3((nrec + 255) / 256), dim3(256), 0, st, rec, nrec, kind, units);
  return hipGetLastError();
}

hipError_t launch_defer_place(const ItemRec* rec, const uint64_t* key, uint32_t n,
                              const uint64_t* dbase, ItemRec* out, hipStream_t st) {
  if (n) hipLaunchKernelGGL(k_defer_place, dim3((n + 255) / 256), dim3(256), 0, st, rec, key, n, dbase, out);
  return hipGetLastError();
}

hipError_t launch_stage_copy(const uint2* stage, const uint64_t* rtag, const uint64_t* roff,
                             const uint64_t* rpos, const uint32_t* rcnt, uint32_t nrec,
                             const ChunkBases& cb, uint64_t m, uint2* out, hipStream_t st) {
  const uint32_t blocks = std::min<uint32_t>((nrec + 3) / 4, 8192u);
  hipLaunchKernelGGL(k_stage_copy, dim3(blocks ? blocks : 1), dim3(256), 0, st, stage, rtag, roff, rpos,
                     rcnt, nrec, cb, m, out);
  return hipGetLastError();
}

}  // namespace hg
