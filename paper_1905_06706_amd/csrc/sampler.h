// sampler.h -- launchers of the preprocessing kernels (prep.hip) and of the
// sampling kernels (sample.hip), and the records they exchange with the host
// driver.
#pragma once

#include "internal.h"

namespace hg {

// persistent grids: workgroups of 4 waves; the number of workgroups comes
// from the tuning table (tune.hip), capped at one wave per chunk
constexpr int kWavesPerBlock = 4;
// type-I items with more tests are split into pieces of kTestChunk tests:
// binomial tests are costly, so smaller items are split than for threshold
// tests, where a piece costs more to schedule than to test
constexpr uint32_t kBigTests = 64;
constexpr uint32_t kBigTestsT0 = 256;
constexpr uint32_t kTestChunk = 64;   // tests per unit of a split type-I item

// one run of a layer's cell: sorted position s of its first vertex, its cell
// A at the level, |V_i^A|, and meta = level | layer << 8
struct Src {
  uint32_t s, A, na, meta;
};

// a deferred item: type-I with more than kBigTests tests, or type-II with
// more than one segment.  meta = level | i << 8 | j << 16 | gap << 24 |
// tri << 31; e = segment exponent (type-II)
struct ItemRec {
  uint32_t a0, na, b0, nb, A, B, meta, e;
};

// dynamic chunk scheduling: waves take chunks of `chunk` units by ticket.
// The wave that finishes chunk c stores the edges it produced in ctot[c] and
// the items it deferred in dtot[c] (null for passes that defer nothing);
// exclusive scans of these give every chunk its output range.
struct Sched {
  unsigned int* next;  // ticket counter (zeroed before each launch)
  uint64_t nunits;
  uint32_t chunk;
  uint32_t nchunks;
  uint32_t pass;       // 0 type-I, 1 split type-I, 2 type-II, 3 segmented type-II
  uint64_t* ctot;
  uint64_t* dtot;
  uint32_t blocks;     // workgroups of the launch
};

// staged output: waves flush blocks of edges to buf at atomically reserved
// positions and record, per flush, (pass, chunk), the edges of the chunk
// flushed before it, its position in buf and its size
struct Stage {
  uint2* buf;
  uint64_t cap;                  // edges that fit in buf
  unsigned long long* cursor;    // edges produced so far
  uint64_t* rtag;                // pass << 32 | chunk
  uint64_t* roff;                // edges of the chunk before this flush
  uint64_t* rpos;
  uint32_t* rcnt;
  unsigned int* nrec;
  uint32_t rcap;
  // 0-1 tests of passes 0-1, 2-3 draws of passes 2-3, 4-5 candidates of
  // passes 2-3, 6 rechecks, 8-11 edges of passes 0-3, 12 decisions within
  // 1e-12 of the boundary, 13 skip quotients within 1e-12 of an integer
  unsigned long long* stats;
  // type-II candidates with |Acc pbar - p_uv| < 1e-12: (su, sv, Acc pbar)
  // for the test against the band 1e-12 pbar after the passes (launch_near2)
  uint4* nbuf;
  unsigned int* ncnt;
  uint32_t ncap;
};

// deferred items: key = chunk << 24 | sequence in chunk; big = the type-I
// split threshold (tests)
struct DeferOut {
  ItemRec* rec;
  uint64_t* key;
  unsigned int* count;
  uint32_t cap;
  uint32_t big;
};

// chunk edge totals of the four passes, scanned in pass order: the start of
// every chunk's edges in the output
struct ChunkBases {
  const uint64_t* base[4];
};

hipError_t launch_points(const Graph& g, double beta, double* w, double* x, hipStream_t st);
hipError_t launch_set_weight_sums(Graph* gd, const double* red, hipStream_t st);
// pts (written): each vertex's point packed in pts_stride(d, model) doubles
// (GIRG w, x_0 .. x_{d-1} and zero padding; HRG r, x), for the gather
__host__ __device__ constexpr int pts_stride(int d, int model) { return model == 1 ? 2 : rec_stride(d, 0); }
hipError_t launch_layer_key(const Graph& g, Graph* gd, const double* w, const double* x,
                            uint64_t* keys, uint32_t* ids, double* pts, uint32_t* flag, hipStream_t st);
hipError_t launch_gather(const Graph& g, const Graph* gd, const uint64_t* keys, const uint32_t* ids,
                         const double* pts, double* sw, double* rec, uint32_t* smort,
                         uint8_t* slayer, uint4* frec, hipStream_t st);
// level tables on the host: comparison level CL(i,j) (Sec. 3.1; HRG by
// search over levels, Sec. 4.3), insertion level I(i), deepest level D, and
// the masks of layer pairs served by neighbouring (CL == level) and distant
// (CL >= level) cell pairs (loop swap, Sec. 3.3), from the layer counts and
// extremes, W and c already in g
void tables_host(Graph& g, int Dcap);
// the pbar table on the device from the uploaded Graph (pb non-null for
// T > 0; L * L * (Dcap + 1) * 2 entries), over a grid
hipError_t launch_pbar(const Graph* gd, int L, int Dcap, Pbar* pb, hipStream_t st);
hipError_t launch_cell_count(const Graph& g, const Graph* gd, const uint32_t* smort,
                             const uint8_t* slayer, uint32_t* cnt, hipStream_t st);
hipError_t launch_sources(const Graph& g, const Graph* gd, const uint32_t* smort,
                          const uint8_t* slayer, const uint32_t* P, uint32_t* cnt,
                          const uint32_t* off, Src* src, CellL* cl, bool fill, hipStream_t st);
// per-cell layer sets: counts (ranks = false), then bases from their scan
// `cnt` and the (first, count) records of every source (ranks = true)
hipError_t launch_cell_layers(const Graph* gd, CellL* cl, uint64_t ne, uint32_t* cnt,
                              const Src* src, uint64_t nsrc, uint2* crec, bool ranks,
                              hipStream_t st);

// sampling passes
hipError_t launch_type1(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                        const uint2* crec, const Src* src, const Sched& sc, const Stage& sg,
                        const DeferOut& dfo, hipStream_t st);
// distant offsets of a cell at levels >= 3 by the parity pattern p of its
// coordinates: dtab[0] = stride, dtab[1 + p] = count, entries at
// dtab[kDistHead + p * stride + t] = sum_k (delta_k + 3) << 3k | gap << 28
// (d = 3: the Morton displacement, delta_k mod 2^10 spread into dimension k's
// bits, | gap << 30);
// only offsets whose first nonzero delta is positive (the other orientation
// of each pair is listed at the other cell)
constexpr int kDistHead = 32;
std::vector<uint32_t> distant_table(int d);
// the same table written to out[0..size) without allocating; returns its
// size (and writes nothing when out is null or cap is smaller), or 0 when a
// row at d >= 3 holds fewer than 64 offsets or a row is longer than
// Offs<d>::nd (k_type2 relies on both)
size_t distant_table_fill(int d, uint32_t* out, size_t cap);

// sources at levels >= lvl_skip are left to launch_type2s (255: none)
hipError_t launch_type2(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                        const uint2* crec, const Src* src, const Sched& sc, const Pbar* pbt,
                        int nlev, const uint32_t* dtab, const Stage& sg, const DeferOut& dfo,
                        uint32_t lvl_skip, hipStream_t st);
// batched type-II sequences of the sources at levels >= 3 (GIRG, d = 2, 3):
// sc covers the same source chunks as the type-II pass, with its own ticket;
// chunk c writes its totals at sc.ctot[c] / sc.dtot[c] and tags its edges
// and deferred pairs as chunk coff + c of the type-II pass
hipError_t launch_type2s(const Graph& g, const Graph* gd, const Verts& v, const CellL* cl,
                         const uint2* crec, const Src* src, const Sched& sc, const Pbar* pbt,
                         int nlev, const uint32_t* dtab2, const Stage& sg, const DeferOut& dfo,
                         uint32_t coff, hipStream_t st);
// the distant offsets per parity split by gap (launch_type2s): head[0] =
// stride, head[1 + 2p] / head[2 + 2p] = gap-1 / gap-2 counts, row p at
// kDistHead + p * stride (gap-1 entries first); returns the size, writes
// nothing when out is null or cap is smaller; 0 if a row is longer than the
// batched kernel holds
size_t seq_table_fill(int d, uint32_t* out, size_t cap);
// the listed type-II candidates inside the band |Acc - p_uv / pbar| < 1e-12
// counted into stats[12] (one small grid; after both type-II passes)
hipError_t launch_near2(const Graph& g, const Graph* gd, const Verts& v, const Pbar* pbt, int nlev,
                        const Stage& sg, hipStream_t st);
// deferred items: units per record (kind 1: test pieces, kind 2: segments)
hipError_t launch_rec_units(const ItemRec* rec, uint32_t nrec, int kind, uint64_t* units,
                            hipStream_t st);
hipError_t launch_big1(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                       const uint64_t* uoff, uint32_t nrec, const Sched& sc, const Stage& sg,
                       hipStream_t st);
hipError_t launch_heavy2(const Graph& g, const Graph* gd, const Verts& v, const ItemRec* rec,
                         const uint64_t* uoff, uint32_t nrec, const Sched& sc, const Pbar* pbt,
                         int nlev, const Stage& sg, hipStream_t st);
// deferred items in (chunk, sequence) order: out[dbase[chunk] + seq] = rec
hipError_t launch_defer_place(const ItemRec* rec, const uint64_t* key, uint32_t n,
                              const uint64_t* dbase, ItemRec* out, hipStream_t st);
// staged blocks to their final positions (one wave per record)
hipError_t launch_stage_copy(const uint2* stage, const uint64_t* rtag, const uint64_t* roff,
                             const uint64_t* rpos, const uint32_t* rcnt, uint32_t nrec,
                             const ChunkBases& cb, uint64_t cap, uint2* out, hipStream_t st);

}  // namespace hg
