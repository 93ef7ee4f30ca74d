// sampler.h -- launchers of the sampler kernels (sampler.hip) and the small
// structures they share with the host driver.
#pragma once

#include "internal.h"

namespace hg {

constexpr int kSampleBlocks = 2048;                 // fixed grid: 8192 waves
constexpr int kSampleWaves = kSampleBlocks * 4;

struct WaveOut {
  uint32_t* count;             // per-wave edge counts (count pass)
  const uint64_t* base;        // per-wave output offsets (write pass)
  uint2* edges;
  unsigned long long* stats;   // 0 tests, 1 draws, 2 candidates, 3 rechecks
};

// a type-II item whose candidate range spans more than one segment
struct HeavyRec {
  uint32_t a0, na, b0, nb, A, B, meta, e;  // meta = level | i << 8 | j << 16 | gap << 24
};

struct HeavyOut {
  HeavyRec* rec;
  uint64_t* key;         // (wave << 24) | sequence within the wave
  unsigned int* count;
  uint32_t cap;
};

hipError_t launch_points(const Graph& g, double beta, double* w, double* x, hipStream_t st);
hipError_t launch_layer_key(const Graph& g, Graph* gd, const double* w, const double* x,
                            uint64_t* keys, uint32_t* ids, uint32_t* flag, hipStream_t st);
hipError_t launch_gather(const Graph& g, const Graph* gd, const uint64_t* keys, const uint32_t* ids,
                         const double* w, const double* x, double* sw, double* sx, uint32_t* smort,
                         uint8_t* slayer, double* aux, hipStream_t st);
hipError_t launch_tables(Graph* gd, int Dcap, Pbar* pb, hipStream_t st);
hipError_t launch_cell_count(const Graph& g, const Graph* gd, const uint32_t* smort,
                             const uint8_t* slayer, uint32_t* cnt, hipStream_t st);
hipError_t launch_sources(const Graph& g, const Graph* gd, const uint32_t* smort,
                          const uint8_t* slayer, uint32_t* cnt, const uint32_t* off, uint64_t* src,
                          bool fill, hipStream_t st);
hipError_t launch_type1(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nsrc, bool write, const WaveOut& wo,
                        hipStream_t st);
hipError_t launch_type2(const Graph& g, const Graph* gd, const Verts& v, const uint32_t* P,
                        const uint64_t* src, uint64_t nsrc, const Pbar* pbt, int nlev, bool write,
                        const WaveOut& wo, const HeavyOut& ho, hipStream_t st);
hipError_t launch_heavy_prep(const void* rec, uint32_t nh, uint64_t* nseg, hipStream_t st);
hipError_t launch_heavy_gather(const void* in, const uint32_t* perm, uint32_t nh, void* out,
                               hipStream_t st);
hipError_t launch_heavy(const Graph& g, const Graph* gd, const Verts& v, const void* rec,
                        const uint64_t* segoff, uint32_t nh, uint64_t nseg, const Pbar* pbt,
                        int nlev, bool write, const WaveOut& wo, hipStream_t st);
size_t heavy_rec_size();

}  // namespace hg
