// tune.h -- launch-shape tuning of the sampling passes.  Only shapes that
// change no result are tuned: the number of workgroups of the persistent
// sampling kernels (waves take chunks by ticket, and every chunk's output is
// placed by its index, so any grid gives the same edge array), and the
// number of concurrent workers of a batch.
#pragma once

#include <cstdint>
#include <string>

namespace hg {

// workload class of a single graph: model, d, binomial (T > 0), floor(log2 n)
struct TuneKey {
  int model, d, binomial, log2n;
  bool operator<(const TuneKey& o) const {
    if (model != o.model) return model < o.model;
    if (d != o.d) return d < o.d;
    if (binomial != o.binomial) return binomial < o.binomial;
    return log2n < o.log2n;
  }
};

TuneKey tune_key(int model, int d, double T, uint64_t n);

// loads GIRG_TUNING_FILE once (every other call below does this first)
void tune_init();

// workgroups of the persistent passes of one graph; `batch` for the graphs
// of a batch (they share the GPU with other instances)
uint32_t tuned_blocks(const TuneKey& k, bool batch);
// the built-in default for a single graph (no table, no environment)
uint32_t default_blocks(const TuneKey& k);
// forced value, else GIRG_BATCH_WORKERS, else the table, else 16
int tuned_batch_workers();

void tune_set_single(const TuneKey& k, uint32_t blocks);
void tune_set_batch(uint32_t blocks, int workers);
void tune_reset();
// forced values while the autotuner times a candidate (0 = none)
void tune_force(uint32_t single_blocks, uint32_t batch_blocks, int batch_workers);

// JSON cache: {"version": 1, "single": [{"model": m, "d": d, "binomial": b,
// "log2n": k, "blocks": g}, ...], "batch": {"blocks": g, "workers": w}}
bool tune_save(const std::string& path, std::string* err);
bool tune_load(const std::string& path, std::string* err);

constexpr uint32_t kMaxBlocks = 8192;
constexpr int kMaxWorkers = 64;

}  // namespace hg
