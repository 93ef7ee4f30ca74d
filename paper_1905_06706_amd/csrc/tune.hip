// tune.hip -- the tuning table of the persistent sampling grids (host code).
// Defaults come from timed runs on MI355X: binomial graphs up to n = 2^22
// finish sooner with 512 workgroups per pass at d <= 2 (type I and type II
// share the GPU; 256 below n = 2^17, which drains sooner) and with 768 at
// d >= 3 from n = 2^18 on (more work per source; at n = 2^17 512 was still
// 2 % faster), larger ones
// with 1024; threshold graphs (one pass) with 1024 from n = 2^17 on and 512
// below (less dispatch and drain); the graphs of a batch with 256, since 16
// instances share the GPU.  The
// autotuner (api.hip) times candidates and stores the best here; the table
// can be saved to and loaded from a JSON file (GIRG_TUNING_FILE is loaded at
// the first lookup).
#include "tune.h"

#include <atomic>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

namespace hg {

namespace {

std::mutex g_mu;
std::map<TuneKey, uint32_t> g_single;
uint32_t g_batch_blocks = 0;  // 0 = default
int g_batch_workers = 0;
std::atomic<uint32_t> g_force_single{0}, g_force_batch{0};
std::atomic<int> g_force_workers{0};
std::once_flag g_env_once;

constexpr uint32_t kDefaultBatchBlocks = 256;
constexpr int kDefaultBatchWorkers = 16;

// binomial graphs run two passes at once, so each takes fewer workgroups;
// threshold graphs have no type-II pass and fill the GPU with one
uint32_t default_single(const TuneKey& k) {
  if (k.binomial) {
    if (k.log2n >= 22) return 1024u;
    if (k.d >= 3) return k.log2n >= 18 ? 768u : 512u;
    return k.log2n < 17 ? 256u : 512u;
  }
  return k.log2n < 17 ? 512u : 1024u;
}

}  // namespace

void tune_init() {
  std::call_once(g_env_once, [] {
    if (const char* p = std::getenv("GIRG_TUNING_FILE")) {
      std::string err;
      if (!tune_load(p, &err)) std::fprintf(stderr, "hipgirg: GIRG_TUNING_FILE ignored: %s\n", err.c_str());
    }
  });
}

namespace {

// --- a small JSON reader for the cache format -------------------------------
struct Tok {
  char kind;  // '{', '}', '[', ']', ':', ',', 's' string, 'n' number, 'e' end
  std::string s;
  double v = 0.0;
};

bool tokenize(const std::string& text, std::vector<Tok>* out, std::string* err) {
  size_t i = 0;
  while (i < text.size()) {
    const char c = text[i];
    if (std::isspace((unsigned char)c)) { ++i; continue; }
    if (c == '{' || c == '}' || c == '[' || c == ']' || c == ':' || c == ',') {
      out->push_back(Tok{c, "", 0.0});
      ++i;
    } else if (c == '"') {
      const size_t j = text.find('"', i + 1);
      if (j == std::string::npos) { *err = "unterminated string"; return false; }
      out->push_back(Tok{'s', text.substr(i + 1, j - i - 1), 0.0});
      i = j + 1;
    } else if (c == '-' || std::isdigit((unsigned char)c)) {
      char* end = nullptr;
      const double v = std::strtod(text.c_str() + i, &end);
      if (end == text.c_str() + i) { *err = "malformed number"; return false; }
      out->push_back(Tok{'n', "", v});
      i = (size_t)(end - text.c_str());
    } else {
      *err = std::string("unexpected character '") + c + "'";
      return false;
    }
  }
  out->push_back(Tok{'e', "", 0.0});
  return true;
}

// an object of string keys and integer values, starting at t[*i] == '{'
bool read_flat_object(const std::vector<Tok>& t, size_t* i, std::map<std::string, long>* kv,
                      std::string* err) {
  if (t[*i].kind != '{') { *err = "expected '{'"; return false; }
  ++*i;
  if (t[*i].kind == '}') { ++*i; return true; }
  for (;;) {
    if (t[*i].kind != 's' || t[*i + 1].kind != ':' || t[*i + 2].kind != 'n') {
      *err = "expected \"key\": number";
      return false;
    }
    const double v = t[*i + 2].v;
    if (v != std::floor(v) || std::fabs(v) > 1e9) { *err = "value of " + t[*i].s + " is not an integer"; return false; }
    (*kv)[t[*i].s] = (long)v;
    *i += 3;
    if (t[*i].kind == ',') { ++*i; continue; }
    if (t[*i].kind == '}') { ++*i; return true; }
    *err = "expected ',' or '}'";
    return false;
  }
}

bool get_int(const std::map<std::string, long>& kv, const char* key, long lo, long hi, long* out,
             std::string* err) {
  auto it = kv.find(key);
  if (it == kv.end()) { *err = std::string("missing \"") + key + "\""; return false; }
  if (it->second < lo || it->second > hi) { *err = std::string("\"") + key + "\" out of range"; return false; }
  *out = it->second;
  return true;
}

}  // namespace

uint32_t default_blocks(const TuneKey& k) { return default_single(k); }

TuneKey tune_key(int model, int d, double T, uint64_t n) {
  int lg = 0;
  while ((n >> (lg + 1)) != 0 && lg < 63) ++lg;
  return TuneKey{model, model == 1 ? 1 : d, T > 0.0 ? 1 : 0, lg};
}

uint32_t tuned_blocks(const TuneKey& k, bool batch) {
  tune_init();
  if (batch) {
    const uint32_t f = g_force_batch.load();
    if (f) return f;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_batch_blocks ? g_batch_blocks : kDefaultBatchBlocks;
  }
  const uint32_t f = g_force_single.load();
  if (f) return f;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_single.find(k);
  return it != g_single.end() ? it->second : default_single(k);
}

int tuned_batch_workers() {
  tune_init();
  const int f = g_force_workers.load();
  if (f) return f;
  if (const char* ev = std::getenv("GIRG_BATCH_WORKERS")) {
    const int v = std::atoi(ev);
    if (v >= 1 && v <= kMaxWorkers) return v;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  return g_batch_workers ? g_batch_workers : kDefaultBatchWorkers;
}

void tune_set_single(const TuneKey& k, uint32_t blocks) {
  tune_init();
  std::lock_guard<std::mutex> lk(g_mu);
  g_single[k] = blocks;
}

void tune_set_batch(uint32_t blocks, int workers) {
  tune_init();
  std::lock_guard<std::mutex> lk(g_mu);
  if (blocks) g_batch_blocks = blocks;
  if (workers) g_batch_workers = workers;
}

void tune_reset() {
  tune_init();
  std::lock_guard<std::mutex> lk(g_mu);
  g_single.clear();
  g_batch_blocks = 0;
  g_batch_workers = 0;
}

void tune_force(uint32_t single_blocks, uint32_t batch_blocks, int batch_workers) {
  g_force_single.store(single_blocks);
  g_force_batch.store(batch_blocks);
  g_force_workers.store(batch_workers);
}

bool tune_save(const std::string& path, std::string* err) {
  std::ostringstream o;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    o << "{\"version\": 1,\n \"single\": [";
    bool first = true;
    for (const auto& e : g_single) {
      o << (first ? "\n  " : ",\n  ") << "{\"model\": " << e.first.model << ", \"d\": " << e.first.d
        << ", \"binomial\": " << e.first.binomial << ", \"log2n\": " << e.first.log2n
        << ", \"blocks\": " << e.second << "}";
      first = false;
    }
    o << "],\n \"batch\": {\"blocks\": " << (g_batch_blocks ? g_batch_blocks : kDefaultBatchBlocks)
      << ", \"workers\": " << (g_batch_workers ? g_batch_workers : kDefaultBatchWorkers) << "}}\n";
  }
  std::ofstream f(path);
  if (!f) { *err = "cannot open " + path + " for writing"; return false; }
  f << o.str();
  if (!f.good()) { *err = "write to " + path + " failed"; return false; }
  return true;
}

bool tune_load(const std::string& path, std::string* err) {
  std::ifstream f(path);
  if (!f) { *err = "cannot open " + path; return false; }
  std::stringstream ss;
  ss << f.rdbuf();
  std::vector<Tok> t;
  if (!tokenize(ss.str(), &t, err)) return false;
  std::map<TuneKey, uint32_t> single;
  long bb = 0, bw = 0;
  size_t i = 0;
  if (t[i].kind != '{') { *err = "expected '{'"; return false; }
  ++i;
  while (t[i].kind != '}') {
    if (t[i].kind != 's' || t[i + 1].kind != ':') { *err = "expected a key"; return false; }
    const std::string key = t[i].s;
    i += 2;
    if (key == "version") {
      if (t[i].kind != 'n' || t[i].v != 1.0) { *err = "unsupported version"; return false; }
      ++i;
    } else if (key == "single") {
      if (t[i].kind != '[') { *err = "\"single\" is not an array"; return false; }
      ++i;
      while (t[i].kind != ']') {
        std::map<std::string, long> kv;
        if (!read_flat_object(t, &i, &kv, err)) return false;
        long model, d, bin, lg, blocks;
        if (!get_int(kv, "model", 0, 1, &model, err) || !get_int(kv, "d", 1, 4, &d, err) ||
            !get_int(kv, "binomial", 0, 1, &bin, err) || !get_int(kv, "log2n", 0, 63, &lg, err) ||
            !get_int(kv, "blocks", 1, kMaxBlocks, &blocks, err))
          return false;
        single[TuneKey{(int)model, (int)d, (int)bin, (int)lg}] = (uint32_t)blocks;
        if (t[i].kind == ',') ++i;
        else if (t[i].kind != ']') { *err = "expected ',' or ']'"; return false; }
      }
      ++i;
    } else if (key == "batch") {
      std::map<std::string, long> kv;
      if (!read_flat_object(t, &i, &kv, err)) return false;
      if (!get_int(kv, "blocks", 1, kMaxBlocks, &bb, err) || !get_int(kv, "workers", 1, kMaxWorkers, &bw, err))
        return false;
    } else {
      *err = "unknown key \"" + key + "\"";
      return false;
    }
    if (t[i].kind == ',') ++i;
    else if (t[i].kind != '}') { *err = "expected ',' or '}'"; return false; }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& e : single) g_single[e.first] = e.second;
  if (bb) g_batch_blocks = (uint32_t)bb;
  if (bw) g_batch_workers = (int)bw;
  return true;
}

}  // namespace hg
