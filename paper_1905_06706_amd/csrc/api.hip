// api.hip -- host driver and C ABI of the gfx950 GIRG / HRG sampler.
//
// One call runs, on one stream:
//   points (optional) -> exact sums and min/max -> layer + Morton keys ->
//   stable radix sort -> sorted SoA -> constant c (App. B.2, when asked) ->
//   level tables -> prefix sums per layer (Lemma 1) -> run sources ->
//   count passes (type-I, type-II, heavy type-II segments) -> one scan of the
//   per-wave counts -> write passes.
// The host only orchestrates and solves the scalar parameter equations (c by
// bisection over sums reduced on the device; R by quadrature).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <atomic>
#include <functional>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/hipgirg.h"
#include "sampler.h"
#include "tune.h"

namespace hg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
static girg_status fail(girg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? GIRG_ENOMEM : GIRG_EDEVICE,                    \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------
void* Arena::raw(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  if (ext_base_) {
    if (failed_ || ext_size_ - ext_used_ < bytes) {
      failed_ = true;
      return nullptr;
    }
    void* p = ext_base_ + ext_used_;
    ext_used_ += bytes;
    return p;
  }
  for (size_t c = cur_; c < chunks_.size(); ++c) {
    Chunk& ch = chunks_[c];
    if (ch.size - ch.used >= bytes) {
      void* p = ch.base + ch.used;
      ch.used += bytes;
      cur_ = c;
      return p;
    }
  }
  const size_t sz = std::max(bytes, (size_t)64 << 20);
  void* p = nullptr;
  if (hipMalloc(&p, sz) != hipSuccess) {
    (void)hipGetLastError();
    failed_ = true;
    return nullptr;
  }
  chunks_.push_back(Chunk{static_cast<char*>(p), sz, bytes});
  cur_ = chunks_.size() - 1;
  return p;
}
void Arena::release() {
  ext_base_ = nullptr;  // an attached buffer belongs to its owner
  ext_size_ = ext_used_ = 0;
  for (auto& c : chunks_) (void)hipFree(c.base);
  chunks_.clear();
  cur_ = 0;
}

// ---------------------------------------------------------------------------
// constant c from the average degree (Sec. 4.1, App. B.2).  f(c) = E[avg
// degree] is monotone in c; its closed form has an error term over E_R, the
// ordered pairs whose saturation radius k exceeds 1/2.  E_R only involves the
// heaviest vertices: with weights sorted in descending order, the partners of
// u form a prefix whose length shrinks as u gets lighter, so prefix sums of w
// and w^(1/T) give each vertex's term in O(1) (the O(|R|) evaluation).
// ---------------------------------------------------------------------------
struct CSolve {
  uint64_t n;
  int d;
  double T, W;
  std::vector<double> h;        // heaviest weights (the tail), descending
  std::vector<double> hp;       // h^(1/T)
  std::vector<double> sw, sw2;  // suffix sums over h: w, w^2
  std::vector<double> sp, sp2;  // suffix sums over h: w^(1/T), w^(2/T)
  // sums over the weights outside h: w, w^2 / W, w^(1/T), (w^2 / W)^(1/T)
  double out_w = 0.0, out_q1 = 0.0, out_p = 0.0, out_q2 = 0.0;
  double wcut;  // every weight not in h is <= wcut

  // a running sum in two doubles (Knuth's two-sum), products added exactly
  // (FMA error term): at least as accurate as a 64-bit long double sum, and
  // several times faster than x87 arithmetic
  struct DSum {
    double hi = 0.0, lo = 0.0;
    void add(double x) {
      const double s = hi + x, bb = s - hi;
      lo += (hi - (s - bb)) + (x - bb);
      hi = s;
    }
    void add_sq(double x) {
      const double p = x * x;
      add(p);
      lo += std::fma(x, x, -p);
    }
    double value() const { return hi + lo; }
  };

  // h must already be in descending order; hp (h^(1/T), same order) may be
  // given, else it is computed here
  void prepare(bool have_hp = false) {
    const size_t K = h.size();
    if (!have_hp) hp.resize(K);
    sw.resize(K + 1);
    sw2.resize(K + 1);
    sp.resize(K + 1);
    sp2.resize(K + 1);
    sw[K] = sw2[K] = sp[K] = sp2[K] = 0.0;
    DSum a, b, e, f;
    for (size_t k = K; k-- > 0;) {
      if (!have_hp) hp[k] = T > 0.0 ? std::pow(h[k], 1.0 / T) : 0.0;
      a.add(h[k]);
      b.add_sq(h[k]);
      e.add(hp[k]);
      f.add_sq(hp[k]);
      sw[k] = a.value();
      sw2[k] = b.value();
      sp[k] = e.value();
      sp2[k] = f.value();
    }
  }

  // a pair (u, v) is in E_R iff w_u w_v > th(c)
  double th(double c) const {
    return T > 0.0 ? std::ldexp(W / std::pow(c, T), -d) : W / std::ldexp(std::pow(c, (double)d), d);
  }
  // E_R within h, i.e. no pair with a weight outside h, at this c (and at
  // every smaller c: th decreases in c)
  bool complete_at(double c) const { return h.empty() || !(h[0] * wcut > th(c)); }

  // expected average degree (App. B.2): E[X_uv] = 1 on E_R and the closed
  // form A x - B x^(1/T) (T = 0: A x), x = w_u w_v / W, elsewhere.  The pairs
  // outside E_R are summed directly from suffix sums over h and the sums over
  // the weights outside h (all of whose pairs are outside E_R when h is
  // complete), so no large excess over E_R is formed and subtracted.
  double f(double c) {
    const double th = this->th(c);
    double A, B = 0.0;
    if (T > 0.0) {
      A = std::pow(c, T) * std::ldexp(1.0, d) / (1.0 - T);
      B = c * std::pow(2.0, d / T) / (1.0 / T - 1.0);
    } else {
      A = std::ldexp(std::pow(c, (double)d), d);
    }
    const double WT = T > 0.0 ? std::pow(W, 1.0 / T) : 1.0;
    const size_t K = h.size();
    const double P = (K ? sp[0] : 0.0) + out_p;
    long double cnt = 0.0L, s1 = 0.0L, s2 = 0.0L;  // s1 = sum x, s2 = sum x^(1/T) off E_R
    size_t m = K;
    for (size_t u = 0; u < K; ++u) {
      const double wu = h[u];
      while (m > 0 && !(wu * h[m - 1] > th)) --m;
      if (m == 0) {
        // no vertex of h from u on has an E_R partner
        s1 += ((long double)W * sw[u] - sw2[u]) / W;
        if (T > 0.0) s2 += ((long double)P * sp[u] - sp2[u]) / WT;
        break;
      }
      const bool self_out = u >= m;
      cnt += (long double)(m - (self_out ? 0 : 1));
      s1 += (long double)(wu / W) * (sw[m] - (self_out ? wu : 0.0) + out_w);
      if (T > 0.0) s2 += (long double)(hp[u] / WT) * (sp[m] - (self_out ? hp[u] : 0.0) + out_p);
    }
    // vertices outside h: every other vertex is a partner off E_R
    s1 += (long double)out_w - out_q1;
    if (T > 0.0) s2 += (long double)out_p * P / WT - out_q2;
    return (double)(((long double)A * s1 - (long double)B * s2 + cnt) / (long double)n);
  }

  // bracket by doubling / halving, then regula falsi on log c with the
  // Anderson-Bjorck scaling of a stale end, until the bracket is a few ulps
  // wide; returns its upper end.  When f hits the target exactly at the upper
  // end (common once the bracket is narrow, and where the secant would stall),
  // a point two ulps below closes the bracket.  f is
  // evaluated exactly wherever h is complete, i.e. at every c up to some
  // bound.  A lower end is only taken where f < target and an upper end where
  // f >= target, so when h is complete at the final upper end (checked by the
  // caller) both ends were evaluated exactly and the root lies between them,
  // whatever inexact values steered the search on the way.
  // A hint (an earlier estimate of c, e.g. from a shorter tail) starts the
  // bracket at hint (1 -+ 1/64), widened by factors of 2 until f changes sign.
  int solve(double target, double* out, double hint = 0.0) {
    double lo = 1.0, hi = 1.0, flo, fhi;
    int it = 0;
    if (hint > 0.0 && std::isfinite(hint)) {
      lo = hint * (1.0 - 1.0 / 64.0);
      hi = hint * (1.0 + 1.0 / 64.0);
      flo = f(lo) - target;
      fhi = f(hi) - target;
      // f increases with c: at most one of these loops runs
      while (!(flo < 0.0)) { hi = lo; fhi = flo; lo *= 0.5; flo = f(lo) - target; if (++it > 2000) return -1; }
      while (fhi < 0.0) { lo = hi; flo = fhi; hi *= 2.0; fhi = f(hi) - target; if (++it > 2000) return -1; }
    } else {
      flo = fhi = f(1.0) - target;
      if (flo < 0.0) {
        while (fhi < 0.0) { lo = hi; flo = fhi; hi *= 2.0; fhi = f(hi) - target; if (++it > 2000) return -1; }
      } else {
        while (!(flo < 0.0)) { hi = lo; fhi = flo; lo *= 0.5; flo = f(lo) - target; if (++it > 2000) return -1; }
      }
    }
    double a = std::log(lo), b = std::log(hi);
    int side = 0;
    for (it = 0; it < 200; ++it) {
      if (!(hi > lo) || hi - lo <= 4.0 * std::ldexp(hi, -52)) break;
      if (fhi == 0.0) {
        const double c = hi - 2.0 * std::ldexp(hi, -52);
        if (!(c > lo)) break;
        const double fc = f(c) - target;
        if (fc < 0.0) { lo = c; a = std::log(c); flo = fc; }
        else { hi = c; b = std::log(c); fhi = fc; }
        side = 0;
        continue;
      }
      double x = (fhi == flo) ? 0.5 * (a + b) : b - fhi * (b - a) / (fhi - flo);
      if (!(x > a && x < b)) x = 0.5 * (a + b);
      double c = std::exp(x);
      if (!(c > lo && c < hi)) {
        c = lo + 0.5 * (hi - lo);
        x = std::log(c);
        if (!(c > lo && c < hi)) break;
      }
      const double fc = f(c) - target;
      if (fc < 0.0) {
        if (side == -1) { const double m = 1.0 - fc / flo; fhi *= m > 0.0 ? m : 0.5; }
        lo = c; a = x; flo = fc;
        side = -1;
      } else {
        if (side == 1) { const double m = 1.0 - fc / fhi; flo *= m > 0.0 ? m : 0.5; }
        hi = c; b = x; fhi = fc;
        side = 1;
      }
    }
    *out = hi;
    return 0;
  }
};

// ---------------------------------------------------------------------------
// per-device context
// ---------------------------------------------------------------------------
struct Ctx {
  int device = -1;
  // external: the device buffers below (and the arena) lie in memory the
  // context does not own (the no-allocation entry point's scratch array);
  // fixed_tuning: the built-in launch shapes, not the tuning table
  bool external = false, fixed_tuning = false;
  Arena ar;
  Graph* gd = nullptr;       // device Graph
  double* red = nullptr;     // 6 doubles
  uint32_t* flag = nullptr;
  unsigned long long* stats = nullptr;  // 16
  unsigned int* hcount = nullptr;
  uint32_t* dtab[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // distant offsets per d
  uint32_t* dtab2[5] = {nullptr, nullptr, nullptr, nullptr, nullptr}; // the same split by gap (d = 2, 3)
  hipStream_t own = nullptr;  // batch workers: the slot's own stream
  bool batch = false;         // a batch worker's context
  // a second stream on which type I and the split type-I pass run beside
  // type II and the segmented type-II pass (fork/join by events)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t rb_done = nullptr;  // end of a readback group (Readback::end)
  // pinned host memory for readbacks: a copy into pageable memory blocks the
  // host once per copy (about 12 us each), into pinned memory the copies of a
  // group complete with one stream synchronisation.  One set per stream.
  struct Pins {
    void* pin = nullptr;
    size_t pin_size = 0;
    void* pin_up = nullptr;  // uploads (the 40 KB Graph among them)
    // direct: no pinned buffers; copies go straight to and from the pageable
    // host memory of their sources and destinations (nothing is allocated)
    bool direct = false;
    Pins() = default;
    Pins(const Pins&) = delete;
    Pins& operator=(const Pins&) = delete;
    ~Pins() {
      if (pin) (void)hipHostFree(pin);
      if (pin_up) (void)hipHostFree(pin_up);
    }
  };
  Pins pins, pins_side;
  // scratch of the c solve's first round, which runs on the side stream while
  // the main stream sorts: an arena and result slots of its own, so that no
  // allocation of the main stream reuses memory still in use there
  Arena ar_side;
  double* red_side = nullptr;  // 8 doubles
  // the c solve's host buffers (the tail and its sums), kept from call to call
  CSolve cs;
  std::vector<double> cs_asc, cs_ascp;
  std::mutex mu;
  // stage timing (HIP events), enabled by girg_set_profiling: a stage's time
  // runs from the event before it to its own, both on the stream it ran on;
  // the passes that overlap are timed on their own streams
  bool profiling = false;
  // profiling mode 2: the passes that otherwise overlap run one after
  // another on the call's stream, so each kernel's time is its own
  bool serial = false;
  std::vector<hipEvent_t> ev;
  std::vector<std::string> ev_name;
  std::vector<double> last_ms;
  std::vector<std::string> last_name;
  void mark(const char* name, hipStream_t st) {
    if (!profiling) return;
    if (ev.size() <= ev_name.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { profiling = false; return; }
      ev.push_back(e);
    }
    (void)hipEventRecord(ev[ev_name.size()], st);
    ev_name.push_back(name);
  }
  void collect() {
    last_ms.clear();
    last_name.clear();
    if (!profiling || ev_name.empty()) return;
    (void)hipEventSynchronize(ev[ev_name.size() - 1]);
    for (size_t k = 1; k < ev_name.size(); ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[k - 1], ev[k]);
      last_ms.push_back(ms);
      last_name.push_back(ev_name[k]);
    }
    ev_name.clear();
  }
  ~Ctx() {
    if (external) {
      ar.release();
      return;
    }
    if (gd) (void)hipFree(gd);
    if (red) (void)hipFree(red);
    if (flag) (void)hipFree(flag);
    if (stats) (void)hipFree(stats);
    if (hcount) (void)hipFree(hcount);
    for (auto t : dtab)
      if (t) (void)hipFree(t);
    for (auto t : dtab2)
      if (t) (void)hipFree(t);
    if (own) (void)hipStreamDestroy(own);
    if (side) (void)hipStreamDestroy(side);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (rb_done) (void)hipEventDestroy(rb_done);
    if (red_side) (void)hipFree(red_side);
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// A group of device-to-host copies staged in the context's pinned buffer:
// begin(bytes) makes room (no copy of an earlier group may be in flight, so
// every group ends with wait()), add() queues one copy, wait() synchronises
// the stream once and moves the data to its destinations.  end() marks the
// end of the group with an event: wait() then waits for that point only, and
// work queued after end() keeps the GPU busy meanwhile.
class Readback {
 public:
  Readback(Ctx& cx, hipStream_t st, bool side = false)
      : cx_(side ? cx.pins_side : cx.pins), st_(st), ev_(side ? nullptr : cx.rb_done) {}
  // a call that returns early (an error) may leave copies in flight that
  // read or write the pinned buffers: drain them before the buffers are reused
  ~Readback() {
    if (nitems_ || up_used_) (void)hipStreamSynchronize(st_);
  }
  hipError_t begin(size_t bytes) {
    if (nitems_) {
      hipError_t e = hipStreamSynchronize(st_);  // an unfinished group: let it land first
      if (e != hipSuccess) return e;
    }
    nitems_ = 0;
    used_ = 0;
    if (cx_.direct) return hipSuccess;
    bytes = (bytes + 4095) & ~(size_t)4095;
    if (bytes <= cx_.pin_size) return hipSuccess;
    if (cx_.pin) (void)hipHostFree(cx_.pin);
    cx_.pin = nullptr;
    cx_.pin_size = 0;
    hipError_t e = hipHostMalloc(&cx_.pin, bytes, hipHostMallocDefault);
    if (e == hipSuccess) cx_.pin_size = bytes;
    return e;
  }
  hipError_t add(void* dst, const void* src, size_t bytes) {
    if (nitems_ == kMaxItems) return hipErrorInvalidValue;  // a group holds at most kMaxItems copies
    if (cx_.direct) {
      items_[nitems_++] = Item{nullptr, 0, 0};
      return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st_);
    }
    const size_t off = (used_ + 15) & ~(size_t)15;
    if (off + bytes > cx_.pin_size) return hipErrorInvalidValue;  // begin() reserved too little
    items_[nitems_++] = Item{dst, off, bytes};
    used_ = off + bytes;
    return hipMemcpyAsync(static_cast<char*>(cx_.pin) + off, src, bytes, hipMemcpyDeviceToHost, st_);
  }
  hipError_t end() {
    if (!ev_) return hipSuccess;
    hipError_t e = hipEventRecord(ev_, st_);
    if (e != hipSuccess) return e;
    ended_ = true;
    up_end_ = up_used_;
    return hipSuccess;
  }
  hipError_t wait() {
    const bool ev = ended_;
    ended_ = false;
    hipError_t e = ev ? hipEventSynchronize(ev_) : hipStreamSynchronize(st_);
    if (e != hipSuccess) return e;
    for (int k = 0; k < nitems_; ++k)
      if (items_[k].dst)
        std::memcpy(items_[k].dst, static_cast<char*>(cx_.pin) + items_[k].off, items_[k].bytes);
    nitems_ = 0;
    used_ = 0;
    // every staged upload queued before the waited point has been read
    if (!ev || up_used_ == up_end_) up_used_ = 0;
    return hipSuccess;
  }
  // host-to-device copy staged in the pinned upload buffer (a pageable source
  // blocks the host once per copy); falls back to a direct copy when the
  // buffer is full.  The staged bytes are reused only after wait().
  hipError_t upload(void* dst, const void* src, size_t bytes) {
    if (cx_.direct) {
      // from pageable memory that the caller may change right after: wait
      hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_);
      return e == hipSuccess ? hipStreamSynchronize(st_) : e;
    }
    if (!cx_.pin_up) {
      if (hipHostMalloc(&cx_.pin_up, kPinUpload, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        cx_.pin_up = nullptr;
      }
    }
    const size_t off = (up_used_ + 255) & ~(size_t)255;
    if (!cx_.pin_up || off + bytes > kPinUpload)
      return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_);
    std::memcpy(static_cast<char*>(cx_.pin_up) + off, src, bytes);
    up_used_ = off + bytes;
    return hipMemcpyAsync(dst, static_cast<char*>(cx_.pin_up) + off, bytes, hipMemcpyHostToDevice, st_);
  }
  static constexpr size_t kPinUpload = 256 << 10;

 private:
  struct Item {
    void* dst;
    size_t off, bytes;
  };
  static constexpr int kMaxItems = 8;
  Ctx::Pins& cx_;
  hipStream_t st_;
  hipEvent_t ev_;
  bool ended_ = false;
  Item items_[kMaxItems];
  int nitems_ = 0;
  size_t used_ = 0;
  size_t up_used_ = 0, up_end_ = 0;
};
constexpr size_t kSmallReadback = 1 << 16;

// contexts per (device, slot): slot 0 serves the single-graph calls, slots
// 1.. the workers of girg_generate_batch (each with its own stream).  The map
// is never destroyed: a context's destructor calls HIP, whose runtime (and a
// profiler attached to it) may already be shut down when static objects are
// destroyed at process exit.  girg_release frees a device's contexts.
static std::mutex g_ctx_mu;
static auto& g_ctx = *new std::map<std::pair<int, int>, std::unique_ptr<Ctx>>();

static girg_status get_ctx(Ctx** out, int slot = 0) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  auto it = g_ctx.find({dev, slot});
  if (it != g_ctx.end()) {
    *out = it->second.get();
    return GIRG_OK;
  }
  std::unique_ptr<Ctx> c(new Ctx());
  c->device = dev;
  HIPCHK(hipMalloc(&c->gd, sizeof(Graph)));
  HIPCHK(hipMalloc(&c->red, 8 * sizeof(double)));
  HIPCHK(hipMalloc(&c->red_side, 8 * sizeof(double)));
  HIPCHK(hipMalloc(&c->flag, sizeof(uint32_t)));
  HIPCHK(hipMalloc(&c->stats, 16 * sizeof(unsigned long long)));
  HIPCHK(hipMalloc(&c->hcount, sizeof(unsigned int)));
  if (slot > 0) HIPCHK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->rb_done, hipEventDisableTiming));
  c->batch = slot > 0;
  // single-graph calls only: the batch's workers already fill the GPU, and
  // twice as many streams on the few hardware queues slowed the batch down
  if (slot == 0) {
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
  }
  *out = c.get();
  g_ctx[{dev, slot}] = std::move(c);
  return GIRG_OK;
}

// side stream: starts after the work queued on st so far; st continues only
// after the work queued on the side stream
// If a call returns between a fork and its join (an error), the guard waits
// for the side stream, so that no kernel still reads scratch memory that the
// next call reuses.
struct SideGuard {
  Ctx& cx;
  bool armed = false;
  ~SideGuard() {
    if (armed) (void)hipStreamSynchronize(cx.side);
  }
};
// work queued on a stream ahead of a host wait for an earlier point of it:
// a call that returns meanwhile (an error) lets that work end first, since
// it uses scratch memory that the next call reuses
struct StreamGuard {
  hipStream_t st;
  bool armed = false;
  ~StreamGuard() {
    if (armed) (void)hipStreamSynchronize(st);
  }
};

static hipError_t fork_side(Ctx& cx, hipStream_t st, bool on, SideGuard& gd) {
  if (!on) return hipSuccess;
  gd.armed = true;
  hipError_t e = hipEventRecord(cx.fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(cx.side, cx.fork, 0);
  return e;
}
static hipError_t join_side(Ctx& cx, hipStream_t st, bool on, SideGuard& gd) {
  if (!on) return hipSuccess;
  hipError_t e = hipEventRecord(cx.join, cx.side);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, cx.join, 0);
  if (e == hipSuccess) gd.armed = false;
  return e;
}

static int bitlen(uint64_t v) {
  int b = 0;
  while (v) { ++b; v >>= 1; }
  return b;
}

// the sums over the weights outside the tail (w, w^2 / W, w^(1/T), (w^2 / W)^(1/T))
static void csolve_take_sums(const double* r, double T, CSolve* cs) {
  cs->out_w = r[0];
  cs->out_q1 = r[1];
  cs->out_p = T > 0.0 ? r[2] : 0.0;
  cs->out_q2 = T > 0.0 ? r[3] : 0.0;
}

// ---------------------------------------------------------------------------
// HRG radius from the average degree (not in the paper).  E[deg] =
// (n-1) E[p] over two independent points; with s = R - r the radial density
// is alpha sinh(alpha (R - s)) / (cosh(alpha R) - 1), and for a fixed pair of
// radii the angular average of p is (1/pi) int_0^pi p dphi, where
// cosh d = cosh(r1 - r2) + 2 sinh r1 sinh r2 sin^2(phi / 2).  Gauss-Legendre
// on panels in s (split where r1 + r2 = R) and in log phi around the angle
// at which d = R.
// ---------------------------------------------------------------------------
namespace rsolve {
constexpr int kN = 12;
static double X[kN], Wt[kN];
static std::once_flag ready;  // the batch's workers may solve radii concurrently
static void init_nodes() {
  for (int i = 0; i < kN; ++i) {
    double z = std::cos(3.141592653589793 * (i + 0.75) / (kN + 0.5));
    for (int it = 0; it < 60; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= kN; ++k) { double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
      const double dp = kN * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        p0 = 1.0; p1 = z;
        for (int k = 2; k <= kN; ++k) { double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k; p0 = p1; p1 = p2; }
        const double dq = kN * (z * p1 - p0) / (z * z - 1.0);
        X[i] = z;
        Wt[i] = 2.0 / ((1.0 - z * z) * dq * dq);
        break;
      }
    }
  }
}
static void init() { std::call_once(ready, init_nodes); }
struct Q {
  double alpha, T, R, coshR, norm;
  double dens(double r) const { return alpha * std::sinh(alpha * r) / norm; }
  double p(double ch) const {
    if (T == 0.0) return ch < coshR ? 1.0 : 0.0;
    const double d = std::acosh(ch < 1.0 ? 1.0 : ch);
    return 1.0 / (std::exp((d - R) / (2.0 * T)) + 1.0);
  }
  double ang_panel(double base, double amp, double a, double b) const {
    double t = 0.0;
    const double hm = 0.5 * (b - a), mid = 0.5 * (a + b);
    for (int k = 0; k < kN; ++k) {
      const double s = std::sin(0.5 * (mid + hm * X[k]));
      t += Wt[k] * p(base + amp * s * s);
    }
    return t * hm;
  }
  double angular(double r1, double r2) const {
    const double base = std::cosh(r1 - r2), amp = 2.0 * std::sinh(r1) * std::sinh(r2);
    const double pi = 3.141592653589793;
    double s2 = amp > 0.0 ? (coshR - base) / amp : (base < coshR ? 2.0 : -1.0);
    double phs = s2 >= 1.0 ? pi : (s2 <= 0.0 ? 0.0 : 2.0 * std::asin(std::sqrt(s2)));
    if (T == 0.0) return phs / pi;
    double t = 0.0;
    if (phs <= 0.0 || phs >= pi) {
      for (int q = 0; q < 6; ++q) t += ang_panel(base, amp, pi * q / 6.0, pi * (q + 1) / 6.0);
      return t / pi;
    }
    // below phi*: panels shrinking towards phi*
    double a = 0.0;
    for (int q = 0; q < 4; ++q) {
      const double b = phs * (1.0 - std::ldexp(1.0, -(q + 1)));
      t += ang_panel(base, amp, a, b);
      a = b;
    }
    t += ang_panel(base, amp, a, phs);
    // above phi*: geometric panels (ratio 1.6)
    a = phs;
    while (a < pi) {
      const double b = std::min(pi, a * 1.6);
      t += ang_panel(base, amp, a, b);
      a = b;
    }
    return t / pi;
  }
};

static double inner(const Q& q, double r1, double a, double b) {
  if (b <= a) return 0.0;
  const int np = std::max(1, (int)std::ceil((b - a) / 0.75));
  double t = 0.0;
  for (int k = 0; k < np; ++k) {
    const double pa = a + (b - a) * k / np, pb = a + (b - a) * (k + 1) / np;
    const double hm = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
    for (int i = 0; i < kN; ++i) {
      const double r2 = mid + hm * X[i];
      t += hm * Wt[i] * q.dens(r2) * q.angular(r1, r2);
    }
  }
  return t;
}

static double expected_degree(uint64_t n, double alpha, double T, double R) {
  init();
  Q q{alpha, T, R, std::cosh(R), std::cosh(alpha * R) - 1.0};
  const int np = std::max(1, (int)std::ceil(R / 0.75));
  double t = 0.0;
  for (int k = 0; k < np; ++k) {
    const double pa = R * k / np, pb = R * (k + 1) / np;
    const double hm = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
    for (int i = 0; i < kN; ++i) {
      const double r1 = mid + hm * X[i];
      const double kink = R - r1;
      t += hm * Wt[i] * q.dens(r1) * (inner(q, r1, 0.0, kink) + inner(q, r1, kink, R));
    }
  }
  return (double)(n - 1) * t;
}

// secant steps on log E[deg] inside a bisection bracket
static int solve(uint64_t n, double alpha, double T, double target, double* out) {
  double lo = std::log((double)n), hi = 2.0 * lo;
  double flo = std::log(expected_degree(n, alpha, T, lo) / target);
  double fhi = std::log(expected_degree(n, alpha, T, hi) / target);
  int it = 0;
  while (flo < 0.0) { hi = lo; fhi = flo; lo *= 0.5; flo = std::log(expected_degree(n, alpha, T, lo) / target); if (++it > 100) return -1; }
  while (fhi > 0.0) { lo = hi; flo = fhi; hi *= 1.5; fhi = std::log(expected_degree(n, alpha, T, hi) / target); if (++it > 200) return -1; }
  for (it = 0; it < 100 && hi - lo > 1e-12 * hi; ++it) {
    double mid = lo + (hi - lo) * flo / (flo - fhi);
    const double span = hi - lo;
    if (!(mid > lo + 0.01 * span && mid < hi - 0.01 * span)) mid = 0.5 * (lo + hi);
    const double fm = std::log(expected_degree(n, alpha, T, mid) / target);
    if (fm == 0.0) { lo = hi = mid; break; }
    if (fm > 0.0) { lo = mid; flo = fm; } else { hi = mid; fhi = fm; }
  }
  *out = 0.5 * (lo + hi);
  return 0;
}
}  // namespace rsolve

// memo of solved radii: R is a pure function of (n, alpha, T, avg_deg)
static std::mutex g_rmemo_mu;
static std::map<std::vector<double>, double> g_rmemo;

static girg_status solve_R_cached(uint64_t n, double alpha, double T, double deg, double* R) {
  const std::vector<double> key{(double)n, alpha, T, deg};
  {
    std::lock_guard<std::mutex> lk(g_rmemo_mu);
    auto it = g_rmemo.find(key);
    if (it != g_rmemo.end()) { *R = it->second; return GIRG_OK; }
  }
  if (rsolve::solve(n, alpha, T, deg, R) != 0) return fail(GIRG_ENOCONV, "hrg_solve_R: no bracket");
  std::lock_guard<std::mutex> lk(g_rmemo_mu);
  g_rmemo[key] = *R;
  return GIRG_OK;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static girg_status validate(const girg_params& p, bool need_beta) {
  if (p.n < 2 || p.n > 0xFFFFFFFFull) return fail(GIRG_EINVAL, "n must be in [2, 2^32-1]");
  if (!(p.T >= 0.0 && p.T < 1.0)) return fail(GIRG_EINVAL, "T must be in [0, 1)");
  if (p.precision != 0 && p.precision != 1) return fail(GIRG_EINVAL, "precision must be 0 or 1");
  if (p.type2_batch != 0 && p.type2_batch != 1) return fail(GIRG_EINVAL, "type2_batch must be 0 or 1");
  if (p.model == 0) {
    if (p.d < 1 || p.d > 4) return fail(GIRG_EINVAL, "d must be in [1, 4]");
    if (need_beta && !(p.beta > 2.0)) return fail(GIRG_EINVAL, "beta must be > 2");
    const bool hasc = p.c > 0.0, hasd = p.avg_deg > 0.0;
    if (hasc == hasd) return fail(GIRG_EINVAL, "exactly one of c > 0 and avg_deg > 0 is required");
    if (p.T > 0.0 && p.avg_deg > 0.0 && p.T < 0.05)
      return fail(GIRG_EINVAL, "solving c needs T = 0 or T >= 0.05; pass c instead");
  } else if (p.model == 1) {
    if (!(p.alpha > 0.5)) return fail(GIRG_EINVAL, "alpha must be > 1/2");
    if (!(p.R > 0.0) && !(p.avg_deg > 0.0)) return fail(GIRG_EINVAL, "R > 0 or avg_deg > 0 is required");
  } else {
    return fail(GIRG_EINVAL, "model must be 0 (GIRG) or 1 (HRG)");
  }
  if (p.T == 0.0 && p.cl_bias > 0) return fail(GIRG_EINVAL, "cl_bias > 0 is inexact at T = 0");
  if (p.cl_bias < -64 || p.cl_bias > 64) return fail(GIRG_EINVAL, "cl_bias out of range");
  return GIRG_OK;
}

// ---------------------------------------------------------------------------
// the sampler over resident points
// ---------------------------------------------------------------------------
// Output placement for batches: called with the edge count once it is known;
// returns where to write them (nullptr: nowhere, the count is still returned).
using Place = std::function<uint32_t*(uint64_t m)>;

static girg_status run_graph(Ctx& cx, const girg_params& p, const double* w, const double* x,
                             uint32_t* edges, uint64_t cap, uint64_t* m_out, girg_info* info,
                             hipStream_t st, const Place* place = nullptr) {
  Arena& ar = cx.ar;
  Graph g;
  std::memset(&g, 0, sizeof(g));
  g.n = (uint32_t)p.n;
  g.model = p.model;
  g.d = p.model == 1 ? 1 : p.d;
  g.Dmax = 32 / g.d;
  g.bits = g.d * g.Dmax;
  g.cl_bias = p.cl_bias;
  g.max_depth = p.max_depth;
  g.precision = p.precision;
  g.T = p.T;
  g.inv_T = p.T > 0.0 ? 1.0 / p.T : 0.0;
  g.alpha = p.alpha;
  g.R = p.R;
  g.coshR = p.model == 1 ? std::cosh(p.R) : 0.0;
  if (p.model == 1 && p.T > 0.0) {
    // p_T(d) = x at d = R + 2T ln(1/x - 1)
    for (int m = 0; m < kHrgTab; ++m) {
      const double x = (double)m / (kHrgTab - 1);
      double c = 0.0;
      if (m == 0) c = INFINITY;
      else if (m < kHrgTab - 1) {
        const double dx = p.R + 2.0 * p.T * std::log(1.0 / x - 1.0);
        c = dx > 0.0 ? std::cosh(dx) : 0.0;
      }
      g.hct[m] = c;
    }
  }
  g.seed_lo = (uint32_t)p.seed;
  g.seed_hi = (uint32_t)(p.seed >> 32);
  const uint64_t n = p.n;
  const int d = g.d;
  if (cx.ev_name.empty()) cx.mark("-", st);

  // exact sum W and min / max of w (GIRG) or r (HRG), then the layer and
  // Morton keys.  W and w0 reach the device Graph from the reduction on the
  // device, so both are read back in one group; the keys of invalid input are
  // computed but never used (the checks below reject it first).
  Readback rb(cx, st);
  for (int i = 0; i < kMaxLayers; ++i) {
    g.ext[i] = p.model == 0 ? 0.0 : __builtin_inf();
  }
  HIPCHK(rb.upload(cx.gd, &g, sizeof(Graph)));
  HIPCHK(hipMemsetAsync(cx.flag, 0, sizeof(uint32_t), st));
  uint64_t* keys = ar.get<uint64_t>(n);
  uint32_t* ids = ar.get<uint32_t>(n);
  double* pts = ar.get<double>(n * (uint64_t)pts_stride(d, p.model));
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (keys)");
  HIPCHK(reduce_terms(ar, w, n, p.model == 0 ? 1 : 0, 0, 1.0, 0.0, cx.red, st));
  if (p.model == 0) HIPCHK(launch_set_weight_sums(cx.gd, cx.red, st));
  cx.mark("-", st);
  HIPCHK(launch_layer_key(g, cx.gd, w, x, keys, ids, pts, cx.flag, st));
  cx.mark("layer_key", st);
  double red[6];
  uint32_t flag = 0;
  HIPCHK(rb.begin(kSmallReadback));
  HIPCHK(rb.add(red, cx.red, sizeof(red)));
  HIPCHK(rb.add(&flag, cx.flag, sizeof(uint32_t)));
  HIPCHK(rb.add(g.count, cx.gd->count, sizeof(g.count)));
  HIPCHK(rb.add(g.ext, cx.gd->ext, sizeof(g.ext)));
  HIPCHK(rb.end());

  // Neither the c solve's first round (it reads the weights and the sums) nor
  // the sort by (layer, Morton code) and the gather need this readback, so
  // they are queued before the host waits for it: the side stream starts
  // from here, and the main stream sorts while the host checks the input.
  // The layer field of the keys is taken 6 bits wide (at most 64 layers); a
  // key has at most 32 + 6 bits, which keeps the number of radix passes.
  const bool csolve = p.model == 0 && !(p.c > 0.0);
  hipStream_t scs = cx.side ? cx.side : st;
  SideGuard cs_guard{cx};
  StreamGuard early{st};
  if (csolve) HIPCHK(fork_side(cx, st, cx.side != nullptr, cs_guard));
  cx.mark("-", st);
  early.armed = true;
  HIPCHK(radix_sort(ar, keys, ids, n, g.bits + 6, st));
  cx.mark("sort", st);
  double* sw = ar.get<double>(n);
  double* rec = ar.get<double>(n * (uint64_t)rec_stride(d, p.model));
  uint32_t* smort = ar.get<uint32_t>(n);
  uint8_t* slayer = ar.get<uint8_t>(n);
  // the mixed path's 16-byte FP32 filter records (GIRG, T > 0, d <= 3)
  const bool frecs = p.precision == 1 && p.model == 0 && p.T > 0.0 && d <= 3;
  uint4* frec = frecs ? ar.get<uint4>(n) : nullptr;
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (sorted arrays)");
  HIPCHK(launch_gather(g, cx.gd, keys, ids, pts, sw, rec, smort, slayer, frec, st));
  cx.mark("gather", st);
  HIPCHK(rb.wait());
  if (p.model == 0) {
    if (!(red[4] > 0.0) || !std::isfinite(red[5]))
      return fail(GIRG_EINVAL, "weights must be finite and > 0");
    g.W = red[0];
    g.w0 = red[4];
    if (bitlen((uint64_t)std::min(red[5] / red[4], 1e19)) > kMaxLayers)
      return fail(GIRG_EINVAL, "weight range exceeds 2^64");
  } else {
    if (!(red[4] >= 0.0) || !(red[5] <= p.R)) return fail(GIRG_EINVAL, "radii must lie in [0, R]");
  }
  if (flag & 1u) return fail(GIRG_EINVAL, p.model == 0 ? "weights must be finite and > 0" : "radii must lie in [0, R]");
  if (flag & 2u) return fail(GIRG_EINVAL, "more than 64 weight layers");
  if (flag & 4u) return fail(GIRG_EINVAL, "positions must lie in [0,1)");
  g.L = 0;
  uint32_t acc = 0;
  for (int i = 0; i < kMaxLayers; ++i) {
    g.lstart[i] = acc;
    acc += (uint32_t)g.count[i];
    if (g.count[i] > 0) g.L = i + 1;
  }
  g.lstart[kMaxLayers] = acc;

  // constant c (App. B.2).  It needs only the heaviest weights (the tail,
  // sorted by value) and sums over the others, both from the unsorted
  // weights, so its first round runs on the side stream (with its own arena,
  // result slots and pinned buffers) while the main stream sorts and gathers.
  // Further rounds, when E_R needs a longer tail, run after the gather.
  Readback rbs(cx, scs, true);
  CSolve& cs = cx.cs;
  int i0 = g.L;
  std::vector<double>& asc = cx.cs_asc;
  std::vector<double>& ascp = cx.cs_ascp;
  double rs[6];
  auto cs_round = [&]() -> girg_status {
    // the tail (layers >= i0), sorted by value, its powers w^(1/T), and the
    // sums over the layers below i0: one readback
    const uint64_t K = n - g.lstart[i0];
    cx.ar_side.reset_all();
    Arena& a2 = cx.ar_side;
    uint64_t* tk = a2.get<uint64_t>(K);
    uint32_t* tv = a2.get<uint32_t>(K);
    unsigned int* tcnt = a2.get<unsigned int>(1);
    double* tp = p.T > 0.0 ? a2.get<double>(K) : nullptr;
    if (a2.failed()) {
      a2.clear_failure();
      return fail(GIRG_ENOMEM, "scratch allocation failed (c solve)");
    }
    HIPCHK(hipMemsetAsync(tcnt, 0, sizeof(unsigned int), scs));
    HIPCHK(launch_tail_collect(w, n, g.w0, i0, tk, tcnt, (uint32_t)K, scs));
    HIPCHK(launch_iota(tv, K, scs));
    HIPCHK(radix_sort(a2, tk, tv, K, 64, scs));  // positive doubles order as integers
    if (tp) HIPCHK(launch_pow_bits(tk, tp, K, 1.0 / p.T, scs));
    const double invT = p.T > 0.0 ? 1.0 / p.T : 0.0;
    HIPCHK(reduce_terms(a2, w, n, p.T > 0.0 ? 4 : 2, 0, g.W, invT, cx.red_side, scs, g.w0, i0));
    asc.assign(K, 0.0);
    ascp.assign(tp ? K : 0, 0.0);
    HIPCHK(rbs.begin(2 * K * sizeof(double) + 4096));
    HIPCHK(rbs.add(asc.data(), tk, K * sizeof(double)));
    if (tp) HIPCHK(rbs.add(ascp.data(), tp, K * sizeof(double)));
    HIPCHK(rbs.add(rs, cx.red_side, 6 * sizeof(double)));
    return GIRG_OK;
  };
  if (csolve) {
    cs.n = n; cs.d = d; cs.T = p.T; cs.W = g.W;
    // heaviest layers first, at least 1024 weights
    uint64_t tail = 0;
    while (i0 > 0 && tail < 1024) { --i0; tail += (uint64_t)g.count[i0]; }
    girg_status s = cs_round();  // on the side stream, forked before the sort
    if (s != GIRG_OK) return s;
  }

  cx.mark("-", st);
  if (p.model == 0) {
    double c = p.c;
    if (csolve) {
      for (;;) {
        HIPCHK(rbs.wait());  // the side stream's round (or st's, with no side stream)
        const uint64_t K = asc.size();
        csolve_take_sums(rs, p.T, &cs);
        cs.h.assign(asc.rbegin(), asc.rend());
        cs.hp.assign(ascp.rbegin(), ascp.rend());
        if (p.T <= 0.0) cs.hp.assign(K, 0.0);
        cs.wcut = 0.0;
        for (int i = i0 - 1; i >= 0; --i)
          if (g.count[i] > 0) { cs.wcut = g.ext[i]; break; }
        cs.prepare(true);
        // (a later round starts from the c of the round before)
        if (cs.solve(p.avg_deg, &c, c) != 0) return fail(GIRG_ENOCONV, "c solve found no bracket");
        if (cs.complete_at(c) || i0 == 0) break;
        // take every layer whose largest weight could pair with the heaviest
        // vertex inside E_R at this c, with a factor 2 of margin for the next
        // solve's c (the next lower layer fails that test, so this grows)
        const double cut = 0.5 * cs.th(c) / cs.h[0];
        while (i0 > 0 && (g.count[i0 - 1] == 0 || g.ext[i0 - 1] > cut)) --i0;
        girg_status s = cs_round();
        if (s != GIRG_OK) return s;
      }
      HIPCHK(join_side(cx, st, cx.side != nullptr, cs_guard));
    }
    g.c = c;
    g.kappa = p.T > 0.0 ? std::pow(c, p.T) : std::pow(c, (double)d);
    if (p.T > 0.0) {
      g.C32 = (float)(std::log2(c) - g.inv_T * std::log2(g.W));
      g.invT32 = (float)g.inv_T;
    }
  }
  cx.mark("c_solve", st);

  // level tables
  const int Dcap = std::min(g.Dmax, (bitlen(n) + 3) / d);
  const int nlev = Dcap + 1;
  Pbar* pbt = nullptr;
  if (p.T > 0.0) {
    pbt = ar.get<Pbar>((uint64_t)std::max(g.L, 1) * std::max(g.L, 1) * nlev * 2);
    if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (pbar)");
  }
  tables_host(g, Dcap);
  HIPCHK(rb.upload(cx.gd, &g, sizeof(Graph)));
  cx.mark("-", st);
  HIPCHK(launch_pbar(cx.gd, g.L, Dcap, pbt, st));
  cx.mark("tables", st);

  // prefix sums per layer at its insertion level
  uint64_t cells = 0;
  for (int i = 0; i < kMaxLayers; ++i) {
    g.pbase[i] = cells;
    if (g.count[i] > 0) cells += (1ull << (d * g.I[i])) + 1;
  }
  g.cells = cells;
  if (cells >= 0xFFFFFFFFull * 4) return fail(GIRG_ENOMEM, "too many cells");
  // per-cell layer sets per level up to the deepest insertion level
  int maxI = 0;
  for (int i = 0; i < g.L; ++i)
    if (g.count[i] > 0 && g.I[i] > maxI) maxI = g.I[i];
  g.moff[0] = 0;
  for (int l = 0; l < kMaxLevels; ++l)
    g.moff[l + 1] = g.moff[l] + (l <= maxI ? (1ull << (d * l)) : 0ull);
  HIPCHK(rb.upload(cx.gd->pbase, g.pbase, sizeof(g.pbase)));
  HIPCHK(rb.upload(cx.gd->moff, g.moff, sizeof(g.moff)));
  uint32_t* P = ar.get<uint32_t>(cells);
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (cells)");
  cx.mark("-", st);
  HIPCHK(hipMemsetAsync(P, 0, cells * sizeof(uint32_t), st));
  HIPCHK(launch_cell_count(g, cx.gd, smort, slayer, P, st));
  HIPCHK(scan_u32(ar, P, P, cells, nullptr, st));
  cx.mark("cells", st);

  // run sources
  uint32_t* scnt = ar.get<uint32_t>(n + 1);
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (sources)");
  HIPCHK(launch_sources(g, cx.gd, smort, slayer, P, scnt, nullptr, nullptr, nullptr, false, st));
  HIPCHK(scan_u32(ar, scnt, scnt, n, scnt + n, st));
  cx.mark("sources_count", st);
  uint32_t nsrc = 0;
  HIPCHK(rb.begin(kSmallReadback));
  HIPCHK(rb.add(&nsrc, scnt + n, sizeof(uint32_t)));
  HIPCHK(rb.wait());
  early.armed = false;  // the main stream has drained
  Src* src = ar.get<Src>(std::max<uint64_t>(nsrc, 1));
  const uint64_t ncl = g.moff[kMaxLevels];
  CellL* cl = ar.get<CellL>(ncl);
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (sources)");
  cx.mark("-", st);
  HIPCHK(hipMemsetAsync(cl, 0, ncl * sizeof(CellL), st));
  HIPCHK(launch_sources(g, cx.gd, smort, slayer, P, nullptr, scnt, src, cl, true, st));
  // (first, count) records of every cell's layers: popcounts, scan, ranks
  uint32_t* ccnt = ar.get<uint32_t>(ncl + 1);
  uint2* crec = ar.get<uint2>(std::max<uint64_t>(nsrc, 1));
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (cell layers)");
  HIPCHK(launch_cell_layers(cx.gd, cl, ncl, ccnt, src, nsrc, crec, false, st));
  HIPCHK(scan_u32(ar, ccnt, ccnt, ncl, nullptr, st));
  HIPCHK(launch_cell_layers(cx.gd, cl, ncl, ccnt, src, nsrc, crec, true, st));
  cx.mark("sources_fill", st);
  if (!cx.dtab[d]) {
    const std::vector<uint32_t> tab = distant_table(d);
    if (tab.empty()) return fail(GIRG_EDEVICE, "distant-offset table rows shorter than a wave");
    uint32_t* t = nullptr;
    HIPCHK(hipMalloc(&t, tab.size() * sizeof(uint32_t)));
    HIPCHK(hipMemcpyAsync(t, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    cx.dtab[d] = t;
  }
  // batched type-II sequences at levels >= 3 (GIRG, d = 2, 3, T > 0)
  const bool batched = p.type2_batch == 1 && p.T > 0.0 && p.model == 0 && (d == 2 || d == 3);
  if (batched && g.L > 32) return fail(GIRG_EINVAL, "type2_batch = 1 needs at most 32 weight layers");
  if (batched && !cx.dtab2[d]) {
    std::vector<uint32_t> tab(seq_table_fill(d, nullptr, 0), 0u);
    if (tab.empty()) return fail(GIRG_EDEVICE, "sequence offset table longer than the kernel holds");
    seq_table_fill(d, tab.data(), tab.size());
    uint32_t* t = nullptr;
    HIPCHK(hipMalloc(&t, tab.size() * sizeof(uint32_t)));
    HIPCHK(hipMemcpyAsync(t, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    cx.dtab2[d] = t;
  }

  Verts v{rec, ids, smort, slayer, frec};
  const bool binomial = p.T > 0.0;

  // staging of the edges: capacity = the caller's; flush records.  The
  // counters sit in one block, cleared by one memset per attempt, 256 bytes
  // apart (atomics of all waves on one cache line slow every pass down):
  // tickets[0..7], deferred counts[64..65], flush records[128], near-boundary
  // candidates[160], cursor (u64) at 192
  unsigned int* ctr = ar.get<unsigned int>(256);
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (counters)");
  unsigned int* tickets = ctr;
  unsigned int* dcount = ctr + 64;
  unsigned int* nrec_d = ctr + 128;
  unsigned int* ncnt = ctr + 160;
  unsigned long long* cursor = reinterpret_cast<unsigned long long*>(ctr + 192);
  // type I (and its split pass) on the side stream, concurrently with type II
  // (and its segments); profiled calls time each pass on its own stream
  const bool overlap = cx.side != nullptr && !(cx.profiling && cx.serial);
  hipStream_t s1 = overlap ? cx.side : st;
  SideGuard sguard{cx};
  // persistent grids: the tuned number of workgroups, at most one wave per chunk
  const uint32_t gblocks = cx.fixed_tuning ? default_blocks(tune_key(p.model, g.d, p.T, p.n))
                                           : tuned_blocks(tune_key(p.model, g.d, p.T, p.n), cx.batch);
  auto grid_for = [&](uint32_t nchunks) {
    const uint32_t need = (nchunks + kWavesPerBlock - 1) / kWavesPerBlock;
    return std::max<uint32_t>(1u, std::min<uint32_t>(gblocks, need));
  };
  auto make_sched = [&](uint64_t nunits, int pass) {
    uint64_t ch = (nunits + 16383) / 16384;
    ch = ((ch + 63) / 64) * 64;
    ch = std::max<uint64_t>(64, std::min<uint64_t>(4096, ch));
    const uint32_t nch = (uint32_t)((nunits + ch - 1) / ch);
    Sched sc{tickets + pass, nunits, (uint32_t)ch, nch, (uint32_t)pass, nullptr, nullptr, grid_for(nch)};
    return sc;
  };
  // type-I and type-II chunks are runs of whole sources
  auto make_sched_src = [&](uint64_t nunits, int pass) {
    uint64_t ch = (nunits + 16383) / 16384;
    ch = std::max<uint64_t>(1, std::min<uint64_t>(64, ch));
    const uint32_t nch = (uint32_t)((nunits + ch - 1) / ch);
    Sched sc{tickets + pass, nunits, (uint32_t)ch, nch, (uint32_t)pass, nullptr, nullptr, grid_for(nch)};
    return sc;
  };
  Sched sch[4] = {make_sched_src(nsrc, 0), make_sched(0, 1),
                  make_sched_src(binomial ? nsrc : 0, 2), make_sched(0, 3)};
  // the type-II pass's chunks: those of k_type2, then (batched) as many of
  // k_type2s over the same sources
  const uint32_t nch2 = sch[2].nchunks * (batched ? 2u : 1u);
  for (int q = 0; q <= 2; q += 2) {
    const uint32_t nc = q == 2 ? nch2 : sch[q].nchunks;
    sch[q].ctot = ar.get<uint64_t>(nc);
    sch[q].dtot = ar.get<uint64_t>(nc);
  }
  uint2* stage = cap ? ar.get<uint2>(cap) : nullptr;
  // every flush but the last of a chunk holds more than 128 edges
  const uint64_t rcap64 = cap / 128 + 2ull * (sch[0].nchunks + nch2) + (1u << 16);
  const uint32_t rcap = (uint32_t)std::min<uint64_t>(rcap64, 0xFFFFFFF0ull);
  uint64_t* rtag = ar.get<uint64_t>(rcap);
  uint64_t* roff = ar.get<uint64_t>(rcap);
  uint64_t* rpos = ar.get<uint64_t>(rcap);
  uint32_t* rcnt = ar.get<uint32_t>(rcap);
  // type-II candidates whose coin lies within 1e-12 of p_uv (expected far
  // fewer than the list holds)
  constexpr uint32_t kNearCap = 1u << 16;
  uint4* nbuf = binomial ? ar.get<uint4>(kNearCap) : nullptr;
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (edge staging)");
  Stage sg{stage, cap, cursor, rtag, roff, rpos, rcnt, nrec_d, rcap, cx.stats, nbuf, ncnt,
           binomial ? kNearCap : 0u};

  // type-I and type-II passes (deferred lists grown once if too small)
  // first capacity: half an entry per source (the workloads measured defer up to
  // about 0.1 per source and per list), at most 2^27; GIRG_DEFER_CAPACITY
  // overrides it, e.g. to exercise the growth
  uint64_t dcap0 = std::min<uint64_t>(std::max<uint64_t>(1u << 16, nsrc / 2 + 1024), 1ull << 27);
  if (const char* ev = std::getenv("GIRG_DEFER_CAPACITY")) {
    const long long v = std::atoll(ev);
    if (v >= 1 && v <= (1ll << 30)) dcap0 = (uint64_t)v;
  }
  uint32_t dcap[2] = {(uint32_t)dcap0, (uint32_t)dcap0};
  ItemRec* drec[2] = {nullptr, nullptr};
  uint64_t* dkey[2] = {nullptr, nullptr};
  unsigned int dn[2] = {0, 0};
  for (int attempt = 0; attempt < 2; ++attempt) {
    Arena::Mark mk = ar.mark();
    for (int q = 0; q < 2; ++q) {
      drec[q] = ar.get<ItemRec>(dcap[q]);
      dkey[q] = ar.get<uint64_t>(dcap[q]);
    }
    if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (deferred items)");
    HIPCHK(hipMemsetAsync(ctr, 0, 256 * sizeof(unsigned int), st));
    HIPCHK(hipMemsetAsync(cx.stats, 0, 16 * sizeof(unsigned long long), st));
    DeferOut df0{drec[0], dkey[0], dcount + 0, dcap[0], p.T > 0.0 ? kBigTests : kBigTestsT0};
    DeferOut df1{drec[1], dkey[1], dcount + 1, dcap[1], 0u};
    cx.mark("-", st);
    HIPCHK(fork_side(cx, st, overlap, sguard));
    cx.mark("-", s1);
    if (sch[0].nchunks) HIPCHK(launch_type1(g, cx.gd, v, cl, crec, src, sch[0], sg, df0, s1));
    cx.mark("type1", s1);
    cx.mark("-", st);
    if (sch[2].nchunks) {
      HIPCHK(launch_type2(g, cx.gd, v, cl, crec, src, sch[2], pbt, nlev, cx.dtab[d], sg, df1,
                          batched ? 3u : 255u, st));
      if (batched) {
        Sched s2 = sch[2];
        s2.next = tickets + 4;
        s2.ctot = sch[2].ctot + sch[2].nchunks;
        s2.dtot = sch[2].dtot + sch[2].nchunks;
        HIPCHK(launch_type2s(g, cx.gd, v, cl, crec, src, s2, pbt, nlev, cx.dtab2[d], sg, df1,
                             sch[2].nchunks, st));
      }
    }
    cx.mark("type2", st);
    HIPCHK(join_side(cx, st, overlap, sguard));
    // where each chunk's deferred items start
    HIPCHK(seg_scan_u64(ar, SegScan{{sch[0].dtot, sch[2].dtot, nullptr, nullptr},
                                {sch[0].nchunks, nch2, 0, 0}, 3u},
                        st));
    HIPCHK(rb.begin(kSmallReadback));
    HIPCHK(rb.add(dn, dcount, 2 * sizeof(unsigned int)));
    HIPCHK(rb.wait());
    if (dn[0] <= dcap[0] && dn[1] <= dcap[1]) break;
    if (attempt == 1) return fail(GIRG_ENOMEM, "deferred item lists overflowed");
    ar.reset(mk);
    dcap[0] = std::max(dcap[0], dn[0]);
    dcap[1] = std::max(dcap[1], dn[1]);
  }

  // deferred items in (chunk, sequence) order, their work units, then their passes
  ItemRec* dsorted[2] = {nullptr, nullptr};
  uint64_t* uoff[2] = {nullptr, nullptr};
  uint64_t nunits[2] = {0, 0};
  cx.mark("-", st);
  HIPCHK(rb.begin(kSmallReadback));
  for (int q = 0; q < 2; ++q) {
    const uint32_t nd = dn[q];
    if (!nd) continue;
    dsorted[q] = ar.get<ItemRec>(nd);
    uoff[q] = ar.get<uint64_t>(nd + 1);
    if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (deferred items)");
    HIPCHK(launch_defer_place(drec[q], dkey[q], nd, sch[q == 0 ? 0 : 2].dtot, dsorted[q], st));
    HIPCHK(launch_rec_units(dsorted[q], nd, q == 0 ? 1 : 2, uoff[q], st));
    HIPCHK(scan_u64(ar, uoff[q], uoff[q], nd, uoff[q] + nd, st));
    HIPCHK(rb.add(nunits + q, uoff[q] + nd, sizeof(uint64_t)));
  }
  if (dn[0] || dn[1]) HIPCHK(rb.wait());
  cx.mark("deferred_prep", st);
  sch[1] = make_sched(nunits[0], 1);
  sch[3] = make_sched(nunits[1], 3);
  for (int q = 1; q <= 3; q += 2) sch[q].ctot = ar.get<uint64_t>(sch[q].nchunks);
  if (ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (deferred passes)");
  HIPCHK(fork_side(cx, st, overlap, sguard));
  cx.mark("-", s1);
  if (sch[1].nchunks) HIPCHK(launch_big1(g, cx.gd, v, dsorted[0], uoff[0], dn[0], sch[1], sg, s1));
  cx.mark("split1", s1);
  cx.mark("-", st);
  if (sch[3].nchunks)
    HIPCHK(launch_heavy2(g, cx.gd, v, dsorted[1], uoff[1], dn[1], sch[3], pbt, nlev, sg, st));
  cx.mark("segments2", st);
  HIPCHK(join_side(cx, st, overlap, sguard));
  cx.mark("-", st);
  if (binomial) HIPCHK(launch_near2(g, cx.gd, v, pbt, nlev, sg, st));
  // where each chunk's edges start, in pass order
  HIPCHK(seg_scan_u64(ar, SegScan{{sch[0].ctot, sch[1].ctot, sch[2].ctot, sch[3].ctot},
                              {sch[0].nchunks, sch[1].nchunks, nch2, sch[3].nchunks}, 1u},
                      st));

  // total, capacity, records, and the counters (final once the passes end)
  unsigned long long mtot = 0;
  unsigned int nrec = 0;
  unsigned long long stt[16];
  HIPCHK(rb.begin(kSmallReadback));
  HIPCHK(rb.add(&mtot, cursor, sizeof(mtot)));
  HIPCHK(rb.add(&nrec, nrec_d, sizeof(nrec)));
  HIPCHK(rb.add(stt, cx.stats, sizeof(stt)));
  HIPCHK(rb.wait());
  // the diagnostics (also for a counting call, which ends with GIRG_EOVERFLOW)
  if (info) {
    for (int q = 0; q < 4; ++q) info->pass_edges[q] = stt[8 + q];
    info->pass_work[0] = stt[0];
    info->pass_work[1] = stt[1];
    info->pass_work[2] = stt[2];
    info->pass_work[3] = stt[3];
    info->pass_cands[2] = stt[4];
    info->pass_cands[3] = stt[5];
    info->type1_edges = stt[8] + stt[9];
    info->type2_edges = stt[10] + stt[11];
    info->tests = stt[0] + stt[1];
    info->draws = stt[2] + stt[3];
    info->candidates = stt[4] + stt[5];
    info->rechecks = stt[6];
    info->near_boundary = stt[12];
    info->skip_ties = stt[13];
    info->sources = nsrc;
    info->heavy_items = dn[1];
    info->split_items = dn[0];
    info->cells = cells;
    info->c = g.c;
    info->W = g.W;
    info->R = g.R;
    info->L = g.L;
    info->D = g.D;
  }
  *m_out = mtot;
  if (info) info->m = mtot;
  if (mtot > cap) {
    cx.collect();  // stage times of a counting call (null buffer, capacity 0)
    return fail(GIRG_EOVERFLOW, "edge capacity too small");
  }
  if (nrec > rcap) return fail(GIRG_ENOMEM, "edge staging records overflowed");
  if (place) edges = (*place)(mtot);

  // staged blocks to their places: chunk start + edges of the chunk before
  if (nrec && edges) {
    const ChunkBases cbs{{sch[0].ctot, sch[1].ctot, sch[2].ctot, sch[3].ctot}};
    HIPCHK(launch_stage_copy(stage, rtag, roff, rpos, rcnt, nrec, cbs, mtot,
                             reinterpret_cast<uint2*>(edges), st));
    cx.mark("order", st);
  }

  HIPCHK(hipStreamSynchronize(st));
  cx.collect();
  return GIRG_OK;
}

// The context of (device, slot), locked for the whole call, then its arena
// cleared.  The reset must come after the lock: a call of another host thread
// may still be allocating from this arena until it releases the lock.
struct CtxLock {
  Ctx* cx = nullptr;
  std::unique_lock<std::mutex> lk;
};
static girg_status lock_ctx(CtxLock* out, int slot = 0) {
  girg_status s = get_ctx(&out->cx, slot);
  if (s != GIRG_OK) return s;
  out->lk = std::unique_lock<std::mutex>(out->cx->mu);
  out->cx->ar.reset_all();
  out->cx->ar.clear_failure();
  return GIRG_OK;
}

// ---------------------------------------------------------------------------
// the no-allocation variant of girg_from_points: every device buffer of a
// call lies in one fixed array of device memory, `scratch`, which each GPU
// holds from the library's first use on it until the process ends
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 512ull << 20;
constexpr uint64_t kNoAllocMaxN = 1ull << 20;
constexpr uint64_t kNoAllocMaxCap = 1ull << 24;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// per device: the address of its copy of `scratch` (the array's name is a
// host-side stand-in, not a device address) and a context whose buffers and
// arena are carved from it
constexpr int kNoAllocDevices = 16;
struct NoAllocSlot {
  bool ready = false;
  unsigned char* ptr = nullptr;
  Ctx cx;
};
static std::mutex g_na_mu;
static NoAllocSlot g_na[kNoAllocDevices];
// the distant-offset tables are built here on the host, then copied once
static uint32_t g_na_tab[1 << 14];

// set-up, once per device, with that device current
static girg_status noalloc_setup(int dev, NoAllocSlot** out) {
  if (dev < 0 || dev >= kNoAllocDevices)
    return fail(GIRG_EINVAL, "girg_from_points_noalloc: device index above 15");
  std::lock_guard<std::mutex> lk(g_na_mu);
  NoAllocSlot& sl = g_na[dev];
  if (!sl.ready) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(GIRG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    unsigned char* base = static_cast<unsigned char*>(ptr);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
      unsigned char* q = base + off;
      off += (bytes + 255) & ~(size_t)255;
      return q;
    };
    Ctx& c = sl.cx;
    c.device = dev;
    c.external = true;
    c.fixed_tuning = true;
    c.pins.direct = true;
    c.pins_side.direct = true;
    c.gd = reinterpret_cast<Graph*>(carve(sizeof(Graph)));
    c.red = reinterpret_cast<double*>(carve(8 * sizeof(double)));
    c.red_side = reinterpret_cast<double*>(carve(8 * sizeof(double)));
    c.flag = reinterpret_cast<uint32_t*>(carve(sizeof(uint32_t)));
    c.stats = reinterpret_cast<unsigned long long*>(carve(16 * sizeof(unsigned long long)));
    c.hcount = reinterpret_cast<unsigned int*>(carve(sizeof(unsigned int)));
    for (int d = 1; d <= 4; ++d) {
      const size_t sz = distant_table_fill(d, g_na_tab, sizeof(g_na_tab) / sizeof(uint32_t));
      if (sz == 0) return fail(GIRG_EDEVICE, "distant-offset table rows shorter than a wave");
      if (sz > sizeof(g_na_tab) / sizeof(uint32_t))
        return fail(GIRG_EDEVICE, "girg_from_points_noalloc: distant table larger than its buffer");
      uint32_t* t = reinterpret_cast<uint32_t*>(carve(sz * sizeof(uint32_t)));
      HIPCHK(hipMemcpy(t, g_na_tab, sz * sizeof(uint32_t), hipMemcpyHostToDevice));
      c.dtab[d] = t;
    }
    for (int d = 2; d <= 3; ++d) {
      const size_t sz = seq_table_fill(d, g_na_tab, sizeof(g_na_tab) / sizeof(uint32_t));
      if (sz == 0 || sz > sizeof(g_na_tab) / sizeof(uint32_t))
        return fail(GIRG_EDEVICE, "girg_from_points_noalloc: sequence table larger than its buffer");
      uint32_t* t = reinterpret_cast<uint32_t*>(carve(sz * sizeof(uint32_t)));
      HIPCHK(hipMemcpy(t, g_na_tab, sz * sizeof(uint32_t), hipMemcpyHostToDevice));
      c.dtab2[d] = t;
    }
    c.ar.attach(reinterpret_cast<char*>(base + off), kScratchBytes - off);
    sl.ptr = base;
    sl.ready = true;
  }
  *out = &sl;
  return GIRG_OK;
}

}  // namespace hg

using namespace hg;

extern "C" {

const char* girg_last_error(void) { return g_err.c_str(); }
const char* girg_version(void) { return "hipgirg 0.1 (gfx950)"; }

girg_status girg_release(void) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  for (auto it = g_ctx.begin(); it != g_ctx.end();) {
    if (it->first.first == dev) it = g_ctx.erase(it);
    else ++it;
  }
  return GIRG_OK;
}

girg_status girg_points(const girg_params* p, double* w, double* x, void* stream) {
  if (!p || !w || !x) return fail(GIRG_EINVAL, "null argument");
  girg_params q = *p;
  if (q.model == 0) {
    if (q.n < 1 || q.n > 0xFFFFFFFFull) return fail(GIRG_EINVAL, "n must be in [1, 2^32-1]");
    if (q.d < 1 || q.d > 4) return fail(GIRG_EINVAL, "d must be in [1, 4]");
    if (!(q.beta > 2.0)) return fail(GIRG_EINVAL, "beta must be > 2");
  } else {
    if (!(q.alpha > 0.5) || !(q.R > 0.0)) return fail(GIRG_EINVAL, "alpha > 1/2 and R > 0 required");
  }
  Graph g;
  std::memset(&g, 0, sizeof(g));
  g.n = (uint32_t)q.n;
  g.d = q.model == 1 ? 1 : q.d;
  g.model = q.model;
  g.alpha = q.alpha;
  g.R = q.R;
  g.seed_lo = (uint32_t)q.seed;
  g.seed_hi = (uint32_t)(q.seed >> 32);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(launch_points(g, q.beta, w, x, st));
  HIPCHK(hipStreamSynchronize(st));
  return GIRG_OK;
}

girg_status girg_from_points(const girg_params* p, const double* w, const double* x,
                             uint32_t* edges, uint64_t cap, uint64_t* m_out, girg_info* info,
                             void* stream) {
  if (!p || !w || !x || !m_out || (!edges && cap)) return fail(GIRG_EINVAL, "null argument");
  girg_status s = validate(*p, false);
  if (s != GIRG_OK) return s;
  if (p->model == 1 && !(p->R > 0.0)) return fail(GIRG_EINVAL, "girg_from_points needs R > 0 for an HRG");
  CtxLock cl;
  if ((s = lock_ctx(&cl)) != GIRG_OK) return s;
  Ctx* cx = cl.cx;
  if (info) std::memset(info, 0, sizeof(*info));
  cx->ev_name.clear();
  return run_graph(*cx, *p, w, x, edges, cap, m_out, info, static_cast<hipStream_t>(stream));
}

girg_status girg_from_points_noalloc(const girg_params* p, const double* w, const double* x,
                                     uint32_t* edges, uint64_t cap, uint64_t* m_out,
                                     girg_info* info, void* stream) {
  if (!p || !w || !x || !m_out || (!edges && cap)) return fail(GIRG_EINVAL, "null argument");
  girg_status s = validate(*p, false);
  if (s != GIRG_OK) return s;
  if (p->model == 0 && !(p->c > 0.0))
    return fail(GIRG_EINVAL, "girg_from_points_noalloc needs c > 0 (solving c keeps host buffers)");
  if (p->model == 1 && !(p->R > 0.0)) return fail(GIRG_EINVAL, "girg_from_points_noalloc needs R > 0");
  if (p->n > kNoAllocMaxN) return fail(GIRG_EINVAL, "girg_from_points_noalloc: n above 2^20");
  if (cap > kNoAllocMaxCap) return fail(GIRG_EINVAL, "girg_from_points_noalloc: cap above 2^24 edges");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  NoAllocSlot* sl = nullptr;
  if ((s = noalloc_setup(dev, &sl)) != GIRG_OK) return s;
  // calls on one device run one at a time and return only after their work
  // on the GPU has ended, so no two of them use the array at once
  std::unique_lock<std::mutex> lk(sl->cx.mu);
  sl->cx.ar.reset_all();
  sl->cx.ar.clear_failure();
  if (info) std::memset(info, 0, sizeof(*info));
  hipStream_t st = static_cast<hipStream_t>(stream);
  s = run_graph(sl->cx, *p, w, x, edges, cap, m_out, info, st);
  if (s != GIRG_OK) {
    (void)hipStreamSynchronize(st);  // an early return may leave work queued on the array
    if (s == GIRG_ENOMEM && sl->cx.ar.failed())
      return fail(GIRG_ENOMEM, "girg_from_points_noalloc: the graph needs more than the fixed 512 MiB "
                               "scratch (" + g_err + ")");
  }
  return s;
}

static girg_status generate_impl(const girg_params* p, uint32_t* edges, uint64_t cap,
                                 uint64_t* m_out, girg_info* info, void* stream, int slot = 0,
                                 const Place* place = nullptr) {
  girg_params q = *p;
  girg_status s = validate(q, q.model == 0);
  if (s != GIRG_OK) return s;
  if (q.model == 1 && !(q.R > 0.0)) {
    s = solve_R_cached(q.n, q.alpha, q.T, q.avg_deg, &q.R);
    if (s != GIRG_OK) return s;
  }
  CtxLock cl;
  if ((s = lock_ctx(&cl, slot)) != GIRG_OK) return s;
  Ctx* cx = cl.cx;
  if (info) std::memset(info, 0, sizeof(*info));
  hipStream_t st = slot > 0 ? cx->own : static_cast<hipStream_t>(stream);
  const int d = q.model == 1 ? 1 : q.d;
  double* w = cx->ar.get<double>(q.n);
  double* x = cx->ar.get<double>(q.n * d);
  if (cx->ar.failed()) return fail(GIRG_ENOMEM, "scratch allocation failed (points)");
  Graph g;
  std::memset(&g, 0, sizeof(g));
  g.n = (uint32_t)q.n;
  g.d = d;
  g.model = q.model;
  g.alpha = q.alpha;
  g.R = q.R;
  g.seed_lo = (uint32_t)q.seed;
  g.seed_hi = (uint32_t)(q.seed >> 32);
  cx->ev_name.clear();
  cx->mark("-", st);
  HIPCHK(launch_points(g, q.beta, w, x, st));
  cx->mark("points", st);
  return run_graph(*cx, q, w, x, edges, cap, m_out, info, st, place);
}

girg_status girg_generate(const girg_params* p, uint32_t* edges, uint64_t cap, uint64_t* m_out,
                          girg_info* info, void* stream) {
  if (!p || !m_out || (!edges && cap)) return fail(GIRG_EINVAL, "null argument");
  return generate_impl(p, edges, cap, m_out, info, stream);
}

girg_status girg_hrg(uint64_t n, double alpha, double T, double R, double avg_deg, uint64_t seed,
                     uint32_t* edges, uint64_t cap, uint64_t* m_out, girg_info* info,
                     void* stream) {
  if (!m_out || (!edges && cap)) return fail(GIRG_EINVAL, "null argument");
  girg_params q;
  std::memset(&q, 0, sizeof(q));
  q.n = n;
  q.d = 1;
  q.model = 1;
  q.alpha = alpha;
  q.T = T;
  q.R = R;
  q.avg_deg = R > 0.0 ? 0.0 : avg_deg;
  q.seed = seed;
  q.max_depth = -1;
  return generate_impl(&q, edges, cap, m_out, info, stream);
}

girg_status girg_generate_batch(const girg_params* p, int32_t count, uint32_t* edges, uint64_t cap,
                                uint64_t* offsets, girg_info* infos, void* stream) {
  if (!p || count < 0 || !offsets || (!edges && cap)) return fail(GIRG_EINVAL, "null argument");
  offsets[0] = 0;
  if (count == 0) return GIRG_OK;
  for (int32_t b = 0; b < count; ++b) {
    girg_params q = p[b];
    girg_status s = validate(q, q.model == 0);
    if (s != GIRG_OK) return fail(s, "instance " + std::to_string(b) + ": " + g_err);
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  // the workers' streams start after the work queued on the caller's stream
  // so far (the edge buffer may be memory that work still reads or writes)
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipEvent_t start_ev = nullptr;
  HIPCHK(hipEventCreateWithFlags(&start_ev, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { (void)hipEventDestroy(e); }
  } start_guard{start_ev};
  HIPCHK(hipEventRecord(start_ev, hs));
  // instances run concurrently, one per worker, each on its own context and
  // stream; an instance's edges go to the caller's buffer at a position
  // reserved once its count is known (completion order), and are put into
  // instance order at the end
  const int nw = std::min<int>(count, tuned_batch_workers());
  // instances are started largest first (expected edges n * degree, ties in
  // instance order), so that no large one starts when the others are done;
  // the order changes no edge array (the edges are put into instance order)
  std::vector<int32_t> order(count);
  for (int32_t b = 0; b < count; ++b) order[b] = b;
  auto cost = [&](int32_t b) {
    const double deg = p[b].avg_deg > 0.0 ? p[b].avg_deg : 16.0;
    return (double)p[b].n * deg;
  };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
  std::atomic<int32_t> next{0};
  std::atomic<bool> stop{false};
  std::mutex cur_mu;
  uint64_t cursor = 0;
  std::vector<uint64_t> m(count, 0), pos(count, 0);
  std::vector<girg_status> st(count, GIRG_OK);
  std::vector<std::string> msg(count);
  auto worker = [&](int slot) {
    (void)hipSetDevice(dev);
    Ctx* wcx = nullptr;
    if (get_ctx(&wcx, slot) != GIRG_OK || hipStreamWaitEvent(wcx->own, start_ev, 0) != hipSuccess) {
      std::lock_guard<std::mutex> lk(cur_mu);
      if (!stop.load()) {
        st[0] = GIRG_EDEVICE;
        msg[0] = "batch worker set-up failed";
      }
      stop.store(true);
      return;
    }
    for (;;) {
      if (stop.load()) return;
      const int32_t k = next.fetch_add(1);
      if (k >= count) return;
      const int32_t b = order[k];
      const girg_params& q = p[b];
      const double deg = q.avg_deg > 0.0 ? q.avg_deg : 16.0;
      uint64_t scap = (uint64_t)(1.25 * 0.5 * deg * (double)q.n) + 4096;
      Place place = [&, b](uint64_t mb) -> uint32_t* {
        std::lock_guard<std::mutex> lk(cur_mu);
        pos[b] = cursor;
        cursor += mb;
        return edges && pos[b] + mb <= cap ? edges + 2 * pos[b] : nullptr;
      };
      for (int attempt = 0; attempt < 2; ++attempt) {
        uint64_t mb = 0;
        // the staging capacity only: edges go where `place` says
        girg_status s = generate_impl(&q, nullptr, scap, &mb, infos ? &infos[b] : nullptr, nullptr,
                                      slot, &place);
        if (s == GIRG_EOVERFLOW && attempt == 0) {
          scap = mb;
          continue;
        }
        st[b] = s;
        m[b] = mb;
        if (s != GIRG_OK) {
          msg[b] = g_err;
          stop.store(true);
        }
        break;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int k = 0; k < nw; ++k) pool.emplace_back(worker, k + 1);
  for (auto& t : pool) t.join();
  for (int32_t b = 0; b < count; ++b)
    if (st[b] != GIRG_OK) return fail(st[b], "instance " + std::to_string(b) + ": " + msg[b]);
  for (int32_t b = 0; b < count; ++b) offsets[b + 1] = offsets[b] + m[b];
  const uint64_t total = offsets[count];
  if (total > cap) return fail(GIRG_EOVERFLOW, "edge capacity too small");
  // completion order -> instance order, through a copy in the scratch arena
  // of the batch's first worker (cached from call to call); the caller's
  // stream waits for the workers' streams first
  bool same = true;
  for (int32_t b = 0; b < count; ++b) same = same && pos[b] == offsets[b];
  if (!same && total) {
    CtxLock cl;
    girg_status s = lock_ctx(&cl, 1);
    if (s != GIRG_OK) return s;
    uint32_t* tmp = cl.cx->ar.get<uint32_t>(total * 2);
    if (!tmp) return fail(GIRG_ENOMEM, "batch reorder: scratch allocation failed");
    for (int k = 0; k < nw; ++k) {
      Ctx* wcx = nullptr;
      if ((s = get_ctx(&wcx, k + 1)) != GIRG_OK) return s;
      HIPCHK(hipStreamSynchronize(wcx->own));
    }
    hipError_t e = hipMemcpyAsync(tmp, edges, total * 2 * sizeof(uint32_t), hipMemcpyDeviceToDevice, hs);
    for (int32_t b = 0; b < count && e == hipSuccess; ++b)
      if (m[b])
        e = hipMemcpyAsync(edges + 2 * offsets[b], tmp + 2 * pos[b], m[b] * 2 * sizeof(uint32_t),
                           hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail(GIRG_EDEVICE, std::string("batch reorder: ") + hipGetErrorString(e));
  }
  return GIRG_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times the candidate grids (and, for batches, worker counts) on
// count-only calls, which run every sampling pass in full but write no edge
// array, and keeps the fastest in the tuning table
// ---------------------------------------------------------------------------
static const uint32_t kSingleCands[] = {256, 512, 768, 1024, 1536, 2048};
static const uint32_t kBatchBlockCands[] = {128, 256, 512, 768, 1024};
static const int kBatchWorkerCands[] = {8, 16};

// RAII: candidate values forced while timing, cleared on every exit
struct ForceGuard {
  ForceGuard(uint32_t sb, uint32_t bb, int bw) { tune_force(sb, bb, bw); }
  ~ForceGuard() { tune_force(0, 0, 0); }
};

static girg_status time_min(const std::function<girg_status()>& call, int reps, double* best_ms) {
  girg_status s = call();  // warm-up
  if (s != GIRG_OK && s != GIRG_EOVERFLOW) return s;
  double best = 1e300;
  for (int r = 0; r < reps; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    s = call();
    const auto t1 = std::chrono::steady_clock::now();
    if (s != GIRG_OK && s != GIRG_EOVERFLOW) return s;
    best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
  }
  *best_ms = best;
  return GIRG_OK;
}

girg_status girg_autotune(const girg_params* p, int32_t reps, void* stream, int32_t* blocks_out) {
  if (!p || reps < 1 || reps > 100) return fail(GIRG_EINVAL, "null argument or reps outside 1..100");
  girg_status s = validate(*p, p->model == 0);
  if (s != GIRG_OK) return s;
  uint32_t best = 0;
  double best_ms = 1e300;
  for (uint32_t cand : kSingleCands) {
    ForceGuard fg(cand, 0, 0);
    double ms = 0.0;
    s = time_min([&] {
          uint64_t m = 0;
          return generate_impl(p, nullptr, 0, &m, nullptr, stream);
        }, reps, &ms);
    if (s != GIRG_OK) return s;
    if (ms < best_ms) { best_ms = ms; best = cand; }
  }
  const int d = p->model == 1 ? 1 : p->d;
  tune_set_single(tune_key(p->model, d, p->T, p->n), best);
  if (blocks_out) *blocks_out = (int32_t)best;
  g_err.clear();  // the count-only runs leave "edge capacity too small"
  return GIRG_OK;
}

girg_status girg_autotune_batch(const girg_params* p, int32_t count, int32_t reps, int32_t* blocks_out,
                                int32_t* workers_out) {
  if (!p || count < 1 || reps < 1 || reps > 100)
    return fail(GIRG_EINVAL, "null argument, count < 1 or reps outside 1..100");
  std::vector<uint64_t> offs((size_t)count + 1);
  uint32_t best_b = 0;
  int best_w = 0;
  double best_ms = 1e300;
  for (int w : kBatchWorkerCands)
    for (uint32_t b : kBatchBlockCands) {
      ForceGuard fg(0, b, w);
      double ms = 0.0;
      girg_status s = time_min([&] {
            return girg_generate_batch(p, count, nullptr, 0, offs.data(), nullptr, nullptr);
          }, reps, &ms);
      if (s != GIRG_OK) return s;
      if (ms < best_ms) { best_ms = ms; best_b = b; best_w = w; }
    }
  tune_set_batch(best_b, best_w);
  if (blocks_out) *blocks_out = (int32_t)best_b;
  if (workers_out) *workers_out = best_w;
  g_err.clear();
  return GIRG_OK;
}

girg_status girg_tuning_get(const girg_params* p, int32_t batch, int32_t* blocks_out,
                            int32_t* workers_out) {
  if (!p) return fail(GIRG_EINVAL, "null argument");
  const int d = p->model == 1 ? 1 : p->d;
  if (blocks_out) *blocks_out = (int32_t)tuned_blocks(tune_key(p->model, d, p->T, p->n), batch != 0);
  if (workers_out) *workers_out = tuned_batch_workers();
  return GIRG_OK;
}

girg_status girg_tuning_set(const girg_params* p, int32_t batch, int32_t blocks, int32_t workers) {
  if (blocks < 1 || blocks > (int32_t)kMaxBlocks) return fail(GIRG_EINVAL, "blocks outside 1..8192");
  if (batch) {
    if (workers < 0 || workers > kMaxWorkers) return fail(GIRG_EINVAL, "workers outside 0..64");
    tune_set_batch((uint32_t)blocks, workers);
    return GIRG_OK;
  }
  if (!p) return fail(GIRG_EINVAL, "null argument");
  if (p->model != 0 && p->model != 1) return fail(GIRG_EINVAL, "model must be 0 or 1");
  if (p->model == 0 && (p->d < 1 || p->d > 4)) return fail(GIRG_EINVAL, "d must be in 1..4");
  const int d = p->model == 1 ? 1 : p->d;
  tune_set_single(tune_key(p->model, d, p->T, p->n), (uint32_t)blocks);
  return GIRG_OK;
}

girg_status girg_tuning_reset(void) {
  tune_reset();
  return GIRG_OK;
}

girg_status girg_tuning_save(const char* path) {
  if (!path) return fail(GIRG_EINVAL, "null path");
  tune_init();
  std::string err;
  if (!tune_save(path, &err)) return fail(GIRG_EINVAL, err);
  return GIRG_OK;
}

girg_status girg_tuning_load(const char* path) {
  if (!path) return fail(GIRG_EINVAL, "null path");
  tune_init();
  std::string err;
  if (!tune_load(path, &err)) return fail(GIRG_EINVAL, "tuning file " + std::string(path) + ": " + err);
  return GIRG_OK;
}

girg_status girg_set_profiling(int32_t on) {
  Ctx* cx = nullptr;
  girg_status s = get_ctx(&cx);
  if (s != GIRG_OK) return s;
  std::lock_guard<std::mutex> lk(cx->mu);
  cx->profiling = on != 0;
  cx->serial = on == 2;
  return GIRG_OK;
}

int32_t girg_stage_times(double* ms, const char** names, int32_t max) {
  Ctx* cx = nullptr;
  if (get_ctx(&cx) != GIRG_OK) return -1;
  std::lock_guard<std::mutex> lk(cx->mu);
  int32_t k = 0;
  for (size_t i = 0; i < cx->last_ms.size() && k < max; ++i) {
    if (cx->last_name[i] == "-") continue;
    if (ms) ms[k] = cx->last_ms[i];
    if (names) names[k] = cx->last_name[i].c_str();
    ++k;
  }
  return k;
}

girg_status girg_solve_c(const double* w_host, uint64_t n, int32_t d, double T, double avg_deg,
                         double* c_out) {
  if (!w_host || !c_out || n < 2) return fail(GIRG_EINVAL, "null argument or n < 2");
  if (d < 1 || d > 4 || !(T >= 0.0 && T < 1.0) || !(avg_deg > 0.0))
    return fail(GIRG_EINVAL, "invalid d, T or avg_deg");
  CSolve cs;
  cs.n = n; cs.d = d; cs.T = T;
  long double W = 0.0L;
  for (uint64_t i = 0; i < n; ++i) W += w_host[i];
  cs.W = (double)W;
  cs.h.assign(w_host, w_host + n);
  std::sort(cs.h.begin(), cs.h.end(), [](double a, double b) { return a > b; });
  cs.wcut = 0.0;
  cs.prepare();
  if (cs.solve(avg_deg, c_out) != 0) return fail(GIRG_ENOCONV, "c solve found no bracket");
  return GIRG_OK;
}

girg_status girg_expected_degree(const double* w_host, uint64_t n, int32_t d, double T, double c,
                                 double* deg_out) {
  if (!w_host || !deg_out || n < 2 || !(c > 0.0)) return fail(GIRG_EINVAL, "invalid argument");
  CSolve cs;
  cs.n = n; cs.d = d; cs.T = T;
  long double W = 0.0L;
  for (uint64_t i = 0; i < n; ++i) W += w_host[i];
  cs.W = (double)W;
  cs.h.assign(w_host, w_host + n);
  std::sort(cs.h.begin(), cs.h.end(), [](double a, double b) { return a > b; });
  cs.wcut = 0.0;
  cs.prepare();
  *deg_out = cs.f(c);
  return GIRG_OK;
}

girg_status hrg_solve_R(uint64_t n, double alpha, double T, double avg_deg, double* R_out) {
  if (!R_out || n < 2 || !(alpha > 0.5) || !(T >= 0.0 && T < 1.0) || !(avg_deg > 0.0))
    return fail(GIRG_EINVAL, "invalid argument");
  return solve_R_cached(n, alpha, T, avg_deg, R_out);
}

girg_status hrg_expected_degree(uint64_t n, double alpha, double T, double R, double* deg_out) {
  if (!deg_out || n < 2 || !(alpha > 0.5) || !(T >= 0.0 && T < 1.0) || !(R > 0.0))
    return fail(GIRG_EINVAL, "invalid argument");
  *deg_out = rsolve::expected_degree(n, alpha, T, R);
  return GIRG_OK;
}

}  // extern "C"
