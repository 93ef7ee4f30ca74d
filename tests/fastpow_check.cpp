// Host check of pow_pos (the FP64 power of the pair probability) against the
// C library's pow: worst relative error over the stated bound
// 2^-52 (6 + 2 |y log2 x|), worst absolute error of min(1, x^y), and exact
// cases.  Prints one JSON object.
#include "fastpow.h"

#include <cmath>
#include <cstdint>
#include <cstdio>

int main() {
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto rnd = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st >> 11) * 0x1p-53;
  };
  double worst = 0.0, worst_abs = 0.0;
  long n = 0;
  for (int i = 0; i < 4000000; ++i) {
    double x, y;
    switch (i % 4) {
      case 0: x = std::exp2(-300.0 + 600.0 * rnd()); y = 1.0 + 9.0 * rnd(); break;  // wide range
      case 1: x = 1.0 + (rnd() - 0.5) * 1e-3; y = 1.0 + 19.0 * rnd(); break;       // near 1
      case 2: x = std::exp2(-60.0 * rnd()); y = 1.0 / (0.05 + 0.95 * rnd()); break; // p in the tested range
      default: x = rnd() * 4.0; y = 0.5 + 4.0 * rnd(); break;
    }
    const double a = hg::pow_pos(x, y), b = std::pow(x, y);
    if (!(b > 1e-300) || std::isinf(b)) continue;
    const double z = std::fabs(y * std::log2(x));
    const double rel = std::fabs(a - b) / b / (0x1p-52 * (6.0 + 2.0 * z));
    if (rel > worst) worst = rel;
    const double pa = a < 1.0 ? a : 1.0, pb = b < 1.0 ? b : 1.0;
    if (std::fabs(pa - pb) > worst_abs) worst_abs = std::fabs(pa - pb);
    ++n;
  }
  // log_pos over the uniforms of the type-II draws, (v + 1) 2^-53, and near 1
  double worst_log = 0.0;
  for (int i = 0; i < 4000000; ++i) {
    double x;
    switch (i % 4) {
      case 0: x = (double)((st >> 11) + 1) * 0x1p-53; break;
      case 1: x = 1.0 - (double)((st >> 11) % 1000000 + 1) * 0x1p-53; break;
      case 2: x = std::exp2(-53.0 * rnd()); break;
      default: x = std::exp2(-600.0 + 1200.0 * rnd()); break;
    }
    rnd();
    const double a = hg::log_pos(x), b = std::log(x);
    if (b == 0.0) {
      if (a != 0.0) worst_log = 1e300;
      continue;
    }
    const double rel = std::fabs(a - b) / std::fabs(b) / (3.0 * 0x1p-52);
    if (rel > worst_log) worst_log = rel;
  }
  std::printf("{\"log_worst_rel_over_bound\": %.17g, \"log1\": %.17g, \"log2\": %.17g, ",
              worst_log, hg::log_pos(1.0), hg::log_pos(2.0));
  std::printf("\"cases\": %ld, \"worst_rel_over_bound\": %.17g, \"worst_abs_capped\": %.17g, "
              "\"p2_10\": %.17g, \"p05_3\": %.17g, \"p1_7\": %.17g, \"px_1\": %.17g, "
              "\"p0\": %.17g, \"pinf_is_inf\": %d, \"tiny\": %.17g}\n",
              n, worst, worst_abs, hg::pow_pos(2.0, 10.0), hg::pow_pos(0.5, 3.0),
              hg::pow_pos(1.0, 7.0), hg::pow_pos(0.3, 1.0), hg::pow_pos(0.0, 2.0),
              (int)std::isinf(hg::pow_pos(INFINITY, 2.0)), hg::pow_pos(1e-300, 5.0));
  return 0;
}
