/*
 * oracle.c -- plain sequential FP64 reference of the GIRG / HRG sampler of
 * arXiv:1905.06706 (Blaesius et al.).  TEST INFRASTRUCTURE: only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * The code follows the paper's steps in the paper's order and notation:
 *   weights / positions (Sec. 2.1, 2.2), the mapping HRG -> GIRG (Sec. 2.3),
 *   weight buckets ("layers", Sec. 3.1), comparison level CL(i,j) and insertion
 *   level I(i) (Sec. 3.1; HRG: search over levels, Sec. 4.3), vertices sorted by
 *   Morton code of their cell (Sec. 3.4, Lemma 1, App. A) with prefix sums,
 *   Algorithm 1 (recursive cell-pair iteration, Sec. 3.3) with the double
 *   counting rules of App. B.1, type-I pairs tested one by one, type-II pairs
 *   sampled by geometric jumps under an upper bound pbar and accepted with
 *   p_uv / pbar (Sec. 3.2).
 * Nothing is blocked, fused or reordered.  The readings taken where the paper
 * is silent are restated briefly at each use.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* error reporting                                                           */
/* ------------------------------------------------------------------------- */
static __thread char g_err[256];
const char* orc_last_error(void) { return g_err; }
static void set_err(const char* msg) {
  strncpy(g_err, msg, sizeof(g_err) - 1);
  g_err[sizeof(g_err) - 1] = 0;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,        */
/* "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011).  One round maps  */
/* (c0,c1,c2,c3) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)); */
/* the key is bumped by the Weyl constants between rounds.                   */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniforms from two 32-bit words: the top 53 bits of hi:lo. */
double orc_u53(uint32_t lo, uint32_t hi) {
  uint64_t v = ((uint64_t)hi << 32) | lo;
  return (double)(v >> 11) * 0x1p-53;
}
double orc_u53_open(uint32_t lo, uint32_t hi) {
  uint64_t v = ((uint64_t)hi << 32) | lo;
  return (double)((v >> 11) + 1) * 0x1p-53;
}

/* Stream layout (our contract; the paper uses thread-local generators,
 * App. B.5).  key = seed.  counter word 3 packs level, layer pair, kind and a
 * high index part. */
enum { KIND_TYPE1 = 0, KIND_TYPE2 = 1, KIND_POINTS = 2, KIND_SEQ = 3 };

static void stream_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

static uint32_t word3(int level, int i, int j, int kind, uint32_t high) {
  return (uint32_t)level | ((uint32_t)i << 6) | ((uint32_t)j << 12) | ((uint32_t)kind << 18) |
         (high << 20);
}

/* ------------------------------------------------------------------------- */
/* Morton code (Sec. 4.2, App. B.3): bitwise interleaving, dimension 0 most   */
/* significant within each group, so (a3a2a1a0, b3b2b1b0) -> a3b3a2b2a1b1a0b0. */
/* Written as the plain bit loop ("FOR").                                    */
/* ------------------------------------------------------------------------- */
uint64_t orc_morton_encode(const uint32_t* coord, int d, int bits) {
  uint64_t code = 0;
  for (int b = bits - 1; b >= 0; b--)
    for (int k = 0; k < d; k++) code = (code << 1) | ((coord[k] >> b) & 1u);
  return code;
}
void orc_morton_decode(uint64_t code, int d, int bits, uint32_t* coord) {
  for (int k = 0; k < d; k++) coord[k] = 0;
  for (int b = 0; b < bits; b++)
    for (int k = 0; k < d; k++) {
      int pos = b * d + (d - 1 - k);
      coord[k] |= (uint32_t)((code >> pos) & 1u) << b;
    }
}

/* ------------------------------------------------------------------------- */
/* Points (Sec. 2.1 GIRG; Sec. 2.2 HRG).                                     */
/* ------------------------------------------------------------------------- */
/* GIRG: power-law weights with exponent beta, w_min = 1, drawn by inverting
 * the Pareto tail P(w > t) = t^{-(beta-1)}; positions uniform on the torus as
 * exact multiples of 2^-53. */
void orc_points_girg(uint64_t n, int d, double beta, uint64_t seed, double* w, double* x) {
  double expo = -1.0 / (beta - 1.0);
  for (uint64_t u = 0; u < n; u++) {
    uint32_t o[4];
    stream_block(seed, (uint32_t)u, 0u, 0u, word3(0, 0, 0, KIND_POINTS, 0), o);
    w[u] = pow(orc_u53_open(o[0], o[1]), expo);
    for (int k = 0; k < d; k++) {
      if (k % 2 == 0) stream_block(seed, (uint32_t)u, (uint32_t)(1 + k / 2), 0u,
                                   word3(0, 0, 0, KIND_POINTS, 0), o);
      int h = k % 2;
      x[u * (uint64_t)d + k] = orc_u53(o[2 * h], o[2 * h + 1]);
    }
  }
}

/* HRG: radius with density alpha sinh(alpha r) / (cosh(alpha R) - 1) on
 * [0, R), by inverting its CDF (cosh(alpha r) - 1) / (cosh(alpha R) - 1);
 * angle theta = 2 pi x with x uniform on [0,1).  A radius that rounds to R or
 * above is clamped to R (the layer formula needs r <= R). */
void orc_points_hrg(uint64_t n, double alpha, double R, uint64_t seed, double* r, double* x) {
  double cm1 = cosh(alpha * R) - 1.0;
  for (uint64_t u = 0; u < n; u++) {
    uint32_t o[4];
    stream_block(seed, (uint32_t)u, 0u, 0u, word3(0, 0, 0, KIND_POINTS, 0), o);
    double U = orc_u53(o[0], o[1]);
    double ru = acosh(1.0 + U * cm1) / alpha;
    r[u] = ru < R ? ru : R;
    stream_block(seed, (uint32_t)u, 1u, 0u, word3(0, 0, 0, KIND_POINTS, 0), o);
    x[u] = orc_u53(o[0], o[1]);
  }
}

/* ------------------------------------------------------------------------- */
/* Expected average degree and estimation of c (Sec. 4.1, App. B.2).          */
/* ------------------------------------------------------------------------- */
static double sum_ld(const double* v, uint64_t n) {
  long double s = 0.0L;
  for (uint64_t i = 0; i < n; i++) s += v[i];
  return (double)s;
}

static int cmp_desc(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x < y) - (x > y);
}

/* f(c) = E[average degree] = (1/n) sum over ordered pairs u != v of
 * E[X_uv] (App. B.2, Eq. deg).  E[X_uv] is 1 on E_R, the pairs whose ball of
 * probability 1 reaches beyond the torus (k > 1/2: T > 0, c^T w_u w_v / W >
 * 2^-d; T = 0, 2^d c^d w_u w_v / W > 1), and elsewhere the closed form of
 * App. B.2: T > 0 A x - B x^{1/T} with x = w_u w_v / W, A = 2^d c^T / (1 - T),
 * B = 2^{d/T} c / (1/T - 1) (Eqs. short, long, shortlong); T = 0
 * ("analogous") (2k)^d = 2^d c^d x.  The paper evaluates the closed form over
 * all pairs and subtracts its excess over E_R; here the pairs outside E_R are
 * summed directly (the same value), so that no large excess is formed and
 * subtracted: with weights in descending order, E_R partners of u are a
 * prefix [0, m_u) and the other partners a suffix, summed from suffix sums. */
typedef struct {
  uint64_t n;
  int d;
  double T, W;
  double* sorted;              /* weights in descending order */
  double *sw, *sw2, *sp, *sp2; /* suffix sums from index k: w, w^2, w^{1/T}, w^{2/T} */
} cctx;

static double f_of_c(const cctx* q, double c) {
  uint64_t n = q->n;
  int d = q->d;
  double T = q->T, W = q->W;
  double cT = T > 0.0 ? pow(c, T) : 0.0;
  double a0 = ldexp(pow(c, (double)d), d); /* T = 0: 2^d c^d */
  double A = T > 0.0 ? cT * ldexp(1.0, d) / (1.0 - T) : a0;
  double B = T > 0.0 ? c * pow(2.0, (double)d / T) / (1.0 / T - 1.0) : 0.0;
  double WT = T > 0.0 ? pow(W, 1.0 / T) : 1.0;
  double Wsum = q->sw[0], P = T > 0.0 ? q->sp[0] : 0.0;
  long double cnt = 0.0L, S1 = 0.0L, S2 = 0.0L; /* S1 = sum w_u w_v, S2 = sum (w_u w_v)^{1/T} off E_R */
  uint64_t m = n;
  for (uint64_t u = 0; u < n; u++) {
    double wu = q->sorted[u];
    /* m = number of v with (u, v) in E_R, v ranging over all vertices */
    while (m > 0) {
      double X = wu * q->sorted[m - 1] / W;
      int in_er = T > 0.0 ? cT * X > ldexp(1.0, -d) : a0 * X > 1.0;
      if (in_er) break;
      m--;
    }
    if (m == 0) {
      /* no vertex from u on has a partner in E_R: all other vertices count */
      S1 += (long double)Wsum * q->sw[u] - q->sw2[u];
      if (T > 0.0) S2 += (long double)P * q->sp[u] - q->sp2[u];
      break;
    }
    int self_out = u >= m; /* u itself lies in the suffix */
    double hu = T > 0.0 ? pow(wu, 1.0 / T) : 0.0;
    cnt += (long double)(m - (self_out ? 0 : 1));
    S1 += (long double)wu * (q->sw[m] - (self_out ? wu : 0.0));
    if (T > 0.0) S2 += (long double)hu * (q->sp[m] - (self_out ? hu : 0.0));
  }
  long double nf = (long double)A * (S1 / W) - (long double)B * (S2 / WT) + cnt;
  return (double)(nf / (long double)n);
}

static void cctx_free(cctx* q) {
  free(q->sorted);
  free(q->sw);
  free(q->sw2);
  free(q->sp);
  free(q->sp2);
}

static int cctx_init(cctx* q, uint64_t n, int d, double T, const double* w) {
  q->n = n; q->d = d; q->T = T;
  q->W = sum_ld(w, n);
  q->sorted = (double*)malloc(sizeof(double) * n);
  q->sw = (double*)malloc(sizeof(double) * (n + 1));
  q->sw2 = (double*)malloc(sizeof(double) * (n + 1));
  q->sp = (double*)malloc(sizeof(double) * (n + 1));
  q->sp2 = (double*)malloc(sizeof(double) * (n + 1));
  if (!q->sorted || !q->sw || !q->sw2 || !q->sp || !q->sp2) { cctx_free(q); return -1; }
  memcpy(q->sorted, w, sizeof(double) * n);
  qsort(q->sorted, n, sizeof(double), cmp_desc);
  /* suffix sums, accumulated from the light end */
  long double a = 0.0L, b = 0.0L, e = 0.0L, f = 0.0L;
  q->sw[n] = q->sw2[n] = q->sp[n] = q->sp2[n] = 0.0;
  for (uint64_t k = n; k-- > 0;) {
    double x = q->sorted[k];
    a += x;
    b += (long double)x * x;
    if (T > 0.0) {
      double h = pow(x, 1.0 / T);
      e += h;
      f += (long double)h * h;
    }
    q->sw[k] = (double)a; q->sw2[k] = (double)b; q->sp[k] = (double)e; q->sp2[k] = (double)f;
  }
  return 0;
}

double orc_expected_avg_degree(uint64_t n, int d, double T, double c, const double* w) {
  cctx q;
  if (cctx_init(&q, n, d, T, w)) return NAN;
  double f = f_of_c(&q, c);
  cctx_free(&q);
  return f;
}

/* Exponential search for a bracket, then bisection in log c (App. B.2: f is
 * monotone in c).  Stops when the geometric midpoint no longer separates the
 * bracket (adjacent doubles) or after 200 halvings; returns the upper end. */
int orc_solve_c(uint64_t n, int d, double T, double avg_deg, const double* w, double* c_out) {
  if (!(avg_deg > 0.0) || n < 2) { set_err("solve_c: avg_deg must be > 0 and n >= 2"); return -1; }
  cctx q;
  if (cctx_init(&q, n, d, T, w)) { set_err("solve_c: out of memory"); return -2; }
  double lo = 1.0, hi = 1.0;
  int it = 0;
  if (f_of_c(&q, 1.0) < avg_deg) {
    while (f_of_c(&q, hi) < avg_deg) {
      lo = hi; hi *= 2.0;
      if (++it > 2000) { cctx_free(&q); set_err("solve_c: no bracket"); return -5; }
    }
  } else {
    while (f_of_c(&q, lo) >= avg_deg) {
      hi = lo; lo *= 0.5;
      if (++it > 2000) { cctx_free(&q); set_err("solve_c: no bracket"); return -5; }
    }
  }
  for (it = 0; it < 200; it++) {
    double mid = sqrt(lo) * sqrt(hi);
    if (!(mid > lo && mid < hi)) break;
    if (f_of_c(&q, mid) < avg_deg) lo = mid; else hi = mid;
  }
  cctx_free(&q);
  *c_out = hi;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* HRG expected average degree (not in the paper).  For independent points   */
/* with the radial density of Sec. 2.2 and uniform angles, the angular       */
/* distance phi is uniform on [0, pi] and                                    */
/*   E[deg] = (n-1) * int int f(r1) f(r2) (1/pi) int_0^pi p(d(r1,r2,phi)) dphi */
/* with cosh d = cosh(r1-r2) + 2 sinh r1 sinh r2 sin^2(phi/2).  Composite     */
/* Gauss-Legendre quadrature with breakpoints at the kink r1 + r2 = R and at */
/* the angle phi* where d = R.                                               */
/* ------------------------------------------------------------------------- */
#define GL_N 16
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;
static void gl_init(void) {
  if (gl_ready) return;
  /* Gauss-Legendre nodes by Newton iteration on the Legendre polynomial P_N. */
  for (int i = 0; i < GL_N; i++) {
    double z = cos(M_PI * (i + 0.75) / (GL_N + 0.5)), p0 = 1.0, p1 = z, dp = 1.0;
    for (int it = 0; it < 100; it++) {
      p0 = 1.0; p1 = z;
      for (int k = 2; k <= GL_N; k++) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
      }
      dp = GL_N * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    p0 = 1.0; p1 = z;
    for (int k = 2; k <= GL_N; k++) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1; p1 = p2;
    }
    dp = GL_N * (z * p1 - p0) / (z * z - 1.0);
    gl_x[i] = z;
    gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  gl_ready = 1;
}

typedef struct { double alpha, T, R, coshR, norm; } hrgq;

static double hrg_density(const hrgq* h, double r) {
  return h->alpha * sinh(h->alpha * r) / h->norm;
}

static double p_T_of_coshd(const hrgq* h, double coshd) {
  double dist = acosh(coshd < 1.0 ? 1.0 : coshd);
  return 1.0 / (exp((dist - h->R) / (2.0 * h->T)) + 1.0);
}

static double gl_panel_p(const hrgq* h, double base, double amp, double a, double b) {
  double hm = 0.5 * (b - a), mid = 0.5 * (a + b), tot = 0.0;
  for (int k = 0; k < GL_N; k++) {
    double sh = sin(0.5 * (mid + hm * gl_x[k]));
    tot += hm * gl_w[k] * p_T_of_coshd(h, base + amp * sh * sh);
  }
  return tot;
}

/* (1/pi) int_0^pi p(d(phi)) dphi.  T = 0: phi* / pi, with phi* the angle at
 * which d = R.  T > 0: panels below phi*, and panels growing geometrically
 * above it (the probability decays like a power of phi there). */
static double angular_prob(const hrgq* h, double r1, double r2) {
  double base = cosh(r1 - r2), amp = 2.0 * sinh(r1) * sinh(r2);
  double s2 = amp > 0.0 ? (h->coshR - base) / amp : (base < h->coshR ? 2.0 : -1.0);
  double phis;
  if (s2 >= 1.0) phis = M_PI;
  else if (s2 <= 0.0) phis = 0.0;
  else phis = 2.0 * asin(sqrt(s2));
  if (h->T == 0.0) return phis / M_PI;
  double tot = 0.0;
  if (phis <= 0.0 || phis >= M_PI) {
    for (int q = 0; q < 4; q++) tot += gl_panel_p(h, base, amp, M_PI * q / 4.0, M_PI * (q + 1) / 4.0);
    return tot / M_PI;
  }
  for (int q = 0; q < 3; q++) tot += gl_panel_p(h, base, amp, phis * q / 3.0, phis * (q + 1) / 3.0);
  double a = phis;
  while (a < M_PI) {
    double b = a * 2.0 < M_PI ? a * 2.0 : M_PI;
    tot += gl_panel_p(h, base, amp, a, b);
    a = b;
  }
  return tot / M_PI;
}

/* int_a^b f(r2) P(r1, r2) dr2 on panels of unit width */
static double hrg_inner(const hrgq* h, double r1, double a, double b) {
  double tot = 0.0;
  if (b <= a) return 0.0;
  int panels = (int)ceil(b - a);
  if (panels < 1) panels = 1;
  for (int q = 0; q < panels; q++) {
    double pa = a + (b - a) * q / panels, pb = a + (b - a) * (q + 1) / panels;
    double hm = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
    for (int k = 0; k < GL_N; k++) {
      double r2 = mid + hm * gl_x[k];
      tot += hm * gl_w[k] * hrg_density(h, r2) * angular_prob(h, r1, r2);
    }
  }
  return tot;
}

double orc_hrg_expected_avg_degree(uint64_t n, double alpha, double T, double R) {
  gl_init();
  hrgq h = {alpha, T, R, cosh(R), cosh(alpha * R) - 1.0};
  double tot = 0.0;
  int panels = (int)ceil(R);
  for (int q = 0; q < panels; q++) {
    double pa = R * q / panels, pb = R * (q + 1) / panels;
    double hm = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
    for (int k = 0; k < GL_N; k++) {
      double r1 = mid + hm * gl_x[k];
      double kink = R - r1; /* at T = 0 every angle connects when r1 + r2 <= R */
      double inner = hrg_inner(&h, r1, 0.0, kink) + hrg_inner(&h, r1, kink, R);
      tot += hm * gl_w[k] * hrg_density(&h, r1) * inner;
    }
  }
  return (double)(n - 1) * tot;
}

/* E[deg] decreases in R.  Bracket around 2 ln n, then regula falsi on
 * log E[deg] with the Illinois modification, to relative width 1e-12. */
int orc_hrg_solve_R(uint64_t n, double alpha, double T, double avg_deg, double* R_out) {
  if (!(avg_deg > 0.0) || n < 2) { set_err("solve_R: avg_deg must be > 0 and n >= 2"); return -1; }
  double lo = 2.0 * log((double)n), hi = lo;
  double flo = orc_hrg_expected_avg_degree(n, alpha, T, lo), fhi = flo;
  int it = 0;
  while (flo < avg_deg) {
    hi = lo; fhi = flo;
    lo *= 0.5;
    flo = orc_hrg_expected_avg_degree(n, alpha, T, lo);
    if (++it > 200) { set_err("solve_R: no bracket"); return -5; }
  }
  while (fhi > avg_deg) {
    lo = hi; flo = fhi;
    hi *= 1.5;
    fhi = orc_hrg_expected_avg_degree(n, alpha, T, hi);
    if (++it > 400) { set_err("solve_R: no bracket"); return -5; }
  }
  double glo = log(flo / avg_deg), ghi = log(fhi / avg_deg); /* glo >= 0 >= ghi */
  int side = 0;
  for (it = 0; it < 200 && (hi - lo) > 1e-12 * hi; it++) {
    double mid = (glo == ghi) ? 0.5 * (lo + hi) : lo + (hi - lo) * glo / (glo - ghi);
    if (!(mid > lo && mid < hi)) mid = 0.5 * (lo + hi);
    double gm = log(orc_hrg_expected_avg_degree(n, alpha, T, mid) / avg_deg);
    if (gm == 0.0) { lo = hi = mid; break; }
    if (gm > 0.0) {
      lo = mid; glo = gm;
      if (side == 1) ghi *= 0.5;
      side = 1;
    } else {
      hi = mid; ghi = gm;
      if (side == -1) glo *= 0.5;
      side = -1;
    }
  }
  *R_out = 0.5 * (lo + hi);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* The sampling run.                                                         */
/* ------------------------------------------------------------------------- */
typedef struct { uint32_t* a; uint64_t n, cap; } vec32;
typedef struct { uint64_t* a; uint64_t n, cap; } vec64;
static int push32(vec32* v, uint32_t x, uint32_t y) {
  if (v->n + 2 > v->cap) {
    uint64_t nc = v->cap ? 2 * v->cap : 1024;
    uint32_t* p = (uint32_t*)realloc(v->a, nc * sizeof(uint32_t));
    if (!p) return -1;
    v->a = p; v->cap = nc;
  }
  v->a[v->n++] = x; v->a[v->n++] = y;
  return 0;
}
static int push64x4(vec64* v, uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  if (v->n + 4 > v->cap) {
    uint64_t nc = v->cap ? 2 * v->cap : 256;
    uint64_t* p = (uint64_t*)realloc(v->a, nc * sizeof(uint64_t));
    if (!p) return -1;
    v->a = p; v->cap = nc;
  }
  v->a[v->n++] = a; v->a[v->n++] = b; v->a[v->n++] = c; v->a[v->n++] = d;
  return 0;
}

struct orc_run {
  orc_params p;
  int L, D, Dmax;
  double W, w0, kappa, coshR;
  int32_t CL[ORC_MAX_LAYERS][ORC_MAX_LAYERS];
  int32_t I[ORC_MAX_LAYERS];
  int64_t count[ORC_MAX_LAYERS];
  double ext[ORC_MAX_LAYERS];   /* GIRG: max weight of the layer; HRG: min radius */
  uint64_t lstart[ORC_MAX_LAYERS + 1];
  uint32_t* P[ORC_MAX_LAYERS];  /* prefix sums at level I(i), 2^{d I(i)} + 1 entries */
  /* per original id */
  int32_t* layer;
  uint64_t* morton;             /* at level Dmax */
  /* sorted order */
  uint32_t* sid;                /* sorted position -> original id */
  uint32_t* spos;               /* original id -> sorted position */
  double* sw;                   /* weight (GIRG) or radius (HRG) */
  double* sx;                   /* n*d */
  /* output */
  vec32 edges, near;
  vec64 ties;
  uint64_t ctr[ORC_NSTATS];
  /* expected numbers of logged near decisions and skip ties over the random
   * draws of this run, given the points: the bounds the parity tests put on
   * the logged counts */
  double near_expect, tie_expect;
  uint64_t lvl_nb[40], lvl_dist[40]; /* visited cell pairs per level */
  int failed;
};

enum {
  S_NBPAIRS = 5, S_DISTPAIRS = 6, S_T1ITEMS = 7, S_T2ITEMS = 8, S_TESTS = 9, S_DRAWS = 10,
  S_CANDS = 11, S_EDGES = 12, S_NEAR = 13, S_TIES = 14, S_SEGS = 15, S_T1EDGES = 17,
  S_T2EDGES = 18, S_SEQS = 21
};

void orc_free(orc_run* r) {
  if (!r) return;
  for (int i = 0; i < ORC_MAX_LAYERS; i++) free(r->P[i]);
  free(r->layer); free(r->morton); free(r->sid); free(r->spos); free(r->sw); free(r->sx);
  free(r->edges.a); free(r->near.a); free(r->ties.a);
  free(r);
}

static int bitlen(uint64_t v) {
  int b = 0;
  while (v) { b++; v >>= 1; }
  return b;
}

/* L-infinity distance on the torus (Sec. 2.1). */
static double torus_dist(const double* a, const double* b, int d) {
  double r = 0.0;
  for (int k = 0; k < d; k++) {
    double delta = fabs(a[k] - b[k]);
    double m = delta < 1.0 - delta ? delta : 1.0 - delta;
    if (m > r) r = m;
  }
  return r;
}

/* Edge probability of Eq. (1), T > 0.  r^d by repeated multiplication. */
static double girg_p(const orc_run* R, double wu, double wv, double r) {
  if (r == 0.0) return 1.0;
  double rd = r;
  for (int k = 1; k < R->p.d; k++) rd *= r;
  double p = R->p.c * pow((wu * wv / R->W) / rd, 1.0 / R->p.T);
  return p < 1.0 ? p : 1.0;
}

/* HRG: cosh of the hyperbolic distance (Sec. 2.2), written with the identity
 * cosh r_u cosh r_v - sinh r_u sinh r_v cos(dtheta)
 *   = cosh(r_u - r_v) + 2 sinh r_u sinh r_v sin^2(dtheta / 2),
 * dtheta = 2 pi dx, which avoids the cancellation of the product form. */
static double hrg_coshd(double ru, double rv, double dx) {
  double s = sin(M_PI * dx);
  return cosh(ru - rv) + 2.0 * sinh(ru) * sinh(rv) * s * s;
}
static double hrg_pT(const orc_run* R, double coshd) {
  double dist = acosh(coshd);
  return 1.0 / (exp((dist - R->p.R) / (2.0 * R->p.T)) + 1.0);
}

/* Morton code of the cell of sorted vertex s at level l. */
static uint64_t cell_of_sorted(const orc_run* R, uint64_t s, int l) {
  return R->morton[R->sid[s]] >> (R->p.d * (R->Dmax - l));
}

/* V_i^A as a range of sorted positions (Lemma 1). */
static void vertex_range(const orc_run* R, int i, int l, uint64_t A, uint64_t* first, uint64_t* num) {
  int sh = R->p.d * (R->I[i] - l);
  uint64_t lo = R->P[i][A << sh], hi = R->P[i][(A + 1) << sh];
  *first = lo; *num = hi - lo;
}

/* Per-dimension torus distance between cell coordinates at level l. */
static void cell_deltas(const orc_run* R, uint64_t A, uint64_t B, int l, uint32_t* delta) {
  uint32_t ca[8], cb[8];
  int d = R->p.d;
  orc_morton_decode(A, d, l, ca);
  orc_morton_decode(B, d, l, cb);
  uint64_t side = (uint64_t)1 << l;
  for (int k = 0; k < d; k++) {
    uint64_t df = ca[k] > cb[k] ? ca[k] - cb[k] : cb[k] - ca[k];
    uint64_t wrap = side - df;
    delta[k] = (uint32_t)(df < wrap ? df : wrap);
  }
}
static int are_neighbours(const orc_run* R, uint64_t A, uint64_t B, int l) {
  uint32_t delta[8];
  cell_deltas(R, A, B, l, delta);
  for (int k = 0; k < R->p.d; k++)
    if (delta[k] > 1) return 0;
  return 1;
}

/* ---- type-I: every pair of V_i^A x V_j^B gets its own coin (Sec. 3.2). ---- */
static void emit(orc_run* R, uint32_t u, uint32_t v, int type) {
  if (push32(&R->edges, u, v)) R->failed = 1;
  R->ctr[S_EDGES]++;
  R->ctr[type ? S_T2EDGES : S_T1EDGES]++;
}
static void near_pair(orc_run* R, uint32_t u, uint32_t v) {
  if (push32(&R->near, u, v)) R->failed = 1;
  R->ctr[S_NEAR]++;
}

/* Probability that a uniform on [0,1) lies within 1e-12 of q in [0,1]: the
 * chance that a coin compared with q is logged as near. */
static double near_mass(double q) {
  double lo = q - 1e-12, hi = q + 1e-12;
  if (lo < 0.0) lo = 0.0;
  if (hi > 1.0) hi = 1.0;
  return hi > lo ? hi - lo : 0.0;
}

static void type1_pair(orc_run* R, int l, uint64_t A, uint64_t B, int i, int j, uint64_t su,
                       uint64_t sv, uint64_t k) {
  const orc_params* p = &R->p;
  uint32_t u = R->sid[su], v = R->sid[sv];
  R->ctr[S_TESTS]++;
  if (p->accept_all) { emit(R, u, v, 0); return; }
  const double* xu = R->sx + su * (uint64_t)p->d;
  const double* xv = R->sx + sv * (uint64_t)p->d;
  double r = torus_dist(xu, xv, p->d);
  if (p->model == 0 && p->T == 0.0) {
    /* threshold variant: edge iff ||x_u - x_v|| <= c (w_u w_v / W)^{1/d} */
    double t = p->c * pow(R->sw[su] * R->sw[sv] / R->W, 1.0 / p->d);
    if (fabs(r - t) <= 1e-12 * t) near_pair(R, u, v);
    /* r / t has a density of order one near 1 over the tested pairs */
    R->near_expect += 2e-12;
    if (r <= t) emit(R, u, v, 0);
    return;
  }
  if (p->model == 1 && p->T == 0.0) {
    /* threshold HRG: edge iff d < R, i.e. cosh d < cosh R (Sec. 4.3) */
    double ch = hrg_coshd(R->sw[su], R->sw[sv], r);
    if (fabs(ch - R->coshR) <= 1e-12 * R->coshR) near_pair(R, u, v);
    R->near_expect += 2e-12;
    if (ch < R->coshR) emit(R, u, v, 0);
    return;
  }
  double prob = p->model == 0 ? girg_p(R, R->sw[su], R->sw[sv], r)
                              : hrg_pT(R, hrg_coshd(R->sw[su], R->sw[sv], r));
  uint64_t blk = k >> 1;
  uint32_t o[4];
  stream_block(p->seed, (uint32_t)blk, (uint32_t)A, (uint32_t)B,
               word3(l, i, j, KIND_TYPE1, (uint32_t)(blk >> 32)), o);
  int h = (int)(k & 1);
  double U = orc_u53(o[2 * h], o[2 * h + 1]);
  if (fabs(U - prob) < 1e-12) near_pair(R, u, v);
  R->near_expect += near_mass(prob);
  if (U < prob) emit(R, u, v, 0);
}

static void type1(orc_run* R, int l, uint64_t A, uint64_t B, int i, int j) {
  uint64_t a0, na, b0, nb;
  vertex_range(R, i, l, A, &a0, &na);
  vertex_range(R, j, l, B, &b0, &nb);
  if (na == 0 || nb == 0) return;
  if (A == B && i == j) {
    if (na < 2) return;
    R->ctr[S_T1ITEMS]++;
    /* only a < b within V_i^A (App. B.1); pair index k = b(b-1)/2 + a */
    for (uint64_t b = 1; b < na; b++)
      for (uint64_t a = 0; a < b; a++) type1_pair(R, l, A, B, i, j, a0 + a, a0 + b, b * (b - 1) / 2 + a);
    return;
  }
  R->ctr[S_T1ITEMS]++;
  for (uint64_t a = 0; a < na; a++)
    for (uint64_t b = 0; b < nb; b++) type1_pair(R, l, A, B, i, j, a0 + a, b0 + b, a * nb + b);
}

/* ---- type-II: geometric jumps under pbar, acceptance p_uv / pbar (Sec. 3.2). ---- */
#define SEG_EXP 5
#define SEG_MAX_BITS 12

/* Upper bound pbar for the layer pair (i,j) at level l with gap g: the maximum
 * weights of the layers and the minimum distance g 2^-l between points of the
 * two cells (GIRG); for the HRG the smallest radii of the layers and the same
 * minimum angular distance. */
static double type2_pbar(const orc_run* R, int l, int i, int j, int g, double* raw) {
  const orc_params* p = &R->p;
  if (p->accept_all) { *raw = 2.0; return 1.0; }
  double dist = ldexp((double)g, -l);
  if (p->model == 0) {
    double dd = dist;
    for (int k = 1; k < p->d; k++) dd *= dist;
    double pb = p->c * pow((R->ext[i] * R->ext[j] / R->W) / dd, 1.0 / p->T);
    *raw = pb; /* before the clamp to 1 */
    return pb < 1.0 ? pb : 1.0;
  }
  double s = sin(M_PI * dist);
  double ch = 1.0 + 2.0 * sinh(R->ext[i]) * sinh(R->ext[j]) * s * s;
  *raw = hrg_pT(R, ch);
  return *raw;
}

/* Chance that the skip quotient q of one draw, q ~ Exp(lambda) with
 * lambda = -ln(1 - pbar), falls within 1e-12 q of an integer j in 1..K, the
 * candidates still in range: about sum_j 2e-12 j lambda e^{-lambda j}
 * = 2e-12 lambda sum_j j r^j with r = 1 - pbar (closed form of the sum). */
static double tie_mass(double pbar, double lambda, double K) {
  if (!(K >= 1.0) || !(pbar > 0.0) || pbar >= 1.0) return 0.0;
  double u = K * lambda, S;
  if (u < 1e-6) {
    S = 0.5 * K * (K + 1.0);
  } else {
    double r = 1.0 - pbar, rK = exp(-u);
    S = r * (1.0 - rK * (1.0 + K * pbar)) / (pbar * pbar);
  }
  return 2e-12 * lambda * S;
}

static int near_pow2(double x) {
  int e;
  double m = frexp(x, &e); /* x = m 2^e, m in [0.5, 1) */
  return m < 0.5 * (1.0 + 4.0 * 0x1p-52) || m > 1.0 - 4.0 * 0x1p-53;
}

static void type2(orc_run* R, int l, uint64_t A, uint64_t B, int i, int j) {
  const orc_params* p = &R->p;
  uint64_t a0, na, b0, nb;
  vertex_range(R, i, l, A, &a0, &na);
  vertex_range(R, j, l, B, &b0, &nb);
  if (na == 0 || nb == 0) return;
  R->ctr[S_T2ITEMS]++;
  uint32_t delta[8];
  cell_deltas(R, A, B, l, delta);
  int g = 0;
  for (int k = 0; k < p->d; k++)
    if ((int)delta[k] - 1 > g) g = (int)delta[k] - 1;
  double pbar_raw;
  double pbar = type2_pbar(R, l, i, j, g, &pbar_raw);
  if (!(pbar > 0.0)) return;
  double Lg = log1p(-pbar);
  uint64_t N = na * nb;
  /* The candidate range [0, N) is cut into segments of G = 2^e candidates,
   * each with its own geometric-jump sequence (exact: the candidates are
   * independent).  e = 5 - ilogb(pbar), raised until at most 2^12 segments. */
  int e = SEG_EXP - ilogb(pbar);
  int emin = bitlen(N - 1) - SEG_MAX_BITS;
  if (e < emin) e = emin;
  uint64_t G = (e >= 63 || ((uint64_t)1 << e) >= N) ? N : ((uint64_t)1 << e);
  uint64_t nseg = (N + G - 1) / G;
  /* a bound within a few ulps of a power of two (before the clamp to 1, which
   * makes 1 exact) may fall on either side of it under another pow, and
   * change the segment size: log the item */
  int tie = near_pow2(pbar_raw) && e > emin;
  for (uint64_t s = 0; s < nseg; s++) {
    uint64_t k = s * G, kend = (s + 1) * G < N ? (s + 1) * G : N;
    R->ctr[S_SEGS]++;
    for (uint32_t t = 0;; t++) {
      uint32_t o[4];
      stream_block(p->seed, t, (uint32_t)A, (uint32_t)B,
                   word3(l, i, j, KIND_TYPE2, (uint32_t)s), o);
      R->ctr[S_DRAWS]++;
      double S = orc_u53_open(o[0], o[1]);
      double Acc = orc_u53(o[2], o[3]);
      /* number of skipped candidates: X ~ Geom_0(pbar) = floor(ln S / ln(1 - pbar)) */
      double q = pbar >= 1.0 ? 0.0 : log(S) / Lg;
      /* a skip length whose quotient lies within 1e-12 (relative) of an
       * integer >= 1 may round either way under another libm; it matters only
       * when it decides a candidate or the end of the segment: log the item */
      double fl = floor(q + 0.5);
      if (pbar < 1.0 && fl >= 1.0 && fabs(q - fl) < 1e-12 * q && q < (double)(kend - k) + 1.0) tie = 1;
      R->tie_expect += tie_mass(pbar, -Lg, (double)(kend - k));
      if (q >= (double)(kend - k)) break;
      k += (uint64_t)q;
      uint64_t a = k / nb, b = k % nb;
      uint64_t su = a0 + a, sv = b0 + b;
      uint32_t u = R->sid[su], v = R->sid[sv];
      R->ctr[S_CANDS]++;
      if (p->accept_all) {
        emit(R, u, v, 1);
      } else {
        double r = torus_dist(R->sx + su * (uint64_t)p->d, R->sx + sv * (uint64_t)p->d, p->d);
        double prob = p->model == 0 ? girg_p(R, R->sw[su], R->sw[sv], r)
                                    : hrg_pT(R, hrg_coshd(R->sw[su], R->sw[sv], r));
        /* the candidate is accepted with probability p_uv / pbar: the
         * coin Acc is near when it lies within 1e-12 of that ratio */
        double ratio = prob / pbar;
        if (fabs(Acc - ratio) < 1e-12) near_pair(R, u, v);
        R->near_expect += near_mass(ratio);
        if (Acc * pbar < prob) emit(R, u, v, 1);
      }
      k += 1;
      if (k >= kend) break;
    }
  }
  if (tie) {
    if (push64x4(&R->ties, a0, na, b0, nb)) R->failed = 1;
    R->ctr[S_TIES]++;
  }
}

/* ---- type-II jump sequences over the cell pairs of one source (ours). ----
 * Sec. 3.2 samples the candidates of a distant cell pair by geometric jumps
 * under pbar.  The jumps need not stop at the end of a cell pair: the
 * candidates of all distant cell pairs that share pbar are independent
 * Bernoulli(pbar) trials too, so one jump sequence can run over their
 * concatenation.  With batch_type2, at every level l >= 3 (GIRG, d = 2 or 3,
 * T > 0; at d = 1 a source has at most one distant cell per gap):
 *  - a source is a cell X at level l with vertices of layer i;
 *  - its distant cells Y are X + delta for the offsets delta of X's parity
 *    table: children of the parent's neighbours that are not neighbours,
 *    with the first nonzero component positive (so each unordered cell pair is
 *    listed at exactly one of its cells), taken in increasing order of
 *    o = sum_k (delta_k + 2 + parity_k) 6^k;
 *  - for each layer j with CL(i,j) >= l and gap g = max_k |delta_k| - 1, the
 *    cell pairs (X, Y) with V_j^Y nonempty and at most 2^(e0 - 4)
 *    candidates, e0 = 5 - ilogb(pbar) (about 2 / pbar; such a pair also fits
 *    one segment of type2()), form a sequence in that order; the candidates
 *    of an item are x |V_j^Y| + y (x in V_i^X, y in V_j^Y), and the items
 *    follow each other;
 *  - draw t of the sequence uses the counter (t, X, g, l | i | j | kind 3);
 *  - the other cell pairs are sampled by type2() as before: the larger ones
 *    (few of their first draws come up empty, and long sequences would hold
 *    many draws) and those of more than one segment.
 * Edges are written with u from the A side (the smaller cell). */
static int batched_level(const orc_run* R, int l) {
  return R->p.batch_type2 && R->p.T > 0.0 && R->p.model == 0 && R->p.d >= 2 && R->p.d <= 3 && l >= 3;
}

/* the distant offsets of parity pattern par with gap g, in increasing o */
static int seq_offsets(int d, int par, int g, int (*delta)[3]) {
  int no = 1, cnt = 0;
  for (int k = 0; k < d; k++) no *= 6;
  for (int o = 0; o < no; o++) {
    int rem = o, dm = 0, first = 0, dl[3] = {0, 0, 0};
    for (int k = 0; k < d; k++) {
      int jk = rem % 6;
      rem /= 6;
      dl[k] = jk - 2 - ((par >> k) & 1);
      int ad = dl[k] < 0 ? -dl[k] : dl[k];
      if (ad > dm) dm = ad;
      if (first == 0) first = dl[k];
    }
    if (dm < 2 || first < 0 || dm - 1 != g) continue;
    for (int k = 0; k < 3; k++) delta[cnt][k] = dl[k];
    cnt++;
  }
  return cnt;
}

typedef struct {
  uint64_t x0, nx, y0, ny, A, B; /* ranges of V_i^X and V_j^Y; A <= B the cells */
  int x_is_a;
} seq_item;

static void run_sequence(orc_run* R, int l, uint64_t X, int i, int j, int g, const seq_item* it,
                         int nit) {
  const orc_params* p = &R->p;
  double pbar_raw;
  double pbar = type2_pbar(R, l, i, j, g, &pbar_raw);
  double lg1 = log1p(-pbar);
  uint64_t total = 0;
  for (int k = 0; k < nit; k++) total += it[k].nx * it[k].ny;
  R->ctr[S_SEQS]++;
  int tie = 0;
  uint64_t pos = 0; /* candidates of the sequence before the next jump */
  int k = 0;        /* item holding position pos */
  uint64_t kstart = 0;
  for (uint64_t t = 0;; t++) {
    uint32_t o[4];
    stream_block(p->seed, (uint32_t)t, (uint32_t)X, (uint32_t)g,
                 word3(l, i, j, KIND_SEQ, (uint32_t)(t >> 32)), o);
    R->ctr[S_DRAWS]++;
    double S = orc_u53_open(o[0], o[1]);
    double Acc = orc_u53(o[2], o[3]);
    /* X ~ Geom_0(pbar) candidates skipped */
    double q = pbar >= 1.0 ? 0.0 : log(S) / lg1;
    double rest = (double)(total - pos);
    double fl = floor(q + 0.5);
    if (pbar < 1.0 && fl >= 1.0 && fabs(q - fl) < 1e-12 * q && q < rest + 1.0) tie = 1;
    R->tie_expect += tie_mass(pbar, -lg1, rest);
    if (q >= rest) break;
    pos += (uint64_t)q;
    while (pos >= kstart + it[k].nx * it[k].ny) { kstart += it[k].nx * it[k].ny; k++; }
    uint64_t loc = pos - kstart;
    uint64_t sx = it[k].x0 + loc / it[k].ny, sy = it[k].y0 + loc % it[k].ny;
    uint32_t ux = R->sid[sx], uy = R->sid[sy];
    uint32_t u = it[k].x_is_a ? ux : uy, v = it[k].x_is_a ? uy : ux;
    R->ctr[S_CANDS]++;
    if (p->accept_all) {
      emit(R, u, v, 1);
    } else {
      double r = torus_dist(R->sx + sx * (uint64_t)p->d, R->sx + sy * (uint64_t)p->d, p->d);
      double puv = p->model == 0 ? girg_p(R, R->sw[sx], R->sw[sy], r)
                                 : hrg_pT(R, hrg_coshd(R->sw[sx], R->sw[sy], r));
      /* accepted with probability p_uv / pbar; near when Acc is within
       * 1e-12 of that ratio */
      if (fabs(Acc - puv / pbar) < 1e-12) near_pair(R, u, v);
      R->near_expect += near_mass(puv / pbar);
      if (pbar * Acc < puv) emit(R, u, v, 1);
    }
    pos += 1;
    if (pos >= total) break;
  }
  if (tie) {
    /* every pair of the sequence may come out differently: log its items */
    for (int q = 0; q < nit; q++) {
      uint64_t a0 = it[q].x_is_a ? it[q].x0 : it[q].y0, na = it[q].x_is_a ? it[q].nx : it[q].ny;
      uint64_t b0 = it[q].x_is_a ? it[q].y0 : it[q].x0, nb = it[q].x_is_a ? it[q].ny : it[q].nx;
      if (push64x4(&R->ties, a0, na, b0, nb)) R->failed = 1;
    }
    R->ctr[S_TIES]++;
  }
}

/* whether the items of sources at level l >= filter level are selected by
 * the source's ancestor (filtered runs) */
static int source_selected(const orc_run* R, int l, uint64_t X) {
  const orc_params* p = &R->p;
  if (!p->filter_mod) return 1;
  if (l < p->filter_level) return !p->filter_skip_top;
  uint64_t anc = X >> (p->d * (l - p->filter_level));
  return (anc % p->filter_mod) == p->filter_rem;
}

static void type2_batched(orc_run* R) {
  const orc_params* p = &R->p;
  int d = p->d;
  static int delta[1296][3];
  seq_item* items = (seq_item*)malloc(sizeof(seq_item) * 1296);
  if (!items) { R->failed = 1; return; }
  for (int l = 3; l <= R->D; l++) {
    if (!batched_level(R, l)) continue;
    uint64_t side = (uint64_t)1 << l;
    for (int i = 0; i < R->L; i++) {
      if (!R->count[i] || R->I[i] < l) continue;
      /* the cells X of layer i at level l: runs of sorted positions */
      uint64_t s = R->lstart[i];
      while (s < R->lstart[i + 1]) {
        uint64_t X = cell_of_sorted(R, s, l), x0, nx;
        vertex_range(R, i, l, X, &x0, &nx);
        s = x0 + nx;
        if (!source_selected(R, l, X)) continue;
        uint32_t cx[8];
        orc_morton_decode(X, d, l, cx);
        int par = 0;
        for (int k = 0; k < d; k++) par |= (int)(cx[k] & 1u) << k;
        for (int g = 1; g <= 2; g++) {
          int no = seq_offsets(d, par, g, delta);
          for (int j = 0; j < R->L; j++) {
            if (!R->count[j] || R->CL[i][j] < l) continue;
            int nit = 0, seq_near = 0;
            for (int t = 0; t < no; t++) {
              uint32_t cy[8];
              for (int k = 0; k < d; k++) cy[k] = (uint32_t)((cx[k] + side + (uint64_t)(int64_t)delta[t][k]) % side);
              uint64_t Y = orc_morton_encode(cy, d, l), y0, ny;
              vertex_range(R, j, l, Y, &y0, &ny);
              if (ny == 0) continue;
              int xa = X < Y;
              uint64_t A = xa ? X : Y, B = xa ? Y : X;
              int ia = xa ? i : j, jb = xa ? j : i;
              double pr;
              double pb = type2_pbar(R, l, ia, jb, g, &pr);
              if (!(pb > 0.0)) continue;
              /* an exponent that another pow could change may move items
               * between the classes below: the sequence's items are logged */
              if (near_pow2(pr)) seq_near = 1;
              uint64_t N = nx * ny;
              int e0 = SEG_EXP - ilogb(pb), e = e0, emin = bitlen(N - 1) - SEG_MAX_BITS;
              if (e < emin) e = emin;
              uint64_t G = (e >= 63 || ((uint64_t)1 << e) >= N) ? N : ((uint64_t)1 << e);
              /* items of more than one segment (the segment rule of type2()),
               * and items of more than 2^(e0 - 4) candidates (about 2 / pbar
               * or more, so that few of their first draws come up empty), are
               * sampled by type2() with their own streams */
              if ((N + G - 1) / G > 1 || (e0 - 4 < 63 && N > ((uint64_t)1 << (e0 - 4)))) {
                type2(R, l, A, B, ia, jb);
                continue;
              }
              R->ctr[S_T2ITEMS]++;
              items[nit].x0 = x0; items[nit].nx = nx; items[nit].y0 = y0; items[nit].ny = ny;
              items[nit].A = A; items[nit].B = B; items[nit].x_is_a = xa;
              nit++;
            }
            if (nit && seq_near) {
              for (int q = 0; q < nit; q++) {
                uint64_t a0 = items[q].x_is_a ? items[q].x0 : items[q].y0;
                uint64_t na = items[q].x_is_a ? items[q].nx : items[q].ny;
                uint64_t b0 = items[q].x_is_a ? items[q].y0 : items[q].x0;
                uint64_t nb = items[q].x_is_a ? items[q].ny : items[q].nx;
                if (push64x4(&R->ties, a0, na, b0, nb)) R->failed = 1;
              }
              R->ctr[S_TIES]++;
            }
            if (nit) run_sequence(R, l, X, i, j, g, items, nit);
          }
        }
      }
    }
  }
  free(items);
}

/* ---- Algorithm 1: recursive iteration of cell pairs (Sec. 3.3). ---- */
static int any_nonempty(const orc_run* R, int l, uint64_t A) {
  /* some layer with I(i) > l has vertices in A (a recursion below l can only
   * touch such layers) */
  for (int i = 0; i < R->L; i++) {
    if (R->count[i] == 0 || R->I[i] <= l) continue;
    uint64_t f, num;
    vertex_range(R, i, l, A, &f, &num);
    if (num) return 1;
  }
  return 0;
}

static void recur(orc_run* R, int l, uint64_t A, uint64_t B, int nb, int selected) {
  const orc_params* p = &R->p;
  if (p->filter_mod && l == p->filter_level) selected = (A % p->filter_mod) == p->filter_rem;
  if (selected && !(p->filter_mod && p->filter_skip_top && l < p->filter_level)) {
    R->ctr[nb ? S_NBPAIRS : S_DISTPAIRS]++;
    if (nb) R->lvl_nb[l]++; else R->lvl_dist[l]++;
    /* for all bucket pairs (i,j) that process (A,B): neighbouring pairs at
     * level l serve pairs with CL(i,j) = l, distant ones those with CL >= l
     * (loop swap, Sec. 3.3).  A <= B; for A = B only i <= j (App. B.1). */
    for (int i = 0; i < R->L; i++) {
      if (R->count[i] == 0) continue;
      for (int j = 0; j < R->L; j++) {
        if (R->count[j] == 0) continue;
        if (A == B && j < i) continue;
        if (nb) {
          if (R->CL[i][j] == l) type1(R, l, A, B, i, j);
        } else {
          /* threshold variants: distant cells hold no edges (their points are
           * farther apart than the cell side, which is at least the threshold);
           * batched runs sample levels >= 3 by source cell afterwards */
          if (R->CL[i][j] >= l && p->T > 0.0 && !batched_level(R, l)) type2(R, l, A, B, i, j);
        }
      }
    }
  }
  if (!nb || l >= R->D) return;
  /* a sampled run: below the filter level the selection is fixed */
  if (!selected && p->filter_mod && l >= p->filter_level) return;
  /* children of neighbouring pairs, A <= B */
  if (!any_nonempty(R, l, A) || !any_nonempty(R, l, B)) return;
  int d = p->d;
  uint64_t nch = (uint64_t)1 << d;
  for (uint64_t x = 0; x < nch; x++)
    for (uint64_t y = 0; y < nch; y++) {
      uint64_t X = (A << d) | x, Y = (B << d) | y;
      if (A == B && Y < X) continue;
      recur(R, l + 1, X, Y, are_neighbours(R, X, Y, l + 1), selected);
    }
}

/* ---- setup: layers, levels, sorted layout ---- */
static const orc_run* g_sort_ctx;
static int cmp_sorted(const void* a, const void* b) {
  uint32_t u = *(const uint32_t*)a, v = *(const uint32_t*)b;
  const orc_run* R = g_sort_ctx;
  if (R->layer[u] != R->layer[v]) return R->layer[u] < R->layer[v] ? -1 : 1;
  if (R->morton[u] != R->morton[v]) return R->morton[u] < R->morton[v] ? -1 : 1;
  return (u > v) - (u < v);
}

orc_run* orc_run_graph(const orc_params* pin, const double* w, const double* x) {
  const orc_params* p = pin;
  uint64_t n = p->n;
  int d = p->d;
  if (n < 1 || n > 0xFFFFFFFFull) { set_err("n must be in [1, 2^32-1]"); return NULL; }
  if (d < 1 || d > 8) { set_err("d must be in [1, 8]"); return NULL; }
  if (p->model == 1 && d != 1) { set_err("HRG requires d = 1"); return NULL; }
  if (!(p->T >= 0.0 && p->T < 1.0)) { set_err("T must be in [0, 1)"); return NULL; }
  if (p->model == 0 && !(p->c > 0.0)) { set_err("c must be > 0"); return NULL; }
  if (p->model == 1 && !(p->R > 0.0)) { set_err("R must be > 0"); return NULL; }
  if (p->T == 0.0 && p->cl_bias > 0) { set_err("cl_bias > 0 is inexact at T = 0"); return NULL; }
  orc_run* R = (orc_run*)calloc(1, sizeof(orc_run));
  if (!R) { set_err("out of memory"); return NULL; }
  R->p = *p;
  R->Dmax = 32 / d;
  R->layer = (int32_t*)malloc(sizeof(int32_t) * n);
  R->morton = (uint64_t*)malloc(sizeof(uint64_t) * n);
  R->sid = (uint32_t*)malloc(sizeof(uint32_t) * n);
  R->spos = (uint32_t*)malloc(sizeof(uint32_t) * n);
  R->sw = (double*)malloc(sizeof(double) * n);
  R->sx = (double*)malloc(sizeof(double) * n * d);
  if (!R->layer || !R->morton || !R->sid || !R->spos || !R->sw || !R->sx) {
    orc_free(R); set_err("out of memory"); return NULL;
  }
  for (uint64_t u = 0; u < n * (uint64_t)d; u++)
    if (!(x[u] >= 0.0 && x[u] < 1.0)) { orc_free(R); set_err("positions must lie in [0,1)"); return NULL; }

  /* weight buckets (Sec. 3.1): max / min weight within a bucket at most 2 */
  if (p->model == 0) {
    R->W = sum_ld(w, n);
    double w0 = w[0];
    for (uint64_t u = 0; u < n; u++) {
      if (!(w[u] > 0.0) || isinf(w[u])) { orc_free(R); set_err("weights must be finite and > 0"); return NULL; }
      if (w[u] < w0) w0 = w[u];
    }
    R->w0 = w0;
    for (uint64_t u = 0; u < n; u++) {
      int li = ilogb(w[u] / w0);
      if (li >= ORC_MAX_LAYERS) { orc_free(R); set_err("weight range exceeds 2^64"); return NULL; }
      R->layer[u] = li;
    }
  } else {
    /* HRG -> GIRG mapping (Sec. 2.3): w = exp((R - r)/2), so the bucket of a
     * vertex is floor(log2 w) = floor((R - r) / (2 ln 2)). */
    R->coshR = cosh(p->R);
    for (uint64_t u = 0; u < n; u++) {
      if (!(w[u] >= 0.0 && w[u] <= p->R)) { orc_free(R); set_err("radii must lie in [0, R]"); return NULL; }
      int li = (int)floor((p->R - w[u]) / (2.0 * 0.6931471805599453));
      if (li >= ORC_MAX_LAYERS) { orc_free(R); set_err("radius range too large"); return NULL; }
      R->layer[u] = li;
    }
  }
  R->L = 0;
  for (int i = 0; i < ORC_MAX_LAYERS; i++) { R->count[i] = 0; R->ext[i] = 0.0; }
  for (uint64_t u = 0; u < n; u++) {
    int li = R->layer[u];
    if (li + 1 > R->L) R->L = li + 1;
    if (R->count[li] == 0 || (p->model == 0 ? w[u] > R->ext[li] : w[u] < R->ext[li])) R->ext[li] = w[u];
    R->count[li]++;
  }

  /* comparison levels (Sec. 3.1): the deepest level whose cell side is at
   * least the connection threshold of the largest weights of the two buckets;
   * HRG: found by search over levels (Sec. 4.3). */
  int Dcap = (bitlen(n) + 3) / d;
  if (Dcap > R->Dmax) Dcap = R->Dmax;
  if (p->model == 0) R->kappa = p->T > 0.0 ? pow(p->c, p->T) : 0.0;
  for (int i = 0; i < ORC_MAX_LAYERS; i++)
    for (int j = 0; j < ORC_MAX_LAYERS; j++) R->CL[i][j] = -1;
  R->D = 0;
  for (int i = 0; i < R->L; i++) {
    if (!R->count[i]) continue;
    for (int j = 0; j < R->L; j++) {
      if (!R->count[j]) continue;
      int l = 0;
      if (p->model == 0 && p->T == 0.0) {
        double tmax = p->c * pow(R->ext[i] * R->ext[j] / R->W, 1.0 / d);
        while (l < Dcap && ldexp(1.0, -(l + 1)) >= tmax) l++;
      } else if (p->model == 0) {
        double V = R->kappa * R->ext[i] * R->ext[j] / R->W;
        while (l < Dcap && ldexp(1.0, -(l + 1) * d) >= V) l++;
      } else {
        double shh = 2.0 * sinh(R->ext[i]) * sinh(R->ext[j]);
        while (l < Dcap) {
          int nl = l + 1;
          if (nl >= 2) {
            double s = sin(M_PI * ldexp(1.0, -nl));
            if (!(1.0 + shh * s * s >= R->coshR)) break;
          }
          l = nl;
        }
      }
      l += p->cl_bias;
      if (l < 0) l = 0;
      if (l > Dcap) l = Dcap;
      if (p->max_depth >= 0 && l > p->max_depth) l = p->max_depth;
      R->CL[i][j] = l;
      if (l > R->D) R->D = l;
    }
  }
  for (int i = 0; i < R->L; i++) {
    R->I[i] = -1;
    if (!R->count[i]) continue;
    for (int j = 0; j < R->L; j++)
      if (R->count[j] && R->CL[i][j] > R->I[i]) R->I[i] = R->CL[i][j];
  }

  /* cells: Morton code at level Dmax; the cell at level l is its top d*l bits */
  for (uint64_t u = 0; u < n; u++) {
    uint32_t q[8];
    for (int k = 0; k < d; k++) q[k] = (uint32_t)(x[u * (uint64_t)d + k] * ldexp(1.0, R->Dmax));
    R->morton[u] = orc_morton_encode(q, d, R->Dmax);
  }
  /* sort by (bucket, Morton code, id): within a bucket this orders vertices by
   * their cell on every level, in particular on I(i) (Sec. 3.4); the paper
   * leaves the tie-break free, we break ties by the finer cells, then by id. */
  for (uint64_t u = 0; u < n; u++) R->sid[u] = (uint32_t)u;
  g_sort_ctx = R;
  qsort(R->sid, n, sizeof(uint32_t), cmp_sorted);
  for (uint64_t s = 0; s < n; s++) {
    uint32_t u = R->sid[s];
    R->spos[u] = (uint32_t)s;
    R->sw[s] = w[u];
    for (int k = 0; k < d; k++) R->sx[s * d + k] = x[u * (uint64_t)d + k];
  }
  uint64_t acc = 0;
  for (int i = 0; i < R->L; i++) { R->lstart[i] = acc; acc += (uint64_t)R->count[i]; }
  R->lstart[R->L] = acc;
  /* prefix sums P_C per bucket at its insertion level (Lemma 1, App. A) */
  for (int i = 0; i < R->L; i++) {
    if (!R->count[i]) continue;
    uint64_t ncell = (uint64_t)1 << (d * R->I[i]);
    R->P[i] = (uint32_t*)calloc(ncell + 1, sizeof(uint32_t));
    if (!R->P[i]) { orc_free(R); set_err("out of memory (cell offsets)"); return NULL; }
    for (uint64_t s = R->lstart[i]; s < R->lstart[i + 1]; s++) R->P[i][cell_of_sorted(R, s, R->I[i]) + 1]++;
    R->P[i][0] = (uint32_t)R->lstart[i];
    for (uint64_t cidx = 1; cidx <= ncell; cidx++) R->P[i][cidx] += R->P[i][cidx - 1];
  }

  recur(R, 0, 0, 0, 1, p->filter_mod == 0 || p->filter_level > 0);
  if (batched_level(R, 3)) type2_batched(R);
  if (R->failed) { orc_free(R); set_err("out of memory (edges)"); return NULL; }
  return R;
}

uint64_t orc_num_edges(const orc_run* r) { return r->edges.n / 2; }
void orc_copy_edges(const orc_run* r, uint32_t* out) { memcpy(out, r->edges.a, r->edges.n * sizeof(uint32_t)); }
uint64_t orc_num_near(const orc_run* r) { return r->near.n / 2; }
void orc_copy_near(const orc_run* r, uint32_t* out) { memcpy(out, r->near.a, r->near.n * sizeof(uint32_t)); }
uint64_t orc_num_ties(const orc_run* r) { return r->ties.n / 4; }
void orc_copy_ties(const orc_run* r, uint64_t* out) { memcpy(out, r->ties.a, r->ties.n * sizeof(uint64_t)); }
void orc_copy_sorted_ids(const orc_run* r, uint32_t* out) { memcpy(out, r->sid, r->p.n * sizeof(uint32_t)); }

void orc_stats(const orc_run* r, double* out) {
  for (int k = 0; k < ORC_NSTATS; k++) out[k] = (double)r->ctr[k];
  out[0] = r->W; out[1] = r->w0; out[2] = r->L; out[3] = r->D; out[4] = r->Dmax;
  out[16] = r->p.model == 0 ? r->kappa : r->coshR;
  out[19] = r->near_expect;
  out[20] = r->tie_expect;
}

void orc_level_counts(const orc_run* r, uint64_t* nb, uint64_t* dist) {
  for (int l = 0; l < 40; l++) { nb[l] = r->lvl_nb[l]; dist[l] = r->lvl_dist[l]; }
}

void orc_tables(const orc_run* r, int32_t* CL, int32_t* I, int64_t* count, double* ext) {
  for (int i = 0; i < ORC_MAX_LAYERS; i++) {
    for (int j = 0; j < ORC_MAX_LAYERS; j++) CL[i * ORC_MAX_LAYERS + j] = r->CL[i][j];
    I[i] = i < r->L ? r->I[i] : -1;
    count[i] = r->count[i];
    ext[i] = r->ext[i];
  }
}

void orc_pair_item(const orc_run* r, uint32_t u, uint32_t v, int64_t* out) {
  int d = r->p.d;
  int i = r->layer[u], j = r->layer[v];
  int cl = r->CL[i][j];
  int level = cl, type = 0;
  for (int l = 2; l <= cl; l++) {
    uint64_t A = r->morton[u] >> (d * (r->Dmax - l)), B = r->morton[v] >> (d * (r->Dmax - l));
    if (!are_neighbours(r, A, B, l)) { level = l; type = 1; break; }
  }
  uint64_t A = r->morton[u] >> (d * (r->Dmax - level)), B = r->morton[v] >> (d * (r->Dmax - level));
  int swapped = 0;
  if (A > B) swapped = 1;
  else if (A == B && j < i) swapped = 1;
  else if (A == B && i == j) {
    /* local order a < b inside V_i^A: sorted position */
    swapped = r->spos[u] > r->spos[v];
  }
  out[0] = level;
  out[1] = (int64_t)(swapped ? B : A);
  out[2] = (int64_t)(swapped ? A : B);
  out[3] = swapped ? j : i;
  out[4] = swapped ? i : j;
  out[5] = type;
  out[6] = swapped;
}

/* The key of an edge in the canonical order of the cell-pair iteration: the
 * item (level, A, B, i, j) that holds the pair, with A <= B and the ordered
 * layer pair of App. B.1, and the pair index k inside it (a |V_j^B| + b, or
 * b (b - 1) / 2 + a with a < b when A = B and i = j, a and b counted from
 * the first sorted positions of V_i^A and V_j^B).  out8[7] = 1 when the edge
 * is written (B side, A side), i.e. not with u from the A side. */
void orc_edge_keys(const orc_run* r, const uint32_t* edges, uint64_t m, int64_t* out8) {
  for (uint64_t e = 0; e < m; e++) {
    uint32_t u = edges[2 * e], v = edges[2 * e + 1];
    int64_t it[7];
    orc_pair_item(r, u, v, it);
    int level = (int)it[0], i = (int)it[3], j = (int)it[4];
    uint64_t A = (uint64_t)it[1], B = (uint64_t)it[2];
    int swapped = (int)it[6];
    uint64_t su = r->spos[swapped ? v : u], sv = r->spos[swapped ? u : v];
    uint64_t a0, na, b0, nb;
    vertex_range(r, i, level, A, &a0, &na);
    vertex_range(r, j, level, B, &b0, &nb);
    uint64_t a = su - a0, b = sv - b0, k;
    if (A == B && i == j) k = b * (b - 1) / 2 + a; /* here a < b */
    else k = a * nb + b;
    int64_t* o = out8 + 8 * e;
    o[0] = level; o[1] = (int64_t)A; o[2] = (int64_t)B; o[3] = i; o[4] = j;
    o[5] = (int64_t)k; o[6] = it[5]; o[7] = swapped;
  }
}
