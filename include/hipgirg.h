/*
 * hipgirg.h -- C ABI of the MI355X (gfx950) sampler for geometric
 * inhomogeneous random graphs (GIRGs) and hyperbolic random graphs (HRGs)
 * after Blaesius, Friedrich, Katzmann, Meyer, Penschuck, Weyand,
 * "Efficiently Generating Geometric Inhomogeneous and Hyperbolic Random
 * Graphs" (arXiv:1905.06706).
 *
 * Conventions shared by every call
 *  - Every call returns a girg_status; no C++ exception crosses the ABI.  On
 *    an error girg_last_error() returns a message (thread-local, valid until
 *    the next call on that thread).
 *  - "device pointer" arguments are HIP device allocations on the current
 *    device; the caller owns them.  The library owns only internal scratch
 *    memory, cached per device and grown on demand (freed by girg_release).
 *  - `stream` is a hipStream_t (passed as void*; NULL = the null stream).
 *    Calls are stream-ordered but synchronise that stream before returning
 *    (they read small results, such as the edge count, back to the host).
 *  - Positions are stored dimension-major: x[k * n + v] is coordinate k of
 *    vertex v.  Vertex ids are 0..n-1 in generation order.
 *  - Edges are written as uint32 pairs (u, v), edges[2e], edges[2e+1], with
 *    u != v and every unordered pair at most once.  Their order is
 *    deterministic: a pure function of the parameters and the seed.
 *  - Randomness: Philox4x32-10 (Salmon et al., SC 2011) keyed by the seed;
 *    the counter packs (level, cell pair, layer pair, kind, index).  Two calls
 *    with equal parameters and seed return identical edge arrays.
 */
#ifndef HIPGIRG_H
#define HIPGIRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GIRG_OK = 0,
  GIRG_EINVAL = -1,    /* invalid parameter (message says which) */
  GIRG_ENOMEM = -2,    /* device or host allocation failed */
  GIRG_EDEVICE = -3,   /* a HIP call failed (no device, launch failure) */
  GIRG_EOVERFLOW = -4, /* edge capacity too small: *m_out holds the edge count
                          needed and *info the call's diagnostics; the edge
                          buffer contents are undefined.  A null buffer with
                          capacity 0 thus counts a graph without storing it */
  GIRG_ENOCONV = -5    /* the c or R solve found no bracket */
} girg_status;

/* Model parameters.
 *  GIRG (model 0), Eq. (1) of Sec. 2.1: p_uv = min(1, c ((w_u w_v / W) /
 *    ||x_u - x_v||^d)^(1/T)) for 0 < T < 1; threshold variant at T = 0: edge
 *    iff ||x_u - x_v|| <= c (w_u w_v / W)^(1/d).  ||.|| is the L-infinity
 *    distance on the torus [0,1)^d.
 *  HRG (model 1), Sec. 2.2: radii r in [0,R) with density
 *    alpha sinh(alpha r) / (cosh(alpha R) - 1), angles uniform; threshold
 *    variant: edge iff the hyperbolic distance is below R; binomial variant:
 *    p_T(d) = 1 / (exp((d - R) / (2T)) + 1).
 * Validation: n in [2, 2^32-1]; GIRG: d in [1, 4], beta > 2, 0 <= T < 1,
 * exactly one of avg_deg > 0 (solve c, Sec. 4.1 / App. B.2) or c > 0;
 * HRG: alpha > 1/2, 0 <= T < 1, R > 0 given or avg_deg > 0 (solve R). */
typedef struct {
  uint64_t n;
  int32_t d;          /* GIRG dimension (HRG: ignored, 1) */
  int32_t model;      /* 0 = GIRG, 1 = HRG */
  double beta;        /* GIRG power-law exponent of the weights (w_min = 1) */
  double T;           /* temperature */
  double avg_deg;     /* expected average degree (0 = use c / R) */
  double c;           /* GIRG constant (0 = solve from avg_deg) */
  double alpha;       /* HRG radial dispersion */
  double R;           /* HRG disk radius (0 = solve from avg_deg) */
  uint64_t seed;
  int32_t precision;  /* 0 = FP64; 1 = FP32 filter with FP64 recheck */
  int32_t max_depth;  /* debug knob, -1 = none: caps the comparison levels */
  int32_t cl_bias;    /* debug knob, 0 = none: shifts the comparison levels
                         (> 0 only for T > 0); every value samples exactly */
  int32_t type2_batch; /* 1: at levels >= 3 of binomial GIRGs with d = 2 or 3,
                          one geometric-jump sequence (Sec. 3.2) runs over the
                          distant cell pairs of a source cell that share the
                          bound pbar and have at most 2^(1 - ilogb(pbar))
                          candidates each (fewer draws; another random
                          stream, the same distribution); needs at most 32
                          weight layers (GIRG_EINVAL otherwise); 0: one
                          sequence per cell pair */
} girg_params;

/* Diagnostics of one call. */
typedef struct {
  uint64_t m;            /* edges */
  uint64_t type1_edges, type2_edges;
  uint64_t tests;        /* type-I pair tests */
  uint64_t draws;        /* type-II geometric draws */
  uint64_t candidates;   /* type-II candidates tested */
  uint64_t rechecks;     /* mixed precision: decisions re-done in FP64 */
  uint64_t sources;      /* (layer, level, cell) runs */
  uint64_t heavy_items;  /* type-II items split into segments */
  uint64_t split_items;  /* type-I items split into pieces of tests */
  uint64_t cells;        /* prefix-sum entries */
  double c, W, R;        /* constants used */
  int32_t L, D;          /* layers, deepest level */
  int32_t reserved[2];
  /* per sampling pass (0 type-I, 1 split type-I items, 2 type-II, 3
   * segmented type-II items): edges, work units (tests for 0-1, draws for
   * 2-3) and type-II candidates */
  uint64_t pass_edges[4], pass_work[4], pass_cands[4];
  /* decisions inside the parity margins (expected about 0): near_boundary =
   * coins within 1e-12 of what they are compared with (type I: |U - p_uv|;
   * type II: |Acc - p_uv / pbar| for the acceptance coin Acc of Sec. 3.2;
   * threshold variants: distance within 1e-12, relative, of the threshold);
   * skip_ties = type-II draws whose skip quotient ln S / ln(1 - pbar) lies
   * within 1e-12 (relative) of an integer >= 1 that can still decide a
   * candidate or the end of the item.  Only such decisions can come out
   * differently under another rounding of the same formulas. */
  uint64_t near_boundary, skip_ties;
} girg_info;

/* girg_generate: points (Sec. 2.1 weights and positions), constant c
 * (App. B.2) when avg_deg > 0, then the sampler of Sec. 3 (Algorithm 1 with
 * type-I tests and type-II geometric jumps).  edges: device pointer to
 * 2*cap uint32.  m_out: host pointer.  info: host pointer or NULL.
 * The sampling passes defer long items to two lists of a first capacity of
 * half an entry per source (at most 2^27); when one overflows, both passes
 * run once more with the lists at their exact sizes (same result, more
 * time).  The environment variable GIRG_DEFER_CAPACITY = 1..2^30, read at
 * every call, sets that first capacity (e.g. to exercise the rerun). */
girg_status girg_generate(const girg_params* p, uint32_t* edges, uint64_t cap, uint64_t* m_out,
                          girg_info* info, void* stream);

/* girg_hrg: HRG of Sec. 2.2 through the GIRG mapping of Sec. 2.3 (w =
 * exp((R - r)/2), x = theta / 2 pi) with the HRG decisions of Sec. 4.3.  R
 * (> 0) is used as given; R = 0 solves it from avg_deg. */
girg_status girg_hrg(uint64_t n, double alpha, double T, double R, double avg_deg, uint64_t seed,
                     uint32_t* edges, uint64_t cap, uint64_t* m_out, girg_info* info, void* stream);

/* girg_from_points: the sampler of Sec. 3 alone (weight layers and levels of
 * Sec. 3.1, type-I tests and type-II geometric jumps of Sec. 3.2, the cell
 * pairs of Algorithm 1 in Sec. 3.3, the Morton layout of Sec. 3.4) over
 * caller-provided points, which is the problem statement of Sec. 2 with the
 * weights and positions given (the paper lets the user supply weights).
 * Device pointers.  GIRG: w = weights (> 0), x = positions in [0,1),
 * dimension-major [d][n]; c given or solved from avg_deg over these weights
 * (App. B.2).  HRG: w = radii in [0, R], x = angle / (2 pi) in [0,1); R must
 * be given (Sec. 2.2, mapped as in Sec. 2.3).  Errors: GIRG_EINVAL for a
 * weight <= 0 or not finite, a position outside [0,1), a radius outside
 * [0, R], more than 64 weight layers; the edge buffer is then untouched. */
girg_status girg_from_points(const girg_params* p, const double* w, const double* x,
                             uint32_t* edges, uint64_t cap, uint64_t* m_out, girg_info* info,
                             void* stream);

/* girg_from_points_noalloc: girg_from_points for callers that cannot allocate
 * device memory (code under HIP graph capture around it, tight serving loops,
 * harnesses that forbid hipMalloc): it calls no hipMalloc, hipFree,
 * hipHostMalloc or other allocating routine.  Every device buffer of the call
 * lies in one fixed array of 512 MiB of device memory that each GPU holds from
 * the library's first use on it until the process ends; the first call on a
 * device looks up that GPU's copy of the array.  Same arguments, edges and
 * info as girg_from_points, with these limits: n <= 2^20, cap <= 2^24 edges,
 * c > 0 given (GIRG; solving c needs host buffers) or R > 0 (HRG); profiling
 * is not recorded.  GIRG_EINVAL for a limit exceeded; GIRG_ENOMEM when the
 * graph's scratch needs more than the array (message says so).  The array
 * keeps the last call's contents; every call clears what must start at zero.
 * Calls on one device share the array: they run one at a time (a lock) and
 * return only after their work on the GPU has ended, so they never overlap;
 * a caller's own kernels must not touch the array's contents. */
girg_status girg_from_points_noalloc(const girg_params* p, const double* w, const double* x,
                                     uint32_t* edges, uint64_t cap, uint64_t* m_out,
                                     girg_info* info, void* stream);

/* girg_points: only the point generation of the models.  GIRG (Sec. 2.1):
 * weights of a power law with exponent beta, drawn as Pareto w = S^(-1/(beta-1))
 * with w_min = 1 (the paper fixes no sampler), positions uniform on the torus
 * as multiples of 2^-53; w[n], x[d][n].  HRG (Sec. 2.2): radii of density
 * alpha sinh(alpha r) / (cosh(alpha R) - 1) on [0, R) by the inverse CDF,
 * angles uniform; r[n], x[n] = angle / (2 pi); R required.  Device pointers
 * owned by the caller; the call draws from the stream's point counters
 * (vertex id, purpose), so any prefix of ids gives the same points. */
girg_status girg_points(const girg_params* p, double* w, double* x, void* stream);

/* girg_solve_c: c for a target average degree over given weights (host
 * pointer), App. B.2: exponential then binary search on the monotone
 * expected average degree f(c). */
girg_status girg_solve_c(const double* w_host, uint64_t n, int32_t d, double T, double avg_deg,
                         double* c_out);

/* girg_expected_degree: f(c) of App. B.2 for given weights (host pointer). */
girg_status girg_expected_degree(const double* w_host, uint64_t n, int32_t d, double T, double c,
                                 double* deg_out);

/* hrg_solve_R: radius R with the given expected average degree (numerical
 * integration over the model of Sec. 2.2; the paper gives no formula). */
girg_status hrg_solve_R(uint64_t n, double alpha, double T, double avg_deg, double* R_out);

/* hrg_expected_degree: expected average degree of an HRG with radius R. */
girg_status hrg_expected_degree(uint64_t n, double alpha, double T, double R, double* deg_out);

/* girg_generate_batch: no passage of the paper defines it; Sec. 5.2 (HRG run
 * time comparison) only notes that one often needs many graphs rather than
 * one huge instance, and then runs instances side by side.  `count`
 * independent GIRGs
 * p[0..count-1], each sampled exactly as girg_generate would; graph b's
 * edges occupy edges[2*offsets[b] .. 2*offsets[b+1]) and carry its own vertex
 * ids.  offsets: host pointer to count+1 entries; infos: host array of count
 * or NULL.  GIRG_EOVERFLOW leaves offsets[count] = edges needed.  Instances
 * run concurrently, each on a worker with its own device scratch and
 * non-blocking stream (the tuned worker count, 16 by default; the
 * environment variable GIRG_BATCH_WORKERS = 1..64 overrides the table);
 * the workers' streams start after the work queued on `stream` before the
 * call, and the edges are put in instance order on `stream`; the call
 * returns when they are in place. */
girg_status girg_generate_batch(const girg_params* p, int32_t count, uint32_t* edges, uint64_t cap,
                                uint64_t* offsets, girg_info* infos, void* stream);

/* Launch-shape tuning.  The sampling passes run as persistent grids whose
 * waves take chunks of work by ticket; every chunk's edges are placed by the
 * chunk's index, so the number of workgroups changes the speed but never an
 * edge or its position.  The library keeps a table: workgroups per workload
 * class (model, d, T > 0, floor(log2 n)) for single graphs, and one
 * (workgroups, workers) pair for batches.  Defaults: 512 workgroups below
 * n = 2^22 for T > 0 and below n = 2^17 for T = 0, else 1024; batches 256
 * and 16 workers.  At the first call the
 * JSON file named by GIRG_TUNING_FILE, if set, is loaded.
 *
 * girg_autotune: times count-only runs of *p (every sampling pass, no edge
 * array) with 256, 512, 768, 1024, 1536 and 2048 workgroups, `reps` runs
 * each (1..100) after one warm-up, and stores the fastest for p's class;
 * *blocks_out (may be NULL) receives it.  Uses the device and `stream` of a
 * girg_generate call.
 * girg_autotune_batch: the same for a batch (p[0..count-1]): 128, 256, 512,
 * 768 and 1024 workgroups per instance with 8 and 16 workers.
 * girg_tuning_get: the values the next call with *p would use (batch != 0:
 * as a batch instance); girg_tuning_set stores them (batch: workers 0 keeps
 * the current count; blocks in 1..8192, workers in 0..64).
 * girg_tuning_save / girg_tuning_load: the table as JSON, {"version": 1,
 * "single": [{"model", "d", "binomial", "log2n", "blocks"}, ...], "batch":
 * {"blocks", "workers"}}; a load that fails leaves the table unchanged
 * (GIRG_EINVAL with the reason).  girg_tuning_reset restores the defaults.
 * Tuning calls on one process share the table; autotuning while other calls
 * run changes their speed, not their results. */
girg_status girg_autotune(const girg_params* p, int32_t reps, void* stream, int32_t* blocks_out);
girg_status girg_autotune_batch(const girg_params* p, int32_t count, int32_t reps, int32_t* blocks_out,
                                int32_t* workers_out);
girg_status girg_tuning_get(const girg_params* p, int32_t batch, int32_t* blocks_out, int32_t* workers_out);
girg_status girg_tuning_set(const girg_params* p, int32_t batch, int32_t blocks, int32_t workers);
girg_status girg_tuning_save(const char* path);
girg_status girg_tuning_load(const char* path);
girg_status girg_tuning_reset(void);

/* Profiling: with girg_set_profiling(1), every later call on this device
 * records HIP events around its stages on the call's own stream; type I and
 * its split pass, which run concurrently with type II and its segmented pass
 * on a second stream of the library's, are timed on that stream, so their
 * times overlap.  girg_set_profiling(2) does the same but runs those passes
 * one after another on the call's stream (same edges), so that each sampling
 * kernel's time is its own, as a kernel trace sees it.  0 turns it off.
 * girg_stage_times copies the durations (milliseconds) and names of the last
 * call's stages (at most `max`; either array may be NULL) and returns how many
 * there were, or -1 on error.  Names stay valid until the next call. */
girg_status girg_set_profiling(int32_t on);
int32_t girg_stage_times(double* ms, const char** names, int32_t max);

/* Frees the scratch memory cached for the current device.  No other call of
 * the library may be in progress on this device meanwhile.  (Other calls are
 * safe to make from several host threads at once: single-graph calls on a
 * device share one context and run one after another.) */
girg_status girg_release(void);

const char* girg_last_error(void);

/* Library version string. */
const char* girg_version(void);

#ifdef __cplusplus
}
#endif
#endif
