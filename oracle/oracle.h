/*
 * oracle.h -- plain, sequential, FP64 reference implementation ("the oracle")
 * of the GIRG sampler and its HRG adaptation from
 *   T. Blaesius, T. Friedrich, M. Katzmann, U. Meyer, M. Penschuck, C. Weyand,
 *   "Efficiently Generating Geometric Inhomogeneous and Hyperbolic Random
 *   Graphs", arXiv:1905.06706.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library: both implement the same random-number contract (Philox4x32-10
 * from its published definition) and the same readings of the paper, each in
 * its own source.
 *
 * Every function states the passage of the paper it follows.  All floating
 * point work is IEEE binary64 with plain <math.h>; the file is compiled with
 * -ffp-contract=off and without fast-math.
 */
#ifndef GIRG_ORACLE_H
#define GIRG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LAYERS 64

/* Parameters of one sampling run over given points (Sec. 2 models, Sec. 3
 * algorithm).  model 0 = GIRG (w = weights, x = torus positions, Eq. (1) /
 * threshold variant); model 1 = HRG (w = radii r, x = angle / (2 pi),
 * Sec. 2.2, mapped to a 1-dimensional GIRG structure as in Sec. 2.3). */
typedef struct orc_params {
  uint64_t n;
  int32_t d;            /* torus dimension (1 for HRG) */
  int32_t model;        /* 0 GIRG, 1 HRG */
  double T;             /* temperature, 0 = threshold variant */
  double c;             /* GIRG constant c of Eq. (1) */
  double alpha, R;      /* HRG parameters */
  uint64_t seed;        /* Philox key */
  int32_t max_depth;    /* < 0: none.  Any value is exact (caps CL). */
  int32_t cl_bias;      /* added to the natural comparison level (T>0 only when > 0) */
  int32_t accept_all;   /* instrumentation: type-I emits every pair, type-II uses
                           pbar = 1 and accepts every candidate (coverage test) */
  int32_t filter_level; /* subtree sampling: with filter_mod > 0, a cell pair at  */
  uint32_t filter_mod;  /* level >= filter_level is processed only if its level-  */
  uint32_t filter_rem;  /* filter_level A-side ancestor a has a % mod == rem      */
  int32_t filter_skip_top; /* with filter_mod > 0: the cell pairs above        */
                           /* filter_level are walked but not sampled, so that  */
                           /* runs over the remainders mod filter_mod and one   */
                           /* run of the top levels alone partition the graph   */
  int32_t batch_type2;     /* 1: at levels >= 3 (GIRG, d = 2, 3, T > 0) the     */
                           /* cell pairs of one source cell X and layer i that  */
                           /* share a bound pbar (layer j, gap g) and have at   */
                           /* most 2^(1 - ilogb(pbar)) candidates run one jump  */
                           /* sequence over their concatenated candidates; the  */
                           /* filter then selects a sequence by X's ancestor    */
} orc_params;

typedef struct orc_run orc_run;

/* ---- random-number contract ------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u53(uint32_t lo, uint32_t hi);      /* [0,1) */
double orc_u53_open(uint32_t lo, uint32_t hi); /* (0,1] */

/* ---- Morton code (Sec. 4.2 / App. B.3) ---------------------------------- */
uint64_t orc_morton_encode(const uint32_t* coord, int d, int bits);
void orc_morton_decode(uint64_t code, int d, int bits, uint32_t* coord);

/* ---- point generation (Sec. 2.1, Sec. 2.2) ------------------------------ */
void orc_points_girg(uint64_t n, int d, double beta, uint64_t seed, double* w, double* x);
void orc_points_hrg(uint64_t n, double alpha, double R, uint64_t seed, double* r, double* x);

/* ---- average degree / constant estimation (Sec. 4.1, App. B.2) --------- */
double orc_expected_avg_degree(uint64_t n, int d, double T, double c, const double* w);
int orc_solve_c(uint64_t n, int d, double T, double avg_deg, const double* w, double* c_out);
/* HRG: expected average degree for radius R (numerical integration) and its
 * inverse by root finding.  The paper gives no formula for R from the
 * average degree: the integral is taken over the model of Sec. 2.2. */
double orc_hrg_expected_avg_degree(uint64_t n, double alpha, double T, double R);
int orc_hrg_solve_R(uint64_t n, double alpha, double T, double avg_deg, double* R_out);

/* ---- sampling (Sec. 3, Algorithm 1, App. B.1) --------------------------- */
/* w: weights (GIRG) or radii (HRG), x: n*d positions, row-major.  Returns
 * NULL and sets orc_last_error() on invalid input. */
orc_run* orc_run_graph(const orc_params* p, const double* w, const double* x);
const char* orc_last_error(void);
void orc_free(orc_run* run);

uint64_t orc_num_edges(const orc_run* run);
void orc_copy_edges(const orc_run* run, uint32_t* out);      /* 2*m, (u,v) pairs */
uint64_t orc_num_near(const orc_run* run);
void orc_copy_near(const orc_run* run, uint32_t* out);       /* 2*k pairs */
uint64_t orc_num_ties(const orc_run* run);
void orc_copy_ties(const orc_run* run, uint64_t* out);       /* 4*k: a0,Na,b0,Nb (sorted positions) */
void orc_copy_sorted_ids(const orc_run* run, uint32_t* out); /* n */

#define ORC_NSTATS 24
/* stats: 0 W, 1 w0 (GIRG) / unused, 2 L, 3 D, 4 Dmax, 5 neighbour cell pairs,
 * 6 distant cell pairs, 7 type-I items, 8 type-II items, 9 tests, 10 draws,
 * 11 candidates, 12 edges, 13 near, 14 ties, 15 segments, 16 kappa / coshR,
 * 17 type-I edges, 18 type-II edges, 19 expected near count, 20 expected
 * skip-tie count (sums over the decisions and draws of the run of the chance
 * that each is logged, given the points) */
void orc_stats(const orc_run* run, double* out);
/* CL (64*64, -1 where a layer is empty), I (64), layer sizes (64),
 * per-layer max weight (GIRG) or min radius (HRG) (64). */
void orc_tables(const orc_run* run, int32_t* CL, int32_t* I, int64_t* count, double* ext);
/* Classify a vertex pair (original ids, u first): writes level, A, B (Morton
 * at that level), i, j, type (0 = type-I, 1 = type-II) and swapped (1 if the
 * item holds the pair as (v,u)). */
void orc_pair_item(const orc_run* run, uint32_t u, uint32_t v, int64_t* out7);
/* For m edges (u, v): level, A, B, i, j, k (the pair index inside the item),
 * type and a flag that is 1 when the edge is not written with u from the A
 * side (App. B.1); out has 8 entries per edge. */
void orc_edge_keys(const orc_run* run, const uint32_t* edges, uint64_t m, int64_t* out8);
/* visited cell pairs (neighbouring, distant) per level 0..39 */
void orc_level_counts(const orc_run* run, uint64_t* nb, uint64_t* dist);

#ifdef __cplusplus
}
#endif
#endif
