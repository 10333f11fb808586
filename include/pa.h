/*
 * pa.h -- C ABI of the MI355X (gfx950) population-annealing library libpa.so.
 *
 * Population annealing (PA) of the 2D Ising model as stated in Russkov,
 * Chulkevich and Shchur, "Algorithm for the replica redistribution in the
 * implementation of parallel annealing method on the hybrid supercomputer
 * architecture": Sec. 2 (the method: Eqs. part-F, part-Q, tau, Free-En) and
 * Sec. 3 (the model: Eq. Ham, the L = 64 periodic lattice and the cooling
 * schedule from beta_0 = 0).  Every step of a call runs in hand-written HIP
 * kernels on the device; the host only builds double-precision tables from an
 * exact integer energy histogram.
 *
 * Conventions
 *  - Every function returns PA_OK (0) or a negative PA_E* code; nothing is
 *    thrown across the ABI.  On error the population, beta and ln Z are left
 *    as they were.
 *  - A context owns all of its device memory (allocated with hipMalloc at
 *    pa_init, sized by the capacity) and is bound to one HIP stream and to the
 *    device that was current at pa_init.  Calls on one context must not
 *    overlap; different contexts are independent.
 *  - Host pointers passed in are only read during the call (copied where
 *    kept); host output buffers are owned by the caller and filled before
 *    the call returns.
 *  - pa_sweep and pa_resample's device work is asynchronous on the stream;
 *    functions returning host values synchronise the stream.
 *  - Spins cross the ABI in the canonical layout: int8 +1/-1, row-major
 *    [R][L][L] (site x of row y at index y*L + x), whatever the device layout.
 *  - Random numbers are Philox4x32-10 (Salmon et al., SC'11), key = (seed low
 *    word, seed high word), counter = ((domain << 28) | group,
 *    (step << 16) | half_sweep, replica slot, population id), domains
 *    INIT = 1, MCMC = 2, RESAMPLE = 3.  The same (seed, population id) gives
 *    the same run bit for bit on any stream, launch shape or layout.
 */
#ifndef PA_H
#define PA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PA_OK = 0,
  PA_EINVAL = -1,    /* bad argument (also: beta not finite, cooling only) */
  PA_ENOMEM = -2,    /* device or host allocation failed                   */
  PA_ECAPACITY = -3, /* resampling would exceed the capacity               */
  PA_EDEVICE = -4,   /* a HIP call failed                                  */
  PA_ESTATE = -5,    /* call out of order (e.g. sweep at another beta)     */
  PA_EEMPTY = -6     /* resampling drew zero copies in total               */
};

enum { PA_FERRO = 0, PA_PMJ = 1 };     /* model                */
enum { PA_INT8 = 0, PA_BITS = 1 };     /* device spin layout   */

typedef struct {
  int32_t L;          /* lattice side, even, 4 <= L <= 128 (checkerboard on
                         a torus needs even L)                               */
  int32_t model;      /* PA_FERRO (J = 1 on every bond, Eq. Ham) or PA_PMJ */
  const int8_t* J;    /* PA_PMJ: host int8 +-1 [2][L][L]; plane 0 is the bond
                         from (x,y) to (x+1,y), plane 1 the bond to (x,y+1);
                         copied at pa_init.  NULL for PA_FERRO.             */
  int64_t R_target;   /* target population R (Sec. 2: resampling keeps the
                         population close to it), 1 <= R_target < 2^31     */
  int64_t capacity;   /* replica slots per buffer; 0 selects
                         R_target + 16*ceil(sqrt(R_target)) + 1024          */
  int32_t layout;     /* PA_INT8: one byte per spin; PA_BITS: one bit per
                         spin, row y in ceil(L/32) uint32 words, site x in
                         bit x%32 of word x/32, bit set = +1                */
  int32_t rows_per_lane; /* sweep launch shape: 0 = tuned default, else 1, 2
                         or 4 lattice rows per lane (must divide L; L/rows
                         <= 64).  Results do not depend on it.             */
  uint64_t seed;      /* Philox key                                          */
  uint32_t population_id; /* Philox counter word 3                          */
  void* stream;       /* hipStream_t to run on; NULL = the null stream      */
} pa_config;

typedef struct {
  int64_t R;          /* population size                                    */
  double beta;
  double e;           /* <E>/N                                              */
  double abs_m;       /* <|M|>/N                                            */
  double m2;          /* <M^2>/N^2                                          */
  double C;           /* beta^2 (<E^2> - <E>^2) / N, from exact sums       */
  int64_t sumE, sumE2, sumAbsM, sumM2;
  int32_t Emin, Emax;
} pa_obs;

typedef struct {       /* device time per kernel class, from HIP events     */
  double ms[6];        /* PA_K_INIT, PA_K_SWEEP, PA_K_HIST, PA_K_COUNTS,
                          PA_K_SCATTER, PA_K_GATHER                         */
  int64_t launches[6];
  int64_t bytes[6];    /* algorithmic bytes moved by the timed launches     */
  int64_t attempts;    /* spin-flip attempts made by the timed sweeps       */
} pa_timing;
enum { PA_K_INIT = 0, PA_K_SWEEP, PA_K_HIST, PA_K_COUNTS, PA_K_SCATTER,
       PA_K_GATHER };

typedef struct pa_ctx pa_ctx;

/* Sec. 2, first step (Eq. part-F, second form, at beta_0 = 0): draw R_target
   replicas with independent uniform spins (INIT stream: site (x,y) takes
   word x%4 of group y*ceil(L/4)+x/4, top bit set = +1), compute E_j and M_j
   (Eq. Ham), set beta = 0, step = 0 and ln Z = N ln 2.  *out receives a new
   context, or NULL on error. */
int pa_init(const pa_config* cfg, pa_ctx** out);

/* Sec. 2, equilibration step: theta checkerboard Metropolis sweeps of every
   replica at the current beta (which `beta` must equal, else PA_ESTATE).
   Colour c = (x+y) mod 2, colour 0 first; a site with a unsatisfied bonds has
   dE = 8 - 4a and is flipped iff dE <= 0 or r < floor(exp(-beta dE) 2^32),
   r = word k%4 of MCMC group y*ceil(L/8)+k/4 (k = x/2) at half sweep 2t+c,
   t counting the sweeps already made at this step.  At most 32767 sweeps
   per step.  Asynchronous. */
int pa_sweep(pa_ctx* c, double beta, int32_t theta);

/* Sec. 2, reweighting and resampling (Eqs. part-Q, tau) from the current
   beta to beta_next >= beta: exact energy histogram on the device; on the
   host, per energy level in ascending order, w = exp(-dbeta (E - Emin)),
   S = sum h w, ln Q = -dbeta Emin + ln(S / R), rho = R_target w / S; copy
   counts n_j = floor(rho) + [r_j < floor(frac(rho) 2^32)] (RESAMPLE word 0
   of slot j at the new step); exclusive scan; gather of the copies (parents
   in slot order, copies contiguous) into the second buffer.  Advances beta
   and the step, adds ln Q to ln Z (Eq. Free-En).  *R_new (may be NULL)
   receives the new population size, also when it exceeds the capacity
   (then PA_ECAPACITY and nothing changes). */
int pa_resample(pa_ctx* c, double beta_next, int64_t* R_new);

/* Sec. 2, measurement after equilibration: population averages from exact
   integer sums over the current population.  Synchronises. */
int pa_observables(pa_ctx* c, pa_obs* out);

/* Eq. Free-En (read with the logarithm): ln Z(beta) = N ln 2 + sum of the
   ln Q of every resampling so far; -beta F = ln Z.  Either pointer may be
   NULL.  No device work. */
int pa_free_energy(pa_ctx* c, double* lnZ, double* lnQ_last);

/* Current population size, beta and step index. */
int pa_state(pa_ctx* c, int64_t* R, double* beta, int32_t* step);

/* Canonical export of the whole population into caller-owned host arrays of
   at least `cap` replicas (spins: cap*L*L bytes); any pointer may be NULL.
   PA_EINVAL if cap < R.  Synchronises. */
int pa_get_population(pa_ctx* c, int8_t* spins, int32_t* E, int32_t* M,
                      int64_t cap);

/* Canonical export of k chosen replicas (slots[i] < R) into host arrays of
   k replicas.  Synchronises. */
int pa_get_replicas(pa_ctx* c, const int64_t* slots, int64_t k, int8_t* spins,
                    int32_t* E, int32_t* M);

/* Copy counts of the last resampling (one per replica of the population
   before it) into a host array of at least `cap` entries; *len receives the
   number written.  Synchronises. */
int pa_get_counts(pa_ctx* c, uint32_t* n, int64_t cap, int64_t* len);

/* Replace the population by R <= capacity replicas given in the canonical
   layout (values must be +-1); E and M are recomputed on the device.  beta,
   step and ln Z are kept.  Synchronises. */
int pa_set_population(pa_ctx* c, const int8_t* spins, int64_t R);

/* Energy histogram of the current population over the levels E = -2N +
   s*i (s = 4 for the ferromagnet, 2 for +-J), i < nbins = 4N/s + 1, into a
   host array of at least `cap` entries; *nbins and *step receive them.
   Synchronises. */
int pa_histogram(pa_ctx* c, uint32_t* h, int64_t cap, int32_t* nbins,
                 int32_t* step);

/* Adaptive temperature step (Sec. 3 remarks that an adaptive step reduces
   the population fluctuations): overlap alpha(dbeta) = sum_E min(h/R,
   h w / S) of the current energy distribution and its reweighting to
   beta + dbeta; and the largest dbeta <= beta_f - beta with alpha >= target
   (the whole interval if it qualifies, else 64 bisection halvings).  Host
   double precision on the device histogram.  Synchronises. */
int pa_overlap(pa_ctx* c, double dbeta, double* alpha);
int pa_bisect_dbeta(pa_ctx* c, double target, double beta_f, double* dbeta);

/* Per-kernel-class device timing with HIP events on the context's stream.
   enable = 1 starts (and zeroes) the counters, 0 stops.  pa_get_timing
   synchronises and reports the totals since the last enable. */
int pa_set_timing(pa_ctx* c, int32_t enable);
int pa_get_timing(pa_ctx* c, pa_timing* out);

void pa_destroy(pa_ctx* c);
const char* pa_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
