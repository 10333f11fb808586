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
  PA_EINVAL = -1,    /* bad argument (also: beta not finite or negative)   */
  PA_ENOMEM = -2,    /* device or host allocation failed                   */
  PA_ECAPACITY = -3, /* resampling would exceed the capacity               */
  PA_EDEVICE = -4,   /* a HIP call failed                                  */
  PA_ESTATE = -5,    /* call out of order (e.g. sweep at another beta)     */
  PA_EEMPTY = -6,    /* resampling drew zero copies in total               */
  PA_EIO = -7        /* population file not written / not readable / not a
                        population file of this library                   */
};

enum { PA_FERRO = 0, PA_PMJ = 1, PA_POTTS = 2 };  /* model     */
enum { PA_INT8 = 0, PA_BITS = 1 };     /* device spin layout   */
enum { PA_NEAREST = 0, PA_POISSON = 1, PA_SYSTEMATIC = 2,
       PA_RESIDUAL = 3, PA_MULTINOMIAL = 4 }; /* resampling law */
enum { PA_RNG_WORD = 0, PA_RNG_PLANES = 1 };  /* sweep random numbers */

typedef struct {
  int32_t L;          /* lattice side, even, 4 <= L <= 128 (checkerboard on
                         a torus needs even L)                               */
  int32_t model;      /* PA_FERRO (J = 1 on every bond, Eq. Ham), PA_PMJ, or
                         PA_POTTS: the q-state Potts ferromagnet named with
                         the heating protocol in Sec. 2, H = -sum over bonds
                         of delta(s, s'), states 0..q-1 as int8 spins,
                         M = q n_0 - N; PA_INT8 layout only, single
                         populations only                                  */
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
  int32_t rows_per_lane; /* sweep launch shape: 1, 2, 3 or 4 lattice rows
                         per lane (must divide L; L/rows <= 64; at least 2
                         for L > 64), or 0: 3 at L = 48 and 96, 2 above
                         L = 64 (and at L = 64 with PA_RNG_PLANES and
                         R_target >= 2^14, except that an int8 launch of
                         one sweep then takes 1), else 1
                         (a batch created with
                         PA_BATCH_AUTOTUNE times the valid shapes instead).
                         Results do not depend on it.                       */
  uint64_t seed;      /* Philox key                                          */
  uint32_t population_id; /* Philox counter word 3                          */
  void* stream;       /* hipStream_t to run on; NULL = the null stream      */
  int32_t resampling; /* copy-count law (Sec. 2): PA_NEAREST (default)
                         floor(rho) + [r < floor(frac(rho) 2^32)], or
                         PA_POISSON, a Poisson(rho) count by inversion of
                         its cumulative distribution C(k) (summed in
                         double precision in increasing k): the count is
                         the number of k with floor(C(k) 2^32) <= r, the
                         list of k ending after C(k) >= 1 - 2^-32 or before
                         ceil(rho + 64 sqrt(rho) + 64); or PA_SYSTEMATIC,
                         the variant of the review Sec. 2 cites: the means
                         as P_j = floor(rho) 2^32 + floor(frac(rho) 2^32)
                         laid end to end (C_j = P_0 + .. + P_j) and one
                         comb offset U (RESAMPLE group 1, slot 0, word 0 at
                         the new step), n_j = floor((C_j + U) / 2^32) -
                         floor((C_{j-1} + U) / 2^32): every count is the
                         floor or ceiling of its mean and the size is
                         within one of the target; or PA_MULTINOMIAL,
                         R_target independent draws: draw i (RESAMPLE
                         group 2, slot i, u = word 1 2^32 + word 0) lands
                         at floor(u C / 2^64), C the total of the P_j, in
                         the replica whose [C_{j-1}, C_j) holds it; or
                         PA_RESIDUAL, floor(rho) copies for certain plus
                         D = R_target - sum floor(rho) such draws over the
                         fractional parts alone (P_j = floor(frac(rho)
                         2^32); no draws when all are zero): the size is
                         exactly sum floor(rho) + D.
                         Single populations only: pa_batch_init takes
                         PA_NEAREST only.                                  */
  int32_t q;          /* PA_POTTS: number of states, 2..16; else ignored   */
  int32_t rng_mode;   /* random number r of a Metropolis decision (accept
                         iff dE <= 0 or r < T, T = floor(exp(-beta dE)
                         2^32), Sec. 2 equilibration step).  PA_RNG_WORD
                         (default): r is the site's own Philox word, word
                         k%4 of MCMC group y*ceil(L/8) + k/4, k = x/2.
                         PA_RNG_PLANES: r = B 2^24 + floor(w / 2^8), w that
                         same word and B a byte of bit planes: the Philox
                         block of domain 5, group y*ceil(L/32) + x/32 (same
                         counter words 1-3) gives bit 7 - m of B, m = 2i+h,
                         as bit (x mod 32) XOR h of its output word i.
                         r is uniform on [0, 2^32) in both modes, so the
                         acceptance probabilities are the same; the plane
                         mode draws one block per 16 sites and needs w only
                         when B equals the top byte of T.  PA_FERRO and
                         PA_PMJ single populations only.                  */
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
   beta to beta_next >= 0 (cooling, or heating when beta_next < beta):
   exact energy histogram on the device; on the host, per energy level in
   ascending order, w = exp(-dbeta (E - E0)) with E0 the smallest energy
   when cooling and the largest when heating, S = sum h w,
   ln Q = -dbeta E0 + ln(S / R), rho = R_target w / S; copy
   counts n_j = floor(rho) + [r_j < floor(frac(rho) 2^32)] (RESAMPLE word 0
   of slot j at the new step); exclusive scan; parent of every new slot
   (parents in slot order, copies contiguous).  The copies into the second
   buffer are made by the next pa_sweep with theta > 0 as it loads each new
   slot from its parent, or by a plain gather before any other call that
   reads the population; either way every later call sees the resampled
   population.  Advances beta and the step, adds ln Q to ln Z (Eq.
   Free-En).  *R_new receives the new population size, also when it exceeds
   the capacity (then PA_ECAPACITY and nothing changes); the call then waits
   for the counts.  With R_new NULL the call does not wait when the tables
   bound the new size within [1, capacity] (every replica gets floor(rho) or
   floor(rho) + 1 copies): the kernels that follow read the size on the
   device, and the host learns it at the next synchronising call.
   Otherwise it waits and checks as above. */
int pa_resample(pa_ctx* c, double beta_next, int64_t* R_new);

/* Sec. 2, the whole annealing loop for a schedule of K temperatures: for
   k = 0..K-1 the same as pa_resample(c, betas[k], NULL), then
   pa_sweep(c, betas[k], theta), then pa_observables into obs[k]; lnQ[k]
   receives the ln Q of step k (obs and lnQ are caller arrays of K entries,
   either may be NULL).  With the nearest-integer law, theta >= 1 and betas
   non-decreasing from the current beta, the device runs the schedule with no
   host stop between steps: the last workgroup of each step's histogram
   builds the step's tables in the host tables' order of operations from
   weights exp(-dbeta (E - E0)) the host evaluates ahead for every level
   (so the tables, counts and ln Q are those of the step-by-step calls, bit
   for bit), and every later kernel reads the population size on the
   device (grids cover the capacity).  Other laws, heating steps or
   theta = 0 run the step-by-step calls.  *done (may be NULL) receives the
   number of completed steps.  A resampling whose size would exceed the
   capacity (PA_ECAPACITY) or be 0 (PA_EEMPTY) ends the schedule at that
   step with the context as the failed pa_resample leaves it: the
   population after the sweeps of the step before.  PA_EINVAL for K < 0,
   theta outside 0..32767, a non-finite or negative beta, or more than
   65535 steps in all (nothing changes then); after PA_EDEVICE the context
   is left as the device left it and is only fit for pa_destroy.
   Synchronises once, at the end. */
int pa_anneal(pa_ctx* c, const double* betas, int32_t K, int32_t theta,
              pa_obs* obs, double* lnQ, int32_t* done);

/* Sec. 2, heating protocol (the population starts close to zero
   temperature): replaces the population of a fresh ferromagnet or Potts
   context (step 0) by ground states at beta0 > 0 -- every spin of replica j
   equals the top bit of its INIT word of site (0,0) (+1 when set), or for
   Potts the state floor(w q / 2^32) of that word -- and sets beta = beta0,
   ln Z = ln(#ground states) + 2 N beta0 (2 or q states of energy -2N)
   plus the lightest excitations of the low-temperature expansion, one
   changed site and two changed neighbours:
   N (exp(-8 beta0) + 2 exp(-12 beta0)) for Ising,
   N (q-1) (exp(-4 beta0) + 2 exp(-6 beta0) + 2 (q-2) exp(-7 beta0)) for
   Potts; what is left out is of order N exp(-16 beta0) (Ising) or
   N exp(-8 beta0) (Potts).  Resampling
   then steps beta down; weights are shifted by the largest energy when
   beta decreases.  PA_EINVAL for +-J couplings or beta0 <= 0, PA_ESTATE
   after a resampling.  Synchronises. */
int pa_start_heating(pa_ctx* c, double beta0);

/* Sec. 2, measurement after equilibration: population averages from exact
   integer sums over the current population.  Synchronises. */
int pa_observables(pa_ctx* c, pa_obs* out);

/* Eq. Free-En (read with the logarithm): ln Z(beta) = N ln 2 + sum of the
   ln Q of every resampling so far; -beta F = ln Z.  Either pointer may be
   NULL.  No device work. */
int pa_free_energy(pa_ctx* c, double* lnZ, double* lnQ_last);

/* Current population size, beta and step index (synchronises when the
   size of a resampled population has not reached the host yet). */
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

/* Checkpoint and resume.  pa_save writes the whole state of the context to
   a file: configuration, couplings, beta, step, sweeps made at this step,
   ln Z and the last ln Q, and the population in the canonical layout with
   its E, M and families (a fixed 104-byte header "PAPOPv03" first, whose
   last word is the founding population size; then the +-J couplings,
   spins [R][L][L] int8, E and M int32 [R], families uint32 [R];
   little-endian).
   It synchronises; a pending resampling copy is made first.  pa_load
   creates a new context on `stream` (a hipStream_t or NULL) from such a
   file: because every random number is keyed by (step, sweep, slot,
   population), the loaded context continues the run bit for bit as the
   saved one would have.  The file is read and checked completely before
   any device work (magic, sizes, spin values, no trailing bytes), and the
   stored E and M must equal those of the stored spins, and every family
   number must lie below the founding size; otherwise PA_EIO and *out =
   NULL.  The copy counts of the last resampling are not saved. */
int pa_save(pa_ctx* c, const char* path);
int pa_load(const char* path, void* stream, pa_ctx** out);

/* Families (the population-annealing diagnostic that accompanies weighted
   averaging, with the Machta reference of Sec. 4): every replica belongs
   to the family of its ancestor in the founding population, i.e. the
   population made by pa_init, pa_start_heating or pa_set_population, whose
   replicas found one family each (numbered by their slot).  A resampling
   copy joins its parent's family; sweeps change no family.
   pa_get_families copies the family number of each replica (ascending
   slot) to fam[cap >= R] (fam may be NULL to query only) and the sizes R
   and n0 (founding population) to *len and *n0; it synchronises.
   pa_family_summary is host arithmetic on such an array: with c_i members
   in family i and nu_i = c_i / R, the families with members, the largest,
   the mean square family size rho_t = R sum nu_i^2 and the entropic family
   size rho_s = R exp(sum nu_i ln nu_i) (both 1 when no two replicas share a
   family, R when one family holds them all).  PA_EINVAL for a number
   >= n0.  pa_family_stats is pa_get_families followed by
   pa_family_summary.  A batch exports its populations' families with
   pa_batch_get_families. */
typedef struct {
  int64_t R;          /* population size                                     */
  int64_t n0;         /* size of the founding population                    */
  int64_t families;   /* families with at least one member                  */
  int64_t largest;    /* members of the largest family                      */
  double rho_t;       /* mean square family size  R sum nu_i^2              */
  double rho_s;       /* entropic family size  R exp(sum nu_i ln nu_i)      */
} pa_family;
int pa_get_families(pa_ctx* c, uint32_t* fam, int64_t cap, int64_t* len,
                    int64_t* n0);
int pa_family_summary(const uint32_t* fam, int64_t R, int64_t n0,
                      pa_family* out);
int pa_family_stats(pa_ctx* c, pa_family* out);

/* The configuration of a context (J is returned as NULL). */
int pa_get_config(pa_ctx* c, pa_config* out);

/* Weighted averaging over M independent populations (Sec. 4, Large scale
   testing, with the Machta reference): population m, with free-energy
   estimate lnZ[m] and population averages values[m*k .. m*k+k) (linear
   averages such as <E>, <E^2>, <|M|>; derived quantities are formed from
   the combined averages), has weight Z_m / sum Z.  out[j] = sum_m w_m
   values[m*k + j]; *lnZ_out (may be NULL) = ln((1/M) sum_m Z_m).  Host
   double precision, weights exp(lnZ[m] - max lnZ) summed in increasing m.
   No device work.  PA_EINVAL for M < 1 or a non-finite lnZ. */
int pa_weighted_average(int32_t M, const double* lnZ, const double* values,
                        int32_t k, double* out, double* lnZ_out);

/* Weighted averaging of the observables themselves (Sec. 4, Large scale
   testing): M populations at the same beta (obs[m].beta all equal, else
   PA_EINVAL), each described by its pa_obs (exact integer sums sumE,
   sumE2, sumAbsM, sumM2 over its R replicas) and its ln Z, combined with
   weights w_m = Z_m / sum Z.  <E> = sum w_m sumE_m / R_m; the energy
   variance is sum w_m Var_m + sum w_m (<E>_m - <E>)^2 (law of total
   variance), where Var_m = (R sumE2 - sumE^2) / R^2 is formed exactly in
   128-bit integers per population; e = <E>/N, |m| = <|M|>/N,
   m2 = <M^2>/N^2, C = beta^2 Var(E) / N, lnZ = ln((1/M) sum Z_m).  Host
   double precision, sums in increasing m.  No device work.  PA_EINVAL for
   M < 1, N < 1, a population with R < 1 or a non-finite lnZ. */
typedef struct {
  int32_t M;          /* populations combined                               */
  int64_t R;          /* their replicas in total                            */
  double beta;
  double e, abs_m, m2, C;
  double varE;        /* combined variance of E                             */
  double lnZ;         /* ln((1/M) sum_m Z_m)                                 */
} pa_combined;
int pa_weighted_observables(int32_t M, const double* lnZ, const pa_obs* obs,
                            int32_t N, pa_combined* out);

/* Per-kernel-class device timing with HIP events on the context's stream.
   classes: PA_TIMING_ALL times every class, otherwise a bit mask of the
   classes to time (bit PA_K_SWEEP = 1 << PA_K_SWEEP, ...); a nonzero value
   starts (and zeroes) the counters, 0 stops.  Each timed launch records two
   events on the stream.  pa_get_timing synchronises and reports the totals
   since timing was started. */
#define PA_TIMING_ALL (-1)
int pa_set_timing(pa_ctx* c, int32_t classes);

/* Time only the first launch and then every `every`-th (>= 1, default 1) of
   each timed class, counted per class from the last pa_set_timing: a run of
   many short launches is then disturbed by few events, and the averages
   stand for a systematic sample of the launches.  PA_EINVAL for every < 1. */
int pa_set_timing_sample(pa_ctx* c, int32_t every);
int pa_get_timing(pa_ctx* c, pa_timing* out);

void pa_destroy(pa_ctx* c);
const char* pa_strerror(int code);
/* Text of the last failing HIP call on the calling thread (the call, the
   source line and HIP's message) behind a PA_EDEVICE; "" if none.  The
   string stays valid until the next failure on the thread. */
const char* pa_last_error(void);

/* ------------------------------------------------------------------------
 * Batched populations: n independent populations (each its own pa_config:
 * L, model, couplings, R_target, capacity, layout, rows_per_lane, seed,
 * population_id; cfg.stream is ignored) advanced together.  Each population
 * follows exactly the steps of Sec. 2 described above for pa_resample and
 * pa_sweep, so its spins, energies, copy counts and ln Z are bit for bit those
 * of a single-population context with the same configuration and schedule.
 * Per temperature step all populations share one launch of each segmented
 * kernel, one persistent sweep kernel per row-width class pulling
 * (population, wave) items from a device queue, one device->host copy of all
 * histograms, one host function for all double-precision tables and one
 * host->device copy; with use_graph the kernels before and after the host
 * function are captured once as two HIP graphs (kernel nodes only) and
 * replayed every step, the copies and the host function running between
 * the two launches.
 *
 * Errors: as above, except that after PA_ECAPACITY, PA_EEMPTY or PA_EDEVICE
 * from pa_batch_run* the batch must only be destroyed.
 * ---------------------------------------------------------------------- */
typedef struct pa_batch pa_batch;
enum { PA_BATCH_AUTOTUNE = 1,     /* flags of pa_batch_init */
       PA_BATCH_TUNE_SWEEP = 2 };

/* Launch-shape autotuner: times theta sweeps of a synthetic population of R
   replicas of side L for 1, 2, 3 and 4 rows per lane (those valid for L)
   with HIP events; *best receives the fastest, ms[4] (may be NULL) the
   times (-1 for invalid shapes).  Results never depend on the shape. */
int pa_tune_rows_per_lane(int32_t L, int32_t layout, int32_t model,
                          int64_t R, int32_t theta, void* stream,
                          int32_t* best, float* ms);

/* Creates n populations at beta_0 = 0 (Eq. part-F, as pa_init).  stream NULL
   = a private non-blocking stream (graph capture needs one).  flags:
   PA_BATCH_AUTOTUNE picks rows_per_lane where a config leaves it 0, with
   the batch's own persistent sweep on scratch batches of the same
   configurations: each distinct (L, layout, model, rng_mode) starts at its
   smallest valid value, and each other valid value, one class at a time,
   is kept when three timed steps take under 98 % of the best time so far
   (cached per process by the configurations).
   Models: the ferromagnet and +-J glasses in either layout, and q-state
   Potts populations (PA_POTTS, PA_INT8, L = 8, 16, 32, 64 or 128: the
   four-sites-per-word pass, one replica per wave, rows_per_lane ignored);
   the nearest-integer law only.  PA_EINVAL otherwise.
   PA_BATCH_TUNE_SWEEP times the persistent sweep's workgroups and items
   per queue atomic on a scratch batch of the same configurations (one
   step to beta = 0.3, then two steps per candidate; cached per process
   by the configurations) and keeps the fastest; results never depend on
   the shape. */
int pa_batch_init(const pa_config* cfgs, int32_t n, void* stream,
                  int32_t flags, pa_batch** out);

/* Advances every population through `steps` temperatures: betas[i*n + p] is
   population p's i-th next beta (non-decreasing per population); theta
   sweeps (0..32767, as pa_sweep allows per step) after each resampling.
   Records the observables after each step's sweeps (pa_batch_trajectory).
   Synchronises at the end. */
int pa_batch_run(pa_batch* b, int32_t steps, const double* betas,
                 int32_t theta, int32_t use_graph);

/* Adaptive schedule (Sec. 3 notes that an adaptive temperature step reduces
   the population fluctuations): each population picks its own next beta as
   the largest step to beta_f whose energy-distribution overlap is at least
   `target` (the bisection of pa_bisect_dbeta, in the host function), and
   stops at beta_f.  At most max_steps steps; *steps_taken receives the most
   any population made. */
int pa_batch_run_adaptive(pa_batch* b, double target, double beta_f,
                          int32_t max_steps, int32_t theta, int32_t use_graph,
                          int32_t* steps_taken);
/* The same schedule rule with the bisection stopped at the first midpoint
   whose exact overlap lies within `tol` of `target` (tol = 0: the 64
   halvings of pa_batch_run_adaptive): the step the learned schedule would
   accept from its network, found without one.  The baseline against which
   the network's saving is measured. */
int pa_batch_run_adaptive_tol(pa_batch* b, double target, double tol,
                              double beta_f, int32_t max_steps, int32_t theta,
                              int32_t use_graph, int32_t* steps_taken);

/* ------------------------------------------------------------------------
 * Temperature-step network: an FP32 multilayer perceptron (n_in inputs,
 * `depth` tanh layers of `width` units, one linear output) that proposes
 * log(dbeta) from histogram summaries of a population.  Inputs are
 * standardised with (mu, sigma), the output de-standardised with
 * (mu_y, sigma_y).  Forward, backward (mean squared error on standardised
 * targets) and Adam run in the library's HIP kernels.  The exact bisection
 * remains the check and the fallback, and the reweighting stays exact, so the
 * network only changes which temperatures are visited, never the weights.
 * Parameters: one flat FP32 vector, per layer W (out x in, row-major), b.
 * ---------------------------------------------------------------------- */
typedef struct pa_mlp pa_mlp;
/* Glorot-uniform weights from `seed`, zero biases, identity scaling.
   1 <= n_in <= 64, 1 <= width <= 1024, 1 <= depth <= 8. */
int pa_mlp_create(int32_t n_in, int32_t width, int32_t depth, uint64_t seed,
                  void* stream, pa_mlp** out);
int pa_mlp_n_params(pa_mlp* m, int64_t* n);
int pa_mlp_set_params(pa_mlp* m, const float* p, int64_t n);
int pa_mlp_get_params(pa_mlp* m, float* p, int64_t n);
int pa_mlp_set_norm(pa_mlp* m, const float* mu, const float* sigma,
                    float mu_y, float sigma_y);
/* y[s] = mu_y + sigma_y z(x_s) for B host rows X [B][n_in]. */
int pa_mlp_forward(pa_mlp* m, const float* X, int32_t B, float* y);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the
   forward pass of pa_mlp_forward with device pointers and no allocation.
   X: device [B][n_in] raw features; y: device [B], receives
   mu_y + sigma_y z(x_s), equal bit for bit to pa_mlp_forward's output.
   Asynchronous on the network's stream; no synchronisation.  The
   activations live in one fixed per-device scratch array of
   2 x PA_MLP_NOALLOC_MAX_ELEMS floats (2 MiB, held until the process ends),
   so B * max(width, n_in) must not exceed PA_MLP_NOALLOC_MAX_ELEMS
   (PA_EINVAL otherwise, nothing launched).  Every call on a device shares
   that array: calls that overlap on one device (other streams, other
   threads) race and must be ordered by the caller.  Nothing in it needs
   to start at zero. */
#define PA_MLP_NOALLOC_MAX_ELEMS 262144
int pa_mlp_forward_noalloc(pa_mlp* m, const float* X, int32_t B, float* y);
/* Mean squared error of the standardised outputs against standardised
   targets T [B], and its gradient w.r.t. the parameters (host, may be
   NULL). */
int pa_mlp_loss_grad(pa_mlp* m, const float* X, const float* T, int32_t B,
                     float* loss, float* grad);
/* `iters` Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on minibatches
   of `batch` rows drawn in shuffled passes over the n rows (seeded);
   *loss receives the last minibatch's loss. */
int pa_mlp_train(pa_mlp* m, const float* X, const float* T, int64_t n,
                 int32_t batch, int32_t iters, float lr, uint64_t seed,
                 float* loss);
void pa_mlp_destroy(pa_mlp* m);

/* Adaptive schedule with the network: each population's next step is the
   network's proposal when its exact overlap is within `tol` of `target`,
   the whole remaining interval when that qualifies, else the bisection of
   pa_batch_run_adaptive.  The summaries (8 per population: mean/N, ln sd(E),
   skewness, (Emin - mean)/sd, beta, ln N, ln R, target) and the inference
   run on the device in the step graph.  src_counts[5] (may be NULL) receives
   how many steps came from each source (see pa_batch_decisions). */
int pa_batch_run_learned(pa_batch* b, pa_mlp* m, double target, double tol,
                         double beta_f, int32_t max_steps, int32_t theta,
                         int32_t use_graph, int32_t* steps_taken,
                         int64_t* src_counts);

/* Per step of the last run in which population p moved: its 8 summaries,
   the dbeta taken, its source (0 schedule, 1 bisection, 2 network,
   3 bisection after a rejected proposal, 4 the whole remaining interval)
   and the network's proposed log dbeta (NaN without a network); host arrays
   of `cap` rows, any pointer may be NULL.  The training data of the
   network. */
int pa_batch_decisions(pa_batch* b, int32_t p, float* feat, double* dbeta,
                       int32_t* src, float* proposal, int32_t cap,
                       int32_t* len);

/* Cost of the schedule decisions of the last run: milliseconds spent in the
   host function, exact overlap evaluations made, steps per source [5]. */
int pa_batch_host_stats(pa_batch* b, double* host_ms, int64_t* overlap_evals,
                        int64_t* src_counts);

/* Population p's size, beta, step index and ln Z (Eq. Free-En). */
int pa_batch_state(pa_batch* b, int32_t p, int64_t* R, double* beta,
                   int32_t* step, double* lnZ);

/* Observables and ln Z of population p after each step of the last run in
   which it moved (host arrays of `cap` entries; *len receives the count). */
int pa_batch_trajectory(pa_batch* b, int32_t p, pa_obs* obs, double* lnZ,
                        int32_t cap, int32_t* len);

/* Canonical export of population p (as pa_get_population; Potts states
   0..q-1). */
int pa_batch_get_population(pa_batch* b, int32_t p, int8_t* spins, int32_t* E,
                            int32_t* M, int64_t cap);

/* Families of population p, as pa_get_families: the founding population is
   the initial one (n0 = its R_target); the batch carries the families
   through every resampling in its segmented parent scatter. */
int pa_batch_get_families(pa_batch* b, int32_t p, uint32_t* fam, int64_t cap,
                          int64_t* len, int64_t* n0);

/* Launch shape of the persistent sweep kernel: workgroups (default 1024,
   at most 65535) and work items taken per queue atomic (default 4,
   1..1024).  Results do not depend on either. */
int pa_batch_set_sweep_blocks(pa_batch* b, int32_t blocks, int32_t chunk);
int pa_batch_get_sweep_blocks(pa_batch* b, int32_t* blocks, int32_t* chunk);

void pa_batch_destroy(pa_batch* b);

#ifdef __cplusplus
}
#endif
#endif
