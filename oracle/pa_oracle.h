/*
 * Oracle for population annealing (PA) of the 2D Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation of the method, written from the paper (Russkov, Chulkevich,
 * Shchur, "Algorithm for the replica redistribution in the implementation of
 * parallel annealing method on the hybrid supercomputer architecture",
 * Sec. 2 "Population annealing algorithm", Eqs. part-F, part-Q, tau,
 * Free-En; Sec. 3, Eq. Ham).  Only the test suite, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the HIP path: it has its own Philox, its own energy function, its own
 * reweighting tables and its own sweep.
 *
 * Every free choice the paper leaves open (RNG stream layout, resampling
 * law, acceptance rounding, summation order) is fixed in pa_oracle.c next
 * to the step it governs.
 */
#ifndef PA_ORACLE_H
#define PA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -2,
  ORC_ECAPACITY = -3,
  ORC_EEMPTY = -6
};

typedef struct orc_pa orc_pa;

typedef struct {
  int64_t R;
  double beta;
  double e;        /* <E>/N            */
  double abs_m;    /* <|M|>/N          */
  double m2;       /* <M^2>/N^2        */
  double C;        /* beta^2 Var(E)/N  */
  int64_t sumE, sumE2, sumAbsM, sumM2;
  int32_t Emin, Emax;
} orc_obs;

/* Philox4x32-10 block: out = philox(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

/* Energy and magnetisation of one L x L configuration (Eq. Ham).
   spins: int8 +-1 row-major [L][L]; J: NULL (ferromagnet, J=1) or int8 +-1
   [2][L][L] (plane 0: bond to the right neighbour, plane 1: bond to the
   neighbour below). */
void orc_energy(int L, const int8_t* J, const int8_t* spins, int32_t* E,
                int32_t* M);

/* Create a population of R_t replicas at beta0 = 0 (uniform spins).
   cap = 0 selects R_t + 16*ceil(sqrt(R_t)) + 1024. */
int orc_create(int L, const int8_t* J, int64_t R_t, int64_t cap,
               uint64_t seed, uint32_t pop, orc_pa** out);
/* The q-state Potts ferromagnet (2 <= q <= 16): states 0..q-1, uniform at
   beta0 = 0 (state floor(w q / 2^32) of the site's INIT word), ln Z = N ln q;
   H = -sum over bonds of delta(s, s'); M = q n_0 - N. */
int orc_create_potts(int L, int q, int64_t R_t, int64_t cap, uint64_t seed,
                     uint32_t pop, orc_pa** out);
void orc_potts_energy(int L, int q, const int8_t* spins, int32_t* E,
                      int32_t* M);
void orc_destroy(orc_pa* p);

/* Heating protocol: replace a fresh ferromagnet population by ground states
   at beta0 > 0 (all +1 or all -1, from the replica's INIT word of site
   (0,0)), ln Z = ln 2 + 2 N beta0. */
int orc_start_heating(orc_pa* p, double beta0);

/* Reweight from the current beta to beta_next (cooling or heating), draw
   copy counts, build the new population.  On error the population is
   unchanged. */
int orc_resample(orc_pa* p, double beta_next, int64_t* R_new);
/* theta checkerboard Metropolis sweeps at the current beta. */
int orc_sweep(orc_pa* p, int theta);
/* The same with the replicas split over nthreads threads (contiguous slot
   ranges); identical results, for timing on every host core. */
int orc_sweep_threads(orc_pa* p, int theta, int nthreads);
int orc_observables(const orc_pa* p, orc_obs* out);
int orc_free_energy(const orc_pa* p, double* lnZ, double* lnQ_last);

int64_t orc_R(const orc_pa* p);
double orc_beta(const orc_pa* p);
int orc_step(const orc_pa* p);
int orc_get_population(const orc_pa* p, int8_t* spins, int32_t* E,
                       int32_t* M, int64_t cap);
int orc_get_counts(const orc_pa* p, uint32_t* n, int64_t cap);
int orc_set_population(orc_pa* p, const int8_t* spins, int64_t R);
/* Histogram of E over the current population; out has 4N+1 entries,
   index E + 2N. */
int orc_histogram(const orc_pa* p, uint32_t* out);
/* Test hook: visit the sites of one colour in a seeded random order instead
   of raster order (0 restores raster order). */
void orc_set_visit_shuffle(orc_pa* p, uint64_t shuffle_seed);

/* Resampling laws: nearest integer (floor of the mean plus a Bernoulli draw
   on its fraction; the default), Poisson (the law the paper names) and
   systematic (one comb of unit-spaced points over the means laid end to
   end, from the review the paper cites for variants of this step). */
#define ORC_NEAREST 0
#define ORC_POISSON 1
#define ORC_SYSTEMATIC 2
#define ORC_RESIDUAL 3   /* floor(rho) copies, draws over the fractions */
#define ORC_MULTINOMIAL 4 /* R_target independent draws of a parent */
int orc_set_resampling(orc_pa* p, int law);
/* The Poisson copy count for mean rho from the 32-bit word r (inversion of
   the cumulative distribution; exposed for its pins). */
uint32_t orc_poisson_draw(double rho, uint32_t r);

/* The reweighting and copy-count step on energies alone (for sampled checks
   at sizes where the whole population does not fit in host memory).
   step_next is the index of the temperature being entered. */
/* Multinomial and residual laws: the replica a 64-bit draw u lands in,
   the first j with floor(u C / 2^64) < cum[j], C = cum[R - 1]. */
int64_t orc_multinomial_pick(uint64_t u, const uint64_t* cum, int64_t R);
int orc_counts(int N, const int32_t* E, int64_t R, int64_t R_t, double dbeta,
               uint64_t seed, uint32_t pop, int step_next, int law,
               uint32_t* n_out, int64_t* R_new, double* lnQ_out);
/* theta sweeps of one replica in place, sweeps t0..t0+theta-1 of step
   `step`, replica slot `slot`. */
int orc_sweep_replica(int L, const int8_t* J, int8_t* spins, int32_t* E,
                      int32_t* M, double beta, uint64_t seed, uint32_t pop,
                      int step, int t0, int theta, uint32_t slot);
/* Families (test infrastructure, like the rest of the oracle): the family
   of each replica is the slot of its ancestor in the population the
   families start from (the initial one, the heating start or a set
   population); *n0 receives that population's size.  orc_family_stats
   summarises a family array: families alive, the largest, rho_t =
   sum_i c_i^2 / R and rho_s = exp(sum_i c_i ln c_i / R). */
int orc_get_families(const orc_pa* p, uint32_t* fam, int64_t cap,
                     int64_t* n0);
int orc_family_stats(const uint32_t* fam, int64_t R, int64_t n0,
                     int64_t* families, int64_t* largest, double* rho_t,
                     double* rho_s);
/* The same for one replica of the q-state Potts ferromagnet. */
int orc_sweep_potts_replica(int L, int q, int8_t* spins, int32_t* E,
                            int32_t* M, double beta, uint64_t seed,
                            uint32_t pop, int step, int t0, int theta,
                            uint32_t slot);

/* Source of the Metropolis random numbers of the Ising sweeps (the
   acceptance rule r < T is the same in both): ORC_RNG_WORD, one Philox word
   per site (the default); ORC_RNG_PLANES, r = B 2^24 + floor(w / 2^8) with
   B a byte of bit planes shared out of one Philox block per 16 colour
   sites and w the site's default word (see site_draw in pa_oracle.c).
   orc_site_draw returns the number site (x, y) uses; orc_sweep_replica_rng
   is orc_sweep_replica with a mode. */
#define ORC_RNG_WORD 0
#define ORC_RNG_PLANES 1
int orc_set_rng_mode(orc_pa* p, int mode);
uint32_t orc_site_draw(int mode, int L, uint64_t seed, uint32_t pop,
                       int step, int half_sweep, uint32_t slot, int y, int x);
int orc_sweep_replica_rng(int L, const int8_t* J, int8_t* spins,
                          int32_t* E, int32_t* M, double beta, uint64_t seed,
                          uint32_t pop, int step, int t0, int theta,
                          uint32_t slot, int rng_mode);

/* Overlap of successive energy distributions for a step dbeta and the
   bisection that picks the largest step meeting a target overlap. */
int orc_overlap(const orc_pa* p, double dbeta, double* alpha);
int orc_bisect_dbeta(const orc_pa* p, double target, double beta_f,
                     double* dbeta);

#ifdef __cplusplus
}
#endif
#endif
