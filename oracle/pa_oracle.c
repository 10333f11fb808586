/*
 * Oracle for population annealing (PA) of the 2D Ising model.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded CPU implementation
 * of the method.  Only the test suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the HIP path.
 *
 * The method (paper Sec. 2, "Population annealing algorithm"):
 *   1. start with R replicas drawn uniformly at beta_0 = 0 (Eq. part-F, the
 *      second one: at infinite temperature every state is equally likely);
 *   2. for each step beta_{i-1} -> beta_i compute the normalised partition
 *      function ratio Q (Eq. part-Q) and the weights tau_j (Eq. tau);
 *   3. resample: replica j gets a random number of exact copies whose mean is
 *      proportional to tau_j, keeping the population near its target;
 *   4. equilibrate every replica with theta MCMC sweeps at beta_i;
 *   5. measure observables over the population;
 *   6. accumulate ln Z(beta_i) = ln Omega + sum_l ln Q_l (Eq. Free-En).
 * The model is the 2D Ising ferromagnet on an L x L periodic square lattice
 * (Sec. 3, Eq. Ham); the +-J Edwards-Anderson glass (a system named in the
 * Introduction and the Discussion) only replaces the coupling of each bond.
 *
 * Readings of the paper fixed here (the paper is silent or garbled on them):
 *   - Eq. Free-En lacks the logarithm and the sign; it is read as
 *     ln Z(beta_i) = ln Omega + sum_{l<=i} ln Q(beta_{l-1}, beta_l) with
 *     ln Omega = N ln 2 for cooling from beta_0 = 0.
 *   - Resampling law: nearest-integer (floor of the mean plus one Bernoulli
 *     draw on its fractional part) by default; Poisson, the law the paper
 *     names, on request (inversion of its cumulative distribution with the
 *     same 32-bit word).  The mean number of copies is
 *     rho_j = R_target * tau_j / R_{i-1}, i.e. population control to the
 *     fixed target R_target.
 *   - MCMC: checkerboard Metropolis, colour 0 ((x+y) even) first; integer
 *     acceptance threshold T = floor(exp(-beta dE) 2^32), accept iff
 *     dE <= 0 or r < T for a 32-bit random word r.
 *   - Weights are shifted by the minimum energy (largest weight 1) and summed
 *     over energy levels in ascending order, in double precision.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *     key (seed low word, seed high word) and counter
 *       c0 = (domain << 28) | group, c1 = (step << 16) | half_sweep,
 *       c2 = replica slot, c3 = population id.
 *
 * ORC_MUTANT (unset in every normal build) plants one plausible mistake so
 * that the test suite can show its pins catch it; see the tests of the
 * oracle's mutants.
 */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif
#include "pa_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define DOMAIN_INIT 1u
#define DOMAIN_MCMC 2u
#define DOMAIN_RESAMPLE 3u
#define DOMAIN_MCMC_PLANES 5u

struct orc_pa {
  int L, N;
  int8_t* J;        /* NULL (ferromagnet) or [2][L][L] */
  int64_t R_t, cap, R;
  uint64_t seed;
  uint32_t pop;
  int8_t* spins;    /* [cap][N] */
  int32_t* E;       /* [cap] */
  int32_t* M;       /* [cap] */
  uint32_t* n;      /* copy counts of the last resampling, [cap] */
  int64_t n_len;
  double beta, lnZ, lnQ_last;
  int step;
  int sweeps_at_step;
  uint64_t shuffle_seed;
  int rng_mode;     /* ORC_RNG_WORD (default) or ORC_RNG_PLANES */
  int law;          /* ORC_NEAREST or ORC_POISSON */
  int q;            /* 0: Ising spins +-1; 2..16: Potts states 0..q-1 */
  uint32_t* fam;    /* family of every replica: the slot of its ancestor in
                       the population the families start from, [cap] */
  int64_t fam_n0;   /* size of that population */
};

/* ---------------------------------------------------------------- Philox */

/* Philox4x32 with 10 rounds, as defined by Salmon et al. (SC'11): each round
   multiplies counter words 0 and 2 by the two round constants, swaps the
   halves and mixes in the key; the key is advanced by the two Weyl
   constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* One random word of the stream layout described at the top of the file. */
static uint32_t draw_word(uint64_t seed, uint32_t domain, uint32_t group,
                          uint32_t step, uint32_t half_sweep, uint32_t slot,
                          uint32_t pop, int word) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = (domain << 28) | group;
  ctr[1] = (step << 16) | half_sweep;
  ctr[2] = slot;
  ctr[3] = pop;
  key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, out);
  return out[word];
}

/* ---------------------------------------------------------------- model */

/* Coupling of the bond from site (x,y) to its right (dir 0) or lower
   (dir 1) neighbour; the ferromagnet has J = 1 on every bond. */
static int bond(const int8_t* J, int L, int dir, int x, int y) {
  if (!J) return 1;
  return J[(size_t)dir * L * L + (size_t)y * L + x];
}

/* Eq. Ham: H = -(J/2) sum over every spin of sigma times each of its four
   neighbours, i.e. minus the coupling-weighted product summed once over the
   2N bonds of the periodic lattice. */
void orc_energy(int L, const int8_t* J, const int8_t* s, int32_t* E,
                int32_t* M) {
  int64_t e = 0, m = 0;
  for (int y = 0; y < L; ++y) {
    for (int x = 0; x < L; ++x) {
      int sv = s[y * L + x];
      int right = (ORC_MUTANT == 5) ? s[((x + 1) % L) * L + y]
                                    : s[y * L + (x + 1) % L];
      int down = s[((y + 1) % L) * L + x];
      e -= bond(J, L, 0, x, y) * sv * right;
      e -= bond(J, L, 1, x, y) * sv * down;
      m += sv;
    }
  }
  *E = (int32_t)e;
  *M = (int32_t)m;
}

/* The q-state Potts ferromagnet (Sec. 2 names it with the heating
   protocol): H = -sum over the 2N bonds of delta(s, s'), so E lies in
   [-2N, 0]; the magnetisation-like integer M = q n_0 - N counts the sites
   in state 0 (its |M| and M^2 averages are the reported moments). */
void orc_potts_energy(int L, int q, const int8_t* s, int32_t* E, int32_t* M) {
  int64_t e = 0, n0 = 0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int sv = s[y * L + x];
      e -= (sv == s[y * L + (x + 1) % L]);
      e -= (sv == s[((y + 1) % L) * L + x]);
      n0 += (sv == 0);
    }
  *E = (int32_t)e;
  *M = (int32_t)((int64_t)q * n0 - (int64_t)L * L);
}

/* floor(w q / 2^32): a state in [0, q) from a 32-bit word */
static int potts_state(uint32_t w, int q) {
  return (int)(((uint64_t)w * (uint64_t)q) >> 32);
}

/* ------------------------------------------------------------- lifetime */

/* Every replica founds its own family. */
static void reset_families(orc_pa* p) {
  for (int64_t j = 0; j < p->R; ++j) p->fam[j] = (uint32_t)j;
  p->fam_n0 = p->R;
}

static int create(int L, const int8_t* J, int q, int64_t R_t, int64_t cap,
                  uint64_t seed, uint32_t pop, orc_pa** out) {
  if (!out) return ORC_EINVAL;
  *out = NULL;
  if (L < 4 || L > 128 || (L % 2) != 0) return ORC_EINVAL;
  if (q != 0 && (q < 2 || q > 16 || J)) return ORC_EINVAL;
  if (R_t < 1 || R_t > ((int64_t)1 << 31)) return ORC_EINVAL;
  if (cap == 0) cap = R_t + 16 * (int64_t)ceil(sqrt((double)R_t)) + 1024;
  if (cap < R_t) return ORC_EINVAL;
  orc_pa* p = (orc_pa*)calloc(1, sizeof(orc_pa));
  if (!p) return ORC_ENOMEM;
  p->L = L;
  p->N = L * L;
  p->R_t = R_t;
  p->cap = cap;
  p->seed = seed;
  p->pop = pop;
  p->q = q;
  size_t N = (size_t)p->N;
  p->spins = (int8_t*)malloc((size_t)cap * N);
  p->E = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  p->M = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  p->n = (uint32_t*)calloc((size_t)cap, sizeof(uint32_t));
  p->fam = (uint32_t*)calloc((size_t)cap, sizeof(uint32_t));
  if (J) {
    p->J = (int8_t*)malloc(2 * N);
    if (p->J) memcpy(p->J, J, 2 * N);
  }
  if (!p->spins || !p->E || !p->M || !p->n || !p->fam || (J && !p->J)) {
    orc_destroy(p);
    return ORC_ENOMEM;
  }
  /* Initial population at beta_0 = 0 (Eq. part-F, second form): every
     state has the same probability, so each spin is an independent fair
     coin.  Site (x,y) takes word x mod 4 of group y*ceil(L/4) + x/4 of the
     INIT stream of its replica; the top bit of the word set means +1. */
  int G4 = (L + 3) / 4;
  for (int64_t j = 0; j < R_t; ++j) {
    int8_t* s = p->spins + (size_t)j * N;
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        uint32_t w = draw_word(seed, DOMAIN_INIT, (uint32_t)(y * G4 + x / 4), 0,
                               0, (uint32_t)j, pop, x % 4);
        /* Potts: a uniform state floor(w q / 2^32) */
        s[y * L + x] = q ? (int8_t)potts_state(w, q) : ((w >> 31) ? 1 : -1);
      }
    if (q) orc_potts_energy(L, q, s, &p->E[j], &p->M[j]);
    else orc_energy(L, p->J, s, &p->E[j], &p->M[j]);
  }
  p->R = R_t;
  reset_families(p);
  p->beta = 0.0;
  /* ln Omega: 2^N (q^N) states, all with weight 1 at beta_0 = 0. */
  p->lnZ = (ORC_MUTANT == 7) ? 0.0 : (double)p->N * log(q ? (double)q : 2.0);
  p->lnQ_last = 0.0;
  p->step = 0;
  p->sweeps_at_step = 0;
  p->n_len = 0;
  *out = p;
  return ORC_OK;
}

int orc_create(int L, const int8_t* J, int64_t R_t, int64_t cap,
               uint64_t seed, uint32_t pop, orc_pa** out) {
  return create(L, J, 0, R_t, cap, seed, pop, out);
}

int orc_create_potts(int L, int q, int64_t R_t, int64_t cap, uint64_t seed,
                     uint32_t pop, orc_pa** out) {
  if (q < 2) return ORC_EINVAL;
  return create(L, NULL, q, R_t, cap, seed, pop, out);
}

void orc_destroy(orc_pa* p) {
  if (!p) return;
  free(p->spins);
  free(p->E);
  free(p->M);
  free(p->n);
  free(p->fam);
  free(p->J);
  free(p);
}

/* ------------------------------------------------------------ resampling */

/* Steps 2-3 of the method (Eqs. part-Q, tau) for a population given by its
   energies E[0..R): computes ln Q for the step dbeta and the copy count of
   every replica.  The resampling draws of slot j come from the RESAMPLE
   stream at step `step_next` (the index of the temperature being entered). */
/* A Poisson(rho) draw from the 32-bit word r by inversion of its cumulative
   distribution.  With P(k) = exp(k log rho - rho - lgamma(k + 1)) and
   C(k) = P(0) + ... + P(k), summed in increasing k, the thresholds are
   U_k = floor(C(k) 2^32) and the draw is the number of thresholds <= r,
   i.e. the smallest k with r < U_k.  The thresholds stop after the first
   k with C(k) >= 1 - 2^-32 (the rest of the mass is below one 32-bit
   step) or before k = ceil(rho + 64 sqrt(rho) + 64). */
uint32_t orc_poisson_draw(double rho, uint32_t r) {
  if (!(rho > 0.0)) return 0u;
  const double kcap = ceil(rho + 64.0 * sqrt(rho) + 64.0);
  const double lr = log(rho);
  double C = 0.0;
  for (uint32_t k = 0;; ++k) {
    if ((double)k >= kcap) return k;      /* every threshold was <= r */
    C = C + exp((double)k * lr - ((ORC_MUTANT == 8) ? 0.0 : rho) -
                lgamma((double)k + 1.0));
    if ((uint64_t)r < (uint64_t)floor(ldexp(C, 32))) return k;
    if (C >= 1.0 - ldexp(1.0, -32)) return k + 1;   /* the last threshold */
  }
}

/* The replica a multinomial draw u lands in: the first j with
   floor(u C / 2^64) < C_j, C = cum[R - 1] the end of the last interval. */
int64_t orc_multinomial_pick(uint64_t u, const uint64_t* cum, int64_t R) {
  const uint64_t x = (uint64_t)(((unsigned __int128)u * cum[R - 1]) >> 64);
  int64_t lo = 0, hi = R - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (x < cum[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

int orc_counts(int N, const int32_t* E, int64_t R, int64_t R_t, double dbeta,
               uint64_t seed, uint32_t pop, int step_next, int law,
               uint32_t* n_out, int64_t* R_new, double* lnQ_out) {
  if (N < 16 || !E || R < 1 || R_t < 1 || !n_out || !isfinite(dbeta) ||
      law < ORC_NEAREST || law > ORC_MULTINOMIAL)
    return ORC_EINVAL;
  for (int64_t j = 0; j < R; ++j)
    if (E[j] < -2 * N || E[j] > 2 * N) return ORC_EINVAL;
  int nlev = 4 * N + 1; /* energies -2N..2N, index E + 2N */
  uint32_t* h = (uint32_t*)calloc((size_t)nlev, sizeof(uint32_t));
  double* w = (double*)calloc((size_t)nlev, sizeof(double));
  double* rh = (double*)calloc((size_t)nlev, sizeof(double));
  uint32_t* f = (uint32_t*)calloc((size_t)nlev, sizeof(uint32_t));
  uint64_t* T = (uint64_t*)calloc((size_t)nlev, sizeof(uint64_t));
  if (!h || !w || !rh || !f || !T) {
    free(h); free(w); free(rh); free(f); free(T);
    return ORC_ENOMEM;
  }
  /* (a) histogram of the energies; the energy the weights are shifted by:
     the smallest one when cooling (dbeta >= 0), the largest when heating,
     so that every weight is at most 1 */
  int32_t Emin = 2 * N + 1, Emax = -2 * N - 1;
  for (int64_t j = 0; j < R; ++j) {
    h[E[j] + 2 * N] += 1;
    if (E[j] < Emin) Emin = E[j];
    if (E[j] > Emax) Emax = E[j];
  }
  if (dbeta < 0.0) Emin = Emax;  /* the shift energy from here on */
  /* (b) Boltzmann factors exp(-dbeta E) shifted, summed per energy level in
     ascending energy order (Eq. part-Q numerator) */
  double S = 0.0;
  for (int e = -2 * N; e <= 2 * N; ++e) {
    uint32_t c = h[e + 2 * N];
    if (c == 0) continue;
    double we = exp(-(dbeta * (double)(e - Emin)));
    w[e + 2 * N] = we;
    double term = (ORC_MUTANT == 6) ? we : (double)c * we;
    S = S + term;
  }
  /* (c) ln Q = ln[(1/R) sum_j exp(-dbeta E_j)] with the shift restored */
  double lnQ = ((ORC_MUTANT == 2) ? (dbeta * (double)Emin)
                                  : (-(dbeta * (double)Emin))) +
               log(S / (double)R);
  /* (d) mean copy number rho = R_target tau / R (Eq. tau); its integer part
     and its fractional part as a 32-bit threshold */
  for (int e = -2 * N; e <= 2 * N; ++e) {
    if (h[e + 2 * N] == 0) continue;
    double rho = ((double)R_t * w[e + 2 * N]) / S;
    rh[e + 2 * N] = rho;
    double fl = floor(rho);
    f[e + 2 * N] = (uint32_t)fl;
    T[e + 2 * N] = (uint64_t)floor(ldexp(rho - fl, 32));
  }
  /* (e) copy counts: floor plus a Bernoulli draw on the fraction, or a
     Poisson draw with mean rho; one 32-bit word per slot either way.
     Systematic resampling instead lays the means end to end in 32.32 fixed
     point, P_j = floor(rho) 2^32 + T, and places one comb of unit-spaced
     teeth offset by a single word U (RESAMPLE group 1, slot 0, word 0 at
     the new step): replica j gets the teeth in its interval,
     n_j = floor((C_j + U) / 2^32) - floor((C_{j-1} + U) / 2^32),
     C_j = P_0 + ... + P_j. */
  int64_t total = 0;
  if (law == ORC_SYSTEMATIC) {
    uint64_t U = draw_word(seed, DOMAIN_RESAMPLE, 1, (uint32_t)step_next, 0,
                           0, pop, 0);
    uint64_t C = 0;
    for (int64_t j = 0; j < R; ++j) {
      int idx = E[j] + 2 * N;
      uint64_t P = ((uint64_t)f[idx] << 32) + T[idx];
      uint32_t nj = (ORC_MUTANT == 11)
                        ? (uint32_t)(((C + U) >> 32) - ((C - (j ? P : 0) + U) >> 32))
                        : (uint32_t)(((C + P + U) >> 32) - ((C + U) >> 32));
      C += P;
      n_out[j] = nj;
      total += nj;
    }
  }
  /* Multinomial resampling: R_target independent draws; draw i (the 64-bit
     number u_i = w1 2^32 + w0 from words 0 and 1 of RESAMPLE group 2, slot
     i, at the new step) lands at x_i = floor(u_i C / 2^64) on the same
     fixed-point axis (C the total of the P_j = floor(rho) 2^32 + T) and
     counts for the replica whose interval [C_{j-1}, C_j) holds it.  A
     64-bit u makes every interval's probability exact to 2^-64 per draw
     (a 32-bit one would quantise it to 2^-32, R_target 2^-32 copies over a
     step: a replica whose expected count is below that could get none).
     Residual resampling keeps floor(rho) copies of every replica for
     certain and makes the remaining D = R_target - sum_j floor(rho_j) draws
     the same way over the fractional parts alone (P_j = T; no draws when
     every fraction is zero). */
  if (law == ORC_MULTINOMIAL || law == ORC_RESIDUAL) {
    uint64_t* cum = (uint64_t*)malloc((size_t)R * sizeof(uint64_t));
    if (!cum) {
      free(h); free(w); free(rh); free(f); free(T);
      return ORC_ENOMEM;
    }
    const int res = (law == ORC_RESIDUAL);
    uint64_t C = 0;
    int64_t floors = 0;
    for (int64_t j = 0; j < R; ++j) {
      int idx = E[j] + 2 * N;
      C += (res ? 0 : ((uint64_t)f[idx] << 32)) + T[idx];
      cum[j] = C;  /* C_j, the end of replica j's interval */
      n_out[j] = res ? f[idx] : 0;
      floors += res ? (int64_t)f[idx] : 0;
    }
    int64_t draws = res ? R_t - floors : R_t;
    if (draws < 0 || C == 0) draws = 0;
    if (ORC_MUTANT == 12) draws = R;
    for (int64_t i = 0; i < draws; ++i) {
      uint64_t u =
          ((uint64_t)draw_word(seed, DOMAIN_RESAMPLE, 2, (uint32_t)step_next,
                               0, (uint32_t)i, pop, 1) << 32) |
          draw_word(seed, DOMAIN_RESAMPLE, 2, (uint32_t)step_next, 0,
                    (uint32_t)i, pop, 0);
      n_out[orc_multinomial_pick(u, cum, R)] += 1;
    }
    free(cum);
    total = floors + draws;
  }
  for (int64_t j = 0; j < R && law != ORC_SYSTEMATIC &&
                      law != ORC_MULTINOMIAL && law != ORC_RESIDUAL;
       ++j) {
    int idx = E[j] + 2 * N;
    uint32_t r = draw_word(seed, DOMAIN_RESAMPLE, 0, (uint32_t)step_next, 0,
                           (uint32_t)j, pop, 0);
    uint32_t nj = (law == ORC_POISSON)
                      ? orc_poisson_draw(rh[idx], r)
                      : f[idx] + ((uint64_t)r < T[idx] ? 1u : 0u);
    n_out[j] = nj;
    total += nj;
  }
  free(h); free(w); free(rh); free(f); free(T);
  if (R_new) *R_new = total;
  if (lnQ_out) *lnQ_out = lnQ;
  return ORC_OK;
}

int orc_resample(orc_pa* p, double beta_next, int64_t* R_new) {
  /* cooling (beta_next >= beta) or heating (beta_next < beta), beta >= 0 */
  if (!p || !isfinite(beta_next) || !(beta_next >= 0.0)) return ORC_EINVAL;
  if (p->step + 1 > 65535) return ORC_EINVAL;
  uint32_t* n = (uint32_t*)malloc((size_t)p->R * sizeof(uint32_t));
  if (!n) return ORC_ENOMEM;
  int64_t total = 0;
  double lnQ = 0.0;
  int rc = orc_counts(p->N, p->E, p->R, p->R_t, beta_next - p->beta, p->seed,
                      p->pop, p->step + 1, p->law, n, &total, &lnQ);
  if (rc != ORC_OK) { free(n); return rc; }
  if (R_new) *R_new = total;
  if (total > p->cap) { free(n); return ORC_ECAPACITY; }
  if (total == 0) { free(n); return ORC_EEMPTY; }
  /* (f) the new population: parents in ascending slot order, each repeated
     n_j times contiguously, exact copies (spins, E and M) */
  size_t N = (size_t)p->N;
  int8_t* ns = (int8_t*)malloc((size_t)p->cap * N);
  int32_t* nE = (int32_t*)malloc((size_t)p->cap * sizeof(int32_t));
  int32_t* nM = (int32_t*)malloc((size_t)p->cap * sizeof(int32_t));
  uint32_t* nF = (uint32_t*)malloc((size_t)p->cap * sizeof(uint32_t));
  if (!ns || !nE || !nM || !nF) {
    free(ns); free(nE); free(nM); free(nF); free(n);
    return ORC_ENOMEM;
  }
  /* a copy belongs to its parent's family */
  int64_t k = 0;
  for (int64_t j = 0; j < p->R; ++j) {
    for (uint32_t c = 0; c < n[j]; ++c) {
      memcpy(ns + (size_t)k * N, p->spins + (size_t)j * N, N);
      nE[k] = p->E[j];
      nM[k] = p->M[j];
      nF[k] = (ORC_MUTANT == 17) ? (uint32_t)j : p->fam[j];
      ++k;
    }
  }
  memcpy(p->n, n, (size_t)p->R * sizeof(uint32_t));
  p->n_len = p->R;
  free(n);
  free(p->spins); free(p->E); free(p->M); free(p->fam);
  p->spins = ns; p->E = nE; p->M = nM; p->fam = nF;
  p->R = total;
  p->beta = beta_next;
  p->step += 1;
  p->sweeps_at_step = 0;
  p->lnQ_last = lnQ;
  /* Eq. Free-En (read with the logarithm): ln Z accumulates ln Q */
  p->lnZ = p->lnZ + lnQ;
  return ORC_OK;
}

/* ---------------------------------------------------------------- sweeps */

/* The 32-bit random number of the colour site (x, y) in half sweep hs of
   step `step`, replica slot `slot`; k = x/2 is its colour rank in the row.
   ORC_RNG_WORD: word k mod 4 of MCMC group y*ceil(L/8) + k/4.
   ORC_RNG_PLANES: r = B * 2^24 + floor(w / 2^8), with w the ORC_RNG_WORD
   number of the same site and B a byte of bit planes: the Philox block of
   domain MCMC_PLANES, group y*ceil(L/32) + x/32 (same step, half sweep,
   slot and population) holds eight planes, plane m = 2i + h (i = 0..3 the
   output word, h = 0 or 1) carrying bit 7 - m of B for the sites of that
   32-site stretch of the row, as bit ((x mod 32) XOR h) of output word i.
   The sites of one colour in a stretch sit at bit positions of one parity,
   so no two of them share a bit.  Both parts of r are independent uniform
   bits, so r is uniform on [0, 2^32) as in the default mode: the
   acceptance probabilities are the same.  A sweep that compares B with the
   top byte of the threshold first needs w only when they are equal. */
static uint32_t site_draw(int mode, int L, uint64_t seed, uint32_t pop,
                          uint32_t step, uint32_t hs, uint32_t slot, int y,
                          int x) {
  const int G8 = (L + 7) / 8;
  const int k = x / 2;
  uint32_t w = draw_word(seed, DOMAIN_MCMC, (uint32_t)(y * G8 + k / 4), step,
                         hs, slot, pop, k % 4);
  if (mode != ORC_RNG_PLANES) return w;
  const int W32 = (L + 31) / 32;
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = (DOMAIN_MCMC_PLANES << 28) | (uint32_t)(y * W32 + x / 32);
  ctr[1] = (step << 16) | hs;
  ctr[2] = slot;
  ctr[3] = pop;
  key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, out);
  uint32_t B = 0;
  for (int m = 0; m < 8; ++m) {
    int pos = (ORC_MUTANT == 18) ? (m & 1) : ((x % 32) ^ (m & 1));
    uint32_t bit = (out[m / 2] >> pos) & 1u;
    B |= bit << (7 - m);
  }
  return (B << 24) | (w >> 8);
}

uint32_t orc_site_draw(int mode, int L, uint64_t seed, uint32_t pop,
                       int step, int half_sweep, uint32_t slot, int y, int x) {
  return site_draw(mode, L, seed, pop, (uint32_t)step, (uint32_t)half_sweep,
                   slot, y, x);
}

static uint64_t splitmix(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Step 4 of the method: theta checkerboard Metropolis sweeps of one replica
   (spins s, energy *E, magnetisation *M) at the inverse temperature whose
   thresholds are T4, T8.  Sites of colour c have (x+y) mod 2 = c; a colour-c
   site with k = x/2 uses word k mod 4 of group y*ceil(L/8) + k/4 of the MCMC
   stream (step, half sweep 2t+c, slot, population), where t counts the
   sweeps made at this step before this one (t0 of them precede the call). */
static void sweep_one(int L, const int8_t* J, int8_t* s, int32_t* E,
                      int32_t* M, uint64_t seed, uint32_t pop, int step,
                      int t0, int theta, uint32_t slot, uint64_t T4,
                      uint64_t T8, uint64_t shuffle_seed, int mode) {
  int half = L * L / 2;
  int* order = (int*)malloc((size_t)half * sizeof(int));
  for (int t = 0; t < theta; ++t) {
    int tt = t0 + t;
    for (int c = 0; c < 2; ++c) {
      int cnt = 0;
      for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x)
          if (((x + y) & 1) == c) order[cnt++] = y * L + x;
      if (shuffle_seed) {
        uint64_t st = shuffle_seed ^ ((uint64_t)slot << 20) ^
                      ((uint64_t)tt << 4) ^ (uint64_t)c;
        for (int i = cnt - 1; i > 0; --i) {
          int r = (int)(splitmix(&st) % (uint64_t)(i + 1));
          int tmp = order[i]; order[i] = order[r]; order[r] = tmp;
        }
      }
      for (int i = 0; i < cnt; ++i) {
        int x = order[i] % L, y = order[i] / L;
        int xl = (x + L - 1) % L, xr = (x + 1) % L;
        int yu = (y + L - 1) % L, yd = (y + 1) % L;
        int sv = s[y * L + x];
        /* unsatisfied bonds: coupling * sigma * neighbour < 0 */
        int a = 0;
        a += (bond(J, L, 0, x, y) * sv * s[y * L + xr] < 0);
        a += (bond(J, L, 0, xl, y) * sv * s[y * L + xl] < 0);
        a += (bond(J, L, 1, x, y) * sv * s[yd * L + x] < 0);
        if (ORC_MUTANT != 1)
          a += (bond(J, L, 1, x, (ORC_MUTANT == 3) ? y : yu) * sv *
                    s[yu * L + x] < 0);
        int dE = 8 - 4 * a;
        uint32_t r = site_draw(mode, L, seed, pop, (uint32_t)step,
                               (uint32_t)(2 * tt + c), slot, y, x);
        int accept;
        if (dE <= 0) accept = 1;
        else if (ORC_MUTANT == 4) accept = (uint64_t)r < (dE == 4 ? T8 : T4);
        else accept = (uint64_t)r < (dE == 4 ? T4 : T8);
        if (accept) {
          s[y * L + x] = (int8_t)(-sv);
          *E += dE;
          *M += 2 * (-sv);
        }
      }
    }
  }
  free(order);
}

/* Metropolis acceptance probabilities exp(-beta dE) for dE = 4, 8 as
   32-bit integer thresholds: accept iff r < floor(p 2^32). */
/* Checkerboard Metropolis for the Potts model: colour 0 first; a colour
   site proposes one of the other q - 1 states uniformly,
   s' = (s + 1 + floor(w q' / 2^32)) mod q with q' = q - 1, and accepts iff
   dE = (#neighbours in s) - (#neighbours in s') <= 0 or r < T[dE],
   T[d] = floor(exp(-beta d) 2^32).  Colour site k = x/2 of row y uses
   Philox group y*ceil(L/4) + k/2: words 2(k%2) (proposal w) and
   2(k%2) + 1 (acceptance r). */
static void sweep_potts_one(int L, int q, int8_t* s, int32_t* E, int32_t* M,
                            uint64_t seed, uint32_t pop, int step, int t0,
                            int theta, uint32_t slot, const uint64_t T[5]) {
  int G4 = (L + 3) / 4;
  for (int t = 0; t < theta; ++t) {
    int tt = t0 + t;
    for (int c = 0; c < 2; ++c) {
      for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
          if (((x + y) & 1) != c) continue;
          int k = x / 2;
          uint32_t ctr[4], key[2], out[4];
          ctr[0] = (DOMAIN_MCMC << 28) | (uint32_t)(y * G4 + k / 2);
          ctr[1] = ((uint32_t)step << 16) | (uint32_t)(2 * tt + c);
          ctr[2] = slot;
          ctr[3] = pop;
          key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
          key[1] = (uint32_t)(seed >> 32);
          orc_philox4x32_10(ctr, key, out);
          uint32_t w = out[2 * (k % 2)], r = out[2 * (k % 2) + 1];
          int sv = s[y * L + x];
          int sn = (sv + 1 + potts_state(w, q - 1)) % q;
          int nb[4] = {s[y * L + (x + 1) % L], s[y * L + (x + L - 1) % L],
                       s[((y + 1) % L) * L + x], s[((y + L - 1) % L) * L + x]};
          int n_old = 0, n_new = 0;
          for (int i = 0; i < 4; ++i) {
            n_old += (nb[i] == sv);
            n_new += (nb[i] == sn);
          }
          int dE = (ORC_MUTANT == 10) ? n_new - n_old : n_old - n_new;
          if (dE <= 0 || (uint64_t)r < T[dE]) {
            s[y * L + x] = (int8_t)sn;
            *E += dE;
            *M += q * ((sn == 0) - (sv == 0));
          }
        }
    }
  }
}

static void potts_thresholds(double beta, uint64_t T[5]) {
  T[0] = (uint64_t)1 << 32;
  for (int d = 1; d <= 4; ++d)
    T[d] = (uint64_t)floor(ldexp(exp(-(beta * (double)d)), 32));
}

static void thresholds(double beta, uint64_t* T4, uint64_t* T8) {
  *T4 = (uint64_t)floor(ldexp(exp(-(beta * 4.0)), 32));
  *T8 = (uint64_t)floor(ldexp(exp(-(beta * 8.0)), 32));
}

int orc_sweep_replica_rng(int L, const int8_t* J, int8_t* spins,
                          int32_t* E, int32_t* M, double beta, uint64_t seed,
                          uint32_t pop, int step, int t0, int theta,
                          uint32_t slot, int rng_mode) {
  if (L < 4 || L > 128 || (L % 2) || !spins || !E || !M || theta < 0 ||
      t0 < 0 || t0 + theta > 32767 || !isfinite(beta) ||
      (rng_mode != ORC_RNG_WORD && rng_mode != ORC_RNG_PLANES))
    return ORC_EINVAL;
  uint64_t T4, T8;
  thresholds(beta, &T4, &T8);
  sweep_one(L, J, spins, E, M, seed, pop, step, t0, theta, slot, T4, T8, 0,
            rng_mode);
  return ORC_OK;
}

int orc_sweep_replica(int L, const int8_t* J, int8_t* spins, int32_t* E,
                      int32_t* M, double beta, uint64_t seed, uint32_t pop,
                      int step, int t0, int theta, uint32_t slot) {
  return orc_sweep_replica_rng(L, J, spins, E, M, beta, seed, pop, step, t0,
                               theta, slot, ORC_RNG_WORD);
}

int orc_sweep_potts_replica(int L, int q, int8_t* spins, int32_t* E,
                            int32_t* M, double beta, uint64_t seed,
                            uint32_t pop, int step, int t0, int theta,
                            uint32_t slot) {
  if (L < 4 || L > 128 || (L % 2) || q < 2 || q > 16 || !spins || !E || !M ||
      theta < 0 || t0 < 0 || t0 + theta > 32767 || !isfinite(beta))
    return ORC_EINVAL;
  uint64_t T[5];
  potts_thresholds(beta, T);
  sweep_potts_one(L, q, spins, E, M, seed, pop, step, t0, theta, slot, T);
  return ORC_OK;
}

int orc_sweep(orc_pa* p, int theta) {
  if (!p || theta < 0) return ORC_EINVAL;
  if (p->sweeps_at_step + theta > 32767) return ORC_EINVAL;
  if (p->q) {
    uint64_t T[5];
    potts_thresholds(p->beta, T);
    for (int64_t j = 0; j < p->R; ++j)
      sweep_potts_one(p->L, p->q, p->spins + (size_t)j * p->N, &p->E[j],
                      &p->M[j], p->seed, p->pop, p->step, p->sweeps_at_step,
                      theta, (uint32_t)j, T);
    p->sweeps_at_step += theta;
    return ORC_OK;
  }
  uint64_t T4, T8;
  thresholds(p->beta, &T4, &T8);
  for (int64_t j = 0; j < p->R; ++j)
    sweep_one(p->L, p->J, p->spins + (size_t)j * p->N, &p->E[j], &p->M[j],
              p->seed, p->pop, p->step, p->sweeps_at_step, theta, (uint32_t)j,
              T4, T8, p->shuffle_seed, p->rng_mode);
  p->sweeps_at_step += theta;
  return ORC_OK;
}

/* The same sweeps with the replicas split into nthreads contiguous ranges,
   one POSIX thread each (for timing the oracle on every host core).  Each
   replica's random numbers are keyed by its own slot, so the result is the
   single-threaded one bit for bit. */
typedef struct {
  orc_pa* p;
  int theta;
  int64_t j0, j1;
  uint64_t T4, T8;
} sweep_range;

static void* sweep_range_run(void* arg) {
  sweep_range* a = (sweep_range*)arg;
  orc_pa* p = a->p;
  for (int64_t j = a->j0; j < a->j1; ++j)
    sweep_one(p->L, p->J, p->spins + (size_t)j * p->N, &p->E[j], &p->M[j],
              p->seed, p->pop, p->step, p->sweeps_at_step, a->theta,
              (uint32_t)j, a->T4, a->T8, p->shuffle_seed, p->rng_mode);
  return NULL;
}

int orc_sweep_threads(orc_pa* p, int theta, int nthreads) {
  if (!p || theta < 0 || nthreads < 1 || nthreads > 1024) return ORC_EINVAL;
  if (p->q || nthreads == 1) return orc_sweep(p, theta);
  if (p->sweeps_at_step + theta > 32767) return ORC_EINVAL;
  uint64_t T4, T8;
  thresholds(p->beta, &T4, &T8);
  sweep_range* a = (sweep_range*)calloc((size_t)nthreads, sizeof(sweep_range));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  int* started = (int*)calloc((size_t)nthreads, sizeof(int));
  if (!a || !th || !started) {
    free(a);
    free(th);
    free(started);
    return ORC_ENOMEM;
  }
  for (int i = 0; i < nthreads; ++i) {
    a[i].p = p;
    a[i].theta = theta;
    a[i].j0 = p->R * i / nthreads;
    a[i].j1 = p->R * (i + 1) / nthreads;
    a[i].T4 = T4;
    a[i].T8 = T8;
    started[i] = pthread_create(&th[i], NULL, sweep_range_run, &a[i]) == 0;
    if (!started[i]) sweep_range_run(&a[i]);
  }
  for (int i = 0; i < nthreads; ++i)
    if (started[i]) pthread_join(th[i], NULL);
  free(a);
  free(th);
  free(started);
  p->sweeps_at_step += theta;
  return ORC_OK;
}

/* ------------------------------------------------------------ observables */

int orc_observables(const orc_pa* p, orc_obs* o) {
  if (!p || !o) return ORC_EINVAL;
  int64_t sE = 0, sE2 = 0, sAM = 0, sM2 = 0;
  int32_t mn = 2 * p->N + 1, mx = -2 * p->N - 1;
  for (int64_t j = 0; j < p->R; ++j) {
    int64_t e = p->E[j], m = p->M[j];
    sE += e;
    sE2 += e * e;
    sAM += m < 0 ? -m : m;
    sM2 += m * m;
    if (p->E[j] < mn) mn = p->E[j];
    if (p->E[j] > mx) mx = p->E[j];
  }
  double R = (double)p->R, N = (double)p->N;
  __int128 var = (__int128)p->R * sE2 - (__int128)sE * sE;
  o->R = p->R;
  o->beta = p->beta;
  o->e = (double)sE / (R * N);
  o->abs_m = (double)sAM / (R * N);
  o->m2 = (double)sM2 / (R * N * N);
  o->C = (((ORC_MUTANT == 15) ? p->beta : (p->beta * p->beta)) * (double)var) /
         ((R * R) * N);
  o->sumE = sE;
  o->sumE2 = sE2;
  o->sumAbsM = sAM;
  o->sumM2 = sM2;
  o->Emin = mn;
  o->Emax = mx;
  return ORC_OK;
}

int orc_free_energy(const orc_pa* p, double* lnZ, double* lnQ_last) {
  if (!p) return ORC_EINVAL;
  if (lnZ) *lnZ = p->lnZ;
  if (lnQ_last) *lnQ_last = p->lnQ_last;
  return ORC_OK;
}

/* -------------------------------------------------------------- accessors */

int64_t orc_R(const orc_pa* p) { return p->R; }
double orc_beta(const orc_pa* p) { return p->beta; }
int orc_step(const orc_pa* p) { return p->step; }

int orc_get_population(const orc_pa* p, int8_t* spins, int32_t* E,
                       int32_t* M, int64_t cap) {
  if (!p || cap < p->R) return ORC_EINVAL;
  if (spins) memcpy(spins, p->spins, (size_t)p->R * p->N);
  if (E) memcpy(E, p->E, (size_t)p->R * sizeof(int32_t));
  if (M) memcpy(M, p->M, (size_t)p->R * sizeof(int32_t));
  return ORC_OK;
}

int orc_get_counts(const orc_pa* p, uint32_t* n, int64_t cap) {
  if (!p || !n || cap < p->n_len) return ORC_EINVAL;
  memcpy(n, p->n, (size_t)p->n_len * sizeof(uint32_t));
  return (int)0;
}

/* The heating protocol (Sec. 2, with the Potts reference): the population
   starts close to zero temperature, at beta0 > 0, in the ground states of
   the ferromagnet, all spins +1 or all -1 with probability 1/2 each (the top
   bit of the INIT word of site (0,0) of the replica decides), and ln Z(beta0)
   is that of the ground states, ln g + 2 N beta0 (g = 2 states, or q for
   Potts, of energy -2N), plus the smallest excitations of each: on a torus
   of side L >= 4 one changed site (N of them, 4 bonds broken) and two
   changed neighbours (2N pairs, 6 bonds broken, or 7 when the two Potts
   states differ).  Taking the logarithm of 1 + these terms, the products of
   two distant excitations cancel the square of the first term, so up to
   terms of order N exp(-16 beta0) (Ising) or N exp(-8 beta0) (Potts):
     Ising: ln Z = ln 2 + 2 N beta0 + N (exp(-8 beta0) + 2 exp(-12 beta0));
     Potts: ln Z = ln q + 2 N beta0
                   + N (q - 1) (exp(-4 beta0) + 2 exp(-6 beta0)
                                + 2 (q - 2) exp(-7 beta0)). */
int orc_start_heating(orc_pa* p, double beta0) {
  if (!p || p->J || p->step != 0 || !isfinite(beta0) || !(beta0 > 0.0))
    return ORC_EINVAL;
  size_t N = (size_t)p->N;
  p->R = p->R_t;
  for (int64_t j = 0; j < p->R; ++j) {
    uint32_t w = draw_word(p->seed, DOMAIN_INIT, 0, 0, 0, (uint32_t)j, p->pop,
                           0);
    int8_t* s = p->spins + (size_t)j * N;
    if (p->q) {  /* the q ground states: every site in one state */
      memset(s, potts_state(w, p->q), N);
      orc_potts_energy(p->L, p->q, s, &p->E[j], &p->M[j]);
    } else {
      memset(s, (w >> 31) ? 1 : -1, N);
      orc_energy(p->L, p->J, s, &p->E[j], &p->M[j]);
    }
  }
  reset_families(p);
  p->beta = beta0;
  /* ln(#ground states) - beta0 E_0 with E_0 = -2N, then the excitations */
  double ex;
  if (p->q)
    ex = (double)p->N * (double)(p->q - 1) *
         (exp(-4.0 * beta0) + 2.0 * exp(-6.0 * beta0) +
          2.0 * (double)(p->q - 2) * exp(-7.0 * beta0));
  else
    ex = (double)p->N * (exp(-8.0 * beta0) + 2.0 * exp(-12.0 * beta0));
  p->lnZ = (log(p->q ? (double)p->q : 2.0) +
            ((ORC_MUTANT == 9) ? 0.0 : 2.0 * (double)p->N * beta0)) +
           ((ORC_MUTANT == 19) ? 0.0 : ex);
  p->lnQ_last = 0.0;
  p->n_len = 0;
  return ORC_OK;
}

int orc_set_population(orc_pa* p, const int8_t* spins, int64_t R) {
  if (!p || !spins || R < 1 || R > p->cap) return ORC_EINVAL;
  for (int64_t i = 0; i < R * p->N; ++i)
    if (p->q ? (spins[i] < 0 || spins[i] >= p->q)
             : (spins[i] != 1 && spins[i] != -1))
      return ORC_EINVAL;
  memcpy(p->spins, spins, (size_t)R * p->N);
  for (int64_t j = 0; j < R; ++j) {
    if (p->q)
      orc_potts_energy(p->L, p->q, p->spins + (size_t)j * p->N, &p->E[j],
                       &p->M[j]);
    else
      orc_energy(p->L, p->J, p->spins + (size_t)j * p->N, &p->E[j], &p->M[j]);
  }
  p->R = R;
  reset_families(p);
  p->n_len = 0;
  return ORC_OK;
}

int orc_get_families(const orc_pa* p, uint32_t* fam, int64_t cap,
                     int64_t* n0) {
  if (!p || !fam || cap < p->R) return ORC_EINVAL;
  memcpy(fam, p->fam, (size_t)p->R * sizeof(uint32_t));
  if (n0) *n0 = p->fam_n0;
  return ORC_OK;
}

/* Family statistics of a population of R replicas whose families are
   numbered 0..n0-1 (fam[j] the family of replica j).  With c_i replicas in
   family i and nu_i = c_i / R: the number of families with c_i > 0, the
   largest c_i, the mean square family size rho_t = R sum_i nu_i^2 =
   sum_i c_i^2 / R, and the entropic family size rho_s = R exp(-S),
   S = -sum_i nu_i ln nu_i, which equals exp(sum_i c_i ln c_i / R).  Sums in
   ascending family order. */
int orc_family_stats(const uint32_t* fam, int64_t R, int64_t n0,
                     int64_t* families, int64_t* largest, double* rho_t,
                     double* rho_s) {
  if (!fam || R < 1 || n0 < 1) return ORC_EINVAL;
  int64_t* c = (int64_t*)calloc((size_t)n0, sizeof(int64_t));
  if (!c) return ORC_ENOMEM;
  for (int64_t j = 0; j < R; ++j) {
    if ((int64_t)fam[j] >= n0) { free(c); return ORC_EINVAL; }
    c[fam[j]] += 1;
  }
  int64_t nf = 0, big = 0, s2 = 0;
  double sl = 0.0;
  for (int64_t i = 0; i < n0; ++i) {
    if (c[i] == 0) continue;
    nf += 1;
    if (c[i] > big) big = c[i];
    s2 += c[i] * c[i];
    sl = sl + (double)c[i] * log((double)c[i]);
  }
  free(c);
  if (families) *families = nf;
  if (largest) *largest = big;
  if (rho_t) *rho_t = (double)s2 / (double)R;
  if (rho_s) *rho_s = (ORC_MUTANT == 16) ? exp(sl) : exp(sl / (double)R);
  return ORC_OK;
}

int orc_histogram(const orc_pa* p, uint32_t* out) {
  if (!p || !out) return ORC_EINVAL;
  memset(out, 0, (size_t)(4 * p->N + 1) * sizeof(uint32_t));
  for (int64_t j = 0; j < p->R; ++j) out[p->E[j] + 2 * p->N] += 1;
  return ORC_OK;
}

int orc_set_resampling(orc_pa* p, int law) {
  if (!p || law < ORC_NEAREST || law > ORC_MULTINOMIAL) return ORC_EINVAL;
  p->law = law;
  return ORC_OK;
}

void orc_set_visit_shuffle(orc_pa* p, uint64_t shuffle_seed) {
  if (p) p->shuffle_seed = shuffle_seed;
}

int orc_set_rng_mode(orc_pa* p, int mode) {
  if (!p || p->q || (mode != ORC_RNG_WORD && mode != ORC_RNG_PLANES))
    return ORC_EINVAL;
  p->rng_mode = mode;
  return ORC_OK;
}

/* ------------------------------------------------------ adaptive schedule */

/* Overlap of the energy distribution at beta with the reweighted one at
   beta + dbeta: alpha = sum_E min(P(E), P'(E)) with P = h/R and
   P' = h w / sum h w, w = exp(-dbeta (E - Emin)).  1 - alpha is the
   fraction of the population the resampling culls on average, the quantity
   an adaptive step (Sec. 3, last paragraph on fluctuations) keeps fixed. */
int orc_overlap(const orc_pa* p, double dbeta, double* alpha) {
  if (!p || !alpha || !isfinite(dbeta) || dbeta < 0.0) return ORC_EINVAL;
  int N = p->N;
  int nlev = 4 * N + 1;
  uint32_t* h = (uint32_t*)calloc((size_t)nlev, sizeof(uint32_t));
  if (!h) return ORC_ENOMEM;
  int32_t Emin = 2 * N + 1;
  for (int64_t j = 0; j < p->R; ++j) {
    h[p->E[j] + 2 * N] += 1;
    if (p->E[j] < Emin) Emin = p->E[j];
  }
  double S = 0.0;
  for (int e = -2 * N; e <= 2 * N; ++e) {
    uint32_t c = h[e + 2 * N];
    if (c == 0) continue;
    double term = (double)c * exp(-(dbeta * (double)(e - Emin)));
    S = S + term;
  }
  double a = 0.0;
  for (int e = -2 * N; e <= 2 * N; ++e) {
    uint32_t c = h[e + 2 * N];
    if (c == 0) continue;
    double pe = (double)c / (double)p->R;
    double qe = ((double)c * exp(-(dbeta * (double)(e - Emin)))) / S;
    a = a + ((ORC_MUTANT == 13) ? (pe < qe ? qe : pe) : (pe < qe ? pe : qe));
  }
  free(h);
  *alpha = a;
  return ORC_OK;
}

/* Largest step dbeta <= beta_f - beta whose overlap is at least target:
   the whole remaining interval if it qualifies, otherwise 64 halvings of
   [0, beta_f - beta] keeping the lower end qualified. */
int orc_bisect_dbeta(const orc_pa* p, double target, double beta_f,
                     double* dbeta) {
  if (!p || !dbeta || !(target > 0.0 && target <= 1.0) || !isfinite(beta_f))
    return ORC_EINVAL;
  double span = beta_f - p->beta;
  if (!(span > 0.0)) { *dbeta = 0.0; return ORC_OK; }
  double a;
  int rc = orc_overlap(p, span, &a);
  if (rc) return rc;
  if (a >= target) { *dbeta = span; return ORC_OK; }
  double lo = 0.0, hi = span;
  for (int it = 0; it < 64; ++it) {
    double mid = 0.5 * (lo + hi);
    rc = orc_overlap(p, mid, &a);
    if (rc) return rc;
    if (a >= target) lo = mid;
    else hi = mid;
  }
  *dbeta = (ORC_MUTANT == 14) ? hi : lo;
  return ORC_OK;
}
