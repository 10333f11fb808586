// Host double-precision arithmetic of the population-annealing step, shared
// by the single-population and the batched paths: reweighting tables from an
// exact energy histogram (Eqs. part-Q, tau), the free-energy increment
// (Eq. Free-En), Metropolis thresholds, observables from exact sums, and the
// overlap / bisection of the adaptive temperature step.
//
// Every quantity is a plain IEEE operation in a fixed order (per energy
// level, ascending energy); the library is compiled with -ffp-contract=off.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <cstdio>
#include <exception>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

namespace pa {

static thread_local char g_last_error[512] = "";

void set_last_error(const char* what, hipError_t e, int line) {
  std::snprintf(g_last_error, sizeof g_last_error, "%s failed at line %d: %s",
                what, line, hipGetErrorString(e));
}

void note_error(const char* text) {
  std::snprintf(g_last_error, sizeof g_last_error, "%s", text ? text : "");
}

void note_exception(const char* what) {
  std::snprintf(g_last_error, sizeof g_last_error,
                "C++ exception stopped at the ABI: %s", what ? what : "");
}

const char* last_error() { return g_last_error; }

bool fault_injected(const char* what) {
  const char* f = std::getenv("PA_FAULT");
  return f && std::strcmp(f, what) == 0;
}

void log_step(const StepLog& s) {
  const char* path = std::getenv("PA_LOG_JSONL");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  char R[32];
  if (s.R >= 0) std::snprintf(R, sizeof R, "%lld", (long long)s.R);
  else std::snprintf(R, sizeof R, "null");
  std::fprintf(f,
               "{\"pop\": %lld, \"step\": %lld, \"beta\": %.17g, "
               "\"dbeta\": %.17g, \"R_prev\": %lld, \"R\": %s, "
               "\"lnQ\": %.17g, \"lnZ\": %.17g, \"overlap\": %.17g, "
               "\"culling\": %.17g, \"e_prev\": %.17g, "
               "\"abs_m_prev\": %.17g, \"C_prev\": %.17g, "
               "\"source\": \"%s\"}\n",
               (long long)s.pop, (long long)s.step, s.beta, s.dbeta,
               (long long)s.R_prev, R, s.lnQ, s.lnZ, s.overlap,
               1.0 - s.overlap, s.e_prev, s.abs_m_prev, s.C_prev,
               s.source ? s.source : "");
  std::fclose(f);
}

static inline int level_energy(int N, int shift, int i) {
  return -2 * N + (i << shift);
}

void occupied_range(const uint32_t* h, int nbins, int* lo, int* hi) {
  int a = 0, b = nbins - 1;
  while (a < nbins && h[a] == 0) ++a;
  while (b >= 0 && h[b] == 0) --b;
  *lo = a;
  *hi = b;
}

// Metropolis acceptance probabilities exp(-beta dE) for dE = 4, 8 as 32-bit
// integer thresholds T = floor(p 2^32) (T = 2^32 accepts always); the kernel
// receives K = 2^32 - T and rejects a random word r iff r + K >= 2^32.
void metropolis_K(double beta, uint64_t* K4, uint64_t* K8) {
  const uint64_t T4 = (uint64_t)std::floor(std::ldexp(std::exp(-(beta * 4.0)), 32));
  const uint64_t T8 = (uint64_t)std::floor(std::ldexp(std::exp(-(beta * 8.0)), 32));
  *K4 = (1ull << 32) - T4;
  *K8 = (1ull << 32) - T8;
}

// Potts acceptance thresholds T[d - 1] = floor(exp(-beta d) 2^32) for an
// energy increase d = 1..4 (beta = 0 gives 2^32: always accept).
void potts_thresholds(double beta, uint64_t Tp[4]) {
  for (int d = 1; d <= 4; ++d)
    Tp[d - 1] = (uint64_t)std::floor(std::ldexp(std::exp(-(beta * (double)d)), 32));
}

int build_tables(const uint32_t* h, int nbins, int shift, int N, int64_t R,
                 int64_t R_t, double dbeta, uint32_t* f, uint32_t* T,
                 TableRange* out) {
  int lo, hi;
  occupied_range(h, nbins, &lo, &hi);
  if (lo > hi || R < 1) return PA_ESTATE;
  // the energy the weights are shifted by: the smallest one when cooling,
  // the largest one when heating (dbeta < 0), so every weight is at most 1
  const int Emin = level_energy(N, shift, dbeta < 0.0 ? hi : lo);
  const int nl = hi - lo + 1;
  // (b) Boltzmann factors shifted by Emin, summed in ascending energy
  std::vector<double> w((size_t)nl, 0.0);
  double S = 0.0;
  for (int i = lo; i <= hi; ++i) {
    if (h[i] == 0) continue;
    const double we =
        std::exp(-(dbeta * (double)(level_energy(N, shift, i) - Emin)));
    w[i - lo] = we;
    const double term = (double)h[i] * we;
    S = S + term;
  }
  // (c) ln Q with the shift restored (Eq. part-Q)
  out->lnQ = (-(dbeta * (double)Emin)) + std::log(S / (double)R);
  // (d) rho = R_target tau / R (Eq. tau): integer part and 32-bit threshold
  for (int i = lo; i <= hi; ++i) {
    f[i - lo] = 0u;
    T[i - lo] = 0u;
    if (h[i] == 0) continue;
    const double rho = ((double)R_t * w[i - lo]) / S;
    const double fl = std::floor(rho);
    f[i - lo] = (uint32_t)fl;
    T[i - lo] = (uint32_t)(uint64_t)std::floor(std::ldexp(rho - fl, 32));
  }
  out->lo = lo;
  out->hi = hi;
  return PA_OK;
}

// Poisson copy-count tables (Sec. 2 names the Poisson law).  For every
// occupied level with mean rho the thresholds U_k = floor(C(k) 2^32) of the
// cumulative distribution C(k) = sum_{i<=k} exp(i log rho - rho -
// lgamma(i + 1)), summed in increasing i; the list stops after the first k
// with C(k) >= 1 - 2^-32 or before k = ceil(rho + 64 sqrt(rho) + 64).  A
// replica's copy count is the number of thresholds <= its 32-bit word.
// Layout (uint32 words): level l (relative to lo) has (base, off, len) at
// 3l; its thresholds are at 3 nl + off.  base counts the zero thresholds
// (every word passes them); thresholds equal to 2^32 (no word passes them)
// are left out.  n_min / n_max bound the new population size exactly.
int build_poisson_tables(const uint32_t* h, int nbins, int shift, int N,
                         int64_t R, int64_t R_t, double dbeta,
                         std::vector<uint32_t>& out, TableRange* tr,
                         int64_t* n_min, int64_t* n_max) {
  int lo, hi;
  occupied_range(h, nbins, &lo, &hi);
  if (lo > hi || R < 1) return PA_ESTATE;
  const int Emin = level_energy(N, shift, dbeta < 0.0 ? hi : lo);
  const int nl = hi - lo + 1;
  // the weights, S and ln Q exactly as for the nearest-integer tables
  std::vector<double> w((size_t)nl, 0.0);
  double S = 0.0;
  for (int i = lo; i <= hi; ++i) {
    if (h[i] == 0) continue;
    const double we =
        std::exp(-(dbeta * (double)(level_energy(N, shift, i) - Emin)));
    w[i - lo] = we;
    const double term = (double)h[i] * we;
    S = S + term;
  }
  tr->lnQ = (-(dbeta * (double)Emin)) + std::log(S / (double)R);
  tr->lo = lo;
  tr->hi = hi;
  out.assign((size_t)3 * nl, 0u);
  int64_t mn = 0, mx = 0;
  const double top = 1.0 - std::ldexp(1.0, -32);
  for (int i = lo; i <= hi; ++i) {
    if (h[i] == 0) continue;
    const double rho = ((double)R_t * w[i - lo]) / S;
    uint32_t base = 0, len = 0;
    const uint32_t off = (uint32_t)(out.size() - (size_t)3 * nl);
    if (rho > 0.0) {
      const double kcap = std::ceil(rho + 64.0 * std::sqrt(rho) + 64.0);
      const double lr = std::log(rho);
      double C = 0.0;
      for (uint32_t k = 0; (double)k < kcap; ++k) {
        C = C + std::exp((double)k * lr - rho - std::lgamma((double)k + 1.0));
        const uint64_t U = (uint64_t)std::floor(std::ldexp(C, 32));
        if (U == 0) {
          ++base;
        } else if (U < (1ull << 32)) {
          out.push_back((uint32_t)U);
          ++len;
        }
        if (C >= top) break;
      }
    }
    out[(size_t)3 * (i - lo) + 0] = base;
    out[(size_t)3 * (i - lo) + 1] = off;
    out[(size_t)3 * (i - lo) + 2] = len;
    mn += (int64_t)h[i] * base;
    mx += (int64_t)h[i] * (base + len);
  }
  *n_min = mn;
  *n_max = mx;
  return PA_OK;
}

void observables_from_hist(const uint32_t* h, int nbins, int shift, int N,
                           int64_t R, double beta, int64_t sumAbsM,
                           int64_t sumM2, pa_obs* o) {
  int64_t sE = 0, sE2 = 0;
  int lo, hi;
  occupied_range(h, nbins, &lo, &hi);
  for (int i = lo; i <= hi; ++i) {
    const int64_t c = h[i], e = level_energy(N, shift, i);
    sE += c * e;
    sE2 += c * e * e;
  }
  observables_from_sums(R, beta, N, sE, sE2, sumAbsM, sumM2,
                        level_energy(N, shift, lo), level_energy(N, shift, hi),
                        o);
}

// The same from the exact sums (a schedule run on the device sends only
// these to the host).
void observables_from_sums(int64_t R, double beta, int N, int64_t sE,
                           int64_t sE2, int64_t sumAbsM, int64_t sumM2,
                           int32_t Emin, int32_t Emax, pa_obs* o) {
  const double Rd = (double)R, Nd = (double)N;
  const __int128 var = (__int128)R * sE2 - (__int128)sE * sE;
  o->R = R;
  o->beta = beta;
  o->e = (double)sE / (Rd * Nd);
  o->abs_m = (double)sumAbsM / (Rd * Nd);
  o->m2 = (double)sumM2 / (Rd * Nd * Nd);
  o->C = ((beta * beta) * (double)var) / ((Rd * Rd) * Nd);
  o->sumE = sE;
  o->sumE2 = sE2;
  o->sumAbsM = sumAbsM;
  o->sumM2 = sumM2;
  o->Emin = Emin;
  o->Emax = Emax;
}

// alpha(dbeta) = sum_E min(h/R, h w / S), w = exp(-dbeta (E - Emin))
double overlap_from_hist(const uint32_t* h, int nbins, int shift, int N,
                         int64_t R, double dbeta) {
  int lo, hi;
  occupied_range(h, nbins, &lo, &hi);
  const int Emin = level_energy(N, shift, lo);
  double S = 0.0;
  for (int i = lo; i <= hi; ++i) {
    if (h[i] == 0) continue;
    const double term = (double)h[i] *
        std::exp(-(dbeta * (double)(level_energy(N, shift, i) - Emin)));
    S = S + term;
  }
  double a = 0.0;
  for (int i = lo; i <= hi; ++i) {
    if (h[i] == 0) continue;
    const double pe = (double)h[i] / (double)R;
    const double qe = ((double)h[i] *
        std::exp(-(dbeta * (double)(level_energy(N, shift, i) - Emin)))) / S;
    a = a + (pe < qe ? pe : qe);
  }
  return a;
}

// Largest dbeta <= span with alpha(dbeta) >= target: the whole span if it
// qualifies, else 64 halvings of [0, span] keeping the lower end qualified.
// With tol > 0 the halving stops at the first midpoint whose overlap is
// within tol of the target (the acceptance test of a proposed step) and
// returns it.
double bisect_from_hist(const uint32_t* h, int nbins, int shift, int N,
                        int64_t R, double target, double span, int* evals,
                        double tol) {
  if (!(span > 0.0)) return 0.0;
  int k = 1;
  double d = span;
  if (overlap_from_hist(h, nbins, shift, N, R, span) < target) {
    double lo = 0.0, hi = span;
    d = -1.0;
    for (int it = 0; it < 64; ++it) {
      const double mid = 0.5 * (lo + hi);
      ++k;
      const double a = overlap_from_hist(h, nbins, shift, N, R, mid);
      if (tol > 0.0 && std::fabs(a - target) <= tol) {
        d = mid;
        break;
      }
      if (a >= target) lo = mid;
      else hi = mid;
    }
    if (d < 0.0) d = lo;
  }
  if (evals) *evals += k;
  return d;
}

}  // namespace pa

extern "C" const char* pa_last_error(void) { return pa::last_error(); }

// Weighted averaging over independent populations (the alternative to one
// large population discussed in Sec. 4 after the Machta reference): each
// population m is weighted by its partition-function estimate Z_m, i.e.
// w_m = exp(ln Z_m - max ln Z) / sum of those, summed in increasing m.
extern "C" int pa_weighted_average(int32_t M, const double* lnZ,
                                   const double* values, int32_t k,
                                   double* out, double* lnZ_out) try {
  if (M < 1 || k < 0 || !lnZ || (k > 0 && (!values || !out))) return PA_EINVAL;
  double mx = lnZ[0];
  for (int32_t m = 0; m < M; ++m) {
    if (!std::isfinite(lnZ[m])) return PA_EINVAL;
    if (lnZ[m] > mx) mx = lnZ[m];
  }
  std::vector<double> w((size_t)M);
  double s = 0.0;
  for (int32_t m = 0; m < M; ++m) {
    w[(size_t)m] = std::exp(lnZ[m] - mx);
    s = s + w[(size_t)m];
  }
  for (int32_t j = 0; j < k; ++j) {
    double a = 0.0;
    for (int32_t m = 0; m < M; ++m)
      a = a + w[(size_t)m] * values[(size_t)m * k + j];
    out[j] = a / s;
  }
  // ln of the mean of the Z_m: the combined estimate of ln Z
  if (lnZ_out) *lnZ_out = mx + std::log(s / (double)M);
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

// Observables of M independent populations at one beta, combined with the
// weights Z_m / sum Z (Sec. 4, Large scale testing).  Each population's
// mean energy is its exact integer sum over its size; its energy variance
// (R sum E^2 - (sum E)^2) / R^2 is formed in 128-bit integers before the
// one conversion, so no population's variance loses digits to
// cancellation.  The combined variance is the law of total variance:
// the weighted mean of the population variances plus the weighted spread
// of the population means about the combined mean.  Sums run over
// ascending m.
extern "C" int pa_weighted_observables(int32_t M, const double* lnZ,
                                       const pa_obs* obs, int32_t N,
                                       pa_combined* out) try {
  if (M < 1 || !lnZ || !obs || !out || N < 1) return PA_EINVAL;
  double mx = lnZ[0];
  for (int32_t m = 0; m < M; ++m) {
    if (!std::isfinite(lnZ[m]) || obs[m].R < 1) return PA_EINVAL;
    if (obs[m].beta != obs[0].beta) return PA_EINVAL;
    if (lnZ[m] > mx) mx = lnZ[m];
  }
  std::vector<double> w((size_t)M), mu((size_t)M), var((size_t)M);
  double s = 0.0, a = 0.0, am = 0.0, m2 = 0.0;
  int64_t Rtot = 0;
  for (int32_t m = 0; m < M; ++m) {
    const pa_obs& o = obs[m];
    const double Rd = (double)o.R;
    w[(size_t)m] = std::exp(lnZ[m] - mx);
    s = s + w[(size_t)m];
    mu[(size_t)m] = (double)o.sumE / Rd;
    const __int128 v = (__int128)o.R * (__int128)o.sumE2 -
                       (__int128)o.sumE * (__int128)o.sumE;
    var[(size_t)m] = (double)v / (Rd * Rd);
    a = a + w[(size_t)m] * mu[(size_t)m];
    am = am + w[(size_t)m] * ((double)o.sumAbsM / Rd);
    m2 = m2 + w[(size_t)m] * ((double)o.sumM2 / Rd);
    Rtot += o.R;
  }
  const double E1 = a / s;
  double within = 0.0, between = 0.0;
  for (int32_t m = 0; m < M; ++m) {
    const double d = mu[(size_t)m] - E1;
    within = within + w[(size_t)m] * var[(size_t)m];
    between = between + w[(size_t)m] * (d * d);
  }
  const double varE = within / s + between / s;
  const double Nd = (double)N, beta = obs[0].beta;
  out->M = M;
  out->R = Rtot;
  out->beta = beta;
  out->e = E1 / Nd;
  out->abs_m = (am / s) / Nd;
  out->m2 = (m2 / s) / (Nd * Nd);
  out->varE = varE;
  out->C = ((beta * beta) * varE) / Nd;
  out->lnZ = mx + std::log(s / (double)M);
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

// Family statistics (the diagnostic that accompanies weighted averaging in
// population annealing): c_i members in family i of n0, R = sum c_i,
// nu_i = c_i / R.  The mean square family size R sum nu_i^2 is
// sum c_i^2 / R (the square sum kept exact in 128 bits); the entropic
// family size R exp(sum nu_i ln nu_i) is exp(sum c_i ln c_i / R).  Both
// equal 1 when every family has one member and R when one family holds
// the whole population.  Sums run over ascending family number.
extern "C" int pa_family_summary(const uint32_t* fam, int64_t R, int64_t n0,
                                 pa_family* out) try {
  if (!fam || !out || R < 1 || n0 < 1 || n0 > (1ll << 32)) return PA_EINVAL;
  std::vector<int64_t> cnt((size_t)n0, 0);
  for (int64_t j = 0; j < R; ++j) {
    if ((int64_t)fam[j] >= n0) return PA_EINVAL;
    cnt[fam[j]] += 1;
  }
  unsigned __int128 sq = 0;
  double cl = 0.0;
  int64_t alive = 0, big = 0;
  for (int64_t i = 0; i < n0; ++i) {
    const int64_t v = cnt[(size_t)i];
    if (v == 0) continue;
    ++alive;
    big = v > big ? v : big;
    sq += (unsigned __int128)v * (unsigned __int128)v;
    cl = cl + (double)v * std::log((double)v);
  }
  out->R = R;
  out->n0 = n0;
  out->families = alive;
  out->largest = big;
  out->rho_t = (double)sq / (double)R;
  out->rho_s = std::exp(cl / (double)R);
  return PA_OK;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}
