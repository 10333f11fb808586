// Host-side table code of the library (reweighting tables, Poisson tables,
// observables, overlap, bisection, weighted averages, family statistics)
// driven over seeded synthetic histograms, for a build under AddressSanitizer
// and UndefinedBehaviorSanitizer.  No GPU call is made.  Exit 0 when every
// call returned and every result is finite and in range.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

using namespace pa;

static int fail(const char* what, int k) {
  std::fprintf(stderr, "tables driver: %s (case %d)\n", what, k);
  return 1;
}

int main() {
  std::mt19937_64 rng(2006);
  for (int k = 0; k < 400; ++k) {
    const int L = 4 + 2 * (int)(rng() % 63);   // 4 .. 128
    const int N = L * L;
    const int shift = (k % 3 == 0) ? 1 : 2;    // +-J or ferromagnet levels
    const int nbins = ((4 * N) >> shift) + 1;
    std::vector<uint32_t> h((size_t)nbins, 0u);
    // a few occupied levels around a random centre, or a single level
    const int c = (int)(rng() % (uint64_t)nbins);
    const int width = (k % 7 == 0) ? 1 : 1 + (int)(rng() % 200);
    int64_t R = 0;
    for (int i = c - width / 2; i <= c + width / 2; ++i) {
      if (i < 0 || i >= nbins) continue;
      const uint32_t v = (uint32_t)(rng() % 5000);
      h[(size_t)i] = v;
      R += v;
    }
    if (R == 0) {
      h[(size_t)c] = 1;
      R = 1;
    }
    const int64_t R_t = 1 + (int64_t)(rng() % (1u << 21));
    const double dbeta = (k % 5 == 0) ? 0.0 : std::ldexp((double)(rng() % 1000), -8);
    std::vector<uint32_t> f((size_t)nbins), T((size_t)nbins);
    TableRange tr;
    if (build_tables(h.data(), nbins, shift, N, R, R_t, dbeta, f.data(),
                     T.data(), &tr) != PA_OK)
      return fail("build_tables", k);
    if (!std::isfinite(tr.lnQ)) return fail("lnQ not finite", k);
    if (k % 4 == 0) {
      std::vector<uint32_t> pt;
      int64_t rmin = 0, rmax = 0;
      TableRange tp;
      const int rc = build_poisson_tables(h.data(), nbins, shift, N, R, R_t,
                                          dbeta, pt, &tp, &rmin, &rmax);
      if (rc != PA_OK && rc != PA_ENOMEM && rc != PA_EINVAL)
        return fail("build_poisson_tables", k);
    }
    pa_obs o{};
    observables_from_hist(h.data(), nbins, shift, N, R, 0.5, 0ull, 0ull, &o);
    const double a = overlap_from_hist(h.data(), nbins, shift, N, R, dbeta);
    if (!(a >= 0.0 && a <= 1.0 + 1e-12)) return fail("overlap range", k);
    int ev = 0;
    const double d = bisect_from_hist(h.data(), nbins, shift, N, R, 0.85,
                                      0.5, &ev, (k & 1) ? 0.02 : 0.0);
    if (!(d >= 0.0 && d <= 0.5)) return fail("bisection range", k);
  }
  // weighted averages and family statistics
  for (int M = 1; M <= 40; ++M) {
    std::vector<double> lnZ((size_t)M), vals((size_t)M * 3), out(3);
    std::vector<pa_obs> obs((size_t)M);
    for (int m = 0; m < M; ++m) {
      lnZ[(size_t)m] = 1000.0 + (double)(rng() % 100) * 0.01;
      for (int j = 0; j < 3; ++j) vals[(size_t)m * 3 + j] = (double)(rng() % 1000);
      pa_obs& q = obs[(size_t)m];
      q.R = 1 + (int64_t)(rng() % 10000);
      q.beta = 0.4;
      q.sumE = -(int64_t)(rng() % 4096) * q.R;
      q.sumE2 = q.sumE / q.R * q.sumE + q.R * 16;
      q.sumAbsM = (int64_t)(rng() % 4096) * q.R;
      q.sumM2 = q.sumAbsM / q.R * q.sumAbsM;
    }
    double lz = 0.0;
    if (pa_weighted_average(M, lnZ.data(), vals.data(), 3, out.data(), &lz))
      return fail("pa_weighted_average", M);
    pa_combined cmb{};
    if (pa_weighted_observables(M, lnZ.data(), obs.data(), 4096, &cmb))
      return fail("pa_weighted_observables", M);
    const int64_t Rf = 1 + (int64_t)(rng() % 5000), n0 = 1 + (int64_t)(rng() % 300);
    std::vector<uint32_t> fam((size_t)Rf);
    for (auto& v : fam) v = (uint32_t)(rng() % (uint64_t)n0);
    pa_family fs{};
    if (pa_family_summary(fam.data(), Rf, n0, &fs)) return fail("pa_family_summary", M);
  }
  std::printf("tables driver ok\n");
  return 0;
}
