// C ABI of libpa.so: host orchestration of the population-annealing hot path
// on one gfx950 device.  All per-replica work runs in the kernels of
// pa_kernels.hip; the host only turns the exact integer energy histogram
// into double-precision per-level tables (Eqs. part-Q, tau, Free-En) and
// keeps beta, the step index and ln Z.
//
// The double-precision host arithmetic is written as plain IEEE operations
// in a fixed order (per energy level, ascending energy) and compiled with
// -ffp-contract=off, so every table entry is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <chrono>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

using namespace pa;

namespace {

struct TimedLaunch {
  int cls;
  hipEvent_t ev0, ev1;
  int64_t bytes, attempts;
  // parts proportional to a population size that was not yet known on the
  // host at launch time; multiplied by it when the launch is harvested
  int64_t bytes_rep, attempts_rep;
  // launches of a schedule run on the device: the index of the population
  // size (in that run's records) the per-replica parts count with; -1 else
  int rseq;
};

// Weight tables of a schedule run on the device: slots of pinned host
// memory, each holding the table of one dbeta (a linear schedule has only a
// few distinct differences); a slot is refilled, least recently used first,
// once the last histogram that read it has reported its sequence number.
constexpr int kWSlots = 16;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace

struct pa_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int L = 0, N = 0, model = 0, layout = 0, W = 0, rpl = 1, lpr = 0, rpw = 0;
  bool rpl_default = false;  // rows per lane left to the library
  int q = 0;  // Potts states (PA_POTTS), else 0
  int rng_mode = PA_RNG_WORD;  // sweep random numbers
  int hist_lo = -1;  // lowest occupied bin of the last histogram (-1: none)
  int64_t R_t = 0, cap = 0, R = 0, stride = 0, ntiles_cap = 0;
  uint64_t seed = 0;
  uint32_t pop = 0;
  double beta = 0.0, lnZ = 0.0, lnQ_last = 0.0;
  int step = 0, sweeps_at_step = 0, cur = 0;
  uint8_t* spins[2] = {nullptr, nullptr};
  int32_t* E[2] = {nullptr, nullptr};
  int32_t* M[2] = {nullptr, nullptr};
  uint32_t* n = nullptr;
  uint32_t* parent = nullptr;
  uint32_t* tile_sum = nullptr;
  uint32_t* tile_off = nullptr;
  uint64_t* tile64 = nullptr;           // systematic law: tile sums of the
  uint64_t* off64 = nullptr;            // fixed-point means and their scan
  uint64_t* cum = nullptr;              // multinomial, residual: interval ends
  // family of every replica (the slot of its ancestor in the population the
  // families start from), double buffered: fam[famcur] is current; a
  // resampling writes the other buffer from the parent map
  uint32_t* fam[2] = {nullptr, nullptr};
  int famcur = 0;
  int64_t fam_n0 = 0;                   // size of the founding population
  // Read-back block, one device->host copy per histogram: the histogram
  // (nbins words, padded to an even count nb2), then scal = [0] sum|M|,
  // [1] sum M^2, [2] unused, [3] energies outside the histogram, all
  // cleared before every histogram, and [4] the size of the last resampled
  // population.
  uint32_t* rb = nullptr;
  uint32_t* hist = nullptr;             // rb
  unsigned long long* scal = nullptr;   // rb + nb2
  uint32_t* tab = nullptr;              // f[nl] then T[nl] of the last step,
                                        // or the Poisson level tables
  size_t tab_words = 0;                 // capacity of tab and h_tab
  int law = PA_NEAREST;
  uint32_t* jbits = nullptr;
  std::vector<int8_t> J;                // host copy of the +-J couplings
  uint32_t* h_rb = nullptr;             // pinned host mirror of rb
  // the histogram kernel writes the read-back block straight into h_rb
  // (through d_hrb, its device address) and raises a flag there, word
  // nb2 + 12, to the sequence number hist_seq; a device counter at word
  // nb2 + 12 of rb finds its last workgroup
  uint32_t* d_hrb = nullptr;
  uint32_t hist_seq = 0;
  uint32_t* h_hist = nullptr;
  unsigned long long* h_scal = nullptr;
  uint32_t* h_tab = nullptr;            // pinned, tab_words words
  int nbins = 0, nb2 = 0, hshift = 0;
  bool hist_valid = false;
  bool rb_zero = false;  // the cleared part of rb is known to be zero
  // pa_resample left the copies to the next sweep: parent[] holds the
  // parent of each of the R new slots, the buffer `cur` still the old
  // population
  bool gather_pending = false;
  // pa_resample did not wait for the new population size: R holds an exact
  // upper bound (grid sizes), the size itself is in scal[4] on the device
  // and reaches the host at the next synchronisation
  bool R_pending = false;
  int64_t n_len = 0;
  uint32_t timing = 0;  // bit k set: launches of class k are timed
  int32_t timing_every = 1;      // time one launch in this many per class
  int64_t timing_count[6] = {};  // launches of each class since the start
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> pool;
  pa_timing acc{};
  int rseq_tag = -1;  // rseq of the launches timed now
  // schedule on the device (pa_anneal): a halt block and one record per
  // step (AnnealRec) on the device, their pinned mirror, the histogram
  // tail's scratch, and the weight-table ring (pinned, read by the kernels
  // through d_w), followed by the word the kernels write the sequence
  // number of the last weights they read to (h_prog; d_prog on the device)
  unsigned char* arec = nullptr;
  unsigned char* h_arec = nullptr;
  int64_t arec_steps = 0;
  double* wscr = nullptr;
  BlockSums* hpart = nullptr;  // the histogram workgroups' parts (256)
  double* h_w = nullptr;
  double* d_w = nullptr;
  uint32_t* h_prog = nullptr;
  uint32_t* d_prog = nullptr;
  uint32_t wseq = 0;  // histograms with weights queued so far
  uint64_t wkey[kWSlots] = {};   // the dbeta of each slot, as bits
  uint32_t wlast[kWSlots] = {};  // the last histogram that reads it
  bool wvalid[kWSlots] = {};
  uint32_t lb_gen = 0;  // launches of the single-pass counts and scatter
};

#define CK(x) PA_HIP(x)

namespace {

// ------------------------------------------------------------------ timing

hipEvent_t take_event(pa_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t t_begin(pa_ctx* c, int cls) {
  if (!(c->timing >> cls & 1u)) return nullptr;
  if (c->timing_count[cls]++ % c->timing_every != 0) return nullptr;
  hipEvent_t e = take_event(c);
  if (e) (void)hipEventRecord(e, c->stream);
  return e;
}

// bytes and attempts of the launch: fixed parts plus parts per replica of
// the current population
void t_end(pa_ctx* c, int cls, hipEvent_t e0, int64_t bytes,
           int64_t attempts, int64_t bytes_rep = 0, int64_t attempts_rep = 0) {
  if (!e0) return;
  hipEvent_t e1 = take_event(c);
  if (!e1) return;
  (void)hipEventRecord(e1, c->stream);
  if (!c->R_pending) {
    bytes += bytes_rep * c->R;
    attempts += attempts_rep * c->R;
    bytes_rep = attempts_rep = 0;
  }
  c->pending.push_back(
      {cls, e0, e1, bytes, attempts, bytes_rep, attempts_rep, c->rseq_tag});
}

// After a stream synchronisation: fold finished launches into the totals.
// Without one (only_done), launches whose end event has not completed stay
// pending.
void t_harvest(pa_ctx* c, bool only_done = false) {
  std::vector<TimedLaunch> keep;
  for (auto& t : c->pending) {
    if (only_done && hipEventQuery(t.ev1) != hipSuccess) {
      keep.push_back(t);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev0, t.ev1) == hipSuccess) {
      c->acc.ms[t.cls] += ms;
      c->acc.launches[t.cls] += 1;
      c->acc.bytes[t.cls] += t.bytes + t.bytes_rep * c->R;
      c->acc.attempts += t.attempts + t.attempts_rep * c->R;
    }
    c->pool.push_back(t.ev0);
    c->pool.push_back(t.ev1);
  }
  (void)hipGetLastError();  // a query of an unfinished event is no error
  c->pending.swap(keep);
}

// size_copied: the caller already queued the copy of scal[4] to the host.
// Waits for the stream by polling it for up to 50 ms, then blocks: a
// blocking wait wakes up tens of microseconds late, which a resampling step
// (a histogram read-back, host tables, the counts) pays at every step.
hipError_t wait_stream(hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50))
      return hipStreamSynchronize(st);
  }
}

// Watches the read-back flag of the last histogram (see compute_hist):
// true once it shows this call's sequence number.  False if the stream
// ends, or fails, without it (the caller then copies and synchronises,
// which also reports a failure).
bool wait_flag(pa_ctx* c) {
  const uint32_t* flag = c->h_rb + c->nb2 + 12;
  for (int64_t k = 0;; ++k) {
    if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == c->hist_seq) return true;
    if ((k & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess)
        return __atomic_load_n(flag, __ATOMIC_ACQUIRE) == c->hist_seq;
      if (e != hipErrorNotReady) return false;
    }
  }
}

// Waits until the kernels have read weight table number `seq` of a
// schedule run on the device (its histogram writes the number to h_prog).
// False if the stream ends, or fails, first.
bool wait_progress(pa_ctx* c, uint32_t seq) {
  for (int64_t k = 0;; ++k) {
    if ((int32_t)(__atomic_load_n(c->h_prog, __ATOMIC_ACQUIRE) - seq) >= 0)
      return true;
    if ((k & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipSuccess)
        return (int32_t)(__atomic_load_n(c->h_prog, __ATOMIC_ACQUIRE) -
                         seq) >= 0;
      if (e != hipErrorNotReady) return false;
    }
  }
}

int sync(pa_ctx* c, bool size_copied = false) {
  if (c->R_pending && !size_copied)
    CK(hipMemcpyAsync(c->h_scal + 4, c->scal + 4, sizeof(unsigned long long),
                      hipMemcpyDeviceToHost, c->stream));
  CK(wait_stream(c->stream));
  if (c->R_pending) {
    c->R = (int64_t)c->h_scal[4];
    c->R_pending = false;
  }
  t_harvest(c);
  return PA_OK;
}

// --------------------------------------------------------- double tables

LatticeArgs lattice_args(pa_ctx* c) {
  LatticeArgs a{};
  a.spins = c->spins[c->cur];
  a.E = c->E[c->cur];
  a.M = c->M[c->cur];
  a.jbits = c->jbits;
  a.R = c->R;
  a.Rdev = c->R_pending ? c->scal + 4 : nullptr;
  a.stride = c->stride;
  a.L = c->L;
  a.lpr = c->lpr;
  a.rpw = c->rpw;
  a.k0 = (uint32_t)(c->seed & 0xFFFFFFFFu);
  a.k1 = (uint32_t)(c->seed >> 32);
  a.pop = c->pop;
  a.step = (uint32_t)c->step;
  a.t0 = c->sweeps_at_step;
  a.one = 1u;
  a.q = c->q;
  if (c->model == PA_POTTS) potts_thresholds(c->beta, a.Tp);
  return a;
}

int run_lattice(pa_ctx* c, LatticeArgs& a, int cls) {
  // one sweep of int8 L = 64 replicas moves as many bytes as it computes
  // attempts: where the library chose two rows per lane, such a launch
  // takes one (one replica per wave, twice the waves in flight; 1.5 %
  // faster at 20480 replicas).  The replica layout and every result are
  // the same in both shapes.
  int rpl = c->rpl;
  if (c->rpl_default && rpl == 2 && c->layout == PA_INT8 && c->L == 64 &&
      a.theta == 1 && c->model != PA_POTTS) {
    rpl = 1;
    a.lpr = 64;
    a.rpw = 1;
  }
  hipEvent_t e0 = t_begin(c, cls);
  if (c->model == PA_POTTS)
    CK(launch_potts(a, c->stream));
  else
    CK(launch_lattice(a, c->W, rpl, c->layout == PA_INT8,
                      c->model == PA_PMJ, c->rng_mode == PA_RNG_PLANES,
                      c->stream));
  t_end(c, cls, e0, 0, 0, (a.init ? 1 : 2) * c->stride + 8,
        (int64_t)c->N * a.theta);
  return PA_OK;
}

// The resampling copies of the last pa_resample when no sweep took them
// over: every new slot receives its parent's lattice, E and M.
int finish_gather(pa_ctx* c) {
  if (!c->gather_pending) return PA_OK;
  if (c->R_pending) {
    const int rs = sync(c);
    if (rs) return rs;
  }
  GatherArgs g{};
  g.src = c->spins[c->cur];
  g.dst = c->spins[c->cur ^ 1];
  g.E_src = c->E[c->cur];
  g.M_src = c->M[c->cur];
  g.E_dst = c->E[c->cur ^ 1];
  g.M_dst = c->M[c->cur ^ 1];
  g.parent = c->parent;
  g.R_new = c->R;
  g.stride = c->stride;
  g.chunks = (int32_t)(c->stride / 16);
  g.chunks_log2 = -1;
  for (int lg = 0; lg < 31; ++lg)
    if ((1 << lg) == g.chunks) g.chunks_log2 = lg;
  hipEvent_t e0 = t_begin(c, PA_K_GATHER);
  CK(launch_gather(g, c->stream));
  t_end(c, PA_K_GATHER, e0, 2 * c->R * c->stride + 20 * c->R, 0);
  c->cur ^= 1;
  c->gather_pending = false;
  return PA_OK;
}

// Exact energy histogram and |M|, M^2 sums of the current population,
// mirrored into pinned host memory.
int compute_hist(pa_ctx* c) {
  if (c->hist_valid) return PA_OK;
  const int rg = finish_gather(c);
  if (rg) return rg;
  // the histogram and moments start from zero (k_counts of the last
  // resampling cleared them unless something else ran since)
  if (!c->rb_zero)
    CK(launch_fill_u32(c->rb, c->nb2 + 8, 0u, c->stream));
  HistArgs h{};
  h.E = c->E[c->cur];
  h.M = c->M[c->cur];
  h.hist = c->hist;
  h.moments = c->scal;
  h.R = c->R;
  h.Rdev = c->R_pending ? c->scal + 4 : nullptr;
  h.twoN = 2 * c->N;
  h.shift = c->hshift;
  h.nbins = c->nbins;
  // the LDS window: every bin when they fit in 64 KB, else 16384 bins from
  // a little below the lowest occupied bin of the last histogram (the
  // middle of the range before the first); bins outside it are counted in
  // the global histogram directly, so the result never depends on it
  h.win_n = std::min(c->nbins, 16384);
  if (h.win_n == c->nbins)
    h.win_lo = 0;
  else if (c->hist_lo >= 0)
    h.win_lo = std::max(0, std::min(c->hist_lo - 1024, c->nbins - h.win_n));
  else
    h.win_lo = (c->nbins - h.win_n) / 2;
  // the kernel's last workgroup sends histogram, moments and population
  // size to the host itself and raises a flag, which the host watches:
  // no copy of its own and no stream synchronisation per step
  const bool mapped = c->d_hrb != nullptr;
  if (mapped) {
    c->hist_seq += 1;
    h.rb = c->rb;
    h.host_rb = c->d_hrb;
    h.host_flag = c->d_hrb + c->nb2 + 12;
    h.counter = c->rb + c->nb2 + 12;
    h.seq = c->hist_seq;
    // hist and the five scalars, rounded up to 16-byte units (nb2 is even,
    // so this stays below the flag word nb2 + 12)
    h.rb_words = (c->nb2 + 10 + 3) & ~3;
  }
  hipEvent_t e0 = t_begin(c, PA_K_HIST);
  CK(launch_hist(h, c->stream));
  t_end(c, PA_K_HIST, e0, 0, 0, 8, 0);
  c->rb_zero = false;
  int rc = PA_OK;
  if (mapped && wait_flag(c)) {
    if (c->R_pending) {
      c->R = (int64_t)c->h_scal[4];
      c->R_pending = false;
      // the launches timed since the size was last known act on this
      // population: their per-replica parts count with its size now, as
      // their events may finish later
      for (auto& t : c->pending) {
        t.bytes += t.bytes_rep * c->R;
        t.attempts += t.attempts_rep * c->R;
        t.bytes_rep = t.attempts_rep = 0;
      }
    }
    t_harvest(c, true);
  } else {
    // histogram, moments and population size in one copy
    CK(hipMemcpyAsync(c->h_rb, c->rb, ((size_t)c->nb2 + 10) * 4,
                      hipMemcpyDeviceToHost, c->stream));
    rc = sync(c, true);
  }
  if (rc) return rc;
  if (fault_injected("energy")) c->h_scal[3] = 1;
  if (c->h_scal[3] != 0) {  // an energy outside [-2N, 2N]
    note_error("a replica's energy lies outside the histogram range");
    return PA_EDEVICE;
  }
  {
    int lo = -1, hi = -1;
    occupied_range(c->h_hist, c->nbins, &lo, &hi);
    c->hist_lo = lo;
  }
  c->hist_valid = true;
  return PA_OK;
}

// Room for `words` table words on the device and in the pinned mirror (the
// Poisson tables grow with the means; allocation happens between steps).
int ensure_tab(pa_ctx* c, size_t words) {
  if (words <= c->tab_words) return PA_OK;
  const size_t nw = words + words / 2;
  uint32_t* d = nullptr;
  uint32_t* h = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), nw * 4) != hipSuccess) {
    (void)hipGetLastError();  // not left for a later launch check
    return PA_ENOMEM;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&h), nw * 4) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d);
    return PA_ENOMEM;
  }
  int rc = sync(c);  // the old tables may still be read
  if (rc) {
    (void)hipFree(d);
    (void)hipHostFree(h);
    return rc;
  }
  (void)hipFree(c->tab);
  (void)hipHostFree(c->h_tab);
  c->tab = d;
  c->h_tab = h;
  c->tab_words = nw;
  return PA_OK;
}

void free_all(pa_ctx* c) {
  for (int b = 0; b < 2; ++b) {
    if (c->spins[b]) (void)hipFree(c->spins[b]);
    if (c->E[b]) (void)hipFree(c->E[b]);
    if (c->M[b]) (void)hipFree(c->M[b]);
    if (c->fam[b]) (void)hipFree(c->fam[b]);
  }
  void* dev[] = {c->n,  c->parent, c->tile_sum, c->tile_off, c->tile64,
                 c->off64, c->cum, c->rb, c->tab, c->jbits, c->arec, c->wscr,
                 c->hpart};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (c->h_rb) (void)hipHostFree(c->h_rb);
  if (c->h_tab) (void)hipHostFree(c->h_tab);
  if (c->h_arec) (void)hipHostFree(c->h_arec);
  if (c->h_w) (void)hipHostFree(c->h_w);
  for (auto& t : c->pending) {
    (void)hipEventDestroy(t.ev0);
    (void)hipEventDestroy(t.ev1);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
}

// Every replica of the current population founds its own family.
int reset_families(pa_ctx* c) {
  CK(launch_iota_u32(c->fam[0], c->R, c->stream));
  c->famcur = 0;
  c->fam_n0 = c->R;
  return PA_OK;
}

template <typename T>
bool dmalloc(T** p, size_t bytes) {
  if (hipMalloc(reinterpret_cast<void**>(p), bytes ? bytes : 16) == hipSuccess)
    return true;
  // the runtime keeps the failure as its last error, which the launch
  // checks of a later, healthy context would read: clear it
  (void)hipGetLastError();
  return false;
}

// canonical int8 [L][L] -> device layout of one replica (stride bytes)
// Buffers of a schedule of K steps run on the device (pa_anneal); called
// with the stream idle, so old buffers may be freed.
int ensure_anneal(pa_ctx* c, int64_t K) {
  const size_t nb = (size_t)c->nbins;
  if (!c->wscr && !dmalloc(&c->wscr, 2 * nb * sizeof(double)))
    return PA_ENOMEM;
  if (!c->hpart && !dmalloc(&c->hpart, 256 * sizeof(BlockSums)))
    return PA_ENOMEM;
  if (!c->h_w) {
    void* h = nullptr;
    if (hipHostMalloc(&h, kWSlots * nb * sizeof(double) + 64,
                      hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      return PA_ENOMEM;
    }
    c->h_w = static_cast<double*>(h);
    void* d = nullptr;
    CK(hipHostGetDevicePointer(&d, h, 0));
    c->d_w = static_cast<double*>(d);
    c->h_prog = reinterpret_cast<uint32_t*>(c->h_w + kWSlots * nb);
    c->d_prog = reinterpret_cast<uint32_t*>(c->d_w + kWSlots * nb);
    *c->h_prog = 0u;
    c->wseq = 0u;
  }
  if (K + 1 > c->arec_steps) {
    const int64_t n = std::max<int64_t>(K + 1, 2 * c->arec_steps);
    const size_t bytes = 64 + (size_t)n * sizeof(AnnealRec);
    unsigned char* d = nullptr;
    void* h = nullptr;
    if (!dmalloc(&d, bytes)) return PA_ENOMEM;
    if (hipHostMalloc(&h, bytes) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(d);
      return PA_ENOMEM;
    }
    if (c->arec) (void)hipFree(c->arec);
    if (c->h_arec) (void)hipHostFree(c->h_arec);
    c->arec = d;
    c->h_arec = static_cast<unsigned char*>(h);
    c->arec_steps = n;
  }
  return PA_OK;
}

void pack_replica(const pa_ctx* c, const int8_t* s, uint8_t* out) {
  std::memset(out, 0, (size_t)c->stride);
  if (c->layout == PA_INT8) {
    std::memcpy(out, s, (size_t)c->N);
    return;
  }
  uint32_t* w = reinterpret_cast<uint32_t*>(out);
  for (int y = 0; y < c->L; ++y)
    for (int x = 0; x < c->L; ++x)
      if (s[y * c->L + x] == 1) w[y * c->W + x / 32] |= 1u << (x % 32);
}

void unpack_replica(const pa_ctx* c, const uint8_t* in, int8_t* s) {
  if (c->layout == PA_INT8) {
    std::memcpy(s, in, (size_t)c->N);
    return;
  }
  const uint32_t* w = reinterpret_cast<const uint32_t*>(in);
  for (int y = 0; y < c->L; ++y)
    for (int x = 0; x < c->L; ++x)
      s[y * c->L + x] = ((w[y * c->W + x / 32] >> (x % 32)) & 1u) ? 1 : -1;
}

}  // namespace

// =================================================================== ABI

extern "C" {

const char* pa_strerror(int code) {
  switch (code) {
    case PA_OK: return "ok";
    case PA_EINVAL: return "invalid argument";
    case PA_ENOMEM: return "out of memory";
    case PA_ECAPACITY: return "population would exceed the capacity";
    case PA_EDEVICE: return "HIP runtime error";
    case PA_ESTATE: return "call out of order";
    case PA_EEMPTY: return "resampling drew no replica";
    case PA_EIO: return "population file could not be written or read";
    default: return "unknown error";
  }
}

int pa_init(const pa_config* cfg, pa_ctx** out) try {
  if (!out) return PA_EINVAL;
  *out = nullptr;
  if (!cfg) return PA_EINVAL;
  const int L = cfg->L;
  if (L < 4 || L > 128 || (L & 1)) return PA_EINVAL;
  if (cfg->model != PA_FERRO && cfg->model != PA_PMJ &&
      cfg->model != PA_POTTS)
    return PA_EINVAL;
  if (cfg->model == PA_PMJ && !cfg->J) return PA_EINVAL;
  if (cfg->layout != PA_INT8 && cfg->layout != PA_BITS) return PA_EINVAL;
  if (cfg->model == PA_POTTS &&
      (cfg->q < 2 || cfg->q > 16 || cfg->layout != PA_INT8))
    return PA_EINVAL;
  if (cfg->resampling < PA_NEAREST || cfg->resampling > PA_MULTINOMIAL)
    return PA_EINVAL;
  if (cfg->rng_mode != PA_RNG_WORD &&
      (cfg->rng_mode != PA_RNG_PLANES || cfg->model == PA_POTTS))
    return PA_EINVAL;
  if (cfg->R_target < 1 || cfg->R_target >= (1ll << 31)) return PA_EINVAL;
  int64_t cap = cfg->capacity;
  if (cap == 0)
    cap = cfg->R_target +
          16 * (int64_t)std::ceil(std::sqrt((double)cfg->R_target)) + 1024;
  if (cap < cfg->R_target || cap >= (1ll << 32)) return PA_EINVAL;
  const int W = (L + 31) / 32;
  int rpl = cfg->rows_per_lane;
  if (rpl == 0)
    rpl = default_rows_per_lane(L, cfg->rng_mode == PA_RNG_PLANES,
                                cfg->R_target);
  if (rpl < 1 || rpl > 4) return PA_EINVAL;
  if (L % rpl != 0 || L / rpl > 64) return PA_EINVAL;
  if (W >= 3 && rpl < 2) return PA_EINVAL;
  if (cfg->model == PA_PMJ) {
    for (int64_t i = 0; i < 2ll * L * L; ++i)
      if (cfg->J[i] != 1 && cfg->J[i] != -1) return PA_EINVAL;
  }

  pa_ctx* c = new (std::nothrow) pa_ctx();
  if (!c) return PA_ENOMEM;
  {
    const hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      set_last_error("hipGetDevice", e, __LINE__);
      delete c;
      return PA_EDEVICE;
    }
  }
  c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  c->L = L;
  c->N = L * L;
  c->model = cfg->model;
  c->layout = cfg->layout;
  c->W = W;
  c->rpl = rpl;
  c->rpl_default = cfg->rows_per_lane == 0;
  c->lpr = L / rpl;
  c->rpw = 64 / c->lpr;
  c->R_t = cfg->R_target;
  c->cap = cap;
  c->seed = cfg->seed;
  c->law = cfg->resampling;
  c->rng_mode = cfg->rng_mode;
  c->pop = cfg->population_id;
  c->stride = (c->layout == PA_INT8) ? round_up(c->N, 16)
                                     : round_up((int64_t)L * W * 4, 16);
  c->q = (c->model == PA_POTTS) ? cfg->q : 0;
  // energy levels: Ising E in [-2N, 2N] (steps of 4 for the ferromagnet,
  // of 2 with +-J couplings); Potts E in [-2N, 0] in steps of 1
  c->hshift = (c->model == PA_FERRO) ? 2 : (c->model == PA_PMJ) ? 1 : 0;
  c->nbins = (c->model == PA_POTTS) ? 2 * c->N + 1
                                    : (4 * c->N >> c->hshift) + 1;
  c->ntiles_cap = (cap + 255) / 256;

  bool ok = true;
  for (int b = 0; b < 2 && ok; ++b) {
    ok = ok && dmalloc(&c->spins[b], (size_t)(cap * c->stride));
    ok = ok && !fault_injected("alloc");  // a failure after the first one
    ok = ok && dmalloc(&c->E[b], (size_t)cap * 4);
    ok = ok && dmalloc(&c->M[b], (size_t)cap * 4);
  }
  ok = ok && dmalloc(&c->n, (size_t)cap * 4);
  ok = ok && dmalloc(&c->parent, (size_t)cap * 4);
  ok = ok && dmalloc(&c->fam[0], (size_t)cap * 4);
  ok = ok && dmalloc(&c->fam[1], (size_t)cap * 4);
  ok = ok && dmalloc(&c->tile_sum, (size_t)c->ntiles_cap * 4);
  ok = ok && dmalloc(&c->tile_off, (size_t)c->ntiles_cap * 4);
  ok = ok && dmalloc(&c->tile64, (size_t)c->ntiles_cap * 8);
  ok = ok && dmalloc(&c->off64, (size_t)c->ntiles_cap * 8);
  if (cfg->resampling == PA_MULTINOMIAL || cfg->resampling == PA_RESIDUAL)
    ok = ok && dmalloc(&c->cum, (size_t)cap * 8);
  c->nb2 = (c->nbins + 1) & ~1;
  ok = ok && dmalloc(&c->rb, ((size_t)c->nb2 + 16) * 4);
  c->tab_words = (size_t)c->nbins * 2;
  ok = ok && dmalloc(&c->tab, c->tab_words * 4);
  ok = ok && dmalloc(&c->jbits, (size_t)2 * L * W * 4);
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&c->h_rb),
                           ((size_t)c->nb2 + 16) * 4) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&c->h_tab),
                           c->tab_words * 4) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();  // a failed allocation is no later launch's error
    free_all(c);
    delete c;
    return PA_ENOMEM;
  }
  c->hist = c->rb;
  c->scal = reinterpret_cast<unsigned long long*>(c->rb + c->nb2);
  c->h_hist = c->h_rb;
  c->h_scal = reinterpret_cast<unsigned long long*>(c->h_rb + c->nb2);
  c->h_rb[c->nb2 + 12] = 0u;
  {
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, c->h_rb, 0) == hipSuccess && d)
      c->d_hrb = static_cast<uint32_t*>(d);
    else
      (void)hipGetLastError();  // the copy path serves instead
  }
  if (c->model == PA_PMJ) c->J.assign(cfg->J, cfg->J + 2ll * L * L);
  // +-J couplings as row bit masks, bit set where J < 0
  std::vector<uint32_t> jb((size_t)2 * L * W, 0u);
  if (c->model == PA_PMJ)
    for (int d = 0; d < 2; ++d)
      for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x)
          if (cfg->J[(size_t)d * L * L + (size_t)y * L + x] < 0)
            jb[((size_t)d * L + y) * W + x / 32] |= 1u << (x % 32);
  int rc = PA_OK;
  {
    const hipError_t e = launch_fill_u32(c->rb + c->nb2 + 12, 4, 0u,
                                         c->stream);
    if (e != hipSuccess) {
      set_last_error("launch_fill_u32", e, __LINE__);
      rc = PA_EDEVICE;
    }
  }
  if (rc == PA_OK) {
    const hipError_t e = hipMemcpyAsync(c->jbits, jb.data(), jb.size() * 4,
                                        hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      set_last_error("hipMemcpyAsync(couplings)", e, __LINE__);
      rc = PA_EDEVICE;
    }
  }
  if (rc == PA_OK) {
    c->R = c->R_t;
    LatticeArgs a = lattice_args(c);
    a.init = 1;
    a.theta = 0;
    rc = run_lattice(c, a, PA_K_INIT);
  }
  if (rc == PA_OK) rc = reset_families(c);
  if (rc == PA_OK) rc = sync(c);
  if (rc != PA_OK) {
    free_all(c);
    delete c;
    return rc;
  }
  c->beta = 0.0;
  // ln Omega: 2^N Ising states, q^N Potts states, all of weight 1 at beta 0
  c->lnZ = (double)c->N * std::log(c->q ? (double)c->q : 2.0);
  c->lnQ_last = 0.0;
  *out = c;
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

void pa_destroy(pa_ctx* c) try {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
} catch (...) {
}

int pa_sweep(pa_ctx* c, double beta, int32_t theta) try {
  if (!c || theta < 0 || !std::isfinite(beta)) return PA_EINVAL;
  if (beta != c->beta) return PA_ESTATE;
  if (c->sweeps_at_step + theta > 32767) return PA_EINVAL;
  if (theta == 0) return PA_OK;
  LatticeArgs a = lattice_args(c);
  metropolis_K(c->beta, &a.K4, &a.K8);
  a.theta = theta;
  const bool fused = c->gather_pending;
  if (fused) {
    // the resampling copies happen on the way in: each new slot loads its
    // parent's lattice from the old buffer and the pass writes the new one
    a.src = c->spins[c->cur];
    a.parent = c->parent;
    a.spins = c->spins[c->cur ^ 1];
    a.E = c->E[c->cur ^ 1];
    a.M = c->M[c->cur ^ 1];
  }
  int rc = run_lattice(c, a, PA_K_SWEEP);
  if (rc) return rc;
  if (fused) {
    c->cur ^= 1;
    c->gather_pending = false;
  }
  c->sweeps_at_step += theta;
  c->hist_valid = false;
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

int pa_resample(pa_ctx* c, double beta_next, int64_t* R_new) try {
  // cooling (beta_next >= beta) or heating (beta_next < beta), beta >= 0
  if (!c || !std::isfinite(beta_next) || !(beta_next >= 0.0))
    return PA_EINVAL;
  if (c->step + 1 > 65535) return PA_EINVAL;
  int rc = compute_hist(c);
  if (rc) return rc;
  const double dbeta = beta_next - c->beta;
  TableRange tr;
  const int nbins = c->nbins;
  int64_t r_min = 0, r_max = 0, draws = 0;
  CountsArgs ca{};
  bool args_tables = false;
  ArgTables at;
  if (c->law == PA_POISSON) {
    std::vector<uint32_t> pt;
    rc = build_poisson_tables(c->h_hist, nbins, c->hshift, c->N, c->R, c->R_t,
                              dbeta, pt, &tr, &r_min, &r_max);
    if (rc) return rc;
    rc = ensure_tab(c, pt.size());
    if (rc) return rc;
    std::memcpy(c->h_tab, pt.data(), pt.size() * 4);
    CK(hipMemcpyAsync(c->tab, c->h_tab, pt.size() * 4, hipMemcpyHostToDevice,
                      c->stream));
    ca.f = c->tab;
    ca.T = nullptr;
    ca.poisson = 1;
  } else {
    rc = build_tables(c->h_hist, nbins, c->hshift, c->N, c->R, c->R_t, dbeta,
                      c->h_tab, c->h_tab + nbins, &tr);
    if (rc) return rc;
    const int nl = tr.hi - tr.lo + 1;
    // only the occupied levels go to the device: f[nl] then T[nl], in the
    // counts kernel's arguments when they fit there (nearest-integer law)
    uint32_t* hf = c->h_tab;
    uint32_t* hT = c->h_tab + nl;
    std::memmove(hT, c->h_tab + nbins, (size_t)nl * 4);
    args_tables = c->law == PA_NEAREST && nl <= kArgLevels;
    if (args_tables) {
      std::memcpy(at.f, hf, (size_t)nl * 4);
      std::memcpy(at.T, hT, (size_t)nl * 4);
    } else {
      CK(hipMemcpyAsync(c->tab, c->h_tab, (size_t)nl * 8,
                        hipMemcpyHostToDevice, c->stream));
    }
    ca.f = c->tab;
    ca.T = c->tab + nl;
    if (c->law == PA_MULTINOMIAL) {
      r_min = r_max = c->R_t;  // exactly R_target draws
      draws = c->R_t;
    } else if (c->law == PA_RESIDUAL) {
      // the floors for certain, then R_target minus their sum drawn over
      // the fractions (none when every fraction is zero): exactly one size
      uint64_t C = 0;
      int64_t floors = 0;
      for (int i = tr.lo; i <= tr.hi; ++i) {
        const uint64_t h = c->h_hist[i];
        C += h * (uint64_t)hT[i - tr.lo];
        floors += (int64_t)h * hf[i - tr.lo];
      }
      draws = c->R_t - floors;
      if (draws < 0 || C == 0) draws = 0;
      r_min = r_max = floors + draws;
      ca.residual = 1;
    } else if (c->law == PA_SYSTEMATIC) {
      // the comb gives floor((C + U) / 2^32) copies in total, C the sum of
      // the fixed-point means: one of two sizes
      uint64_t C = 0;
      for (int i = tr.lo; i <= tr.hi; ++i)
        C += (uint64_t)c->h_hist[i] *
             (((uint64_t)hf[i - tr.lo] << 32) + (uint64_t)hT[i - tr.lo]);
      r_min = (int64_t)(C >> 32);
      r_max = r_min + 1;
    } else {
      // every replica at level l gets f or f + 1 copies, f + 1 only where
      // its threshold is nonzero
      for (int i = tr.lo; i <= tr.hi; ++i) {
        const int64_t h = c->h_hist[i];
        r_min += h * (int64_t)hf[i - tr.lo];
        r_max += h * ((int64_t)hf[i - tr.lo] + (hT[i - tr.lo] ? 1 : 0));
      }
    }
  }
  const int lo = tr.lo, nl = tr.hi - tr.lo + 1;
  const double lnQ = tr.lnQ;
  // (e) copy counts and their exclusive scan; the counts kernel also clears
  // the histogram and moments for the next step (their copy to the host
  // precedes it on the stream)
  ca.E = c->E[c->cur];
  ca.clear = c->rb;
  ca.nclear = c->nb2 + 8;
  ca.n = c->n;
  ca.tile_sum = c->tile_sum;
  ca.R = c->R;
  ca.twoN = 2 * c->N;
  ca.shift = c->hshift;
  ca.lvl0 = lo;
  ca.nlvl = nl;
  ca.k0 = (uint32_t)(c->seed & 0xFFFFFFFFu);
  ca.k1 = (uint32_t)(c->seed >> 32);
  ca.pop = c->pop;
  ca.step_next = (uint32_t)(c->step + 1);
  const int64_t ntiles = (c->R + 255) / 256;
  // the size need not reach the host now when it cannot be out of range and
  // the caller did not ask for it: the next synchronisation brings it
  const bool forced_full = fault_injected("capacity");
  const bool deferred =
      !R_new && r_min >= 1 && r_max <= c->cap && !forced_full;
  // up to 256 tiles of the plain counts kernel, the parent map scans the
  // tile sums itself and writes the new size: it runs now, before the size
  // is checked (the parent map and the second family buffer are scratch
  // until the step commits)
  const bool scatter_scans = (c->law == PA_NEAREST || c->law == PA_POISSON) &&
                             ntiles <= 256;
  hipEvent_t e0 = t_begin(c, PA_K_COUNTS);
  if (c->law == PA_MULTINOMIAL || c->law == PA_RESIDUAL)
    CK(launch_multi_counts(ca, draws, c->tile64, c->off64, c->cum,
                           c->stream));
  else if (c->law == PA_SYSTEMATIC)
    CK(launch_sys_counts(ca, c->tile64, c->off64, c->stream));
  else if (args_tables)
    CK(launch_counts_args(ca, at, c->stream));
  else
    CK(launch_counts(ca, c->stream));
  if (!scatter_scans)
    CK(launch_scan(c->tile_sum, c->tile_off, ntiles, c->scal + 4, c->stream));
  t_end(c, PA_K_COUNTS, e0, 8 * c->R + 8 * ntiles, 0);
  if (scatter_scans) {
    e0 = t_begin(c, PA_K_SCATTER);
    CK(launch_scatter_scan(c->n, c->tile_sum, c->R, c->cap, c->parent,
                           c->fam[c->famcur], c->fam[c->famcur ^ 1],
                           c->scal + 4, c->stream));
    t_end(c, PA_K_SCATTER, e0, 4 * c->R, 0, 4, 0);
  }
  c->rb_zero = true;
  const int64_t R_old = c->R;
  if (!deferred) {
    CK(hipMemcpyAsync(c->h_scal + 4, c->scal + 4, sizeof(unsigned long long),
                      hipMemcpyDeviceToHost, c->stream));
    rc = sync(c);
    if (rc) return rc;
    const int64_t total =
        forced_full ? c->cap + 1 : (int64_t)c->h_scal[4];
    if (R_new) *R_new = total;
    if (total > c->cap) {
      c->n_len = 0;
      return PA_ECAPACITY;
    }
    if (total == 0) {
      c->n_len = 0;
      return PA_EEMPTY;
    }
    c->R = total;
  } else {
    c->R = r_max;
    c->R_pending = true;
  }
  // (f) parent of every new slot; the copies into the other buffer are left
  // to the next sweep, which reads every new slot from its parent
  if (!scatter_scans) {
    e0 = t_begin(c, PA_K_SCATTER);
    CK(launch_scatter(c->n, c->tile_off, R_old, c->cap, c->parent,
                      c->fam[c->famcur], c->fam[c->famcur ^ 1], c->stream));
    t_end(c, PA_K_SCATTER, e0, 4 * R_old, 0, 4, 0);
  }
  c->famcur ^= 1;
  c->n_len = R_old;
  c->gather_pending = true;
  if (std::getenv("PA_LOG_JSONL")) {
    StepLog sl{};
    pa_obs o{};
    observables_from_hist(c->h_hist, c->nbins, c->hshift, c->N, R_old,
                          c->beta, (int64_t)c->h_scal[0],
                          (int64_t)c->h_scal[1], &o);
    sl.pop = c->pop;
    sl.step = c->step + 1;
    sl.R_prev = R_old;
    sl.R = c->R_pending ? -1 : c->R;
    sl.beta = beta_next;
    sl.dbeta = dbeta;
    sl.lnQ = lnQ;
    sl.lnZ = c->lnZ + lnQ;
    sl.overlap = overlap_from_hist(c->h_hist, c->nbins, c->hshift, c->N,
                                   R_old, dbeta);
    sl.e_prev = o.e;
    sl.abs_m_prev = o.abs_m;
    sl.C_prev = o.C;
    sl.source = "caller";
    log_step(sl);
  }
  c->beta = beta_next;
  c->step += 1;
  c->sweeps_at_step = 0;
  c->lnQ_last = lnQ;
  c->lnZ = c->lnZ + lnQ;  // Eq. Free-En, read with the logarithm
  c->hist_valid = false;
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

int pa_anneal(pa_ctx* c, const double* betas, int32_t K, int32_t theta,
              pa_obs* obs, double* lnQ, int32_t* done) try {
  if (done) *done = 0;
  if (!c || K < 0 || (K > 0 && !betas) || theta < 0 || theta > 32767)
    return PA_EINVAL;
  if ((int64_t)c->step + K > 65535) return PA_EINVAL;
  // the device runs the schedule alone for the nearest-integer law when
  // beta never decreases and every step sweeps; else the same calls one by
  // one
  bool on_device = c->law == PA_NEAREST && theta > 0;
  double prev = c->beta;
  for (int k = 0; k < K; ++k) {
    if (!std::isfinite(betas[k]) || !(betas[k] >= 0.0)) return PA_EINVAL;
    if (betas[k] < prev) on_device = false;
    prev = betas[k];
  }
  if (K == 0) return PA_OK;
  if (!on_device) {
    for (int k = 0; k < K; ++k) {
      int rc = pa_resample(c, betas[k], nullptr);
      if (rc == PA_OK && theta > 0) rc = pa_sweep(c, betas[k], theta);
      pa_obs o{};
      if (rc == PA_OK && obs) rc = pa_observables(c, &o);
      if (rc) return rc;
      if (obs) obs[k] = o;
      if (lnQ) lnQ[k] = c->lnQ_last;
      if (done) *done = k + 1;
    }
    return PA_OK;
  }
  int rc = PA_OK;
  if (c->R_pending) {
    rc = sync(c);
    if (rc) return rc;
  }
  rc = finish_gather(c);
  if (rc) return rc;
  rc = ensure_anneal(c, K);
  if (rc) return rc;
  AnnealHalt* d_halt = reinterpret_cast<AnnealHalt*>(c->arec);
  AnnealRec* d_rec = reinterpret_cast<AnnealRec*>(c->arec + 64);
  CK(launch_fill_u32(reinterpret_cast<uint32_t*>(c->arec), 16, 0u,
                     c->stream));
  // the single-pass scan's status words: no generation in them may match a
  // launch of this call (the memory may hold anything from earlier use)
  CK(launch_fill_u32(reinterpret_cast<uint32_t*>(c->tile64),
                     2 * c->ntiles_cap, 0u, c->stream));
  if (!c->rb_zero) CK(launch_fill_u32(c->rb, c->nb2 + 8, 0u, c->stream));
  const int cur0 = c->cur, fam0 = c->famcur, step0 = c->step;
  const int sw0 = c->sweeps_at_step;
  const double beta0 = c->beta, lnZ0 = c->lnZ, lnQ0 = c->lnQ_last;
  const int64_t R0 = c->R, cap = c->cap, nb = c->nbins;
  // the single-pass counts and parent map: its two counters after the halt
  // record and the range sums
  uint32_t* lb_ctr = reinterpret_cast<uint32_t*>(c->arec + 32);
  HistArgs h{};
  h.hist = c->hist;
  h.moments = c->scal;
  h.twoN = 2 * c->N;
  h.shift = c->hshift;
  h.nbins = c->nbins;
  h.win_n = std::min(c->nbins, 16384);
  if (h.win_n == c->nbins)
    h.win_lo = 0;
  else if (c->hist_lo >= 0)
    h.win_lo = std::max(0, std::min(c->hist_lo - 1024, c->nbins - h.win_n));
  else
    h.win_lo = (c->nbins - h.win_n) / 2;
  h.counter = c->rb + c->nb2 + 12;
  h.halt = d_halt;
  h.part = c->hpart;
  h.Rw = c->scal + 4;
  h.wscr = c->wscr;
  h.R_t = c->R_t;
  ArgWeights wk{};
  // timed launches are tagged with their record while the loop runs, on
  // every way out of it too
  struct TagReset {
    pa_ctx* c;
    ~TagReset() { c->rseq_tag = -1; }
  } tag_reset{c};
  // the sizes stay on the device until the end: grids cover the capacity
  c->R = cap;
  c->R_pending = true;
  for (int k = 0; k <= K; ++k) {
    // (a) histogram of the population at the current beta; for k < K the
    // tables of the step to betas[k] from it (Eqs. part-Q, tau)
    h.E = c->E[c->cur];
    h.M = c->M[c->cur];
    h.R = (k == 0) ? R0 : cap;
    h.Rdev = (k == 0) ? nullptr : c->scal + 4;
    h.rec = d_rec + k;
    h.step = (uint32_t)k;
    h.wtab = nullptr;
    h.tab_f = c->tab;
    h.tab_T = c->tab + nb;
    h.progress = nullptr;
    if (k < K) {
      // w = exp(-dbeta (E - E0)) for E - E0 = d 2^shift, every level the
      // histogram may start at: the slot holding this dbeta's table, else
      // the least recently used one, refilled once its last reader is done
      const double dbeta = betas[k] - c->beta;
      uint64_t key;
      std::memcpy(&key, &dbeta, sizeof key);
      int slot = -1;
      for (int i = 0; i < kWSlots && slot < 0; ++i)
        if (c->wvalid[i] && c->wkey[i] == key) slot = i;
      double* w;
      if (slot >= 0) {
        w = c->h_w + (size_t)slot * nb;
      } else {
        slot = 0;
        for (int i = 0; i < kWSlots; ++i) {
          if (!c->wvalid[i]) {
            slot = i;
            break;
          }
          if ((int32_t)(c->wlast[i] - c->wlast[slot]) < 0) slot = i;
        }
        if (c->wvalid[slot] && !wait_progress(c, c->wlast[slot])) {
          CK(wait_stream(c->stream));
          note_error("a histogram of the schedule did not report its weights");
          return PA_EDEVICE;
        }
        w = c->h_w + (size_t)slot * nb;
        for (int64_t d = 0; d < nb; ++d)
          w[d] = std::exp(-(dbeta * (double)(d << c->hshift)));
        c->wkey[slot] = key;
        c->wvalid[slot] = true;
      }
      // the first levels also in the kernel's arguments
      std::memcpy(wk.w, w, (size_t)std::min<int64_t>(nb, kArgWeights) * 8);
      const uint32_t seq = ++c->wseq;
      c->wlast[slot] = seq;
      h.wtab = c->d_w + (size_t)slot * nb;
      h.progress = c->d_prog;
      h.wseq = seq;
    }
    c->rseq_tag = k;
    hipEvent_t e0 = t_begin(c, PA_K_HIST);
    CK(launch_hist_sched(h, wk, c->stream));
    t_end(c, PA_K_HIST, e0, 0, 0, 8, 0);
    if (k == K) break;
    // (b) copy counts with the device tables, the new size and the parent
    // of every new slot; the counts clear the histogram for the next step
    CountsArgs ca{};
    ca.E = c->E[c->cur];
    ca.f = c->tab;
    ca.T = c->tab + nb;
    ca.n = c->n;
    ca.tile_sum = c->tile_sum;
    ca.clear = c->rb;
    ca.nclear = c->nb2 + 8;
    ca.R = cap;
    ca.Rdev = &d_rec[k].Rc;
    ca.lvl_dev = &d_rec[k].lo;
    ca.twoN = 2 * c->N;
    ca.shift = c->hshift;
    ca.k0 = (uint32_t)(c->seed & 0xFFFFFFFFu);
    ca.k1 = (uint32_t)(c->seed >> 32);
    ca.pop = c->pop;
    ca.step_next = (uint32_t)(step0 + k + 1);
    if (c->ntiles_cap > kLookbackTiles) {
      e0 = t_begin(c, PA_K_COUNTS);
      CK(launch_counts(ca, c->stream));
      CK(launch_scan_dev(c->tile_sum, c->tile_off, c->ntiles_cap, c->scal + 4,
                         cap, d_halt, (uint32_t)k, c->stream));
      t_end(c, PA_K_COUNTS, e0, 8 * c->ntiles_cap, 0, 8, 0);
      e0 = t_begin(c, PA_K_SCATTER);
      CK(launch_scatter_dev(c->n, c->tile_off, cap, &d_rec[k].Rc, cap,
                            c->parent, c->fam[c->famcur],
                            c->fam[c->famcur ^ 1], c->stream));
      t_end(c, PA_K_SCATTER, e0, 0, 0, 4, 0);
    } else {
    LookbackArgs lb{};
    lb.status = reinterpret_cast<unsigned long long*>(c->tile64);
    lb.ticket = lb_ctr;
    lb.done = lb_ctr + 1;
    lb.gen = ++c->lb_gen;
    lb.ntiles = c->ntiles_cap;
    lb.cap = cap;
    lb.parent = c->parent;
    lb.fam_src = c->fam[c->famcur];
    lb.fam_dst = c->fam[c->famcur ^ 1];
    lb.total = c->scal + 4;
    lb.halt = d_halt;
    lb.step = (uint32_t)k;
    e0 = t_begin(c, PA_K_COUNTS);
    CK(launch_counts_scatter(ca, lb, c->stream));
    t_end(c, PA_K_COUNTS, e0, 8 * c->ntiles_cap, 0, 12, 0);
    }
    c->famcur ^= 1;
    // (c) theta sweeps at betas[k], each new slot loaded from its parent
    c->beta = betas[k];
    c->step = step0 + k + 1;
    c->sweeps_at_step = 0;
    LatticeArgs a = lattice_args(c);
    metropolis_K(c->beta, &a.K4, &a.K8);
    a.theta = theta;
    a.src = c->spins[c->cur];
    a.parent = c->parent;
    a.spins = c->spins[c->cur ^ 1];
    a.E = c->E[c->cur ^ 1];
    a.M = c->M[c->cur ^ 1];
    c->rseq_tag = k + 1;
    rc = run_lattice(c, a, PA_K_SWEEP);
    if (rc) return rc;
    c->cur ^= 1;
    c->sweeps_at_step = theta;
  }
  c->rseq_tag = -1;
  const size_t rec_bytes = 64 + (size_t)(K + 1) * sizeof(AnnealRec);
  CK(hipMemcpyAsync(c->h_arec, c->arec, rec_bytes, hipMemcpyDeviceToHost,
                    c->stream));
  CK(wait_stream(c->stream));
  const AnnealHalt hh = *reinterpret_cast<const AnnealHalt*>(c->h_arec);
  const AnnealRec* rec = reinterpret_cast<const AnnealRec*>(c->h_arec + 64);
  const int kd = hh.code ? (int)hh.step : K;
  // timed launches: their per-replica parts with the size they acted on
  for (auto& t : c->pending) {
    if (t.rseq < 0) continue;
    const int64_t Rs = (int64_t)rec[t.rseq].R;
    t.bytes += t.bytes_rep * Rs;
    t.attempts += t.attempts_rep * Rs;
    t.bytes_rep = t.attempts_rep = 0;
    t.rseq = -1;
  }
  // ln Q of every completed step from its sum S, in the host tables' order
  // of operations (Eq. part-Q), and the observables after its sweeps
  double lnZ = lnZ0, lq = lnQ0, bprev = beta0;
  for (int k = 0; k < kd; ++k) {
    const double dbeta = betas[k] - bprev;
    const int Emin = -2 * c->N + (rec[k].lo << c->hshift);
    const double q = (-(dbeta * (double)Emin)) +
                     std::log(rec[k].S / (double)(int64_t)rec[k].R);
    lnZ = lnZ + q;  // Eq. Free-En, read with the logarithm
    lq = q;
    if (lnQ) lnQ[k] = q;
    if (obs) {
      const AnnealRec& r = rec[k + 1];
      observables_from_sums((int64_t)r.R, betas[k], c->N, r.sumE, r.sumE2,
                            (int64_t)r.sumAbsM, (int64_t)r.sumM2,
                            -2 * c->N + (r.lo << c->hshift),
                            -2 * c->N + ((r.lo + r.nl - 1) << c->hshift),
                            &obs[k]);
    }
    bprev = betas[k];
  }
  c->lnZ = lnZ;
  c->lnQ_last = lq;
  c->R_pending = false;
  c->gather_pending = false;
  c->hist_valid = false;
  c->rb_zero = false;
  if (kd == K) {
    c->R = (int64_t)rec[K].R;
    c->n_len = (int64_t)rec[K - 1].R;
    c->hist_lo = rec[K].lo;
  } else if (hh.code == kHaltWait) {
    note_error("a wait of the single-pass scan for an earlier tile gave up");
    rc = PA_EDEVICE;
  } else {
    // as after the failed pa_resample of step kd: the population after the
    // sweeps of step kd - 1, in the buffers it was left in
    c->cur = cur0 ^ (kd & 1);
    c->famcur = fam0 ^ (kd & 1);
    c->step = step0 + kd;
    c->beta = kd ? betas[kd - 1] : beta0;
    c->sweeps_at_step = kd ? theta : sw0;
    c->R = (int64_t)rec[kd].R;
    c->n_len = 0;
    rc = hh.code == kHaltCapacity ? PA_ECAPACITY
         : hh.code == kHaltEmpty  ? PA_EEMPTY
                                  : PA_EDEVICE;
    if (rc == PA_EDEVICE)
      note_error("a replica's energy lies outside the histogram range");
  }
  t_harvest(c);
  if (done) *done = kd;
  return rc;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_start_heating(pa_ctx* c, double beta0) try {
  if (!c || !std::isfinite(beta0) || !(beta0 > 0.0)) return PA_EINVAL;
  if (c->model == PA_PMJ) return PA_EINVAL;
  if (c->step != 0) return PA_ESTATE;
  int rc = sync(c);
  if (rc) return rc;
  c->gather_pending = false;
  c->R = c->R_t;
  LatticeArgs a = lattice_args(c);
  a.init = 2;
  a.theta = 0;
  rc = run_lattice(c, a, PA_K_INIT);
  if (rc) return rc;
  rc = reset_families(c);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  c->beta = beta0;
  // ln Z(beta0): the ground states (2 Ising, q Potts) of energy -2N, and to
  // first order their lightest excitations on a torus of side >= 4: one
  // changed site (4 broken bonds) and two changed neighbours (6 broken
  // bonds, or 7 for two different new Potts states)
  const double n = (double)c->N;
  double excited;
  if (c->q) {
    const double e4 = std::exp(-4.0 * beta0), e6 = std::exp(-6.0 * beta0),
                 e7 = std::exp(-7.0 * beta0);
    excited = n * (double)(c->q - 1) *
              (e4 + 2.0 * e6 + 2.0 * (double)(c->q - 2) * e7);
  } else {
    const double e8 = std::exp(-8.0 * beta0), e12 = std::exp(-12.0 * beta0);
    excited = n * (e8 + 2.0 * e12);
  }
  c->lnZ = (std::log(c->q ? (double)c->q : 2.0) + 2.0 * n * beta0) + excited;
  c->lnQ_last = 0.0;
  c->sweeps_at_step = 0;
  c->n_len = 0;
  c->hist_valid = false;
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

int pa_observables(pa_ctx* c, pa_obs* o) try {
  if (!c || !o) return PA_EINVAL;
  int rc = compute_hist(c);
  if (rc) return rc;
  observables_from_hist(c->h_hist, c->nbins, c->hshift, c->N, c->R, c->beta,
                        (int64_t)c->h_scal[0], (int64_t)c->h_scal[1], o);
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

int pa_free_energy(pa_ctx* c, double* lnZ, double* lnQ_last) try {
  if (!c) return PA_EINVAL;
  if (lnZ) *lnZ = c->lnZ;
  if (lnQ_last) *lnQ_last = c->lnQ_last;
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

int pa_state(pa_ctx* c, int64_t* R, double* beta, int32_t* step) try {
  if (!c) return PA_EINVAL;
  if (R && c->R_pending) {
    const int rc = sync(c);
    if (rc) return rc;
  }
  if (R) *R = c->R;
  if (beta) *beta = c->beta;
  if (step) *step = c->step;
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

int pa_get_population(pa_ctx* c, int8_t* spins, int32_t* E, int32_t* M,
                      int64_t cap) try {
  if (!c) return PA_EINVAL;
  int rc = sync(c);  // the population size, if still on the device
  if (rc) return rc;
  if (cap < c->R) return PA_EINVAL;
  rc = finish_gather(c);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  if (spins) {
    if (c->layout == PA_INT8) {
      CK(hipMemcpy2D(spins, (size_t)c->N, c->spins[c->cur], (size_t)c->stride,
                     (size_t)c->N, (size_t)c->R, hipMemcpyDeviceToHost));
    } else {
      std::vector<uint8_t> tmp((size_t)(c->R * c->stride));
      CK(hipMemcpy(tmp.data(), c->spins[c->cur], tmp.size(),
                   hipMemcpyDeviceToHost));
      for (int64_t j = 0; j < c->R; ++j)
        unpack_replica(c, tmp.data() + j * c->stride, spins + j * c->N);
    }
  }
  if (E) CK(hipMemcpy(E, c->E[c->cur], (size_t)c->R * 4, hipMemcpyDeviceToHost));
  if (M) CK(hipMemcpy(M, c->M[c->cur], (size_t)c->R * 4, hipMemcpyDeviceToHost));
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

int pa_get_replicas(pa_ctx* c, const int64_t* slots, int64_t k, int8_t* spins,
                    int32_t* E, int32_t* M) try {
  if (!c || (k > 0 && !slots) || k < 0) return PA_EINVAL;
  int rc = sync(c);  // the population size, if still on the device
  if (rc) return rc;
  for (int64_t i = 0; i < k; ++i)
    if (slots[i] < 0 || slots[i] >= c->R) return PA_EINVAL;
  rc = finish_gather(c);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  std::vector<uint8_t> tmp((size_t)c->stride);
  for (int64_t i = 0; i < k; ++i) {
    const int64_t j = slots[i];
    if (spins) {
      CK(hipMemcpy(tmp.data(), c->spins[c->cur] + j * c->stride, tmp.size(),
                   hipMemcpyDeviceToHost));
      unpack_replica(c, tmp.data(), spins + i * c->N);
    }
    if (E) CK(hipMemcpy(E + i, c->E[c->cur] + j, 4, hipMemcpyDeviceToHost));
    if (M) CK(hipMemcpy(M + i, c->M[c->cur] + j, 4, hipMemcpyDeviceToHost));
  }
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

int pa_get_counts(pa_ctx* c, uint32_t* n, int64_t cap, int64_t* len) try {
  if (!c || (c->n_len > 0 && !n) || cap < c->n_len) return PA_EINVAL;
  int rc = sync(c);
  if (rc) return rc;
  if (c->n_len > 0)
    CK(hipMemcpy(n, c->n, (size_t)c->n_len * 4, hipMemcpyDeviceToHost));
  if (len) *len = c->n_len;
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

int pa_set_population(pa_ctx* c, const int8_t* spins, int64_t R) try {
  if (!c || !spins || R < 1 || R > c->cap) return PA_EINVAL;
  for (int64_t i = 0; i < R * c->N; ++i)
    if (c->q ? (spins[i] < 0 || spins[i] >= c->q)
             : (spins[i] != 1 && spins[i] != -1))
      return PA_EINVAL;
  int rc = sync(c);
  if (rc) return rc;
  c->gather_pending = false;  // the new population replaces the pending one
  std::vector<uint8_t> tmp((size_t)(R * c->stride));
  for (int64_t j = 0; j < R; ++j)
    pack_replica(c, spins + j * c->N, tmp.data() + j * c->stride);
  CK(hipMemcpy(c->spins[c->cur], tmp.data(), tmp.size(), hipMemcpyHostToDevice));
  c->R = R;
  LatticeArgs a = lattice_args(c);
  a.theta = 0;
  rc = run_lattice(c, a, PA_K_SWEEP);
  if (rc) return rc;
  rc = reset_families(c);
  if (rc) return rc;
  rc = sync(c);
  if (rc) return rc;
  c->hist_valid = false;
  c->n_len = 0;
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

int pa_get_families(pa_ctx* c, uint32_t* fam, int64_t cap, int64_t* len,
                    int64_t* n0) try {
  if (!c) return PA_EINVAL;
  int rc = sync(c);  // the population size, if still on the device
  if (rc) return rc;
  if (fam && cap < c->R) return PA_EINVAL;
  if (fam)
    CK(hipMemcpy(fam, c->fam[c->famcur], (size_t)c->R * 4,
                 hipMemcpyDeviceToHost));
  if (len) *len = c->R;
  if (n0) *n0 = c->fam_n0;
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

int pa_family_stats(pa_ctx* c, pa_family* out) try {
  if (!c || !out) return PA_EINVAL;
  int rc = sync(c);
  if (rc) return rc;
  std::vector<uint32_t> f((size_t)c->R);
  int64_t len = 0, n0 = 0;
  rc = pa_get_families(c, f.data(), (int64_t)f.size(), &len, &n0);
  if (rc) return rc;
  return pa_family_summary(f.data(), len, n0, out);
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_histogram(pa_ctx* c, uint32_t* h, int64_t cap, int32_t* nbins,
                 int32_t* step) try {
  if (!c || (h && cap < c->nbins)) return PA_EINVAL;
  int rc = compute_hist(c);
  if (rc) return rc;
  if (h) std::memcpy(h, c->h_hist, (size_t)c->nbins * 4);
  if (nbins) *nbins = c->nbins;
  if (step) *step = 1 << c->hshift;
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

int pa_overlap(pa_ctx* c, double dbeta, double* alpha) try {
  if (!c || !alpha || !std::isfinite(dbeta) || dbeta < 0.0) return PA_EINVAL;
  int rc = compute_hist(c);
  if (rc) return rc;
  *alpha = overlap_from_hist(c->h_hist, c->nbins, c->hshift, c->N, c->R,
                             dbeta);
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

int pa_bisect_dbeta(pa_ctx* c, double target, double beta_f, double* dbeta) try {
  if (!c || !dbeta || !(target > 0.0 && target <= 1.0) ||
      !std::isfinite(beta_f))
    return PA_EINVAL;
  int rc = compute_hist(c);
  if (rc) return rc;
  *dbeta = bisect_from_hist(c->h_hist, c->nbins, c->hshift, c->N, c->R,
                            target, beta_f - c->beta);
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

int pa_set_timing(pa_ctx* c, int32_t classes) try {
  if (!c) return PA_EINVAL;
  int rc = sync(c);
  if (rc) return rc;
  c->timing = (classes == PA_TIMING_ALL) ? 0x3Fu : ((uint32_t)classes & 0x3Fu);
  if (c->timing) c->acc = pa_timing{};
  for (auto& n : c->timing_count) n = 0;
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

int pa_set_timing_sample(pa_ctx* c, int32_t every) try {
  if (!c || every < 1) return PA_EINVAL;
  c->timing_every = every;
  for (auto& n : c->timing_count) n = 0;
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

int pa_get_config(pa_ctx* c, pa_config* out) try {
  if (!c || !out) return PA_EINVAL;
  pa_config k{};
  k.L = c->L;
  k.model = c->model;
  k.J = nullptr;
  k.R_target = c->R_t;
  k.capacity = c->cap;
  k.layout = c->layout;
  k.rows_per_lane = c->rpl;
  k.seed = c->seed;
  k.population_id = c->pop;
  k.stream = c->stream;
  k.resampling = c->law;
  k.q = c->q;
  k.rng_mode = c->rng_mode;
  *out = k;
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

}  // extern "C"

namespace {

// Population file: a fixed header, the couplings (+-J only), then the
// population in the canonical layout.  Little-endian, as the host.
constexpr char kMagic[8] = {'P', 'A', 'P', 'O', 'P', 'v', '0', '4'};
struct FileHeader {
  char magic[8];
  int64_t R_target, capacity, seed, R;
  double beta, lnZ, lnQ_last;
  int32_t L, model, layout, rows_per_lane;
  uint32_t population_id;
  int32_t step, sweeps_at_step, resampling;
  int32_t q;
  uint32_t fam_n0;  // size of the founding population of the families
  int32_t rng_mode, reserved;
};
static_assert(sizeof(FileHeader) == 8 + 4 * 8 + 3 * 8 + 12 * 4,
              "population file header must have no padding");

struct File {
  FILE* f = nullptr;
  explicit File(FILE* g) : f(g) {}
  ~File() {
    if (f) std::fclose(f);
  }
  bool write(const void* p, size_t n) { return std::fwrite(p, 1, n, f) == n; }
  bool read(void* p, size_t n) { return std::fread(p, 1, n, f) == n; }
};

}  // namespace

extern "C" {

int pa_save(pa_ctx* c, const char* path) try {
  if (!c || !path) return PA_EINVAL;
  int rc = sync(c);  // the population size, if still on the device
  if (rc) return rc;
  const int64_t R = c->R;
  std::vector<int8_t> spins((size_t)R * c->N);
  std::vector<int32_t> E((size_t)R), M((size_t)R);
  rc = pa_get_population(c, spins.data(), E.data(), M.data(), R);
  if (rc) return rc;
  std::vector<uint32_t> fam((size_t)R);
  int64_t flen = 0, n0 = 0;
  rc = pa_get_families(c, fam.data(), R, &flen, &n0);
  if (rc) return rc;
  FileHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.R_target = c->R_t;
  h.capacity = c->cap;
  h.seed = (int64_t)c->seed;
  h.R = R;
  h.beta = c->beta;
  h.lnZ = c->lnZ;
  h.lnQ_last = c->lnQ_last;
  h.L = c->L;
  h.model = c->model;
  h.layout = c->layout;
  h.rows_per_lane = c->rpl;
  h.population_id = c->pop;
  h.step = c->step;
  h.sweeps_at_step = c->sweeps_at_step;
  h.resampling = c->law;
  h.q = c->q;
  h.fam_n0 = (uint32_t)n0;
  h.rng_mode = c->rng_mode;
  File f(std::fopen(path, "wb"));
  if (!f.f) return PA_EIO;
  bool ok = f.write(&h, sizeof h);
  if (c->model == PA_PMJ) ok = ok && f.write(c->J.data(), c->J.size());
  ok = ok && f.write(spins.data(), spins.size());
  ok = ok && f.write(E.data(), E.size() * 4);
  ok = ok && f.write(M.data(), M.size() * 4);
  ok = ok && f.write(fam.data(), fam.size() * 4);
  ok = (std::fflush(f.f) == 0) && ok;
  return ok ? PA_OK : PA_EIO;
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_load(const char* path, void* stream, pa_ctx** out) try {
  if (!out) return PA_EINVAL;
  *out = nullptr;
  if (!path) return PA_EINVAL;
  // everything is read and checked before any device work
  File f(std::fopen(path, "rb"));
  if (!f.f) return PA_EIO;
  FileHeader h{};
  if (!f.read(&h, sizeof h) || std::memcmp(h.magic, kMagic, 8) != 0)
    return PA_EIO;
  if (h.L < 4 || h.L > 128 || (h.L & 1) || h.R < 1 || h.R > h.capacity ||
      h.capacity >= (1ll << 32) ||
      (h.model != PA_FERRO && h.model != PA_PMJ && h.model != PA_POTTS) ||
      (h.model == PA_POTTS && (h.q < 2 || h.q > 16)) ||
      h.step < 0 || h.step > 65535 || h.sweeps_at_step < 0 ||
      h.sweeps_at_step > 32767 || !std::isfinite(h.beta) || !(h.beta >= 0.0) ||
      h.resampling < PA_NEAREST || h.resampling > PA_MULTINOMIAL ||
      h.fam_n0 < 1 || (int64_t)h.fam_n0 > h.capacity ||
      (h.rng_mode != PA_RNG_WORD && h.rng_mode != PA_RNG_PLANES) ||
      h.reserved != 0)
    return PA_EIO;
  const int64_t N = (int64_t)h.L * h.L;
  // the body's size follows from the header: check it before allocating
  {
    const long here = std::ftell(f.f);
    if (here < 0 || std::fseek(f.f, 0, SEEK_END) != 0) return PA_EIO;
    const long end = std::ftell(f.f);
    if (end < 0 || std::fseek(f.f, here, SEEK_SET) != 0) return PA_EIO;
    const int64_t want = (h.model == PA_PMJ ? 2 * N : 0) + h.R * N + 12 * h.R;
    if ((int64_t)(end - here) != want) return PA_EIO;
  }
  std::vector<int8_t> J;
  if (h.model == PA_PMJ) {
    J.resize((size_t)(2 * N));
    if (!f.read(J.data(), J.size())) return PA_EIO;
  }
  std::vector<int8_t> spins((size_t)(h.R * N));
  std::vector<int32_t> E((size_t)h.R), M((size_t)h.R);
  std::vector<uint32_t> fam((size_t)h.R);
  if (!f.read(spins.data(), spins.size()) || !f.read(E.data(), E.size() * 4) ||
      !f.read(M.data(), M.size() * 4) || !f.read(fam.data(), fam.size() * 4))
    return PA_EIO;
  for (uint32_t v : fam)
    if (v >= h.fam_n0) return PA_EIO;
  char extra;
  if (f.read(&extra, 1)) return PA_EIO;  // trailing bytes: not our file
  for (int8_t v : spins)
    if (h.model == PA_POTTS ? (v < 0 || v >= h.q) : (v != 1 && v != -1))
      return PA_EIO;
  pa_config cfg{};
  cfg.L = h.L;
  cfg.model = h.model;
  cfg.J = J.empty() ? nullptr : J.data();
  cfg.R_target = h.R_target;
  cfg.capacity = h.capacity;
  cfg.layout = h.layout;
  cfg.rows_per_lane = h.rows_per_lane;
  cfg.seed = (uint64_t)h.seed;
  cfg.population_id = h.population_id;
  cfg.stream = stream;
  cfg.resampling = h.resampling;
  cfg.q = h.q;
  cfg.rng_mode = h.rng_mode;
  pa_ctx* c = nullptr;
  int rc = pa_init(&cfg, &c);
  if (rc) return rc == PA_EINVAL ? PA_EIO : rc;
  rc = pa_set_population(c, spins.data(), h.R);
  // the energies and magnetisations the file holds must be the ones of its
  // spins
  std::vector<int32_t> E2((size_t)h.R), M2((size_t)h.R);
  if (!rc) rc = pa_get_population(c, nullptr, E2.data(), M2.data(), h.R);
  if (!rc && (E2 != E || M2 != M)) rc = PA_EIO;
  if (!rc && hipMemcpy(c->fam[0], fam.data(), fam.size() * 4,
                       hipMemcpyHostToDevice) != hipSuccess)
    rc = PA_EDEVICE;
  if (rc) {
    pa_destroy(c);
    return rc;
  }
  c->famcur = 0;
  c->fam_n0 = h.fam_n0;
  c->beta = h.beta;
  c->lnZ = h.lnZ;
  c->lnQ_last = h.lnQ_last;
  c->step = h.step;
  c->sweeps_at_step = h.sweeps_at_step;
  c->n_len = 0;
  c->hist_valid = false;
  *out = c;
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

int pa_get_timing(pa_ctx* c, pa_timing* out) try {
  if (!c || !out) return PA_EINVAL;
  int rc = sync(c);
  if (rc) return rc;
  *out = c->acc;
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

}  // extern "C"
