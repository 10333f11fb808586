// HIP kernels (gfx950) of the population-annealing hot path.
//
//  k_lattice   init at beta_0 = 0 / theta checkerboard Metropolis sweeps /
//              energy and magnetisation of every replica (paper Sec. 2,
//              first and equilibration steps; Eq. Ham).  One replica's
//              lattice lives in the VGPRs of L/RPL lanes of one wave, bit
//              packed (lane = RPL consecutive rows, 32 sites per register);
//              vertical neighbours come from the adjacent lanes through
//              ds_bpermute, horizontal ones from in-register shifts.  The
//              lattice is read from HBM once and written once per call,
//              whatever theta is.  After a resampling the call reads every
//              new slot from its parent in the other buffer, so the
//              resampling copy needs no pass of its own.
//  k_hist      exact energy histogram + |M| and M^2 sums (Eqs. part-Q/tau
//              need only the energy distribution).
//  k_counts    copy counts floor(rho) + Bernoulli(frac rho) per replica from
//              the host's per-level tables (or a Poisson count: the number
//              of the level's CDF thresholds below the replica's word),
//              plus one partial sum per tile;
//              clears the histogram of the next step on the way.
//  k_scan      exclusive scan of the tile sums (single workgroup).
//  k_scatter   per-tile scan of the counts -> parent index of every new slot
//              (and its family, the parent's family).
//  k_gather    copy of every parent's lattice, E and M into its new slots of
//              the second buffer (one wave per slot for replicas of 1 KB and
//              more, else a flat array of 16-byte units with four in flight
//              per thread), when no sweep follows the resampling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "pa_device.h"
#include "pa_internal.h"
#include "pa_lattice.h"

namespace pa {

// ------------------------------------------------------------- lattice pass

template <int W, int RPL, bool INT8, bool GLASS, bool PLANES>
__global__ __launch_bounds__(256) void k_lattice(const LatticeArgs a) {
  lattice_pass<W, RPL, INT8, GLASS, PLANES>(
      a, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

// -------------------------------------------------------------- histogram

// Workgroup histogram in LDS over the window of bins the host expects the
// energies in.  In every wave the lanes whose bin equals that of the lowest
// pending lane add as one (at low temperatures most replicas share an energy,
// and 64 lanes adding 1 to one LDS word would serialise); the rest add their
// own 1.  The |M| and M^2 sums are reduced over the workgroup before one
// atomic each, and every nonzero window bin is added to the global
// histogram once per workgroup.
constexpr int kHistU = 8;

// Lane q's value of v, the same in every lane (q uniform).
__device__ __forceinline__ double readlane_f64(double v, int q) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, q);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), q);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Levels per piece of the term array of the table tail in LDS.
constexpr int kTermPiece = 4096;

// The end of a step's histogram in a schedule run on the device, in its last
// workgroup (the histogram, moments and sums are final): the occupied range
// and exact energy sums the workgroups added up, then, with weights given,
// the nearest-integer tables of Eqs. part-Q/tau in the operation order of
// the host's: terms h w per level, their sum S in ascending level order, and
// per level rho = R_target w / S, f = floor(rho), T = floor(frac(rho)
// 2^32).  The terms of up to kTermPiece levels at a time go to LDS (every
// load of a piece in flight at once); one wave then adds them in level order
// (empty levels and the padding add +0, which leaves every partial sum as it
// is, as the host's skipping them does).  The population counted is R.
// Finally the weights' sequence number goes to *progress, in host memory:
// the host may then reuse their slot.
__device__ void anneal_tail(const HistArgs& a, const double* wk, int64_t R,
                            double* tl) {
  __shared__ double s_S;
  __shared__ BlockSums s_red[4];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // the workgroups' parts, one per thread, summed over the workgroup
  BlockSums acc{};
  if (tid < (int)gridDim.x) acc = a.part[tid];
  for (int off = 32; off > 0; off >>= 1) {
    acc.sAbsM += __shfl_down(acc.sAbsM, off, 64);
    acc.sM2 += __shfl_down(acc.sM2, off, 64);
    acc.sE += __shfl_down(acc.sE, off, 64);
    acc.sE2 += __shfl_down(acc.sE2, off, 64);
    acc.lo_rev = max(acc.lo_rev, (uint32_t)__shfl_down((int)acc.lo_rev, off, 64));
    acc.hi1 = max(acc.hi1, (uint32_t)__shfl_down((int)acc.hi1, off, 64));
  }
  if (lane == 0) s_red[wid] = acc;
  __syncthreads();
  acc = s_red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
    acc.sAbsM += s_red[i].sAbsM;
    acc.sM2 += s_red[i].sM2;
    acc.sE += s_red[i].sE;
    acc.sE2 += s_red[i].sE2;
    acc.lo_rev = max(acc.lo_rev, s_red[i].lo_rev);
    acc.hi1 = max(acc.hi1, s_red[i].hi1);
  }
  const int lo = a.nbins - (int)acc.lo_rev, hi = (int)acc.hi1 - 1;
  // a bad energy stops the schedule here: no tables, no replicas from now on
  const bool bad = a.moments[3] != 0ull;
  const int nl = (hi >= lo && !bad) ? hi - lo + 1 : 0;
  double S = 0.0;
  if (a.wtab && nl > 0) {
    constexpr int PT = kTermPiece / 256;  // levels per thread and piece
    double sum = 0.0;
    for (int p0 = 0; p0 < nl; p0 += kTermPiece) {
      const int n = min(kTermPiece, nl - p0);
      const int npad = (n + 31) & ~31;
      uint32_t h[PT];
      double w[PT];
#pragma unroll
      for (int c = 0; c < PT; ++c) {
        const int l = p0 + c * 256 + tid;
        const bool in = c * 256 + tid < n;
        h[c] = in ? a.hist[lo + l] : 0u;
        w[c] = in ? (l < kArgWeights ? wk[l] : a.wtab[l]) : 0.0;
      }
#pragma unroll
      for (int c = 0; c < PT; ++c) {
        const int i = c * 256 + tid;
        if (i < npad) tl[i] = (double)h[c] * w[c];
        if (i < n) a.wscr[p0 + i] = w[c];
      }
      __syncthreads();
      if (wid == 0) {
        for (int i0 = 0; i0 < npad; i0 += 32) {
          double v[32];
#pragma unroll
          for (int u = 0; u < 32; ++u) v[u] = tl[i0 + u];
#pragma unroll
          for (int u = 0; u < 32; ++u) sum = sum + v[u];
        }
      }
      __syncthreads();
    }
    if (tid == 0) s_S = sum;
    __syncthreads();
    S = s_S;
    const double Rt = (double)a.R_t;
    for (int l = tid; l < nl; l += blockDim.x) {
      uint32_t f = 0u, T = 0u;
      if (a.hist[lo + l]) {
        const double rho = (Rt * a.wscr[l]) / S;
        const double fl = floor(rho);
        f = (uint32_t)fl;
        T = (uint32_t)(uint64_t)floor(ldexp(rho - fl, 32));
      }
      a.tab_f[l] = f;
      a.tab_T[l] = T;
    }
  }
  if (tid == 0) {
    AnnealRec r;
    r.R = (unsigned long long)R;
    r.Rc = bad ? 0ull : (unsigned long long)R;
    r.sumAbsM = acc.sAbsM;
    r.sumM2 = acc.sM2;
    r.sumE = acc.sE;
    r.sumE2 = acc.sE2;
    r.S = S;
    r.lo = lo;
    r.nl = nl;
    *a.rec = r;
    if (bad) {
      if (a.halt->code == 0u) {
        a.halt->code = kHaltEnergy;
        a.halt->step = a.step;
        a.halt->total = 0ull;
      }
      *a.Rw = 0ull;
    }
    if (a.progress)
      __hip_atomic_store(a.progress, a.wseq, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The histogram pass; SCHED: a step of a schedule on the device, which also
// adds up the occupied range and the exact energy sums and ends in
// anneal_tail (weights wk in the arguments).
template <bool SCHED>
__device__ __forceinline__ void hist_body(const HistArgs& a, const double* wk) {
  extern __shared__ __attribute__((aligned(16))) uint32_t sh[];
  __shared__ unsigned long long red[2][4];
  __shared__ long long red_e[2][4];
  __shared__ uint32_t red_r[2][4];
  for (int i = threadIdx.x; i < a.win_n; i += blockDim.x) sh[i] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long sam = 0ull, sm2 = 0ull;
  long long se = 0, se2 = 0;
  uint32_t lo_rev = 0u, hi1 = 0u;
  const int64_t R = a.Rdev ? min((int64_t)*a.Rdev, a.R) : a.R;
  // kHistU replicas per lane and pass, their loads all issued before any is
  // counted; the loop bound is uniform over the workgroup, so every wave
  // runs whole
  constexpr int U = kHistU;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * U; base < R;
       base += (int64_t)gridDim.x * blockDim.x * U) {
    int32_t e[U], m[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = base + (int64_t)u * blockDim.x + threadIdx.x;
      e[u] = j < R ? a.E[j] : 0;
      m[u] = j < R ? a.M[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int w = -1;
      if (base + (int64_t)u * blockDim.x + threadIdx.x < R) {
        const int idx = (e[u] + a.twoN) >> a.shift;
        if (idx < 0 || idx >= a.nbins) {  // corrupt energy: report, never index
          atomicAdd(&a.moments[3], 1ull);
        } else {
          w = idx - a.win_lo;
          if (w < 0 || w >= a.win_n) {
            atomicAdd(&a.hist[idx], 1u);
            w = -1;
          }
          if (SCHED) {
            const long long ee = e[u];
            se += ee;
            se2 += ee * ee;
            lo_rev = max(lo_rev, (uint32_t)(a.nbins - idx));
            hi1 = max(hi1, (uint32_t)(idx + 1));
          }
        }
        const int mm = m[u];
        sam += (unsigned long long)(mm < 0 ? -mm : mm);
        sm2 += (unsigned long long)((long long)mm * mm);
      }
      const unsigned long long pend = __ballot(w >= 0);
      if (pend) {
        const int first = __builtin_ctzll(pend);
        const int lb = __shfl(w, first, 64);
        const unsigned long long same = __ballot(w == lb);
        if (lane == first) atomicAdd(&sh[lb], (uint32_t)__popcll(same));
        else if (w >= 0 && w != lb) atomicAdd(&sh[w], 1u);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sam += __shfl_down(sam, off, 64);
    sm2 += __shfl_down(sm2, off, 64);
    if (SCHED) {
      se += __shfl_down(se, off, 64);
      se2 += __shfl_down(se2, off, 64);
      lo_rev = max(lo_rev, (uint32_t)__shfl_down((int)lo_rev, off, 64));
      hi1 = max(hi1, (uint32_t)__shfl_down((int)hi1, off, 64));
    }
  }
  if (lane == 0) {
    red[0][wid] = sam;
    red[1][wid] = sm2;
    if (SCHED) {
      red_e[0][wid] = se;
      red_e[1][wid] = se2;
      red_r[0][wid] = lo_rev;
      red_r[1][wid] = hi1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s0 = 0ull, s1 = 0ull;
    long long t0 = 0, t1 = 0;
    uint32_t r0 = 0u, r1 = 0u;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      s0 += red[0][i];
      s1 += red[1][i];
      if (SCHED) {
        t0 += red_e[0][i];
        t1 += red_e[1][i];
        r0 = max(r0, red_r[0][i]);
        r1 = max(r1, red_r[1][i]);
      }
    }
    if (SCHED) {
      // the workgroup's part, added up by the last workgroup (no device
      // atomics on shared words)
      BlockSums b{};
      b.sAbsM = s0;
      b.sM2 = s1;
      b.sE = t0;
      b.sE2 = t1;
      b.lo_rev = r0;
      b.hi1 = r1;
      a.part[blockIdx.x] = b;
    } else {
      atomicAdd(&a.moments[0], s0);
      atomicAdd(&a.moments[1], s1);
    }
  }
  // the window's nonzero bins to the global histogram (a step of a schedule
  // knows its workgroup's occupied range: only that part)
  int m0 = 0, m1 = a.win_n;
  if (SCHED) {
    __shared__ int s_m[2];
    if (threadIdx.x == 0) {
      uint32_t r0 = 0u, r1 = 0u;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        r0 = max(r0, red_r[0][i]);
        r1 = max(r1, red_r[1][i]);
      }
      s_m[0] = max(0, (a.nbins - (int)r0) - a.win_lo);
      s_m[1] = min(a.win_n, (int)r1 - a.win_lo);
    }
    __syncthreads();
    m0 = s_m[0];
    m1 = s_m[1];
  }
  for (int i = m0 + threadIdx.x; i < m1; i += blockDim.x)
    if (sh[i]) atomicAdd(&a.hist[a.win_lo + i], sh[i]);
  if (!SCHED && !a.host_rb) return;
  // the last workgroup to finish sends the read-back block to the host, or
  // ends the step of a schedule on the device: every workgroup's additions
  // are made before its count (release), the last one reads them after
  // (acquire)
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (SCHED) {
    __syncthreads();  // every wave is past the window before it is reused
    anneal_tail(a, wk, R, reinterpret_cast<double*>(sh));
    if (threadIdx.x == 0) *a.counter = 0u;
    return;
  }
  // to host memory, then the flag after a system-scope fence
  // 16-byte units (rb_words is a multiple of 4; both blocks 16-byte aligned)
  const uint4* src = reinterpret_cast<const uint4*>(a.rb);
  uint4* dst = reinterpret_cast<uint4*>(a.host_rb);
  for (int i = threadIdx.x; i < a.rb_words / 4; i += blockDim.x)
    dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    *a.counter = 0u;
    __threadfence_system();
    __hip_atomic_store(a.host_flag, a.seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(256) void k_hist(HistArgs a) {
  hist_body<false>(a, nullptr);
}

static_assert(sizeof(HistArgs) + sizeof(ArgWeights) <= 4096,
              "kernel arguments of one launch stay within 4 KB");

__global__ __launch_bounds__(256) void k_hist_sched(HistArgs a,
                                                    ArgWeights w) {
  hist_body<true>(a, w.w);
}

// ------------------------------------------------------------ copy counts

// Workgroup-wide exclusive scan of one value per thread (256 threads);
// returns the exclusive prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds,
                                                    uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  uint32_t wbase = 0u, tot = 0u;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    const uint32_t x = lds[i];
    if (i < wid) wbase += x;
    tot += x;
  }
  *total = tot;
  return wbase + incl - v;
}

// The copy count of replica j (nearest-integer or Poisson law) from the
// level tables f, T.
__device__ __forceinline__ uint32_t count_of(const CountsArgs& a, int64_t j,
                                            const uint32_t* f,
                                            const uint32_t* T) {
  uint32_t nj = 0u;
  const int l = ((a.E[j] + a.twoN) >> a.shift) - a.lvl0;
  const uint4 b = philox10(make_uint4(kDomainResample << 28,
                                      a.step_next << 16, (uint32_t)j, a.pop),
                           a.k0, a.k1);
  if (l >= 0 && l < a.nlvl) {
    if (a.poisson) {
      // the number of the level's thresholds <= r (they are sorted)
      const uint32_t base = f[3 * l], off = f[3 * l + 1], len = f[3 * l + 2];
      const uint32_t* U = f + 3 * a.nlvl + off;
      uint32_t lo = 0, hi = len;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (U[mid] <= b.x) lo = mid + 1;
        else hi = mid;
      }
      nj = base + lo;
    } else {
      nj = f[l] + (b.x < T[l] ? 1u : 0u);
    }
  }
  return nj;
}

__device__ __forceinline__ void counts_body(const CountsArgs& a0,
                                            const uint32_t* f,
                                            const uint32_t* T,
                                            uint32_t* lds) {
  CountsArgs a = a0;
  if (a0.Rdev) a.R = min((int64_t)*a0.Rdev, a0.R);
  if (a0.lvl_dev) {
    a.lvl0 = a0.lvl_dev[0];
    a.nlvl = a0.lvl_dev[1];
  }
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = j; i < a.nclear; i += (int64_t)gridDim.x * blockDim.x)
    a.clear[i] = 0u;
  uint32_t nj = 0u;
  if (j < a.R) {
    nj = count_of(a, j, f, T);
    a.n[j] = nj;
  }
  uint32_t total;
  (void)block_excl_scan(nj, lds, &total);
  if (threadIdx.x == 0) a.tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_counts(CountsArgs a) {
  __shared__ uint32_t lds[8];
  counts_body(a, a.f, a.T, lds);
}

// The same with the level tables in the kernel arguments.
__global__ __launch_bounds__(256) void k_counts_args(CountsArgs a,
                                                     ArgTables t) {
  __shared__ uint32_t lds[8];
  counts_body(a, t.f, t.T, lds);
}

// ------------------------------------------------- systematic resampling
// The mean copy numbers in 32.32 fixed point, P_j = f 2^32 + T from the
// nearest-integer tables, laid end to end (C_j = P_0 + ... + P_j, exact
// integer sums); one comb of unit-spaced points offset by the word U gives
// n_j = floor((C_j + U) / 2^32) - floor((C_{j-1} + U) / 2^32).

// (the residual law draws over the fractional parts alone: P_j = T)
__device__ __forceinline__ uint64_t sys_mean(const CountsArgs& a, int64_t j) {
  const int l = ((a.E[j] + a.twoN) >> a.shift) - a.lvl0;
  if (l < 0 || l >= a.nlvl) return 0ull;
  return (a.residual ? 0ull : ((uint64_t)a.f[l] << 32)) + (uint64_t)a.T[l];
}

__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v,
                                                      uint64_t* lds,
                                                      uint64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  uint64_t wbase = 0ull, tot = 0ull;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    const uint64_t x = lds[i];
    if (i < wid) wbase += x;
    tot += x;
  }
  *total = tot;
  return wbase + incl - v;
}

// Per 256-replica tile: the sum of P_j (and the read-back clear of k_counts).
__global__ __launch_bounds__(256) void k_sys_tiles(CountsArgs a,
                                                   uint64_t* tile64) {
  __shared__ uint64_t lds[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = j; i < a.nclear; i += (int64_t)gridDim.x * blockDim.x)
    a.clear[i] = 0u;
  uint64_t tot;
  (void)block_excl_scan64(j < a.R ? sys_mean(a, j) : 0ull, lds, &tot);
  if (threadIdx.x == 0) tile64[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the tile sums of P (64-bit).
__global__ __launch_bounds__(1024) void k_scan64(const uint64_t* tile64,
                                                 uint64_t* off64,
                                                 int64_t ntiles) {
  __shared__ uint64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (ntiles + 1023) / 1024;
  const int64_t b = tid * per;
  const int64_t e = (b + per < ntiles) ? b + per : ntiles;
  uint64_t s = 0ull;
  for (int64_t i = b; i < e; ++i) s += tile64[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t v = (tid >= off) ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = part[tid] - s;
  for (int64_t i = b; i < e; ++i) {
    off64[i] = run;
    run += tile64[i];
  }
}

// Copy counts from the comb, and the per-tile sums of the counts.
__global__ __launch_bounds__(256) void k_sys_counts(CountsArgs a,
                                                    const uint64_t* off64) {
  __shared__ uint64_t l64[4];
  __shared__ uint32_t l32[8];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t P = j < a.R ? sys_mean(a, j) : 0ull;
  uint64_t tot;
  const uint64_t C = off64[blockIdx.x] + block_excl_scan64(P, l64, &tot);
  // the comb offset: word 0 of RESAMPLE group 1, slot 0, at the new step
  const uint64_t U = philox10(make_uint4((kDomainResample << 28) | 1u,
                                         a.step_next << 16, 0u, a.pop),
                              a.k0, a.k1).x;
  const uint32_t nj =
      j < a.R ? (uint32_t)(((C + P + U) >> 32) - ((C + U) >> 32)) : 0u;
  if (j < a.R) a.n[j] = nj;
  uint32_t total;
  (void)block_excl_scan(nj, l32, &total);
  if (threadIdx.x == 0) a.tile_sum[blockIdx.x] = total;
}

// ------------------------------------------------ multinomial resampling
// R_target independent draws on the same fixed-point axis: draw i (word 0 of
// RESAMPLE group 2, slot i, at the new step) lands at x_i = floor(u_i C / 2^32)
// and counts for the replica whose interval [C_{j-1}, C_j) holds it.
// The residual law starts every count at floor(rho) and draws the rest,
// R_target - sum floor(rho), over the fractional parts (P_j = T).

// Interval ends C_j of every replica, and its count before the draws.
__global__ __launch_bounds__(256) void k_multi_cum(CountsArgs a,
                                                   const uint64_t* off64,
                                                   uint64_t* cum) {
  __shared__ uint64_t l64[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t P = j < a.R ? sys_mean(a, j) : 0ull;
  uint64_t tot;
  const uint64_t C = off64[blockIdx.x] + block_excl_scan64(P, l64, &tot);
  if (j < a.R) {
    cum[j] = C + P;
    uint32_t n0 = 0u;
    if (a.residual) {  // the certain copies
      const int l = ((a.E[j] + a.twoN) >> a.shift) - a.lvl0;
      if (l >= 0 && l < a.nlvl) n0 = a.f[l];
    }
    a.n[j] = n0;
  }
}

// One thread per draw: the first j with x < C_j, counted with an atomic
// increment (the counts do not depend on the order of the increments).
__global__ __launch_bounds__(256) void k_multi_draw(CountsArgs a,
                                                    const uint64_t* cum,
                                                    int64_t draws) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= draws) return;
  const uint64_t total = cum[a.R - 1];
  const uint4 b = philox10(make_uint4((kDomainResample << 28) | 2u,
                                      a.step_next << 16, (uint32_t)i, a.pop),
                           a.k0, a.k1);
  // a 64-bit uniform u from words 0 and 1, and x = floor(u total / 2^64):
  // every replica's probability is exact to 2^-64 per draw
  const uint64_t u = ((uint64_t)b.y << 32) | b.x;
  const uint64_t x = __umul64hi(u, total);
  int64_t lo = 0, hi = a.R - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (x < cum[mid]) hi = mid;
    else lo = mid + 1;
  }
  atomicAdd(&a.n[lo], 1u);
}

// Per-tile sums of the counts (for the scan and the parent scatter).
__global__ __launch_bounds__(256) void k_count_tiles(CountsArgs a) {
  __shared__ uint32_t lds[8];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t total;
  (void)block_excl_scan(j < a.R ? a.n[j] : 0u, lds, &total);
  if (threadIdx.x == 0) a.tile_sum[blockIdx.x] = total;
}

// Single workgroup of 1024 threads: exclusive scan of ntiles tile sums.
// New size of a resampling in a schedule on the device: 0 and sizes above
// the capacity stop the schedule (the first such step is recorded) and
// leave no replicas for the kernels after it; once it has stopped, every
// size is 0.
__device__ __forceinline__ unsigned long long checked_total(
    unsigned long long t, int64_t cap, AnnealHalt* halt, uint32_t step) {
  if (!halt) return t;
  if (halt->code != 0u) return 0ull;
  if (t != 0ull && t <= (unsigned long long)cap) return t;
  halt->code = t ? kHaltCapacity : kHaltEmpty;
  halt->step = step;
  halt->total = t;
  return 0ull;
}

__global__ __launch_bounds__(1024) void k_scan(const uint32_t* tile_sum,
                                               uint32_t* tile_off,
                                               int64_t ntiles,
                                               unsigned long long* total,
                                               int64_t cap,
                                               AnnealHalt* halt,
                                               uint32_t step) {
  __shared__ unsigned long long part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (ntiles + 1023) / 1024;
  const int64_t b = tid * per;
  const int64_t e = (b + per < ntiles) ? b + per : ntiles;
  unsigned long long s = 0ull;
  for (int64_t i = b; i < e; ++i) s += tile_sum[i];
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    unsigned long long v = (tid >= off) ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  unsigned long long run = part[tid] - s;
  for (int64_t i = b; i < e; ++i) {
    tile_off[i] = (uint32_t)run;
    run += tile_sum[i];
  }
  if (tid == 1023) *total = checked_total(part[1023], cap, halt, step);
}

__global__ __launch_bounds__(256) void k_scatter(
    const uint32_t* n, const uint32_t* tile_off, int64_t R, int64_t cap,
    uint32_t* parent, const uint32_t* fam_src, uint32_t* fam_dst,
    const unsigned long long* Rdev) {
  __shared__ uint32_t lds[8];
  if (Rdev) R = min((int64_t)*Rdev, R);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nj = (j < R) ? n[j] : 0u;
  uint32_t total;
  const uint32_t ex = block_excl_scan(nj, lds, &total);
  const int64_t o = (int64_t)tile_off[blockIdx.x] + ex;
  const uint32_t fj = (nj && fam_src) ? fam_src[j] : 0u;
  for (uint32_t t = 0; t < nj; ++t)
    if (o + t < cap) {
      parent[o + t] = (uint32_t)j;
      if (fam_dst) fam_dst[o + t] = fj;
    }
}

// The parent map of a population of at most kScatterTiles tiles without a
// scan of its own: every workgroup sums the tile sums before its tile (in
// tile order, as k_scan does), and workgroup 0 also the total, the new size.
constexpr int kScatterTiles = 256;

__global__ __launch_bounds__(256) void k_scatter_scan(
    const uint32_t* n, const uint32_t* tile_sum, int64_t ntiles, int64_t R,
    int64_t cap, uint32_t* parent, const uint32_t* fam_src, uint32_t* fam_dst,
    unsigned long long* total_out) {
  __shared__ uint32_t lds[8];
  __shared__ uint32_t base_sh;
  // the tile sums before this tile, one per lane, then summed
  const uint32_t v = (threadIdx.x < blockIdx.x) ? tile_sum[threadIdx.x] : 0u;
  uint32_t before;
  (void)block_excl_scan(v, lds, &before);
  if (threadIdx.x == 0) base_sh = before;
  __syncthreads();
  if (blockIdx.x == 0) {
    const uint32_t w = (threadIdx.x < ntiles) ? tile_sum[threadIdx.x] : 0u;
    uint32_t all;
    (void)block_excl_scan(w, lds, &all);
    if (threadIdx.x == 0) *total_out = all;
  }
  __syncthreads();  // every wave has read lds before its next use
  const uint32_t base = base_sh;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nj = (j < R) ? n[j] : 0u;
  uint32_t tile_total;
  const uint32_t ex = block_excl_scan(nj, lds, &tile_total);
  const int64_t o = (int64_t)base + ex;
  const uint32_t fj = (nj && fam_src) ? fam_src[j] : 0u;
  for (uint32_t t = 0; t < nj; ++t)
    if (o + t < cap) {
      parent[o + t] = (uint32_t)j;
      if (fam_dst) fam_dst[o + t] = fj;
    }
}

// ------------------------------------------ single-pass counts and scatter

// Polls of an earlier tile's status before the wait gives up (each poll
// sleeps about 64 cycles first: some tens of milliseconds in all).
constexpr int kLookbackPolls = 1 << 20;

// Status word of a tile: the launch's generation (28 bits), the kind (1:
// the tile's own sum, 2: the inclusive prefix through it) and the value (34
// bits: sizes stay below 2^33, the capacity being below 2^32).
constexpr unsigned long long kLbValue = (1ull << 34) - 1ull;
__device__ __forceinline__ unsigned long long lb_word(uint32_t gen,
                                                      uint32_t kind,
                                                      unsigned long long v) {
  return ((unsigned long long)gen << 36) | ((unsigned long long)kind << 34) |
         (v & kLbValue);
}

// Copy counts of a tile of 256 replicas, the exclusive prefix of the tile
// sums before it and the parent of every new slot of the tile, in one pass.
// The tile is the workgroup's ticket, so every earlier tile belongs to a
// workgroup that has already started; a workgroup publishes its tile's sum
// before it waits for anything, and waits only for earlier tiles.
__global__ __launch_bounds__(256) void k_counts_scatter(CountsArgs a0,
                                                        LookbackArgs s) {
  __shared__ uint32_t lds[8];
  __shared__ uint32_t s_tile;
  __shared__ unsigned long long s_prefix;
  if (threadIdx.x == 0) s_tile = atomicAdd(s.ticket, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  CountsArgs a = a0;
  if (a0.Rdev) a.R = min((int64_t)*a0.Rdev, a0.R);
  if (a0.lvl_dev) {
    a.lvl0 = a0.lvl_dev[0];
    a.nlvl = a0.lvl_dev[1];
  }
  const int64_t j = (int64_t)tile * blockDim.x + threadIdx.x;
  for (int64_t i = j; i < a.nclear; i += s.ntiles * blockDim.x)
    a.clear[i] = 0u;
  const uint32_t fj = (j < a.R && s.fam_src) ? s.fam_src[j] : 0u;
  uint32_t nj = 0u;
  if (j < a.R) {
    nj = count_of(a, j, a.f, a.T);
    a.n[j] = nj;
  }
  uint32_t agg;
  const uint32_t ex = block_excl_scan(nj, lds, &agg);
  const uint32_t gen = s.gen & 0x0FFFFFFFu;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (tile == 0) {
      if (lane == 0) {
        __hip_atomic_store(&s.status[0], lb_word(gen, 2u, agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_prefix = 0ull;
      }
    } else {
      if (lane == 0)
        __hip_atomic_store(&s.status[tile], lb_word(gen, 1u, agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned long long prefix = 0ull;
      bool failed = false;
      // windows of 64 earlier tiles, lane 0 the nearest, until one of them
      // holds an inclusive prefix (tile 0 always does)
      for (int64_t end = tile; end > 0; end -= 64) {
        const int64_t p = end - 1 - lane;
        unsigned long long w = 0ull;
        bool ready = p < 0;
        for (int k = 0; !ready && k < kLookbackPolls; ++k) {
          w = __hip_atomic_load(&s.status[p], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
          ready = (uint32_t)(w >> 36) == gen && ((w >> 34) & 3ull) != 0ull;
          if (!ready) __builtin_amdgcn_s_sleep(1);
        }
        if (!__all(ready)) {
          failed = true;
          break;
        }
        const bool incl = p >= 0 && ((w >> 34) & 3ull) == 2ull;
        const unsigned long long im = __ballot(incl);
        // the lanes up to the nearest inclusive prefix, or the whole window
        const int upto = im ? __builtin_ctzll(im) : 63;
        unsigned long long v =
            (p >= 0 && lane <= upto) ? (w & kLbValue) : 0ull;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        prefix += v;
        if (im) break;
      }
      if (lane == 0) {
        if (failed) {
          if (atomicCAS(&s.halt->code, 0u, (uint32_t)kHaltWait) == 0u)
            s.halt->step = s.step;
          prefix = 0ull;
        }
        __hip_atomic_store(&s.status[tile], lb_word(gen, 2u, prefix + agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_prefix = prefix;
      }
    }
  }
  __syncthreads();
  const unsigned long long base = s_prefix;
  const int64_t o = (int64_t)(base + ex);
  for (uint32_t t = 0; t < nj; ++t)
    if (o + t < s.cap) {
      s.parent[o + t] = (uint32_t)j;
      if (s.fam_dst) s.fam_dst[o + t] = fj;
    }
  if (threadIdx.x == 0) {
    if (tile == (uint32_t)(s.ntiles - 1))
      *s.total = checked_total(base + agg, s.cap, s.halt, s.step);
    if (atomicAdd(s.done, 1u) == (uint32_t)(s.ntiles - 1)) {
      *s.ticket = 0u;
      *s.done = 0u;
    }
  }
}

// ---------------------------------------------------------------- gather

// Replicas of at least 64 units (1 KB): one wave per new slot, each lane
// copying every 64th 16-byte unit, one parent index per lane.
__global__ __launch_bounds__(256) void k_gather(GatherArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (k >= a.R_new) return;
  const uint32_t p = a.parent[k];
  const uint4* src = reinterpret_cast<const uint4*>(a.src + (size_t)p * a.stride);
  uint4* dst = reinterpret_cast<uint4*>(a.dst + (size_t)k * a.stride);
  for (int c = lane; c < a.chunks; c += 64) dst[c] = src[c];
  if (lane == 0) {
    a.E_dst[k] = a.E_src[p];
    a.M_dst[k] = a.M_src[p];
  }
}

// Smaller replicas: the copies as one flat array of 16-byte units (new slot
// k, chunk c); a workgroup copies a contiguous tile of 1024 units,
// consecutive threads take consecutive units, and every thread has four
// units in flight (all loads before the stores).
__global__ __launch_bounds__(256) void k_gather_flat(GatherArgs a) {
  constexpr int U = 4;
  const int64_t total = a.R_new * (int64_t)a.chunks;
  // each workgroup copies one contiguous tile of U * 256 units
  const int64_t stride = blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * (U * 256) + threadIdx.x;
  uint4 v[U];
  int64_t k[U];
  int c[U];
  uint32_t p[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t it = first + u * stride;
    if (it >= total) {
      k[u] = -1;
      c[u] = 0;
    } else if (a.chunks_log2 >= 0) {  // every benchmark layout
      k[u] = it >> a.chunks_log2;
      c[u] = (int)(it & ((1 << a.chunks_log2) - 1));
    } else {
      k[u] = it / a.chunks;
      c[u] = (int)(it - k[u] * a.chunks);
    }
    p[u] = k[u] >= 0 ? a.parent[k[u]] : 0u;
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (k[u] >= 0)
      v[u] = reinterpret_cast<const uint4*>(a.src + (size_t)p[u] * a.stride)[c[u]];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k[u] < 0) continue;
    reinterpret_cast<uint4*>(a.dst + (size_t)k[u] * a.stride)[c[u]] = v[u];
    if (c[u] == 0) {
      a.E_dst[k[u]] = a.E_src[p[u]];
      a.M_dst[k[u]] = a.M_src[p[u]];
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// p[i] = i: every replica founds its own family.
__global__ void k_iota_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

// --------------------------------------------------------------- launchers

template <int W, int RPL, bool PLANES>
static hipError_t launch_lattice_w(const LatticeArgs& a, bool int8, bool glass,
                                   dim3 grid, hipStream_t st) {
  if (int8) {
    if (glass) hipLaunchKernelGGL((k_lattice<W, RPL, true, true, PLANES>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_lattice<W, RPL, true, false, PLANES>), grid, dim3(256), 0, st, a);
  } else {
    if (glass) hipLaunchKernelGGL((k_lattice<W, RPL, false, true, PLANES>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_lattice<W, RPL, false, false, PLANES>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template <int W, int RPL>
static hipError_t launch_lattice_p(const LatticeArgs& a, bool int8, bool glass,
                                   bool planes, dim3 grid, hipStream_t st) {
  return planes ? launch_lattice_w<W, RPL, true>(a, int8, glass, grid, st)
                : launch_lattice_w<W, RPL, false>(a, int8, glass, grid, st);
}

hipError_t launch_lattice(const LatticeArgs& a, int W, int RPL, bool int8,
                          bool glass, bool planes, hipStream_t st) {
  const int64_t waves = (a.R + a.rpw - 1) / a.rpw;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  switch (W * 8 + RPL) {
    case 1 * 8 + 1: return launch_lattice_p<1, 1>(a, int8, glass, planes, grid, st);
    case 1 * 8 + 2: return launch_lattice_p<1, 2>(a, int8, glass, planes, grid, st);
    case 1 * 8 + 3: return launch_lattice_p<1, 3>(a, int8, glass, planes, grid, st);
    case 1 * 8 + 4: return launch_lattice_p<1, 4>(a, int8, glass, planes, grid, st);
    case 2 * 8 + 1: return launch_lattice_p<2, 1>(a, int8, glass, planes, grid, st);
    case 2 * 8 + 2: return launch_lattice_p<2, 2>(a, int8, glass, planes, grid, st);
    case 2 * 8 + 3: return launch_lattice_p<2, 3>(a, int8, glass, planes, grid, st);
    case 2 * 8 + 4: return launch_lattice_p<2, 4>(a, int8, glass, planes, grid, st);
    case 3 * 8 + 2: return launch_lattice_p<3, 2>(a, int8, glass, planes, grid, st);
    case 3 * 8 + 3: return launch_lattice_p<3, 3>(a, int8, glass, planes, grid, st);
    case 3 * 8 + 4: return launch_lattice_p<3, 4>(a, int8, glass, planes, grid, st);
    case 4 * 8 + 2: return launch_lattice_p<4, 2>(a, int8, glass, planes, grid, st);
    case 4 * 8 + 3: return launch_lattice_p<4, 3>(a, int8, glass, planes, grid, st);
    case 4 * 8 + 4: return launch_lattice_p<4, 4>(a, int8, glass, planes, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hist(const HistArgs& a, hipStream_t st) {
  // at most one workgroup per compute unit, each over kHistU or more
  // replicas per lane: the window merge and the moment atomics are per
  // workgroup
  int64_t blocks = (a.R + 256 * kHistU - 1) / (256 * kHistU);
  if (blocks < 1) blocks = 1;
  if (blocks > 256) blocks = 256;
  if (a.win_n < 0 || a.win_n > 16384 || a.win_lo < 0 ||
      a.win_lo + a.win_n > a.nbins)
    return hipErrorInvalidValue;
  const size_t shm = (size_t)a.win_n * sizeof(uint32_t);
  hipLaunchKernelGGL(k_hist, dim3((unsigned)blocks), dim3(256), shm, st, a);
  return hipGetLastError();
}

hipError_t launch_hist_sched(const HistArgs& a, const ArgWeights& w,
                             hipStream_t st) {
  int64_t blocks = (a.R + 256 * kHistU - 1) / (256 * kHistU);
  if (blocks < 1) blocks = 1;
  if (blocks > 256) blocks = 256;
  if (a.win_n < 0 || a.win_n > 16384 || a.win_lo < 0 ||
      a.win_lo + a.win_n > a.nbins || !a.rec || !a.part || !a.halt || !a.Rw)
    return hipErrorInvalidValue;
  // LDS: the window, then the table tail's terms (kTermPiece doubles)
  const size_t shm = std::max((size_t)a.win_n * sizeof(uint32_t),
                              (size_t)kTermPiece * sizeof(double));
  hipLaunchKernelGGL(k_hist_sched, dim3((unsigned)blocks), dim3(256), shm, st,
                     a, w);
  return hipGetLastError();
}

hipError_t launch_counts_args(const CountsArgs& a, const ArgTables& t,
                              hipStream_t st) {
  if (a.nlvl > kArgLevels || a.poisson) return hipErrorInvalidValue;
  const int64_t blocks = (a.R + 255) / 256;
  hipLaunchKernelGGL(k_counts_args, dim3((unsigned)blocks), dim3(256), 0, st,
                     a, t);
  return hipGetLastError();
}

hipError_t launch_scatter_scan(const uint32_t* n, const uint32_t* tile_sum,
                               int64_t R, int64_t cap, uint32_t* parent,
                               const uint32_t* fam_src, uint32_t* fam_dst,
                               unsigned long long* total, hipStream_t st) {
  const int64_t blocks = (R + 255) / 256;
  if (blocks > kScatterTiles) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scatter_scan, dim3((unsigned)(blocks ? blocks : 1)),
                     dim3(256), 0, st, n, tile_sum, blocks, R, cap, parent,
                     fam_src, fam_dst, total);
  return hipGetLastError();
}

hipError_t launch_counts_scatter(const CountsArgs& a, const LookbackArgs& s,
                                 hipStream_t st) {
  const int64_t blocks = (a.R + 255) / 256;
  if (blocks != s.ntiles || blocks <= 0 || blocks > kLookbackTiles ||
      s.cap >= (1ll << 32) || a.poisson || !s.halt || !s.total ||
      !s.status || !s.ticket || !s.done)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_counts_scatter, dim3((unsigned)blocks), dim3(256), 0,
                     st, a, s);
  return hipGetLastError();
}

hipError_t launch_scan_dev(const uint32_t* tile_sum, uint32_t* tile_off,
                           int64_t ntiles, unsigned long long* total,
                           int64_t cap, AnnealHalt* halt, uint32_t step,
                           hipStream_t st) {
  if (!halt) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tile_sum, tile_off,
                     ntiles, total, cap, halt, step);
  return hipGetLastError();
}

hipError_t launch_scatter_dev(const uint32_t* n, const uint32_t* tile_off,
                              int64_t R, const unsigned long long* Rdev,
                              int64_t cap, uint32_t* parent,
                              const uint32_t* fam_src, uint32_t* fam_dst,
                              hipStream_t st) {
  const int64_t blocks = (R + 255) / 256;
  if (!Rdev) return hipErrorInvalidValue;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, st, n,
                     tile_off, R, cap, parent, fam_src, fam_dst, Rdev);
  return hipGetLastError();
}

hipError_t launch_counts(const CountsArgs& a, hipStream_t st) {
  const int64_t blocks = (a.R + 255) / 256;
  hipLaunchKernelGGL(k_counts, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sys_counts(const CountsArgs& a, uint64_t* tile64,
                             uint64_t* off64, hipStream_t st) {
  const int64_t blocks = (a.R + 255) / 256;
  hipLaunchKernelGGL(k_sys_tiles, dim3((unsigned)blocks), dim3(256), 0, st, a,
                     tile64);
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, tile64, off64,
                     blocks);
  hipLaunchKernelGGL(k_sys_counts, dim3((unsigned)blocks), dim3(256), 0, st, a,
                     off64);
  return hipGetLastError();
}

hipError_t launch_multi_counts(const CountsArgs& a, int64_t draws,
                               uint64_t* tile64, uint64_t* off64,
                               uint64_t* cum, hipStream_t st) {
  const int64_t blocks = (a.R + 255) / 256;
  hipLaunchKernelGGL(k_sys_tiles, dim3((unsigned)blocks), dim3(256), 0, st, a,
                     tile64);
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, tile64, off64,
                     blocks);
  hipLaunchKernelGGL(k_multi_cum, dim3((unsigned)blocks), dim3(256), 0, st, a,
                     off64, cum);
  if (draws > 0)  // the host passes no draws when the weights are all zero
    hipLaunchKernelGGL(k_multi_draw, dim3((unsigned)((draws + 255) / 256)),
                       dim3(256), 0, st, a, cum, draws);
  hipLaunchKernelGGL(k_count_tiles, dim3((unsigned)blocks), dim3(256), 0, st,
                     a);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* tile_sum, uint32_t* tile_off,
                       int64_t ntiles, unsigned long long* total,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tile_sum, tile_off,
                     ntiles, total, (int64_t)0, (AnnealHalt*)nullptr, 0u);
  return hipGetLastError();
}

hipError_t launch_scatter(const uint32_t* n, const uint32_t* tile_off,
                          int64_t R, int64_t cap, uint32_t* parent,
                          const uint32_t* fam_src, uint32_t* fam_dst,
                          hipStream_t st) {
  const int64_t blocks = (R + 255) / 256;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, st, n,
                     tile_off, R, cap, parent, fam_src, fam_dst,
                     (const unsigned long long*)nullptr);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t st) {
  if (a.R_new <= 0) return hipSuccess;
  if (a.chunks >= 64) {
    const int64_t blocks = (a.R_new + 3) / 4;  // four slots per workgroup
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, st, a);
  } else {
    const int64_t units = a.R_new * (int64_t)a.chunks;
    const int64_t blocks = (units + 4 * 256 - 1) / (4 * 256);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_flat, dim3((unsigned)blocks), dim3(256), 0, st,
                       a);
  }
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_iota_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace pa
