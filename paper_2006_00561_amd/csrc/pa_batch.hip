// Batched population annealing: many independent populations (uneven L and
// R, ferromagnets and +-J glasses) advanced together, one set of launches
// per temperature step for all of them.
//
// Each population is the method of the paper's Sec. 2 on its own (its own
// Philox key and population id, its own schedule, its own ln Z), so every
// population's trajectory is bit for bit the one the single-population path
// (pa_init / pa_resample / pa_sweep) produces.  What changes is the launch
// structure:
//   - segmented kernels (grid y = population) for the histogram, copy
//     counts, scan and parent scatter, reading every population's size from
//     device memory;
//   - one persistent sweep kernel per row-width class that pulls (population,
//     wave) work items from a device queue, largest lattices first, and
//     loads every new slot straight from its parent (the resampling copy
//     costs no pass of its own; a separate gather runs only for populations
//     without sweeps at the new temperature);
//   - one device->host copy of all histograms, one host function building
//     every population's double-precision tables (and next beta), one
//     host->device copy of all tables per step;
//   - the kernels before and after the host function have no host-side size
//     dependence, so each sequence is captured once as a HIP graph of kernel
//     nodes and replayed every step; the two copies and the host function
//     run between the two graph launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <exception>
#include <new>
#include <numeric>
#include <tuple>
#include <vector>

#include "pa.h"
#include "pa_device.h"
#include "pa_internal.h"
#include "pa_lattice.h"
#include "pa_potts.h"

namespace pa {

// Sweep classes: one per lattice variant (row words W, rows per lane, spin
// layout, model), so a persistent launch carries the code of one variant.
// Sweep classes: 64 Ising variants (W, rows per lane, layout, model), then
// the Potts pass for L = 8, 16, 32, 64, 128.
constexpr int kIsingClasses = 128;
constexpr int kClasses = kIsingClasses + 5;
__host__ __device__ constexpr int sweep_class(int W, int rpl, int int8,
                                              int glass, int planes) {
  return ((((W - 1) * 4 + (rpl - 1)) * 2 + int8) * 2 + glass) + 64 * planes;
}
__host__ __device__ constexpr int potts_class(int mpr) {
  return kIsingClasses + (mpr == 1 ? 0 : mpr == 2 ? 1 : mpr == 4 ? 2 : mpr == 8 ? 3 : 4);
}

// -------------------------------------------------------------- kernels

// One-dimensional grid: gx workgroups of 2048 replicas per population.
__global__ __launch_bounds__(256) void k_bhist(const BatchPop* P,
                                               const int64_t* R,
                                               const int32_t* cur,
                                               unsigned long long* mom,
                                               unsigned long long* flags,
                                               int lds_bins, int gx) {
  extern __shared__ uint32_t sh[];
  const int p = blockIdx.x / gx;
  const int bx = blockIdx.x - p * gx;
  const int64_t Rp = R[p];
  if ((int64_t)bx * 256 * 8 >= Rp) return;  // whole block
  const BatchPop& q = P[p];
  const int c = cur[p];
  const int32_t* E = q.E[c];
  const int32_t* M = q.M[c];
  const int twoN = 2 * q.L * q.L;
  const bool lds = q.nbins <= lds_bins;
  if (lds) {
    for (int i = threadIdx.x; i < q.nbins; i += blockDim.x) sh[i] = 0u;
    __syncthreads();
  }
  unsigned long long sam = 0ull, sm2 = 0ull;
  const int64_t j0 = (int64_t)bx * 256 * 8;
  const int64_t j1 = min(j0 + 256 * 8, Rp);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const int idx = (E[j] + twoN) >> q.shift;
    if (idx < 0 || idx >= q.nbins) {
      atomicAdd(&flags[0], 1ull);
      continue;
    }
    if (lds) atomicAdd(&sh[idx], 1u);
    else atomicAdd(&q.hist[idx], 1u);
    const int m = M[j];
    sam += (unsigned long long)(m < 0 ? -m : m);
    sm2 += (unsigned long long)((long long)m * m);
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < q.nbins; i += blockDim.x)
      if (sh[i]) atomicAdd(&q.hist[i], sh[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sam += __shfl_down(sam, off, 64);
    sm2 += __shfl_down(sm2, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&mom[2 * p], sam);
    atomicAdd(&mom[2 * p + 1], sm2);
  }
}

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v,
                                                       uint32_t* lds,
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
  for (int i = 0; i < 4; ++i) {
    const uint32_t x = lds[i];
    if (i < wid) wbase += x;
    tot += x;
  }
  *total = tot;
  return wbase + incl - v;
}

__global__ __launch_bounds__(256) void k_bcounts(const BatchPop* P,
                                                 const BatchStep* S,
                                                 const int64_t* R,
                                                 const int32_t* cur) {
  __shared__ uint32_t lds[4];
  const int p = blockIdx.y;
  const int64_t Rp = R[p];
  if (!S[p].active || (int64_t)blockIdx.x * 256 >= Rp) return;  // whole block
  const BatchPop& q = P[p];
  const BatchStep& st = S[p];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t nj = 0u;
  if (j < Rp) {
    const int32_t* E = q.E[cur[p]];
    const int l = ((E[j] + 2 * q.L * q.L) >> q.shift) - st.lvl0;
    const uint4 b = philox10(make_uint4(kDomainResample << 28, st.step << 16,
                                        (uint32_t)j, q.pop),
                             q.k0, q.k1);
    if (l >= 0 && l < st.nlvl)
      nj = q.tab[l] + (b.x < q.tab[q.nbins + l] ? 1u : 0u);
    q.n[j] = nj;
  }
  uint32_t total;
  (void)block_excl_scan256(nj, lds, &total);
  if (threadIdx.x == 0) q.tile_sum[blockIdx.x] = total;
}

// One workgroup per population: scan of its tile sums, its new size.
__global__ __launch_bounds__(1024) void k_bscan(const BatchPop* P,
                                                const BatchStep* S,
                                                const int64_t* R,
                                                int64_t* Rnew,
                                                unsigned long long* flags) {
  __shared__ unsigned long long part[1024];
  const int p = blockIdx.x;
  if (!S[p].active) {
    if (threadIdx.x == 0) Rnew[p] = R[p];
    return;
  }
  const BatchPop& q = P[p];
  const int tid = threadIdx.x;
  const int64_t ntiles = (R[p] + 255) / 256;
  const int64_t per = (ntiles + 1023) / 1024;
  const int64_t b = tid * per;
  const int64_t e = (b + per < ntiles) ? b + per : ntiles;
  unsigned long long s = 0ull;
  for (int64_t i = b; i < e; ++i) s += q.tile_sum[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned long long v = (tid >= off) ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  unsigned long long run = part[tid] - s;
  for (int64_t i = b; i < e; ++i) {
    q.tile_off[i] = (uint32_t)run;
    run += q.tile_sum[i];
  }
  if (tid == 1023) {
    const int64_t tot = (int64_t)part[1023];
    Rnew[p] = tot;
    if (tot > q.cap) atomicOr(&flags[1], 1ull);
    if (tot == 0) atomicOr(&flags[1], 2ull);
  }
}

__global__ __launch_bounds__(256) void k_bscatter(const BatchPop* P,
                                                  const BatchStep* S,
                                                  const int64_t* R,
                                                  const int32_t* cur) {
  __shared__ uint32_t lds[4];
  const int p = blockIdx.y;
  const int64_t Rp = R[p];
  if (!S[p].active || (int64_t)blockIdx.x * 256 >= Rp) return;  // whole block
  const BatchPop& q = P[p];
  const int c = cur[p];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t nj = (j < Rp) ? q.n[j] : 0u;
  uint32_t total;
  const uint32_t ex = block_excl_scan256(nj, lds, &total);
  const int64_t o = (int64_t)q.tile_off[blockIdx.x] + ex;
  // a copy joins its parent's family (the other family buffer becomes
  // current when the commit adopts the new population)
  const uint32_t fj = nj ? q.fam[c][j] : 0u;
  for (uint32_t t = 0; t < nj; ++t)
    if (o + t < q.cap) {
      q.parent[o + t] = (uint32_t)j;
      q.fam[c ^ 1][o + t] = fj;
    }
}

// Grid-stride over row groups of every population (grid y = population).
// Only populations without sweeps at the new temperature: the sweep kernel
// reads every other population's new slots from their parents directly.
__global__ __launch_bounds__(256) void k_bgather(const BatchPop* P,
                                                 const BatchStep* S,
                                                 const int64_t* Rnew,
                                                 const int32_t* cur) {
  const int p = blockIdx.y;
  if (!S[p].active || S[p].theta > 0) return;
  const BatchPop& q = P[p];
  const int64_t Rn = min(Rnew[p], q.cap);
  const int c = cur[p];
  const int lane = threadIdx.x & 63;
  const int sub = lane >> q.lpr_log2;
  const int c0 = lane & ((1 << q.lpr_log2) - 1);
  const int64_t rows_per_wave = 64 >> q.lpr_log2;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
       w * rows_per_wave < Rn; w += waves) {
    const int64_t k = w * rows_per_wave + sub;
    if (k >= Rn) continue;
    const uint32_t par = q.parent[k];
    const uint4* src =
        reinterpret_cast<const uint4*>(q.spins[c] + (size_t)par * q.stride);
    uint4* dst = reinterpret_cast<uint4*>(q.spins[c ^ 1] + (size_t)k * q.stride);
    for (int ch = c0; ch < q.chunks; ch += (1 << q.lpr_log2)) dst[ch] = src[ch];
    if (c0 == 0) {
      q.E[c ^ 1][k] = q.E[c][par];
      q.M[c ^ 1][k] = q.M[c][par];
    }
  }
}

// Single workgroup: adopt the new populations, then lay out the sweep work
// queue (items = waves of rpw replicas) of every sweep class, in the sorted
// population order (class c's prefix sums sit at first_c + c + i).
__global__ __launch_bounds__(256) void k_bcommit(
    const BatchPop* P, const BatchStep* S, int64_t* R, const int64_t* Rnew,
    int32_t* cur, const int32_t* order, int n, const int32_t* cls_first,
    const int32_t* cls_count, int64_t* prefix, unsigned long long* queue,
    int commit) {
  if (commit) {
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
      if (!S[p].active) continue;
      const int64_t rn = Rnew[p];
      if (rn >= 1 && rn <= P[p].cap) {
        R[p] = rn;
        cur[p] ^= 1;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kClasses && cls_count[threadIdx.x] > 0) {
    const int w = threadIdx.x;
    int64_t acc = 0;
    const int f = cls_first[w];
    for (int i = 0; i < cls_count[w]; ++i) {
      const int p = order[f + i];
      prefix[f + w + i] = acc;
      if (S[p].active && S[p].theta > 0) acc += (R[p] + P[p].rpw - 1) / P[p].rpw;
    }
    prefix[f + w + cls_count[w]] = acc;
    queue[w] = 0ull;
  }
}

// Histogram summaries of every population (one workgroup each), from its
// exact energy histogram: mean/N, log of the energy standard deviation,
// skewness, (Emin - mean)/sd, beta, log N, log R and the overlap target.
// Double precision, rounded to FP32 for the network.
__global__ __launch_bounds__(256) void k_bfeatures(const BatchPop* P,
                                                   const BatchStep* S,
                                                   const int64_t* R,
                                                   float* feat) {
  __shared__ double red[256];
  __shared__ int mn[256];
  const int p = blockIdx.x;
  const BatchPop& q = P[p];
  const int N = q.L * q.L;
  const double Rd = (double)R[p];
  auto level = [&](int i) { return (double)(-2 * N + (i << q.shift)); };
  auto block_sum = [&](double v) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };
  double s1 = 0.0;
  int imin = q.nbins;
  for (int i = threadIdx.x; i < q.nbins; i += 256) {
    const uint32_t h = q.hist[i];
    if (h) {
      s1 += (double)h * level(i);
      imin = min(imin, i);
    }
  }
  mn[threadIdx.x] = imin;
  const double mean = block_sum(s1) / Rd;
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      mn[threadIdx.x] = min(mn[threadIdx.x], mn[threadIdx.x + off]);
    __syncthreads();
  }
  const int i0 = mn[0];
  double s2 = 0.0, s3 = 0.0;
  for (int i = threadIdx.x; i < q.nbins; i += 256) {
    const uint32_t h = q.hist[i];
    if (h) {
      const double d = level(i) - mean;
      s2 += (double)h * d * d;
      s3 += (double)h * d * d * d;
    }
  }
  const double var = block_sum(s2) / Rd;
  const double m3 = block_sum(s3) / Rd;
  if (threadIdx.x == 0) {
    const double sd = sqrt(var > 1e-3 ? var : 1e-3);
    float* f = feat + (size_t)p * kFeatures;
    f[0] = (float)(mean / N);
    f[1] = (float)log(sd);
    f[2] = (float)(var > 0.0 ? m3 / (var * sqrt(var)) : 0.0);
    f[3] = (float)((level(i0) - mean) / sd);
    f[4] = (float)S[p].beta;
    f[5] = (float)log((double)N);
    f[6] = (float)log(Rd);
    f[7] = (float)S[p].target;
  }
}

// log dbeta proposals of the network (de-standardised) next to the features.
__global__ void k_bpred(const float* z, float* pred, int n, float mu_y,
                        float sigma_y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) pred[p] = mu_y + sigma_y * z[p];
}

// Persistent sweep kernel of one lattice variant: every wave pulls work
// items (population, wave of replicas) from the class queue until the queue
// is exhausted; every wave reaches the exit once the counter passes the
// total, which k_bcommit fixed before the launch.
template <int W, int RPL, bool INT8, bool GLASS, bool PLANES>
__global__ __launch_bounds__(256) void k_bsweep(
    const BatchPop* P, const BatchStep* S, const int64_t* R,
    const int32_t* cur, const int32_t* order, const int64_t* prefix,
    unsigned long long* queue, int first, int count, int chunk,
    uint32_t one) {
  constexpr int cls =
      sweep_class(W, RPL, INT8 ? 1 : 0, GLASS ? 1 : 0, PLANES ? 1 : 0);
  const int lane = threadIdx.x & 63;
  const int64_t* pre = prefix + first + cls;
  const int64_t total = pre[count];
  // items are taken `chunk` at a time: one atomic per chunk
  int64_t item = 0, end = 0;
  while (true) {
    if (item == end) {
      int it = 0;
      if (lane == 0) it = (int)atomicAdd(&queue[cls], (unsigned long long)chunk);
      item = (int64_t)__shfl(it, 0, 64);
      end = item + chunk;
    }
    if (item >= total) break;
    const int64_t this_item = item++;
    int lo = 0, hi = count - 1;  // last i with pre[i] <= this_item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= this_item) lo = mid;
      else hi = mid - 1;
    }
    const int p = order[first + lo];
    const BatchPop& q = P[p];
    const BatchStep& st = S[p];
    const int c = cur[p];
    LatticeArgs a;
    // the population was resampled at this step (k_bcommit made buffer c
    // current): each new slot is read from its parent in buffer c ^ 1
    a.spins = q.spins[c];
    a.src = q.spins[c ^ 1];
    a.parent = q.parent;
    a.Rdev = nullptr;
    a.E = q.E[c];
    a.M = q.M[c];
    a.jbits = q.jbits;
    a.R = R[p];
    a.stride = q.stride;
    a.L = q.L;
    a.lpr = q.lpr;
    a.rpw = q.rpw;
    a.K4 = st.K4;
    a.K8 = st.K8;
    a.one = one;
    a.k0 = q.k0;
    a.k1 = q.k1;
    a.pop = q.pop;
    a.step = st.step;
    a.t0 = 0;
    a.theta = st.theta;
    a.init = 0;
    lattice_pass<W, RPL, INT8, GLASS, PLANES>(a, this_item - pre[lo]);
  }
}

// Persistent Potts pass of one lattice size, with up to four waves per
// workgroup as in the single-population kernel: each wave takes one replica
// (rpw = 1), all the workgroup's waves run the pass together (its barriers
// are the workgroup's; each wave keeps its own threshold table), and a wave
// past the queue's end runs the pass inactive.  Thread 0 takes one item per
// wave with a single atomic and shares the base through LDS; the loop ends
// for the whole workgroup at once, when the base passes the total.
template <int MPR>
__global__ __launch_bounds__(256) void k_bpotts(
    const BatchPop* P, const BatchStep* S, const int64_t* R,
    const int32_t* cur, const int32_t* order, const int64_t* prefix,
    unsigned long long* queue, int first, int count, uint32_t one) {
  extern __shared__ uint32_t lds_words[];
  __shared__ unsigned long long s_base;
  constexpr int cls = potts_class(MPR);
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int64_t* pre = prefix + first + cls;
  const int64_t total = pre[count];
  while (true) {
    if (threadIdx.x == 0)
      s_base = atomicAdd(&queue[cls], (unsigned long long)wpb);
    __syncthreads();
    const int64_t base = (int64_t)s_base;
    __syncthreads();  // every wave has read the base before the next take
    if (base >= total) break;
    const int64_t mine = base + wave;
    const bool active = mine < total;
    // an inactive wave looks up a valid item (the base) for its arguments
    const int64_t it = (int64_t)__builtin_amdgcn_readfirstlane(
        (uint32_t)(active ? mine : base));
    int lo = 0, hi = count - 1;  // last i with pre[i] <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int p = __builtin_amdgcn_readfirstlane(order[first + lo]);
    const BatchPop& q = P[p];
    const BatchStep& st = S[p];
    const int c = cur[p];
    LatticeArgs a{};
    a.spins = q.spins[c];
    a.src = q.spins[c ^ 1];  // every new slot reads its parent
    a.parent = q.parent;
    a.Rdev = nullptr;
    a.E = q.E[c];
    a.M = q.M[c];
    a.R = R[p];
    a.stride = q.stride;
    a.L = q.L;
    a.one = one;
    a.k0 = q.k0;
    a.k1 = q.k1;
    a.pop = q.pop;
    a.step = st.step;
    a.t0 = 0;
    a.theta = st.theta;
    a.init = 0;
    a.q = q.q;
    for (int d = 0; d < 4; ++d) a.Tp[d] = st.Tp[d];
    potts_swar_pass<MPR>(a, it - pre[lo], active, lds_words);
    __syncthreads();  // the next items overwrite the tables and lattices
  }
}

}  // namespace pa

using namespace pa;

// ================================================================= host

namespace {

struct PopHost {
  BatchPop d;        // the device description (pointers into the arenas)
  int64_t R_t = 0;
  int N = 0, model = 0;
  double beta = 0.0, lnZ = 0.0, lnQ_last = 0.0;
  int step = 0;
  size_t rb_hist = 0;  // offset of the histogram in the readback block
  int moved = 0;       // the population moved in the previous step
  size_t up_tab = 0;   // offset of the tables in the upload block
};

struct TuneKey {
  int L, layout, model, rng_mode;
  bool operator<(const TuneKey& o) const {
    return std::tie(L, layout, model, rng_mode) <
           std::tie(o.L, o.layout, o.model, o.rng_mode);
  }
};
}  // namespace

struct pa_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n = 0;
  std::vector<PopHost> pops;
  BatchPop* d_pops = nullptr;
  // readback block: R[n] | flags[4] (sticky) | mom[2n] | features[n][8]
  // | predictions[n] | histograms
  uint8_t* d_rb = nullptr;
  uint8_t* h_rb = nullptr;
  size_t rb_bytes = 0, rb_clear_off = 0;
  size_t off_flags = 0, off_mom = 0, off_feat = 0, off_pred = 0;
  // upload block: BatchStep[n] | tables
  uint8_t* d_up = nullptr;
  uint8_t* h_up = nullptr;
  size_t up_bytes = 0;
  // device control
  int64_t* d_Rnew = nullptr;
  int32_t* d_cur = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_cls_first = nullptr;
  int32_t* d_cls_count = nullptr;
  int64_t* d_prefix = nullptr;
  unsigned long long* d_queue = nullptr;
  std::vector<void*> allocs;
  int cls_first[kClasses] = {0}, cls_count[kClasses] = {0};
  int64_t max_cap = 0;
  int lds_bins = 0;
  // persistent sweep shape: 4 waves per SIMD, and 4 work items per queue
  // atomic (one atomic per item serialised the queue counter: 3.9 ms per
  // step of the 64-instance glass batch against 2.3 ms with 4)
  int sweep_blocks = 1024;
  int sweep_chunk = 4;
  // temperature-step network (learned mode) and its acceptance tolerance
  pa_mlp* mlp = nullptr;
  pa_mlp* graph_mlp = nullptr;  // the network the graph was built with
  uint64_t graph_mlp_gen = 0;   // and its scratch/scale generation
  double tol = 0.02;
  double bisect_tol = 0.0;      // mode 1: 0 = the exact 64 halvings
  // schedule
  int mode = 0;                 // 0 explicit schedule, 1 bisection, 2 learned
  std::vector<double> sched;    // [steps][n]
  int sched_steps = 0, pos = 0;
  double beta_f = 0.0, target = 0.0;
  int theta = 0;
  int adaptive_max_steps = 0;
  // trajectory of observables after each step's sweeps
  std::vector<pa_obs> traj;
  std::vector<double> traj_lnZ;
  // per step and population: the features, the step taken and its source
  std::vector<float> dec_feat;
  std::vector<float> dec_prop;   // the network's log dbeta (NaN without one)
  std::vector<double> dec_dbeta;
  std::vector<int32_t> dec_src;
  int64_t src_count[5] = {0, 0, 0, 0, 0};
  int64_t overlap_evals = 0;  // exact overlap evaluations by the host
  double host_ms = 0.0;       // time spent in the host function
  int record = 0;
  int rec_rows = 0;      // rows of the per-step records allocated so far
  int rec_rows_max = 0;  // rows the run can need
  int n_active = 0;      // populations that moved in the last host step
  // graphs of the kernels before and after the host function
  hipGraph_t graph = nullptr, graph2 = nullptr;
  hipGraphExec_t exec = nullptr, exec2 = nullptr;
  int host_err = 0;
  int64_t attempts = 0;
};

namespace {

int64_t* rb_R(pa_batch* b) { return reinterpret_cast<int64_t*>(b->h_rb); }
unsigned long long* rb_flags(pa_batch* b) {
  return reinterpret_cast<unsigned long long*>(b->h_rb + b->off_flags);
}
unsigned long long* rb_mom(pa_batch* b) {
  return reinterpret_cast<unsigned long long*>(b->h_rb + b->off_mom);
}
const float* rb_feat(pa_batch* b) {
  return reinterpret_cast<const float*>(b->h_rb + b->off_feat);
}
const float* rb_pred(pa_batch* b) {
  return reinterpret_cast<const float*>(b->h_rb + b->off_pred);
}
BatchStep* up_steps(pa_batch* b) {
  return reinterpret_cast<BatchStep*>(b->h_up);
}

// Per-step records grow with the run (an adaptive run's length is unknown).
void grow_records(pa_batch* b, int rows) {
  if (rows <= b->rec_rows) return;
  rows = std::min(std::max(rows, 2 * b->rec_rows), b->rec_rows_max);
  const size_t n = (size_t)rows * b->n;
  b->traj.resize(n, pa_obs{});
  b->traj_lnZ.resize(n, 0.0);
  b->dec_feat.resize(n * kFeatures, 0.0f);
  b->dec_dbeta.resize(n, 0.0);
  b->dec_prop.resize(n, 0.0f);
  b->dec_src.resize(n, -1);
  b->rec_rows = rows;
}

// The host part of one step, between the two kernel sequences:
// observables of every population after the previous sweeps, the next beta
// of every population, its tables and Metropolis thresholds.
void host_step(void* ud) {
  pa_batch* b = static_cast<pa_batch*>(ud);
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t* R = rb_R(b);
  const unsigned long long* mom = rb_mom(b);
  BatchStep* st = up_steps(b);
  const bool last = (b->mode == 0) ? (b->pos >= b->sched_steps)
                                   : (b->pos >= b->adaptive_max_steps);
  grow_records(b, b->pos + 1);
  int active = 0;
  for (int p = 0; p < b->n; ++p) {
    PopHost& q = b->pops[p];
    const uint32_t* h = reinterpret_cast<const uint32_t*>(b->h_rb + q.rb_hist);
    if (b->record && q.moved) {
      pa_obs o;
      observables_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p], q.beta,
                            (int64_t)mom[2 * p], (int64_t)mom[2 * p + 1], &o);
      const size_t at = (size_t)(b->pos - 1) * b->n + p;
      if (at < b->traj.size()) {
        b->traj[at] = o;
        b->traj_lnZ[at] = q.lnZ;
      }
    }
    BatchStep& s = st[p];
    s.active = 0;
    s.beta = q.beta;
    s.target = b->target;
    q.moved = 0;
    if (last) continue;
    double beta_next;
    int src = 0;
    if (b->mode == 0) {
      beta_next = b->sched[(size_t)b->pos * b->n + p];
    } else {
      if (!(q.beta < b->beta_f)) continue;
      const double span = b->beta_f - q.beta;
      double d = -1.0;
      int ev = 1;
      // the remaining interval whenever it qualifies
      if (overlap_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p], span) >=
          b->target) {
        d = span;
        src = 4;
      } else if (b->mode == 2) {
        // the network's proposal, kept if its exact overlap is within tol
        const double prop = std::exp((double)rb_pred(b)[p]);
        if (prop > 0.0 && prop < span) {
          ++ev;
          const double a =
              overlap_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p], prop);
          if (std::fabs(a - b->target) <= b->tol) {
            d = prop;
            src = 2;
          }
        }
        if (d < 0.0) src = 3;  // fallback
      } else {
        src = 1;
      }
      // the exact bisection; as the baseline of the network, the bisection
      // that stops as soon as a midpoint passes the network's own test
      if (d < 0.0)
        d = bisect_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p], b->target,
                             span, &ev, b->mode == 1 ? b->bisect_tol : 0.0);
      b->overlap_evals += ev;
      beta_next = (d == span) ? b->beta_f : q.beta + d;
      if (!(beta_next > q.beta)) beta_next = b->beta_f;  // no progress
    }
    if (!(beta_next >= q.beta) || q.step + 1 > 65535) {
      b->host_err = PA_EINVAL;
      continue;
    }
    uint32_t* f = reinterpret_cast<uint32_t*>(b->h_up + q.up_tab);
    TableRange tr;
    if (build_tables(h, q.d.nbins, q.d.shift, q.N, R[p], q.R_t,
                     beta_next - q.beta, f, f + q.d.nbins, &tr) != PA_OK) {
      b->host_err = PA_ESTATE;
      continue;
    }
    {
      const size_t at = (size_t)b->pos * b->n + p;
      if (at < b->dec_src.size()) {
        std::memcpy(&b->dec_feat[at * kFeatures], rb_feat(b) + (size_t)p * kFeatures,
                    sizeof(float) * kFeatures);
        b->dec_dbeta[at] = beta_next - q.beta;
        b->dec_prop[at] = b->mlp ? rb_pred(b)[p] : std::nanf("");
        b->dec_src[at] = src;
      }
      b->src_count[src] += 1;
    }
    metropolis_K(beta_next, &s.K4, &s.K8);
    if (q.d.q) potts_thresholds(beta_next, s.Tp);
    s.lvl0 = tr.lo;
    s.nlvl = tr.hi - tr.lo + 1;
    s.step = (uint32_t)(q.step + 1);
    s.theta = b->theta;
    s.active = 1;
    ++active;
    q.lnQ_last = tr.lnQ;
    q.lnZ = q.lnZ + tr.lnQ;  // Eq. Free-En, read with the logarithm
    if (std::getenv("PA_LOG_JSONL")) {
      static const char* kSrc[5] = {"schedule", "bisection", "network",
                                    "fallback", "rest"};
      pa_obs o{};
      observables_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p], q.beta,
                            (int64_t)mom[2 * p], (int64_t)mom[2 * p + 1], &o);
      StepLog sl{};
      sl.pop = q.d.pop;
      sl.step = q.step + 1;
      sl.R_prev = R[p];
      sl.R = -1;  // drawn on the device after this decision
      sl.beta = beta_next;
      sl.dbeta = beta_next - q.beta;
      sl.lnQ = tr.lnQ;
      sl.lnZ = q.lnZ;
      sl.overlap = overlap_from_hist(h, q.d.nbins, q.d.shift, q.N, R[p],
                                     beta_next - q.beta);
      sl.e_prev = o.e;
      sl.abs_m_prev = o.abs_m;
      sl.C_prev = o.C;
      sl.source = kSrc[src];
      log_step(sl);
    }
    q.beta = beta_next;
    q.step += 1;
    q.moved = 1;
    s.beta = beta_next;
  }
  b->n_active = active;
  b->pos += 1;
  b->host_ms += std::chrono::duration<double, std::milli>(
                    std::chrono::steady_clock::now() - t0).count();
}

#define BK(x) PA_HIP(x)

// Kernels of one step before the host function.
int enqueue_front(pa_batch* b) {
  hipStream_t st = b->stream;
  const size_t clear = b->rb_bytes - b->rb_clear_off;
  BK(launch_fill_u32(reinterpret_cast<uint32_t*>(b->d_rb + b->rb_clear_off),
                     (int64_t)(clear / 4), 0u, st));
  const int64_t* dR = reinterpret_cast<const int64_t*>(b->d_rb);
  unsigned long long* dflags =
      reinterpret_cast<unsigned long long*>(b->d_rb + b->off_flags);
  unsigned long long* dmom =
      reinterpret_cast<unsigned long long*>(b->d_rb + b->off_mom);
  float* dfeat = reinterpret_cast<float*>(b->d_rb + b->off_feat);
  const unsigned gx = (unsigned)((b->max_cap + 2047) / 2048);
  hipLaunchKernelGGL(k_bhist, dim3(gx * (unsigned)b->n), dim3(256),
                     (size_t)b->lds_bins * 4, st, b->d_pops, dR, b->d_cur,
                     dmom, dflags, b->lds_bins, (int)gx);
  BK(hipGetLastError());
  hipLaunchKernelGGL(k_bfeatures, dim3(b->n), dim3(256), 0, st, b->d_pops,
                     reinterpret_cast<const BatchStep*>(b->d_up), dR, dfeat);
  BK(hipGetLastError());
  if (b->mlp) {
    const int rc = mlp_infer_on(b->mlp, dfeat, b->n, st);
    if (rc) return rc;
    float mu_y, sig_y;
    mlp_out_scale(b->mlp, &mu_y, &sig_y);
    hipLaunchKernelGGL(k_bpred, dim3((b->n + 255) / 256), dim3(256), 0, st,
                       mlp_output_dev(b->mlp),
                       reinterpret_cast<float*>(b->d_rb + b->off_pred), b->n,
                       mu_y, sig_y);
    BK(hipGetLastError());
  }
  return PA_OK;
}

template <int W, int RPL, bool PLANES>
hipError_t launch_bsweep_wrp(int int8, int glass, unsigned blocks,
                             hipStream_t st, const BatchPop* P,
                             const BatchStep* S, const int64_t* R,
                             const int32_t* cur, const int32_t* order,
                             const int64_t* prefix, unsigned long long* queue,
                             int first, int count, int chunk) {
  const dim3 g(blocks), t(256);
  if (int8 && glass)
    hipLaunchKernelGGL((k_bsweep<W, RPL, true, true, PLANES>), g, t, 0, st, P, S, R, cur, order, prefix, queue, first, count, chunk, 1u);
  else if (int8)
    hipLaunchKernelGGL((k_bsweep<W, RPL, true, false, PLANES>), g, t, 0, st, P, S, R, cur, order, prefix, queue, first, count, chunk, 1u);
  else if (glass)
    hipLaunchKernelGGL((k_bsweep<W, RPL, false, true, PLANES>), g, t, 0, st, P, S, R, cur, order, prefix, queue, first, count, chunk, 1u);
  else
    hipLaunchKernelGGL((k_bsweep<W, RPL, false, false, PLANES>), g, t, 0, st, P, S, R, cur, order, prefix, queue, first, count, chunk, 1u);
  return hipGetLastError();
}

template <int W, int RPL>
hipError_t launch_bsweep_wr(int int8, int glass, int planes, unsigned blocks,
                            hipStream_t st, const BatchPop* P,
                            const BatchStep* S, const int64_t* R,
                            const int32_t* cur, const int32_t* order,
                            const int64_t* prefix, unsigned long long* queue,
                            int first, int count, int chunk) {
  return planes ? launch_bsweep_wrp<W, RPL, true>(int8, glass, blocks, st, P,
                                                  S, R, cur, order, prefix,
                                                  queue, first, count, chunk)
                : launch_bsweep_wrp<W, RPL, false>(int8, glass, blocks, st, P,
                                                   S, R, cur, order, prefix,
                                                   queue, first, count, chunk);
}

// The persistent Potts pass of class k (see potts_class): as many waves as
// the Ising sweep has, up to four per workgroup.
hipError_t launch_bpotts(int k, int blocks, int chunk, hipStream_t st,
                         const BatchPop* P, const BatchStep* S,
                         const int64_t* R, const int32_t* cur,
                         const int32_t* order, const int64_t* prefix,
                         unsigned long long* queue, int first, int count) {
  const int mi = k - kIsingClasses;
  const int mpr = 1 << mi;
  const int64_t N = (int64_t)64 * mpr * mpr;
  const int wpb = N <= 4096 ? 4 : N <= 8192 ? 2 : 1;  // <= 17 KB of LDS
  const size_t shm = (size_t)wpb * (72 + N);
  (void)chunk;  // one item per wave per atomic
  const dim3 grid((unsigned)(4 * blocks / wpb)), block(64 * wpb);
#define PA_BP(m)                                                           \
  hipLaunchKernelGGL(k_bpotts<m>, grid, block, shm, st, P, S, R, cur,      \
                     order, prefix, queue, first, count, 1u)
  switch (mpr) {
    case 1: PA_BP(1); break;
    case 2: PA_BP(2); break;
    case 4: PA_BP(4); break;
    case 8: PA_BP(8); break;
    case 16: PA_BP(16); break;
    default: return hipErrorInvalidValue;
  }
#undef PA_BP
  return hipGetLastError();
}

// The persistent sweep of sweep class k (see sweep_class).
hipError_t launch_bsweep(int k, int blocks, int chunk, hipStream_t st,
                         const BatchPop* P, const BatchStep* S,
                         const int64_t* R, const int32_t* cur,
                         const int32_t* order, const int64_t* prefix,
                         unsigned long long* queue, int first, int count) {
  const int planes = k >> 6, kk = k & 63;
  const int glass = kk & 1, int8 = (kk >> 1) & 1, rpl = (kk >> 2) % 4 + 1,
            W = (kk >> 2) / 4 + 1;
  const unsigned bl = (unsigned)blocks;
#define PA_BS(w, r) \
  launch_bsweep_wr<w, r>(int8, glass, planes, bl, st, P, S, R, cur, order, \
                         prefix, queue, first, count, chunk)
  switch (W * 8 + rpl) {
    case 1 * 8 + 1: return PA_BS(1, 1);
    case 1 * 8 + 2: return PA_BS(1, 2);
    case 1 * 8 + 3: return PA_BS(1, 3);
    case 1 * 8 + 4: return PA_BS(1, 4);
    case 2 * 8 + 1: return PA_BS(2, 1);
    case 2 * 8 + 2: return PA_BS(2, 2);
    case 2 * 8 + 3: return PA_BS(2, 3);
    case 2 * 8 + 4: return PA_BS(2, 4);
    case 3 * 8 + 2: return PA_BS(3, 2);
    case 3 * 8 + 3: return PA_BS(3, 3);
    case 3 * 8 + 4: return PA_BS(3, 4);
    case 4 * 8 + 2: return PA_BS(4, 2);
    case 4 * 8 + 3: return PA_BS(4, 3);
    case 4 * 8 + 4: return PA_BS(4, 4);
    default: return hipErrorInvalidValue;
  }
#undef PA_BS
}

// Kernels of one step after the host function.
int enqueue_back(pa_batch* b) {
  hipStream_t st = b->stream;
  int64_t* dR = reinterpret_cast<int64_t*>(b->d_rb);
  unsigned long long* dflags =
      reinterpret_cast<unsigned long long*>(b->d_rb + b->off_flags);
  const BatchStep* dS = reinterpret_cast<const BatchStep*>(b->d_up);
  const unsigned tiles = (unsigned)((b->max_cap + 255) / 256);
  hipLaunchKernelGGL(k_bcounts, dim3(tiles, b->n), dim3(256), 0, st, b->d_pops,
                     dS, dR, b->d_cur);
  BK(hipGetLastError());
  hipLaunchKernelGGL(k_bscan, dim3(b->n), dim3(1024), 0, st, b->d_pops, dS, dR,
                     b->d_Rnew, dflags);
  BK(hipGetLastError());
  hipLaunchKernelGGL(k_bscatter, dim3(tiles, b->n), dim3(256), 0, st,
                     b->d_pops, dS, dR, b->d_cur);
  BK(hipGetLastError());
  hipLaunchKernelGGL(k_bgather, dim3(256, b->n), dim3(256), 0, st, b->d_pops,
                     dS, b->d_Rnew, b->d_cur);
  BK(hipGetLastError());
  hipLaunchKernelGGL(k_bcommit, dim3(1), dim3(256), 0, st, b->d_pops, dS, dR,
                     b->d_Rnew, b->d_cur, b->d_order, b->n, b->d_cls_first,
                     b->d_cls_count, b->d_prefix, b->d_queue, 1);
  BK(hipGetLastError());
  for (int k = 0; k < kClasses; ++k) {
    if (b->cls_count[k] == 0) continue;
    if (k >= kIsingClasses)
      BK(launch_bpotts(k, b->sweep_blocks, b->sweep_chunk, st, b->d_pops, dS,
                       dR, b->d_cur, b->d_order, b->d_prefix, b->d_queue,
                       b->cls_first[k], b->cls_count[k]));
    else
      BK(launch_bsweep(k, b->sweep_blocks, b->sweep_chunk, st, b->d_pops, dS,
                       dR, b->d_cur,
                       b->d_order, b->d_prefix, b->d_queue, b->cls_first[k],
                       b->cls_count[k]));
  }
  return PA_OK;
}

int check_flags(pa_batch* b) {
  const unsigned long long* fl = rb_flags(b);
  if (b->host_err) return b->host_err;
  if (fl[0]) {
    note_error("a population's energy lies outside its histogram range");
    return PA_EDEVICE;
  }
  if (fl[1] & 1ull) return PA_ECAPACITY;
  if (fl[1] & 2ull) return PA_EEMPTY;
  return PA_OK;
}

// Waits for the stream by polling it for up to 50 ms, then blocks (a
// blocking wait wakes up tens of microseconds late, which every step of a
// batch would pay).
hipError_t poll_stream(hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50))
      return hipStreamSynchronize(st);
  }
}

// The host part of a step between the two kernel sequences: all
// histograms down, synchronise, the host function, all tables up.  The
// copies and the host function stay outside the graphs.
int host_between(pa_batch* b) {
  BK(hipMemcpyAsync(b->h_rb, b->d_rb, b->rb_bytes, hipMemcpyDeviceToHost,
                    b->stream));
  BK(poll_stream(b->stream));
  const int rc = check_flags(b);
  if (rc) return rc;
  host_step(b);
  if (b->host_err) return b->host_err;
  BK(hipMemcpyAsync(b->d_up, b->h_up, b->up_bytes, hipMemcpyHostToDevice,
                    b->stream));
  return PA_OK;
}

// One step with individual launches.
int step_eager(pa_batch* b) {
  int rc = enqueue_front(b);
  if (!rc) rc = host_between(b);
  if (!rc) rc = enqueue_back(b);
  return rc;
}

// Captures a kernel sequence as a graph (kernel nodes only: clearing uses a
// fill kernel, and no copy or host callback is recorded).
int capture(pa_batch* b, int (*enqueue)(pa_batch*), hipGraphExec_t* out,
            hipGraph_t* g_out) {
  BK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
  const int rc = enqueue(b);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != PA_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) set_last_error("hipStreamEndCapture", e, __LINE__);
    return rc ? rc : PA_EDEVICE;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    set_last_error("hipGraphInstantiate", ei, __LINE__);
    return PA_EDEVICE;
  }
  *out = x;
  *g_out = g;
  return PA_OK;
}

void drop_graph(pa_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec2) (void)hipGraphExecDestroy(b->exec2);
  if (b->graph2) (void)hipGraphDestroy(b->graph2);
  b->exec = b->exec2 = nullptr;
  b->graph = b->graph2 = nullptr;
}

int build_graph(pa_batch* b) {
  const uint64_t gen = mlp_generation(b->mlp);
  if (b->exec && b->exec2 && b->graph_mlp == b->mlp && b->graph_mlp_gen == gen)
    return PA_OK;
  drop_graph(b);
  b->graph_mlp = b->mlp;
  b->graph_mlp_gen = gen;
  int rc = capture(b, enqueue_front, &b->exec, &b->graph);
  if (rc == PA_OK) rc = capture(b, enqueue_back, &b->exec2, &b->graph2);
  if (rc != PA_OK) drop_graph(b);
  return rc;
}

// One step with the two captured kernel sequences.
int step_graph(pa_batch* b) {
  BK(hipGraphLaunch(b->exec, b->stream));
  const int rc = host_between(b);
  if (rc) return rc;
  BK(hipGraphLaunch(b->exec2, b->stream));
  return PA_OK;
}

void free_batch(pa_batch* b) {
  drop_graph(b);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->h_rb) (void)hipHostFree(b->h_rb);
  if (b->h_up) (void)hipHostFree(b->h_up);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

template <typename T>
bool balloc(pa_batch* b, T** p, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();  // not left for a later launch check to read
    return false;
  }
  b->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return true;
}

int64_t round_up16(int64_t v) { return (v + 15) / 16 * 16; }

}  // namespace

// =================================================================== ABI

extern "C" {

int pa_tune_rows_per_lane(int32_t L, int32_t layout, int32_t model,
                          int64_t R, int32_t theta, void* stream,
                          int32_t* best, float* ms) {
  return tune_rows_per_lane(L, layout, model, PA_RNG_WORD, R, theta, stream,
                            best, ms);
}

}  // extern "C"

namespace pa {

// The launch shape of a single population's sweep that takes least time:
// every valid rows-per-lane of one test population (R replicas, theta
// sweeps at beta = 0.4, after a warm-up), in the given random-number mode.
int tune_rows_per_lane(int32_t L, int32_t layout, int32_t model,
                       int32_t rng_mode, int64_t R, int32_t theta,
                       void* stream, int32_t* best, float* ms) try {
  if (!best || L < 4 || L > 128 || (L & 1) || R < 1 || theta < 1)
    return PA_EINVAL;
  const int cand[4] = {1, 2, 3, 4};
  float t[4] = {-1.f, -1.f, -1.f, -1.f};
  std::vector<int8_t> J;
  if (model == PA_PMJ) {
    J.assign((size_t)2 * L * L, 1);
    for (size_t i = 0; i < J.size(); i += 3) J[i] = -1;
  }
  int bi = -1;
  for (int k = 0; k < 4; ++k) {
    const int rpl = cand[k];
    if (L % rpl || L / rpl > 64 || ((L + 31) / 32 >= 3 && rpl < 2)) continue;
    pa_config cfg{};
    cfg.L = L;
    cfg.model = model;
    cfg.J = J.empty() ? nullptr : J.data();
    cfg.R_target = R;
    cfg.layout = layout;
    cfg.rows_per_lane = rpl;
    cfg.seed = 12345;
    cfg.stream = stream;
    cfg.rng_mode = rng_mode;
    pa_ctx* c = nullptr;
    int rc = pa_init(&cfg, &c);
    if (rc) return rc;
    rc = pa_resample(c, 0.4, nullptr);
    if (!rc) rc = pa_sweep(c, 0.4, 1);  // warm-up
    if (!rc) rc = pa_set_timing(c, 1 << PA_K_SWEEP);
    if (!rc) rc = pa_sweep(c, 0.4, theta);
    if (!rc) rc = pa_sweep(c, 0.4, theta);
    pa_timing tm{};
    if (!rc) rc = pa_get_timing(c, &tm);
    pa_destroy(c);
    if (rc) return rc;
    t[k] = (float)(tm.ms[PA_K_SWEEP] / 2.0);
    if (bi < 0 || t[k] < t[bi]) bi = k;
  }
  if (bi < 0) return PA_EINVAL;
  *best = cand[bi];
  if (ms)
    for (int k = 0; k < 4; ++k) ms[k] = t[k];
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

// Rows per lane of a batch, timed with the batch's own persistent sweep
// on scratch batches of the same configurations.  Each distinct (L,
// layout, model, stream) whose configurations leave rows_per_lane 0 starts
// at its smallest valid value; then, one class at a time, every other
// valid value is tried and kept when three steps (theta = 4 at beta = 0.3,
// after one untimed step, no graph) take under 98 % of the best time so
// far.  Potts populations have no rows per lane.  out[p] is 0 where the
// configuration is not tuned.  Cached per process by the configurations.
int tune_batch_rows(const pa_config* cfgs, int n, void* stream,
                    std::vector<int>* out) {
  // the cache is shared by threads; the tuning itself runs unlocked
  static std::mutex mu;
  static std::map<std::vector<int64_t>, std::vector<int>> cache;
  std::vector<int64_t> key;
  for (int p = 0; p < n; ++p) {
    const pa_config& c = cfgs[p];
    key.insert(key.end(), {c.L, c.R_target, c.layout, c.model, c.q,
                           c.rng_mode, c.rows_per_lane});
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return PA_OK;
    }
  }
  auto valid = [](int L, int r) {
    return L % r == 0 && L / r <= 64 && !((L + 31) / 32 >= 3 && r < 2);
  };
  std::vector<pa_config> work(cfgs, cfgs + n);
  std::map<TuneKey, std::vector<int>> members;
  for (int p = 0; p < n; ++p) {
    const pa_config& c = cfgs[p];
    if (c.model != PA_POTTS && c.rows_per_lane == 0)
      members[TuneKey{c.L, c.layout, c.model, c.rng_mode}].push_back(p);
  }
  std::map<TuneKey, int> cur;
  for (const auto& kv : members) {
    int r = 1;
    while (!valid(kv.first.L, r)) ++r;  // r <= 2 for every even L <= 128
    cur[kv.first] = r;
    for (int p : kv.second) work[p].rows_per_lane = r;
  }
  std::vector<int> res(n, 0);
  if (!members.empty()) {
    const std::vector<double> betas((size_t)3 * n, 0.3);
    auto timed = [&](double* ms) -> int {
      pa_batch* t = nullptr;
      int rc = pa_batch_init(work.data(), n, stream, 0, &t);
      if (rc) return rc;
      rc = pa_batch_run(t, 1, betas.data(), 4, 0);
      if (rc == PA_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = pa_batch_run(t, 3, betas.data(), 4, 0);
        *ms = std::chrono::duration<double, std::milli>(
                  std::chrono::steady_clock::now() - t0).count();
      }
      pa_batch_destroy(t);
      return rc;
    };
    double best = 0.0;
    int rc = timed(&best);
    if (rc) return rc;
    for (const auto& kv : members) {
      for (int r = 1; r <= 4; ++r) {
        if (r == cur[kv.first] || !valid(kv.first.L, r)) continue;
        for (int p : kv.second) work[p].rows_per_lane = r;
        double ms = 0.0;
        rc = timed(&ms);
        if (rc) return rc;
        if (ms < 0.98 * best) {
          best = ms;
          cur[kv.first] = r;
        } else {
          for (int p : kv.second) work[p].rows_per_lane = cur[kv.first];
        }
      }
    }
    for (const auto& kv : members)
      for (int p : kv.second) res[p] = cur[kv.first];
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = res;
  }
  *out = res;
  return PA_OK;
}

// Launch shape of the persistent sweep (workgroups, items per queue
// atomic) that runs the given populations fastest: a scratch batch of the
// same configurations takes one step to beta = 0.3, then each candidate
// times two more steps at that beta (theta = 4, no graph), timed on the
// host around the synchronising run.  Cached per process by the list of
// (L, R, layout, model, q, stream) of the populations.
int tune_sweep_shape(const pa_config* cfgs, int n, void* stream,
                     int* blocks, int* chunk) {
  static std::mutex mu;
  static std::map<std::vector<int64_t>, std::pair<int, int>> cache;
  std::vector<int64_t> key;
  for (int p = 0; p < n; ++p) {
    const pa_config& c = cfgs[p];
    key.insert(key.end(), {c.L, c.R_target, c.layout, c.model, c.q,
                           c.rng_mode, c.rows_per_lane});
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      *blocks = it->second.first;
      *chunk = it->second.second;
      return PA_OK;
    }
  }
  static const int cand[][2] = {{1024, 4}, {512, 4}, {2048, 4},
                                {1024, 8}, {2048, 8}, {1024, 2}};
  pa_batch* t = nullptr;
  int rc = pa_batch_init(cfgs, n, stream, PA_BATCH_AUTOTUNE, &t);
  if (rc) return rc;
  std::vector<double> betas((size_t)2 * n, 0.3);
  rc = pa_batch_run(t, 1, betas.data(), 2, 0);
  double best = -1.0;
  int bb = 1024, bc = 4;
  for (const auto& c : cand) {
    if (rc) break;
    rc = pa_batch_set_sweep_blocks(t, c[0], c[1]);
    if (rc) break;
    const auto t0 = std::chrono::steady_clock::now();
    rc = pa_batch_run(t, 2, betas.data(), 4, 0);
    const double ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t0).count();
    if (!rc && (best < 0.0 || ms < best)) {
      best = ms;
      bb = c[0];
      bc = c[1];
    }
  }
  pa_batch_destroy(t);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = {bb, bc};
  }
  *blocks = bb;
  *chunk = bc;
  return PA_OK;
}

}  // namespace pa

extern "C" {

int pa_batch_init(const pa_config* cfgs, int32_t n, void* stream,
                  int32_t flags, pa_batch** out) try {
  if (!out) return PA_EINVAL;
  *out = nullptr;
  if (!cfgs || n < 1 || n > 4096) return PA_EINVAL;
  for (int p = 0; p < n; ++p) {
    const pa_config& c = cfgs[p];
    if (c.L < 4 || c.L > 128 || (c.L & 1)) return PA_EINVAL;
    if (c.model != PA_FERRO && c.model != PA_PMJ && c.model != PA_POTTS)
      return PA_EINVAL;
    // Potts populations: the four-sites-per-word pass (L = 8, 16, 32, 64,
    // 128), one byte per state
    if (c.model == PA_POTTS &&
        (c.q < 2 || c.q > 16 || c.layout != PA_INT8 ||
         (c.L != 8 && c.L != 16 && c.L != 32 && c.L != 64 && c.L != 128)))
      return PA_EINVAL;
    if (c.model == PA_PMJ && !c.J) return PA_EINVAL;
    if (c.layout != PA_INT8 && c.layout != PA_BITS) return PA_EINVAL;
    if (c.resampling != PA_NEAREST) return PA_EINVAL;  // single path only
    if (c.rng_mode != PA_RNG_WORD &&
        (c.rng_mode != PA_RNG_PLANES || c.model == PA_POTTS))
      return PA_EINVAL;
    if (c.R_target < 1 || c.R_target >= (1ll << 31)) return PA_EINVAL;
    const int rpl = c.model == PA_POTTS ? 0 : c.rows_per_lane;  // Potts: unused
    if (rpl < 0 || rpl > 4) return PA_EINVAL;
    if (rpl && (c.L % rpl || c.L / rpl > 64 || ((c.L + 31) / 32 >= 3 && rpl < 2)))
      return PA_EINVAL;
    if (c.model == PA_PMJ)
      for (int64_t i = 0; i < 2ll * c.L * c.L; ++i)
        if (c.J[i] != 1 && c.J[i] != -1) return PA_EINVAL;
  }
  // rows per lane chosen with the batch's own sweep, before anything is
  // allocated for this batch
  std::vector<int> tuned;
  if (flags & PA_BATCH_AUTOTUNE) {
    const int rc = tune_batch_rows(cfgs, n, stream, &tuned);
    if (rc) return rc;
  }
  pa_batch* b = new (std::nothrow) pa_batch();
  if (!b) return PA_ENOMEM;
  if (hip_ok(hipGetDevice(&b->device), "hipGetDevice", __LINE__)) {
    delete b;
    return PA_EDEVICE;
  }
  b->stream = reinterpret_cast<hipStream_t>(stream);
  if (!b->stream) {  // graph capture needs a stream other than the null one
    if (hip_ok(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking),
               "hipStreamCreateWithFlags", __LINE__)) {
      delete b;
      return PA_EDEVICE;
    }
    b->own_stream = true;
  }
  b->n = n;
  b->pops.resize(n);
  // layout of the readback and upload blocks
  b->off_flags = (size_t)8 * n;
  b->off_mom = b->off_flags + 32;
  b->off_feat = b->off_mom + (size_t)16 * n;
  b->off_pred = b->off_feat + (size_t)4 * kFeatures * n;
  size_t rb = (size_t)round_up16((int64_t)(b->off_pred + (size_t)4 * n));
  b->rb_clear_off = b->off_mom;  // moments, features and histograms
  size_t up = round_up16((int64_t)sizeof(BatchStep) * n);
  int max_bins = 0;
  for (int p = 0; p < n; ++p) {
    const pa_config& c = cfgs[p];
    PopHost& q = b->pops[p];
    BatchPop& d = q.d;
    int rpl = c.model == PA_POTTS ? 1 : c.rows_per_lane;
    const bool planes = c.rng_mode == PA_RNG_PLANES;
    if (rpl == 0 && !tuned.empty() && tuned[p] > 0) rpl = tuned[p];
    if (rpl == 0) rpl = default_rows_per_lane(c.L, planes, c.R_target);
    d.L = c.L;
    d.planes = planes ? 1 : 0;
    d.W = (c.L + 31) / 32;
    d.rpl = rpl;
    d.lpr = c.L / rpl;
    d.rpw = 64 / d.lpr;
    d.shift = (c.model == PA_FERRO) ? 2 : (c.model == PA_PMJ) ? 1 : 0;
    // Potts energies lie in [-2N, 0]
    d.nbins = c.model == PA_POTTS ? 2 * c.L * c.L + 1
                                  : ((4 * c.L * c.L) >> d.shift) + 1;
    d.q = c.model == PA_POTTS ? c.q : 0;
    if (d.q) {  // one replica per wave
      d.lpr = 64;
      d.rpw = 1;
    }
    d.glass = c.model == PA_PMJ;
    d.int8 = c.layout == PA_INT8;
    d.stride = d.int8 ? round_up16((int64_t)c.L * c.L)
                      : round_up16((int64_t)c.L * d.W * 4);
    d.chunks = (int32_t)(d.stride / 16);
    int lg = 0;
    while ((1 << lg) < d.chunks && lg < 6) ++lg;
    d.lpr_log2 = lg;
    d.cap = c.capacity ? c.capacity
                       : c.R_target +
                             16 * (int64_t)std::ceil(std::sqrt((double)c.R_target)) +
                             1024;
    d.k0 = (uint32_t)(c.seed & 0xFFFFFFFFu);
    d.k1 = (uint32_t)(c.seed >> 32);
    d.pop = c.population_id;
    q.R_t = c.R_target;
    q.N = c.L * c.L;
    q.model = c.model;
    q.lnZ = (double)q.N * std::log(d.q ? (double)d.q : 2.0);
    q.rb_hist = rb;
    rb += (size_t)d.nbins * 4;
    q.up_tab = up;
    up += (size_t)d.nbins * 8;
    max_bins = std::max(max_bins, d.nbins);
    b->max_cap = std::max(b->max_cap, d.cap);
    if (d.cap < c.R_target || d.cap >= (1ll << 32)) {
      free_batch(b);
      delete b;
      return PA_EINVAL;
    }
  }
  b->rb_bytes = (size_t)round_up16((int64_t)rb);
  b->up_bytes = (size_t)round_up16((int64_t)up);
  b->lds_bins = std::min(max_bins, 16384);
  bool ok = true;
  ok = ok && balloc(b, &b->d_rb, b->rb_bytes);
  ok = ok && balloc(b, &b->d_up, b->up_bytes);
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_rb), b->rb_bytes) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_up), b->up_bytes) == hipSuccess;
  ok = ok && balloc(b, &b->d_Rnew, (size_t)8 * n);
  ok = ok && balloc(b, &b->d_cur, (size_t)4 * n);
  ok = ok && balloc(b, &b->d_order, (size_t)4 * n);
  ok = ok && balloc(b, &b->d_cls_first, 4 * kClasses);
  ok = ok && balloc(b, &b->d_cls_count, 4 * kClasses);
  ok = ok && balloc(b, &b->d_prefix, (size_t)8 * (n + kClasses));
  ok = ok && balloc(b, &b->d_queue, 8 * kClasses);
  ok = ok && balloc(b, &b->d_pops, sizeof(BatchPop) * n);
  for (int p = 0; p < n && ok; ++p) {
    BatchPop& d = b->pops[p].d;
    const size_t cap = (size_t)d.cap;
    for (int k = 0; k < 2 && ok; ++k) {
      ok = ok && balloc(b, &d.spins[k], cap * (size_t)d.stride);
      ok = ok && balloc(b, &d.E[k], cap * 4);
      ok = ok && balloc(b, &d.M[k], cap * 4);
    }
    ok = ok && balloc(b, &d.n, cap * 4);
    ok = ok && balloc(b, &d.parent, cap * 4);
    ok = ok && balloc(b, &d.fam[0], cap * 4);
    ok = ok && balloc(b, &d.fam[1], cap * 4);
    ok = ok && balloc(b, &d.tile_sum, (cap / 256 + 2) * 4);
    ok = ok && balloc(b, &d.tile_off, (cap / 256 + 2) * 4);
    d.hist = reinterpret_cast<uint32_t*>(b->d_rb + b->pops[p].rb_hist);
    d.tab = reinterpret_cast<uint32_t*>(b->d_up + b->pops[p].up_tab);
    if (cfgs[p].model == PA_PMJ) {
      uint32_t* jb = nullptr;
      ok = ok && balloc(b, &jb, (size_t)2 * d.L * d.W * 4);
      d.jbits = jb;
    }
  }
  if (!ok) {
    (void)hipGetLastError();  // a failed allocation is no later launch's error
    free_batch(b);
    delete b;
    return PA_ENOMEM;
  }
  // population order: by sweep class, then by L descending
  auto cls_of = [&](int p) {
    const BatchPop& x = b->pops[p].d;
    return x.q ? potts_class(x.L / 8)
               : sweep_class(x.W, x.rpl, x.int8, x.glass, x.planes);
  };
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    if (cls_of(a) != cls_of(c)) return cls_of(a) < cls_of(c);
    return b->pops[a].d.L > b->pops[c].d.L;
  });
  int cf[kClasses] = {0}, cc[kClasses] = {0};
  for (int i = n - 1; i >= 0; --i) cf[cls_of(order[i])] = i;
  for (int i = 0; i < n; ++i) cc[cls_of(order[i])] += 1;
  for (int k = 0; k < kClasses; ++k) {
    b->cls_first[k] = cc[k] ? cf[k] : 0;
    b->cls_count[k] = cc[k];
  }
  int rc = PA_OK;
  std::vector<BatchPop> dp(n);
  for (int p = 0; p < n; ++p) dp[p] = b->pops[p].d;
  std::vector<int32_t> cur0(n, 0);
  rc = hip_ok(hipMemcpy(b->d_pops, dp.data(), sizeof(BatchPop) * n,
                        hipMemcpyHostToDevice), "hipMemcpy(populations)",
              __LINE__);
  if (!rc)
    rc = hip_ok(hipMemcpy(b->d_order, order.data(), 4 * n,
                          hipMemcpyHostToDevice), "hipMemcpy(order)", __LINE__);
  if (!rc)
    rc = hip_ok(hipMemcpy(b->d_cls_first, b->cls_first, 4 * kClasses,
                          hipMemcpyHostToDevice), "hipMemcpy(classes)",
                __LINE__);
  if (!rc)
    rc = hip_ok(hipMemcpy(b->d_cls_count, b->cls_count, 4 * kClasses,
                          hipMemcpyHostToDevice), "hipMemcpy(classes)",
                __LINE__);
  if (!rc)
    rc = hip_ok(hipMemcpy(b->d_cur, cur0.data(), 4 * n, hipMemcpyHostToDevice),
                "hipMemcpy(buffers)", __LINE__);
  // couplings and the initial populations (the INIT stream of each)
  std::memset(b->h_rb, 0, b->rb_bytes);
  std::memset(b->h_up, 0, b->up_bytes);
  if (rc == PA_OK)
    rc = hip_ok(hipMemcpy(b->d_up, b->h_up, b->up_bytes, hipMemcpyHostToDevice),
                "hipMemcpy(upload block)", __LINE__);
  for (int p = 0; p < n && rc == PA_OK; ++p) {
    const pa_config& c = cfgs[p];
    BatchPop& d = b->pops[p].d;
    rb_R(b)[p] = c.R_target;
    if (c.model == PA_PMJ) {
      std::vector<uint32_t> jb((size_t)2 * d.L * d.W, 0u);
      for (int k = 0; k < 2; ++k)
        for (int y = 0; y < d.L; ++y)
          for (int x = 0; x < d.L; ++x)
            if (c.J[(size_t)k * d.L * d.L + (size_t)y * d.L + x] < 0)
              jb[((size_t)k * d.L + y) * d.W + x / 32] |= 1u << (x % 32);
      rc = hip_ok(hipMemcpy(const_cast<uint32_t*>(d.jbits), jb.data(),
                            jb.size() * 4, hipMemcpyHostToDevice),
                  "hipMemcpy(couplings)", __LINE__);
    }
    LatticeArgs a{};
    a.spins = d.spins[0];
    a.E = d.E[0];
    a.M = d.M[0];
    a.jbits = d.jbits;
    a.R = c.R_target;
    a.stride = d.stride;
    a.L = d.L;
    a.lpr = d.lpr;
    a.rpw = d.rpw;
    a.k0 = d.k0;
    a.k1 = d.k1;
    a.pop = d.pop;
    a.one = 1u;
    a.init = 1;
    a.q = d.q;
    if (rc == PA_OK)
      rc = hip_ok(d.q ? launch_potts(a, b->stream)
                      : launch_lattice(a, d.W, d.rpl, d.int8, d.glass,
                                       d.planes != 0, b->stream),
                  "initial lattice pass", __LINE__);
    // every initial replica founds its own family
    if (rc == PA_OK)
      rc = hip_ok(launch_iota_u32(d.fam[0], c.R_target, b->stream),
                  "initial families", __LINE__);
  }
  // the whole readback block: sizes, zeroed sticky error flags, moments
  if (rc == PA_OK)
    rc = hip_ok(hipMemcpyAsync(b->d_rb, b->h_rb, b->rb_bytes,
                               hipMemcpyHostToDevice, b->stream),
                "hipMemcpyAsync(readback block)", __LINE__);
  if (rc == PA_OK)
    rc = hip_ok(hipStreamSynchronize(b->stream), "hipStreamSynchronize",
                __LINE__);
  if (rc == PA_OK && (flags & PA_BATCH_TUNE_SWEEP)) {
    int tb = 0, tc = 0;
    rc = tune_sweep_shape(cfgs, n, stream, &tb, &tc);
    if (rc == PA_OK) {
      b->sweep_blocks = tb;
      b->sweep_chunk = tc;
    }
  }
  if (rc != PA_OK) {
    free_batch(b);
    delete b;
    return rc;
  }
  *out = b;
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

void pa_batch_destroy(pa_batch* b) try {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  delete b;
} catch (...) {
}

static int batch_run(pa_batch* b, int steps, int use_graph) {
  b->host_err = 0;
  b->pos = 0;
  const int total = steps + 1;  // the extra pass only measures
  b->record = 1;
  b->traj.clear();
  b->traj_lnZ.clear();
  b->dec_feat.clear();
  b->dec_dbeta.clear();
  b->dec_prop.clear();
  b->dec_src.clear();
  b->rec_rows = 0;
  b->rec_rows_max = steps;
  grow_records(b, std::min(steps, 256));
  for (auto& c : b->src_count) c = 0;
  b->overlap_evals = 0;
  b->host_ms = 0.0;
  if (b->mlp) {
    const int rc = mlp_prepare(b->mlp, b->n);
    if (rc) return rc;
  }
  // current beta and target of every population for the first summaries
  BK(hipStreamSynchronize(b->stream));
  BatchStep* st = up_steps(b);
  for (int p = 0; p < b->n; ++p) {
    st[p].beta = b->pops[p].beta;
    st[p].target = b->target;
    st[p].active = 0;
  }
  BK(hipMemcpyAsync(b->d_up, b->h_up, sizeof(BatchStep) * b->n,
                    hipMemcpyHostToDevice, b->stream));
  if (use_graph) {
    const int rc = build_graph(b);
    if (rc) return rc;
  }
  for (int i = 0; i < total; ++i) {
    const int rc = use_graph ? step_graph(b) : step_eager(b);
    if (rc) return rc;
    // an adaptive run ends once every population has reached beta_f (this
    // pass recorded the observables of their last step)
    if (b->mode != 0 && b->n_active == 0) break;
  }
  BK(hipStreamSynchronize(b->stream));
  return check_flags(b);
}

int pa_batch_run(pa_batch* b, int32_t steps, const double* betas,
                 int32_t theta, int32_t use_graph) try {
  // theta <= 32767: the half-sweep index 2t + c fills 16 counter bits
  if (!b || steps < 1 || !betas || theta < 0 || theta > 32767)
    return PA_EINVAL;
  for (int64_t i = 0; i < (int64_t)steps * b->n; ++i)
    if (!std::isfinite(betas[i])) return PA_EINVAL;
  b->mode = 0;
  b->mlp = nullptr;
  b->sched.assign(betas, betas + (size_t)steps * b->n);
  b->sched_steps = steps;
  b->theta = theta;
  return batch_run(b, steps, use_graph);
} catch (const std::bad_alloc&) {
  return PA_ENOMEM;
} catch (const std::exception& e) {
  ::pa::note_exception(e.what());
  return PA_EDEVICE;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_batch_run_adaptive(pa_batch* b, double target, double beta_f,
                          int32_t max_steps, int32_t theta, int32_t use_graph,
                          int32_t* steps_taken) {
  return pa_batch_run_adaptive_tol(b, target, 0.0, beta_f, max_steps, theta,
                                   use_graph, steps_taken);
}

int pa_batch_run_adaptive_tol(pa_batch* b, double target, double tol,
                              double beta_f, int32_t max_steps, int32_t theta,
                              int32_t use_graph, int32_t* steps_taken) try {
  if (!b || !(target > 0.0 && target <= 1.0) || !std::isfinite(beta_f) ||
      !(tol >= 0.0) || max_steps < 1 || theta < 0 || theta > 32767)
    return PA_EINVAL;
  b->mode = 1;
  b->bisect_tol = tol;
  b->mlp = nullptr;
  b->target = target;
  b->beta_f = beta_f;
  b->adaptive_max_steps = max_steps;
  b->theta = theta;
  int rc = batch_run(b, max_steps, use_graph);
  if (steps_taken) {
    int mx = 0;
    for (auto& q : b->pops) mx = std::max(mx, q.step);
    *steps_taken = mx;
  }
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

int pa_batch_run_learned(pa_batch* b, pa_mlp* m, double target, double tol,
                         double beta_f, int32_t max_steps, int32_t theta,
                         int32_t use_graph, int32_t* steps_taken,
                         int64_t* src_counts) try {
  if (!b || !m || !(target > 0.0 && target <= 1.0) || !(tol >= 0.0) ||
      !std::isfinite(beta_f) || max_steps < 1 || theta < 0 || theta > 32767)
    return PA_EINVAL;
  if (mlp_n_in(m) != kFeatures) return PA_EINVAL;
  b->mode = 2;
  b->mlp = m;
  b->target = target;
  b->tol = tol;
  b->beta_f = beta_f;
  b->adaptive_max_steps = max_steps;
  b->theta = theta;
  int rc = batch_run(b, max_steps, use_graph);
  if (steps_taken) {
    int mx = 0;
    for (auto& q : b->pops) mx = std::max(mx, q.step);
    *steps_taken = mx;
  }
  if (src_counts)
    for (int k = 0; k < 5; ++k) src_counts[k] = b->src_count[k];
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

int pa_batch_host_stats(pa_batch* b, double* host_ms, int64_t* overlap_evals,
                        int64_t* src_counts) try {
  if (!b) return PA_EINVAL;
  if (host_ms) *host_ms = b->host_ms;
  if (overlap_evals) *overlap_evals = b->overlap_evals;
  if (src_counts)
    for (int k = 0; k < 5; ++k) src_counts[k] = b->src_count[k];
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

int pa_batch_decisions(pa_batch* b, int32_t p, float* feat, double* dbeta,
                       int32_t* src, float* proposal, int32_t cap,
                       int32_t* len) try {
  if (!b || p < 0 || p >= b->n || cap < 0) return PA_EINVAL;
  const int steps = (int)(b->dec_src.size() / b->n);
  int k = 0;
  for (int i = 0; i < steps && k < cap; ++i) {
    const size_t at = (size_t)i * b->n + p;
    if (b->dec_src[at] < 0) continue;  // the population did not move
    if (feat)
      std::memcpy(feat + (size_t)k * kFeatures, &b->dec_feat[at * kFeatures],
                  sizeof(float) * kFeatures);
    if (dbeta) dbeta[k] = b->dec_dbeta[at];
    if (src) src[k] = b->dec_src[at];
    if (proposal) proposal[k] = b->dec_prop[at];
    ++k;
  }
  if (len) *len = k;
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

int pa_batch_state(pa_batch* b, int32_t p, int64_t* R, double* beta,
                   int32_t* step, double* lnZ) try {
  if (!b || p < 0 || p >= b->n) return PA_EINVAL;
  BK(hipStreamSynchronize(b->stream));
  if (R) *R = rb_R(b)[p];
  if (beta) *beta = b->pops[p].beta;
  if (step) *step = b->pops[p].step;
  if (lnZ) *lnZ = b->pops[p].lnZ;
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

int pa_batch_trajectory(pa_batch* b, int32_t p, pa_obs* obs, double* lnZ,
                        int32_t cap, int32_t* len) try {
  if (!b || p < 0 || p >= b->n) return PA_EINVAL;
  const int steps = b->n ? (int)(b->traj.size() / b->n) : 0;
  int k = 0;
  for (int i = 0; i < steps && k < cap; ++i) {
    const pa_obs& o = b->traj[(size_t)i * b->n + p];
    if (o.R == 0) continue;  // the population had stopped
    if (obs) obs[k] = o;
    if (lnZ) lnZ[k] = b->traj_lnZ[(size_t)i * b->n + p];
    ++k;
  }
  if (len) *len = k;
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

int pa_batch_get_population(pa_batch* b, int32_t p, int8_t* spins, int32_t* E,
                            int32_t* M, int64_t cap) try {
  if (!b || p < 0 || p >= b->n) return PA_EINVAL;
  BK(hipStreamSynchronize(b->stream));
  const BatchPop& d = b->pops[p].d;
  int32_t cur = 0;
  BK(hipMemcpy(&cur, b->d_cur + p, 4, hipMemcpyDeviceToHost));
  int64_t R = 0;
  BK(hipMemcpy(&R, b->d_rb + 8 * (size_t)p, 8, hipMemcpyDeviceToHost));
  if (cap < R) return PA_EINVAL;
  const int N = d.L * d.L;
  if (spins) {
    std::vector<uint8_t> tmp((size_t)(R * d.stride));
    BK(hipMemcpy(tmp.data(), d.spins[cur], tmp.size(), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < R; ++j) {
      const uint8_t* in = tmp.data() + j * d.stride;
      int8_t* s = spins + j * N;
      if (d.int8) {
        std::memcpy(s, in, (size_t)N);
      } else {
        const uint32_t* w = reinterpret_cast<const uint32_t*>(in);
        for (int y = 0; y < d.L; ++y)
          for (int x = 0; x < d.L; ++x)
            s[y * d.L + x] = ((w[y * d.W + x / 32] >> (x % 32)) & 1u) ? 1 : -1;
      }
    }
  }
  if (E) BK(hipMemcpy(E, d.E[cur], (size_t)R * 4, hipMemcpyDeviceToHost));
  if (M) BK(hipMemcpy(M, d.M[cur], (size_t)R * 4, hipMemcpyDeviceToHost));
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

int pa_batch_get_families(pa_batch* b, int32_t p, uint32_t* fam, int64_t cap,
                          int64_t* len, int64_t* n0) try {
  if (!b || p < 0 || p >= b->n) return PA_EINVAL;
  BK(hipStreamSynchronize(b->stream));
  const BatchPop& d = b->pops[p].d;
  int32_t cur = 0;
  BK(hipMemcpy(&cur, b->d_cur + p, 4, hipMemcpyDeviceToHost));
  int64_t R = 0;
  BK(hipMemcpy(&R, b->d_rb + 8 * (size_t)p, 8, hipMemcpyDeviceToHost));
  if (fam && cap < R) return PA_EINVAL;
  if (fam) BK(hipMemcpy(fam, d.fam[cur], (size_t)R * 4, hipMemcpyDeviceToHost));
  if (len) *len = R;
  if (n0) *n0 = b->pops[p].R_t;
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

int pa_batch_get_sweep_blocks(pa_batch* b, int32_t* blocks,
                              int32_t* chunk) try {
  if (!b || !blocks || !chunk) return PA_EINVAL;
  *blocks = b->sweep_blocks;
  *chunk = b->sweep_chunk;
  return PA_OK;
} catch (...) {
  ::pa::note_exception("unknown exception");
  return PA_EDEVICE;
}

int pa_batch_set_sweep_blocks(pa_batch* b, int32_t blocks, int32_t chunk) try {
  if (!b || blocks < 1 || blocks > 65535 || chunk < 1 || chunk > 1024)
    return PA_EINVAL;
  drop_graph(b);
  b->sweep_blocks = blocks;
  b->sweep_chunk = chunk;
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
