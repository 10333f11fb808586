// Internal interfaces between the C ABI (pa_api.hip) and the kernels
// (pa_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pa.h"

namespace pa {

struct LatticeArgs {
  uint8_t* spins;         // buffer base; replica j at spins + j * stride
  int32_t* E;
  int32_t* M;
  // resampling copies fused into the pass: when parent is set, replica j is
  // read from src + parent[j] * stride (the other buffer) instead of its own
  // slot, and written to its own slot of `spins`
  const uint8_t* src;
  const uint32_t* parent;
  // when set, the replica count is min(*Rdev, R): R is then only a bound
  // (the grid size) and the exact count is still on the device
  const unsigned long long* Rdev;
  const uint32_t* jbits;  // +-J couplings, [2][L][W] bits, set where J < 0
  int64_t R;              // replicas to process
  int64_t stride;         // bytes per replica (multiple of 16)
  int32_t L;
  int32_t lpr;            // lanes per replica = L / rows per lane
  int32_t rpw;            // replicas per wave = 64 / lpr
  uint64_t K4, K8;        // 2^32 - T for the Metropolis thresholds
                          // T = floor(exp(-beta dE) 2^32), dE = 4, 8
  uint32_t one;           // the constant 1, opaque to the compiler
  uint32_t k0, k1;        // Philox key
  uint32_t pop, step;
  int32_t t0, theta;      // first sweep index at this step, sweep count
  int32_t init;           // 1: draw the spins from the INIT stream;
                          // 2: ferromagnet ground states (heating start)
  // q-state Potts pass only: the number of states and the acceptance
  // thresholds T[d - 1] = floor(exp(-beta d) 2^32), d = 1..4
  int32_t q;
  uint64_t Tp[4];
};

// One record per temperature step of a schedule run on the device
// (pa_anneal), written by the last workgroup of the step's histogram: the
// population it counted, its exact sums and the reweighting sum of the
// step's tables (64 bytes).
struct AnnealRec {
  unsigned long long R;   // replicas counted
  unsigned long long Rc;  // replicas the copy counts read: R, or 0 once the
                          // schedule has stopped
  unsigned long long sumAbsM, sumM2;
  long long sumE, sumE2;
  double S;               // sum of h w over the occupied levels, in order
  int32_t lo, nl;         // first occupied level, level count (0: none)
};
static_assert(sizeof(AnnealRec) == 64, "record layout");

// The first step of such a schedule that failed, 0 while none has
// (kHaltWait: a wait of the single-pass scan for an earlier tile gave up).
enum { kHaltCapacity = 1, kHaltEmpty = 2, kHaltEnergy = 3, kHaltWait = 4 };
struct AnnealHalt {
  uint32_t code, step;      // step: index of the failed resampling
  unsigned long long total; // the new size that failed (capacity, empty)
};

// One workgroup's part of a step's histogram: its moment sums, exact energy
// sums and occupied range (lo_rev = max of nbins - bin, hi1 = max of bin +
// 1; both 0 when it counted nothing); the last workgroup adds them up.
struct BlockSums {
  unsigned long long sAbsM, sM2;
  long long sE, sE2;
  uint32_t lo_rev, hi1;
  uint32_t pad[2];
};
static_assert(sizeof(BlockSums) == 48, "block sums layout");

// The first kArgWeights weights exp(-dbeta d 2^shift) of a step, in the
// histogram kernel's arguments (no read from host memory for them).
constexpr int kArgWeights = 440;
struct ArgWeights {
  double w[kArgWeights];
};

struct HistArgs {
  const int32_t* E;
  const int32_t* M;
  uint32_t* hist;
  unsigned long long* moments;  // [0] sum |M|, [1] sum M^2, [3] bad energies
  int64_t R;
  const unsigned long long* Rdev;  // as in LatticeArgs
  int32_t twoN, shift, nbins;
  // bins [win_lo, win_lo + win_n) are counted in LDS first (win_n <= 16384);
  // a replica outside the window goes to the global histogram directly
  int32_t win_lo, win_n;
  // when host_rb is set, the last workgroup to finish copies the read-back
  // block (rb_words words, a multiple of 4, from `rb`, which holds hist and
  // the moments) to
  // host memory and then writes `seq` to *host_flag; `counter` (device,
  // zero between calls) finds that workgroup
  const uint32_t* rb;
  uint32_t* host_rb;
  uint32_t* host_flag;
  uint32_t* counter;
  uint32_t seq;
  int32_t rb_words;
  // schedule on the device (rec set): the last workgroup writes *rec and,
  // with wtab set, the nearest-integer tables of the step (f to tab_f, T to
  // tab_T, levels from rec->lo) from the weights wtab[d] = exp(-dbeta d
  // 2^shift) the host computed (d >= kArgWeights read there, the others
  // from the arguments), through the scratch wscr (nbins doubles);
  // a bad energy stops the schedule (*halt, and *Rw = 0 so that every later
  // kernel of it finds no replicas)
  AnnealRec* rec;
  AnnealHalt* halt;
  unsigned long long* Rw;
  const double* wtab;
  double* wscr;
  uint32_t* tab_f;
  uint32_t* tab_T;
  int64_t R_t;
  uint32_t step;
  // with weights: their sequence number, written to *progress (host
  // memory) once they are read
  uint32_t* progress;
  uint32_t wseq;
  BlockSums* part;  // one per workgroup (at most 256)
};

struct CountsArgs {
  const int32_t* E;
  const uint32_t* f;  // integer part of rho per level (from lvl0)
  const uint32_t* T;  // 32-bit threshold of the fractional part per level
  uint32_t* n;
  uint32_t* tile_sum;
  uint32_t* clear;    // words [0, nclear) set to zero on the way (may be null)
  int64_t nclear;
  // Poisson law: when set, f points to the level table of
  // build_poisson_tables (T is unused)
  int32_t poisson;
  // multinomial kernels: residual law (floor(rho) copies kept, the draws
  // over the fractional parts only)
  int32_t residual;
  int64_t R;
  int32_t twoN, shift, lvl0, nlvl;
  uint32_t k0, k1, pop, step_next;
  // schedule on the device: the replica count min(*Rdev, R) and the level
  // range (lvl_dev[0], lvl_dev[1]) come from the step's record
  const unsigned long long* Rdev;
  const int32_t* lvl_dev;
};

// Single-pass counts, scan and parent map of a schedule on the device: each
// workgroup takes the next tile from *ticket, publishes its tile's sum in
// status[tile] and looks back over the earlier tiles for its prefix
// (decoupled look-back); *done finds the last workgroup, which resets both
// counters.  Status words carry the launch's generation, so the array
// needs no clearing.
struct LookbackArgs {
  unsigned long long* status;  // [ntiles]
  uint32_t* ticket;
  uint32_t* done;
  uint32_t gen;                // 28 bits used
  int64_t ntiles;
  int64_t cap;
  uint32_t* parent;
  const uint32_t* fam_src;
  uint32_t* fam_dst;
  unsigned long long* total;   // the new size (0 once the schedule stops)
  AnnealHalt* halt;
  uint32_t step;
};

// Nearest-integer tables of at most kArgLevels occupied levels, passed by
// value in the kernel arguments: no upload of their own.
constexpr int kArgLevels = 448;
struct ArgTables {
  uint32_t f[kArgLevels];
  uint32_t T[kArgLevels];
};

struct GatherArgs {
  const uint8_t* src;
  uint8_t* dst;
  const int32_t* E_src;
  const int32_t* M_src;
  int32_t* E_dst;
  int32_t* M_dst;
  const uint32_t* parent;
  int64_t R_new;
  int64_t stride;   // bytes per replica, multiple of 16
  int32_t chunks;      // stride / 16
  int32_t chunks_log2; // log2(chunks) when it is a power of two, else -1
};

// ---- batched populations (pa_batch.hip)
struct BatchPop {          // static description of one population
  uint8_t* spins[2];
  int32_t* E[2];
  int32_t* M[2];
  uint32_t* n;             // copy counts            [cap]
  uint32_t* parent;        // parent of each new slot [cap]
  uint32_t* fam[2];        // family of each replica  [cap], buffer cur
  uint32_t* tile_sum;      // per 256-replica tile   [cap/256 + 1]
  uint32_t* tile_off;
  uint32_t* hist;          // energy histogram       [nbins]
  uint32_t* tab;           // f[nbins] then T[nbins]
  const uint32_t* jbits;   // +-J couplings or null
  int64_t cap, stride;
  int32_t L, W, rpl, lpr, rpw, nbins, shift, glass, int8, chunks, lpr_log2;
  int32_t q;               // Potts states (0: Ising)
  uint32_t k0, k1, pop;
  int32_t planes;          // sweep random numbers: 1 bit planes, 0 words
  int32_t pad_;
};

struct BatchStep {         // per population, rewritten by the host each step
  uint64_t K4, K8;         // Metropolis thresholds at the new beta
  uint64_t Tp[4];          // Potts: T[d - 1] = floor(exp(-beta d) 2^32)
  double beta;             // the population's beta after this step
  double target;           // overlap target of the adaptive schedule
  int32_t lvl0, nlvl;      // table range (histogram levels)
  uint32_t step;           // index of the temperature being entered
  int32_t theta;           // sweeps at the new beta
  int32_t active;          // 0: the population does not move this step
  int32_t pad;
};

// Sweep shape when the caller leaves rows_per_lane at 0 and nothing is
// tuned: three rows per lane fill whole waves at L = 48 and 96 (16 and 32
// lanes per replica), where the tuner measured them fastest; two rows above
// L = 64 keep the registers in bounds; one row otherwise.  The plane stream
// takes two rows at L = 64 from 2^14 replicas: a lane then resolves the
// ties of 64 draws per half sweep, merged two words into one, in fewer
// passes per draw than of 32, and int8 replicas still move as whole
// kilobytes, two per wave.  Whole int8 anneals against one row: +4.5 % at
// R = 20480 and +7.5 % at 65536 with theta = 10, +4.7 % at 65536 with
// theta = 3, equal at 32768 and 65536 with theta = 1, -1.5 % at 20480
// with theta = 1; bit-packed +8 % at 65536 with theta = 10.
inline int default_rows_per_lane(int L, bool planes = false,
                                 int64_t R = 0) {
  if (planes && L == 64 && R >= (1 << 14)) return 2;
  return (L == 48 || L == 96) ? 3 : (L > 64 ? 2 : 1);
}

// Fastest rows-per-lane of a single population's sweep, timed on a test
// population (pa_batch.hip; pa_tune_rows_per_lane is its word-stream form).
int tune_rows_per_lane(int32_t L, int32_t layout, int32_t model,
                       int32_t rng_mode, int64_t R, int32_t theta,
                       void* stream, int32_t* best, float* ms);

// Rows per lane of each population of a batch (0 where not tuned), timed
// with the batch's own persistent sweep on scratch batches (pa_batch.hip).
int tune_batch_rows(const pa_config* cfgs, int n, void* stream,
                    std::vector<int>* out);

// Fastest persistent-sweep launch shape of a batch of these populations,
// timed on a scratch batch (pa_batch.hip).
int tune_sweep_shape(const pa_config* cfgs, int n, void* stream,
                     int* blocks, int* chunk);

// Histogram summaries fed to the temperature-step network (kFeatures per
// population, computed on the device from the exact histogram).
constexpr int kFeatures = 8;



// ---- temperature-step network (pa_mlp.hip), used by the batch
int mlp_prepare(pa_mlp* m, int B);
int mlp_infer_on(pa_mlp* m, const float* X, int B, hipStream_t st);
const float* mlp_output_dev(pa_mlp* m);
void mlp_out_scale(const pa_mlp* m, float* mu_y, float* sigma_y);
int mlp_n_in(const pa_mlp* m);
uint64_t mlp_generation(const pa_mlp* m);

// ---- diagnostics: text of the last failing HIP call on this thread
void set_last_error(const char* what, hipError_t e, int line);
// a C++ exception stopped at the ABI (reported as PA_EDEVICE)
void note_exception(const char* what);
// another device-side inconsistency reported as PA_EDEVICE
void note_error(const char* text);

// PA_OK, or PA_EDEVICE with the failed call recorded.
inline int hip_ok(hipError_t e, const char* what, int line) {
  if (e == hipSuccess) return PA_OK;
  set_last_error(what, e, line);
  return PA_EDEVICE;
}

// Evaluate a HIP call; on failure record it and return PA_EDEVICE.
#define PA_HIP(x)                                   \
  do {                                              \
    const hipError_t pa_e_ = (x);                   \
    if (pa_e_ != hipSuccess) {                      \
      ::pa::set_last_error(#x, pa_e_, __LINE__);    \
      return PA_EDEVICE;                            \
    }                                               \
  } while (0)

// ---- host double-precision helpers (pa_tables.hip)
struct TableRange {
  int lo, hi;    // occupied histogram levels; tables hold levels lo..hi
  double lnQ;    // ln Q of the step (Eq. part-Q)
};
void occupied_range(const uint32_t* h, int nbins, int* lo, int* hi);
void metropolis_K(double beta, uint64_t* K4, uint64_t* K8);
void potts_thresholds(double beta, uint64_t Tp[4]);
int build_tables(const uint32_t* h, int nbins, int shift, int N, int64_t R,
                 int64_t R_t, double dbeta, uint32_t* f, uint32_t* T,
                 TableRange* out);
int build_poisson_tables(const uint32_t* h, int nbins, int shift, int N,
                         int64_t R, int64_t R_t, double dbeta,
                         std::vector<uint32_t>& out, TableRange* tr,
                         int64_t* n_min, int64_t* n_max);
double overlap_from_hist(const uint32_t* h, int nbins, int shift, int N,
                         int64_t R, double dbeta);
void observables_from_hist(const uint32_t* h, int nbins, int shift, int N,
                           int64_t R, double beta, int64_t sumAbsM,
                           int64_t sumM2, pa_obs* o);
void observables_from_sums(int64_t R, double beta, int N, int64_t sumE,
                           int64_t sumE2, int64_t sumAbsM, int64_t sumM2,
                           int32_t Emin, int32_t Emax, pa_obs* o);
double bisect_from_hist(const uint32_t* h, int nbins, int shift, int N,
                        int64_t R, double target, double span,
                        int* evals = nullptr, double tol = 0.0);

// ---- debug and metrics hooks, read from the environment at each use
// (pa_tables.hip):
//   PA_FAULT=alloc|energy|capacity  force a failure from the host: pa_init's
//     device allocations fail; the next histogram reports an energy outside
//     its range; the next resampling exceeds the capacity
//   PA_LOG_JSONL=<path>  append one JSON object per resampling step
bool fault_injected(const char* what);
struct StepLog {
  int64_t pop, step, R_prev, R;  // R < 0: the new size is still on the device
  double beta, dbeta, lnQ, lnZ, overlap;
  double e_prev, abs_m_prev, C_prev;  // observables before the resampling
  const char* source;                 // how the step was chosen
};
void log_step(const StepLog& s);

// ---- kernel launchers (pa_kernels.hip)
hipError_t launch_lattice(const LatticeArgs& a, int W, int RPL, bool int8,
                          bool glass, bool planes, hipStream_t st);
hipError_t launch_hist(const HistArgs& a, hipStream_t st);
// the histogram of a step of a schedule on the device (a.rec set), the
// first weights in the arguments (a.wtab holds them all)
hipError_t launch_hist_sched(const HistArgs& a, const ArgWeights& w,
                             hipStream_t st);
// parent map of at most 256 tiles with its own scan of the tile sums (the
// new size to *total)
hipError_t launch_scatter_scan(const uint32_t* n, const uint32_t* tile_sum,
                               int64_t R, int64_t cap, uint32_t* parent,
                               const uint32_t* fam_src, uint32_t* fam_dst,
                               unsigned long long* total, hipStream_t st);
// copy counts of the nearest-integer law with the tables in the arguments
hipError_t launch_counts_args(const CountsArgs& a, const ArgTables& t,
                              hipStream_t st);
hipError_t launch_potts(const LatticeArgs& a, hipStream_t st);
hipError_t launch_sys_counts(const CountsArgs& a, uint64_t* tile64,
                             uint64_t* off64, hipStream_t st);
hipError_t launch_multi_counts(const CountsArgs& a, int64_t draws,
                               uint64_t* tile64, uint64_t* off64,
                               uint64_t* cum, hipStream_t st);
hipError_t launch_counts(const CountsArgs& a, hipStream_t st);
hipError_t launch_scan(const uint32_t* tile_sum, uint32_t* tile_off,
                       int64_t ntiles, unsigned long long* total,
                       hipStream_t st);
hipError_t launch_scatter(const uint32_t* n, const uint32_t* tile_off,
                          int64_t R, int64_t cap, uint32_t* parent,
                          const uint32_t* fam_src, uint32_t* fam_dst,
                          hipStream_t st);
hipError_t launch_gather(const GatherArgs& a, hipStream_t st);
// (at most kLookbackTiles tiles: with more, the waits for earlier tiles
// cost more than the two launches they save)
constexpr int64_t kLookbackTiles = 256;
hipError_t launch_counts_scatter(const CountsArgs& a, const LookbackArgs& s,
                                 hipStream_t st);
// counts, scan and parent map in three launches for more tiles: the old
// size is read from *Rdev (R and cap bound the grid); a new size of 0 or
// above cap stops the schedule (*halt, and the size written is 0)
hipError_t launch_scan_dev(const uint32_t* tile_sum, uint32_t* tile_off,
                           int64_t ntiles, unsigned long long* total,
                           int64_t cap, AnnealHalt* halt, uint32_t step,
                           hipStream_t st);
hipError_t launch_scatter_dev(const uint32_t* n, const uint32_t* tile_off,
                              int64_t R, const unsigned long long* Rdev,
                              int64_t cap, uint32_t* parent,
                              const uint32_t* fam_src, uint32_t* fam_dst,
                              hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t st);

}  // namespace pa
