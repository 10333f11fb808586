// Internal interfaces between the C ABI (pa_api.hip) and the kernels
// (pa_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

struct LatticeArgs {
  uint8_t* spins;         // buffer base; replica j at spins + j * stride
  int32_t* E;
  int32_t* M;
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
  int32_t init;           // draw the spins from the INIT stream
};

struct HistArgs {
  const int32_t* E;
  const int32_t* M;
  uint32_t* hist;
  unsigned long long* moments;  // [0] sum |M|, [1] sum M^2, [3] bad energies
  int64_t R;
  int32_t twoN, shift, nbins, use_lds;
};

struct CountsArgs {
  const int32_t* E;
  const uint32_t* f;  // integer part of rho per level (from lvl0)
  const uint32_t* T;  // 32-bit threshold of the fractional part per level
  uint32_t* n;
  uint32_t* tile_sum;
  int64_t R;
  int32_t twoN, shift, lvl0, nlvl;
  uint32_t k0, k1, pop, step_next;
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
  int32_t chunks;   // stride / 16
  int32_t lpr_log2; // log2 of the lanes that copy one row
};

hipError_t launch_lattice(const LatticeArgs& a, int W, int RPL, bool int8,
                          bool glass, hipStream_t st);
hipError_t launch_hist(const HistArgs& a, hipStream_t st);
hipError_t launch_counts(const CountsArgs& a, hipStream_t st);
hipError_t launch_scan(const uint32_t* tile_sum, uint32_t* tile_off,
                       int64_t ntiles, unsigned long long* total,
                       hipStream_t st);
hipError_t launch_scatter(const uint32_t* n, const uint32_t* tile_off,
                          int64_t R, int64_t cap, uint32_t* parent,
                          hipStream_t st);
hipError_t launch_gather(const GatherArgs& a, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

}  // namespace pa
