// Issue-rate probe of the vector ALU of gfx950 for the instruction classes
// the Metropolis pass is made of, the measured ceiling its roofline is
// priced against.  Each lane runs `iters` rounds of eight independent
// dependency chains (enough to hide the pipeline latency at any occupancy)
// of one instruction kind; the result is folded into one word per lane and
// written only if it equals a value it cannot take, so nothing is removed.
//
//   kind 0  v_bitop3_b32 (three-input xor)
//   kind 1  v_mad_u64_u32 (32 x 32 -> 64 multiply-add)
//   kind 2  v_xor_b32 (two-input)
//   kind 3  Philox4x32-10 blocks, the generator of the sweep
//
// The vector instruction count per round is fixed by the source; the host
// divides it by the event-timed kernel duration.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_device.h"
#include "pa_probe.h"

namespace {

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(uint32_t* sink, int iters,
                                               uint32_t seed) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[8], b = seed ^ t, c = seed * 0x9E3779B9u + t;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = t * (2u * i + 1u) + seed;
  uint64_t m[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) m[i] = a[i];
  for (int it = 0; it < iters; ++it) {
    if (KIND == 0) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = pa::xor3(a[i], b + i, c);
      b += 1u;
    } else if (KIND == 1) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          m[i] = (uint64_t)(uint32_t)m[i] * (uint64_t)(b | 1u) + m[i];
      b += 2u;
    } else if (KIND == 2) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = (a[i] ^ b) ^ a[(i + 1) & 7];
      b += 1u;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint4 o = pa::philox10(make_uint4(a[i], b, t, seed), seed, c);
        a[i] ^= o.x ^ o.y ^ o.z ^ o.w;
      }
      b += 1u;
    }
  }
  uint32_t acc = 0u;
#pragma unroll
  for (int i = 0; i < 8; ++i) acc ^= a[i] ^ (uint32_t)m[i] ^ (uint32_t)(m[i] >> 32);
  if (acc == 0xFFFFFFFFu && b == 0u) sink[t & 255u] = acc;
}

}  // namespace

extern "C" int pa_probe_valu(int32_t kind, int32_t blocks, int32_t iters,
                             void* stream, double* ms) {
  if (!ms || kind < 0 || kind > 3 || blocks < 1 || iters < 1) return -1;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint32_t* sink = nullptr;
  if (hipMalloc(&sink, 256 * sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return -2;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = -4;
  for (int rep = 0; rc == 0 && rep < 2; ++rep) {  // the first run warms up
    if (hipEventRecord(e0, st) != hipSuccess) rc = -4;
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, st, sink, iters, 7u); break;
      case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, st, sink, iters, 7u); break;
      case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, st, sink, iters, 7u); break;
      default: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, st, sink, iters, 7u); break;
    }
    if (rc == 0 && hipGetLastError() != hipSuccess) rc = -4;
    if (rc == 0 && hipEventRecord(e1, st) != hipSuccess) rc = -4;
    if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -4;
    float f = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = -4;
    *ms = f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  return rc;
}
