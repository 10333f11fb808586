// Lattice pass of the q-state Potts ferromagnet for gfx950 (Sec. 2 names the
// model with the heating protocol): H = -sum over the 2N bonds of
// delta(s, s'), states 0..q-1 stored one byte per site.
//
// One wave per replica, up to 4 replicas per workgroup (at most 16 KB of LDS
// per workgroup): the replica's L x L lattice is staged in LDS, swept theta
// times in place with checkerboard Metropolis, then written back with its
// energy and M = q n_0 - N.
// As in the Ising pass, a pass after a resampling loads every new slot from
// its parent in the other buffer, so the resampling copy costs no pass of its
// own.
//
// Random numbers: colour site k = x/2 of row y takes Philox group
// y*ceil(L/4) + k/2 of the MCMC stream (half sweep 2t + c): words 2(k%2)
// (proposal) and 2(k%2) + 1 (acceptance).  The proposal is one of the other
// q - 1 states, s' = (s + 1 + floor(w (q-1) / 2^32)) mod q; it is accepted iff
// dE = (#neighbours in s) - (#neighbours in s') <= 0 or r < T[dE],
// T[d] = floor(exp(-beta d) 2^32).  The initial state takes
// floor(w q / 2^32) of the site's INIT word (word x%4 of group
// y*ceil(L/4) + x/4), the ground-state start the same of word 0 of group 0
// for every site.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_device.h"
#include "pa_internal.h"
#include "pa_potts.h"

namespace pa {

__global__ __launch_bounds__(256) void k_potts(const LatticeArgs a) {
  extern __shared__ uint32_t lds_words[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int L = a.L, N = L * L, q = a.q;
  const int64_t R = a.Rdev ? min((int64_t)*a.Rdev, a.R) : a.R;
  if ((int64_t)blockIdx.x * wpb >= R) return;  // the whole workgroup is idle
  const int64_t rep = (int64_t)blockIdx.x * wpb + wave;
  // a wave past the population keeps to the workgroup barriers only
  const bool active = rep < R;
  const uint32_t slot = (uint32_t)(active ? rep : 0);
  const int G4 = (L + 3) >> 2;
  const int nw = N >> 2;  // L is even, so N is a multiple of 4
  uint32_t* lw = lds_words + (size_t)wave * nw;
  int8_t* lat = reinterpret_cast<int8_t*>(lw);
  uint8_t* dst = a.spins + (size_t)slot * (size_t)a.stride;
  const uint8_t* src =
      a.parent ? a.src + (size_t)a.parent[slot] * (size_t)a.stride : dst;

  if (!active) {
  } else if (a.init == 2) {
    const uint4 b = philox10(make_uint4(kDomainInit << 28, 0u, slot, a.pop),
                             a.k0, a.k1);
    const uint32_t st = mulhi_q(b.x, (uint32_t)q);
    const uint32_t word = st * 0x01010101u;
    for (int i = lane; i < nw; i += 64) lw[i] = word;
  } else if (a.init) {
    for (int g = lane; g < L * G4; g += 64) {
      const int y = g / G4, x0 = (g - y * G4) * 4;
      const uint4 b = philox10(make_uint4((kDomainInit << 28) | (uint32_t)g,
                                          0u, slot, a.pop),
                               a.k0, a.k1);
      const uint32_t w[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (x0 + j < L) lat[y * L + x0 + j] = (int8_t)mulhi_q(w[j], (uint32_t)q);
    }
  } else {
    const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
    for (int i = lane; i < nw; i += 64) lw[i] = s32[i];
  }
  __syncthreads();

  // work item g = y*G4 + m (a Philox group: sites 2m and 2m+1 of colour c
  // in row y); lane items advance by 64 = dy rows and dm groups
  const int dy = 64 / G4, dm = 64 - dy * G4;
  const int y_first = lane / G4, m_first = lane - y_first * G4;
  for (int t = 0; t < a.theta; ++t) {
    for (int c = 0; c < 2; ++c) {
      const uint32_t ctr1 = (a.step << 16) | (uint32_t)(2 * (a.t0 + t) + c);
      int y = y_first, m = m_first;
      for (int g = lane; active && g < L * G4; g += 64) {
        const uint4 b = philox10(make_uint4((kDomainMcmc << 28) | (uint32_t)g,
                                            ctr1, slot, a.pop),
                                 a.k0, a.k1);
        const int yu = (y == 0) ? L - 1 : y - 1, yd = (y == L - 1) ? 0 : y + 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = 2 * m + h;
          if (k >= (L >> 1)) break;
          const int x = 2 * k + ((y + c) & 1);
          const int xl = (x == 0) ? L - 1 : x - 1, xr = (x == L - 1) ? 0 : x + 1;
          const uint32_t w = h ? b.z : b.x, r = h ? b.w : b.y;
          const int sv = lat[y * L + x];
          int sn = sv + 1 + (int)mulhi_q(w, (uint32_t)(q - 1));
          if (sn >= q) sn -= q;
          const int n0 = lat[y * L + xl], n1 = lat[y * L + xr],
                    n2 = lat[yu * L + x], n3 = lat[yd * L + x];
          const int dE = ((n0 == sv) + (n1 == sv) + (n2 == sv) + (n3 == sv)) -
                         ((n0 == sn) + (n1 == sn) + (n2 == sn) + (n3 == sn));
          if (dE <= 0 || (uint64_t)r < a.Tp[dE - 1]) lat[y * L + x] = (int8_t)sn;
        }
        y += dy;
        m += dm;
        if (m >= G4) {
          m -= G4;
          ++y;
        }
      }
      __syncthreads();  // the other colour reads these sites
    }
  }

  if (!active) return;  // no barrier follows
  // energy and M of the final state
  int e = 0, z = 0;
  {
    const int ey = 64 / L, ex = 64 - ey * L;  // site i advances by 64
    int y = lane / L, x = lane - (lane / L) * L;
    for (int i = lane; i < N; i += 64) {
      const int sv = lat[i];
      e -= (sv == lat[y * L + ((x == L - 1) ? 0 : x + 1)]);
      e -= (sv == lat[((y == L - 1) ? 0 : y + 1) * L + x]);
      z += (sv == 0);
      y += ey;
      x += ex;
      if (x >= L) {
        x -= L;
        ++y;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_down(e, off, 64);
    z += __shfl_down(z, off, 64);
  }
  uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
  for (int i = lane; i < nw; i += 64) d32[i] = lw[i];
  if (lane == 0) {
    a.E[rep] = e;
    a.M[rep] = q * z - N;
  }
}

template <int MPR>
__global__ __launch_bounds__(256) void k_potts_swar(const LatticeArgs a) {
  extern __shared__ uint32_t lds_words[];
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int64_t R = a.Rdev ? min((int64_t)*a.Rdev, a.R) : a.R;
  if ((int64_t)blockIdx.x * wpb >= R) return;  // the whole workgroup is idle
  const int64_t rep = (int64_t)blockIdx.x * wpb + wave;
  potts_swar_pass<MPR>(a, rep, rep < R, lds_words);
}

hipError_t launch_potts(const LatticeArgs& a, hipStream_t st) {
  if (a.R <= 0) return hipSuccess;
  const int64_t N = (int64_t)a.L * a.L;
  const int wpb = N <= 4096 ? 4 : N <= 8192 ? 2 : 1;  // <= 16 KB of LDS
  const int64_t blocks = (a.R + wpb - 1) / wpb;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(64 * wpb);
  const size_t shm = (size_t)(wpb * (72 + N));  // a table and a lattice per wave
  switch (a.L) {
    case 8: hipLaunchKernelGGL(k_potts_swar<1>, grid, block, shm, st, a); break;
    case 16: hipLaunchKernelGGL(k_potts_swar<2>, grid, block, shm, st, a); break;
    case 32: hipLaunchKernelGGL(k_potts_swar<4>, grid, block, shm, st, a); break;
    case 64: hipLaunchKernelGGL(k_potts_swar<8>, grid, block, shm, st, a); break;
    case 128: hipLaunchKernelGGL(k_potts_swar<16>, grid, block, shm, st, a); break;
    default:
      hipLaunchKernelGGL(k_potts, grid, block, (size_t)(wpb * N), st, a);
  }
  return hipGetLastError();
}

}  // namespace pa
