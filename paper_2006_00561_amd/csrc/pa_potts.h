// Potts lattice pass with four sites per 32-bit word, shared by the
// single-population kernel (pa_potts.hip) and the persistent batched kernel
// (pa_batch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_device.h"
#include "pa_internal.h"

namespace pa {

__device__ __forceinline__ uint32_t mulhi_q(uint32_t w, uint32_t q) {
  return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

// The same pass for L = 8 MPR with MPR = 1, 2, 4, 8 or 16 (the dwords per
// colour row), four sites per VALU word.  In LDS the replica is split by
// colour: colour c holds the L/2 sites x = 2k + p of row y (p = (y + c) & 1)
// as bytes k of MPR dwords, so one dword holds the four sites k = 4m..4m+3.
// Their neighbours are dwords of the other colour: the same dword in rows
// y - 1, y + 1 and y, and in row y the same dword moved by one byte towards
// k + 1 (p = 1) or k - 1 (p = 0).  States fit in four bits, so the number of
// unequal neighbours of all four sites is a sum of four (a ^ b) + 0x0F masks
// per byte, for the current and the proposed states alike; the four
// acceptance decisions then take the carry of r + K[dE] (K = 2^32 - T, from
// a nine-entry table indexed by dE + 4, zero for dE <= 0).  The Philox words,
// and so the results, are the generic pass's.
//
// A lane keeps one dword column m = lane % MPR and the rows y = lane / MPR +
// 64 i / MPR; the row step is even (or there is one row per lane), so p is
// fixed per lane and colour and every address moves by 64 dwords per row
// step, except the wrapped neighbour rows of the first and last steps.

// 16 per byte where the bytes of a and b differ (bytes at most 15).
__device__ __forceinline__ uint32_t neq16(uint32_t a, uint32_t b) {
  return ((a ^ b) + 0x0F0F0F0Fu) & 0x10101010u;
}

// One wave's replica `rep` (active) of a workgroup whose waves all call this
// together (the barriers are the workgroup's).  lds_words holds one
// nine-entry threshold table per wave (its replica's beta; the waves of a
// batch workgroup may hold different populations), then 2 NWC dwords per
// wave.
template <int MPR>
__device__ __forceinline__ void potts_swar_pass(const LatticeArgs& a,
                                                int64_t rep, bool active,
                                                uint32_t* lds_words) {
  constexpr int L = 8 * MPR, N = L * L;
  constexpr int NWC = L * MPR;          // dwords per colour
  constexpr int DY = 64 / MPR;          // row step of a lane
  constexpr int IT = (NWC + 63) / 64;   // row steps
  constexpr int G4 = L / 4;             // Philox groups per row
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int q = a.q;
  const uint32_t slot =
      __builtin_amdgcn_readfirstlane((uint32_t)(active ? rep : 0));
  // K[e] for e = dE + 4: 0 for dE <= 0, 2^32 - T[dE - 1] above
  uint64_t* ktab = reinterpret_cast<uint64_t*>(lds_words + 18 * wave);
  if (lane < 9)
    ktab[lane] = lane <= 4 ? 0ull : (1ull << 32) - a.Tp[lane - 5];
  uint32_t* A = lds_words + 18 * wpb + (size_t)wave * 2 * NWC;
  uint8_t* dst = a.spins + (size_t)slot * (size_t)a.stride;
  const uint8_t* src =
      a.parent ? a.src + (size_t)a.parent[slot] * (size_t)a.stride : dst;
  const bool lane_on = active && lane < NWC;

  // staging: natural dwords 2d, 2d + 1 (sites 8j..8j+7 of row y, d =
  // y MPR + j) give dword d of each colour; the even sites belong to colour
  // y & 1
  if (!active) {
  } else if (a.init == 2) {
    const uint4 b = philox10(make_uint4(kDomainInit << 28, 0u, slot, a.pop),
                             a.k0, a.k1);
    const uint32_t word = mulhi_q(b.x, (uint32_t)q) * 0x01010101u;
    for (int i = lane; i < 2 * NWC; i += 64) A[i] = word;
  } else {
    for (int d = lane; d < NWC; d += 64) {
      const int y = d / MPR, j = d % MPR;
      uint32_t lo, hi;
      if (a.init) {
        const uint32_t g = (uint32_t)(y * G4 + 2 * j);
        const uint4 b0 = philox10(
            make_uint4((kDomainInit << 28) | g, 0u, slot, a.pop), a.k0, a.k1);
        const uint4 b1 = philox10(
            make_uint4((kDomainInit << 28) | (g + 1), 0u, slot, a.pop), a.k0,
            a.k1);
        const uint32_t uq = (uint32_t)q;
        lo = mulhi_q(b0.x, uq) | (mulhi_q(b0.y, uq) << 8) |
             (mulhi_q(b0.z, uq) << 16) | (mulhi_q(b0.w, uq) << 24);
        hi = mulhi_q(b1.x, uq) | (mulhi_q(b1.y, uq) << 8) |
             (mulhi_q(b1.z, uq) << 16) | (mulhi_q(b1.w, uq) << 24);
      } else {
        const uint2 v = reinterpret_cast<const uint2*>(src)[d];
        lo = v.x;
        hi = v.y;
      }
      const int c0 = y & 1;
      A[c0 * NWC + d] = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
      A[(c0 ^ 1) * NWC + d] = __builtin_amdgcn_perm(hi, lo, 0x07050301u);
    }
  }
  __syncthreads();

  const int m = lane % MPR, y0 = lane / MPR;
  const int base = y0 * MPR + m;                           // dword of row y0
  const int up0 = ((y0 + L - 1) % L) * MPR + m;            // row above, step 0
  const int dn_last = ((y0 + (IT - 1) * DY + 1) % L) * MPR + m;  // row below,
                                                                // last step
  const uint32_t qm1 = (uint32_t)(q - 1);
  const uint32_t ge_add = (uint32_t)(128 - q) * 0x01010101u;
  const uint32_t qq = (uint32_t)q * 0x01010101u;
  for (int t = 0; t < a.theta; ++t) {
    for (int c = 0; c < 2; ++c) {
      const uint32_t ctr1 = (a.step << 16) | (uint32_t)(2 * (a.t0 + t) + c);
      uint32_t* Sc = A + c * NWC;
      const uint32_t* B = A + (c ^ 1) * NWC;
      const int p = (y0 + c) & 1;
      const int mn = p ? (m + 1) % MPR : (m + MPR - 1) % MPR;
      const int hn = y0 * MPR + mn;
      // byte k + 1 (p = 1) or k - 1 (p = 0) of the row: a byte permute of
      // the dword and its neighbour dword
      const uint32_t hsel = p ? 0x04030201u : 0x02010007u;
      if (lane_on) {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
          const int o = 64 * i;
          const uint32_t S = Sc[base + o];
          const uint32_t H0 = B[base + o];
          const uint32_t H1 = __builtin_amdgcn_perm(B[hn + o], H0, hsel);
          const uint32_t U = B[i == 0 ? up0 : base + o - MPR];
          const uint32_t D = B[i == IT - 1 ? dn_last : base + o + MPR];
          const uint32_t g0 = (uint32_t)(2 * (base + o));  // y G4 + 2 m
          const uint4 b0 = philox10(
              make_uint4((kDomainMcmc << 28) | g0, ctr1, slot, a.pop), a.k0,
              a.k1);
          const uint4 b1 = philox10(
              make_uint4((kDomainMcmc << 28) | (g0 + 1), ctr1, slot, a.pop),
              a.k0, a.k1);
          // proposals s' = (s + 1 + floor(w (q - 1) / 2^32)) mod q, bytewise
          const uint32_t P = mulhi_q(b0.x, qm1) | (mulhi_q(b0.z, qm1) << 8) |
                             (mulhi_q(b1.x, qm1) << 16) |
                             (mulhi_q(b1.z, qm1) << 24);
          uint32_t Sn = S + P + 0x01010101u;
          {
            // 0x80 in the bytes at or above q, widened to 0x7F, masks q off
            const uint32_t t = (Sn + ge_add) & 0x80808080u;
            Sn -= (t - (t >> 7)) & qq;
          }
          const uint32_t NO =
              neq16(S, H0) + neq16(S, H1) + neq16(S, U) + neq16(S, D);
          const uint32_t NN =
              neq16(Sn, H0) + neq16(Sn, H1) + neq16(Sn, U) + neq16(Sn, D);
          // byte i: 16 (dE_i + 4), dE = unequal(s') - unequal(s); half of
          // it is the byte offset of K[dE + 4]
          const uint32_t Dv = NN + 0x40404040u - NO;
          const char* kb = reinterpret_cast<const char*>(ktab);
          const uint32_t r0 = reject_bit(
              b0.y, a.one,
              *reinterpret_cast<const uint64_t*>(kb + ((Dv >> 1) & 0x7Fu)));
          const uint32_t r1 = reject_bit(
              b0.w, a.one,
              *reinterpret_cast<const uint64_t*>(kb + ((Dv >> 9) & 0x7Fu)));
          const uint32_t r2 = reject_bit(
              b1.y, a.one,
              *reinterpret_cast<const uint64_t*>(kb + ((Dv >> 17) & 0x7Fu)));
          const uint32_t r3 = reject_bit(
              b1.w, a.one,
              *reinterpret_cast<const uint64_t*>(kb + ((Dv >> 25) & 0x7Fu)));
          // 0xFF in the bytes whose proposal is rejected
          const uint32_t rj = r0 | (r1 << 8) | (r2 << 16) | (r3 << 24);
          const uint32_t keep = (rj << 8) - rj;
          Sc[base + o] = (S & keep) | (Sn & ~keep);
        }
      }
      __syncthreads();  // the other colour reads these sites
    }
  }

  if (!active) return;  // no barrier follows
  // E = (number of unequal bonds) - 2N, each bond counted once from its
  // colour-0 end; M = q n_0 - N
  int e = 0, nz = 0;
  for (int d = lane; d < NWC; d += 64) {
    const int y = d / MPR, j = d % MPR;
    const int pp = y & 1;  // colour 0 sits at x = 2k + (y & 1)
    const int jn = pp ? (j + 1) % MPR : (j + MPR - 1) % MPR;
    const uint32_t* B = A + NWC;
    const uint32_t S = A[d], H0 = B[d];
    const uint32_t H1 = __builtin_amdgcn_perm(B[y * MPR + jn], H0,
                                              pp ? 0x04030201u : 0x02010007u);
    const uint32_t NO = neq16(S, H0) + neq16(S, H1) +
                        neq16(S, B[((y + L - 1) % L) * MPR + j]) +
                        neq16(S, B[((y + 1) % L) * MPR + j]);
    e += (int)((((NO >> 4) * 0x01010101u) >> 24) & 0xFFu);
    nz += __builtin_popcount((S + 0x0F0F0F0Fu) & 0x10101010u) +
          __builtin_popcount((H0 + 0x0F0F0F0Fu) & 0x10101010u);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_down(e, off, 64);
    nz += __shfl_down(nz, off, 64);
  }
  uint2* d64 = reinterpret_cast<uint2*>(dst);
  for (int d = lane; d < NWC; d += 64) {
    const int c0 = (d / MPR) & 1;
    const uint32_t ev = A[c0 * NWC + d], od = A[(c0 ^ 1) * NWC + d];
    d64[d] = make_uint2(__builtin_amdgcn_perm(od, ev, 0x05010400u),
                        __builtin_amdgcn_perm(od, ev, 0x07030602u));
  }
  if (lane == 0) {
    a.E[rep] = e - 2 * N;
    a.M[rep] = q * (N - nz) - N;
  }
}

}  // namespace pa
