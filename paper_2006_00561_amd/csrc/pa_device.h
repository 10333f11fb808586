// Device helpers for the gfx950 population-annealing kernels: the Philox
// counter generator and bit-sliced operations on lattice rows.
//
// A lattice row of L sites is held as W32 = ceil(L/32) 32-bit words, site x
// in bit x%32 of word x/32, bit set = spin +1; bits at x >= L are zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

constexpr uint32_t kDomainInit = 1u;
constexpr uint32_t kDomainMcmc = 2u;
constexpr uint32_t kDomainResample = 3u;
// bit planes of the sweep's second random-number mode
constexpr uint32_t kDomainMcmcPlanes = 5u;

// Three-input XOR in one VALU instruction (gfx950 v_bitop3_b32, truth
// table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by the round constants, a swap of the halves and a
// xor with the key, the key stepping by the Weyl constants between rounds.
// The key arrives in kernel arguments, so its schedule stays in scalar
// registers.  Counter words 1 and 3 are uniform in every caller, so the
// first round folds them into the key on the scalar unit; each later round
// is two v_mad_u64_u32 and two v_bitop3_b32.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
  {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ (c.y ^ k0), (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ (c.w ^ k1), (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
#pragma unroll
  for (int i = 1; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                   xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Truth tables of v_bitop3_b32 are written as expressions over the bit
// patterns of its three sources: source 0 is 0xF0, source 1 0xCC, source 2
// 0xAA (entry {s0, s1, s2} of the table is bit s0*4 + s1*2 + s2).
constexpr uint32_t kS0 = 0xF0u, kS1 = 0xCCu, kS2 = 0xAAu;

// One bit of a bit-sliced borrow chain against a constant: with b the bits
// of the minuend's plane, br the incoming borrow and t all ones where the
// constant's bit is 1, the outgoing borrow is t ? (~b | br) : (~b & br).
__device__ __forceinline__ uint32_t borrow_step(uint32_t b, uint32_t br,
                                                uint32_t t) {
  constexpr uint32_t tt =
      ((kS2 & (~kS0 | kS1)) | (~kS2 & ~kS0 & kS1)) & 0xFFu;
  return __builtin_amdgcn_bitop3_b32(b, br, t, tt);
}

// e & ~(b ^ t): the equality mask after one more plane.
__device__ __forceinline__ uint32_t equal_step(uint32_t e, uint32_t b,
                                               uint32_t t) {
  constexpr uint32_t tt = (kS0 & ~(kS1 ^ kS2)) & 0xFFu;
  return __builtin_amdgcn_bitop3_b32(e, b, t, tt);
}

// Bit-sliced comparison of eight planes against a byte: P[k] holds bit k of
// every position's byte B (k = 0 least significant), tm[k] is all ones
// where bit k of the constant byte t is set.  lt gets B < t, eq B == t, per
// bit position.
__device__ __forceinline__ void compare_byte(const uint32_t P[8],
                                             const uint32_t tm[8],
                                             uint32_t& lt, uint32_t& eq) {
  uint32_t br = ~P[0] & tm[0];
  uint32_t e = ~(P[0] ^ tm[0]);
#pragma unroll
  for (int k = 1; k < 8; ++k) {
    br = borrow_step(P[k], br, tm[k]);
    e = equal_step(e, P[k], tm[k]);
  }
  lt = br;
  eq = e;
}

// acc * 4 + bit as one v_lshl_add_u32.  Written as an instruction so that the
// compiler keeps one shift-add per decision instead of re-associating the
// chain into wider trees.
__device__ __forceinline__ uint32_t shl2_add(uint32_t acc, uint32_t bit) {
  uint32_t out;
  asm("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(out) : "v"(acc), "v"(bit));
  return out;
}

// 1 iff r >= T, given K = 2^32 - T: the high word of r * one + K, a single
// v_mad_u64_u32 (`one` is 1 at run time).
__device__ __forceinline__ uint32_t reject_bit(uint32_t r, uint32_t one,
                                               uint64_t K) {
  return (uint32_t)(((uint64_t)r * one + K) >> 32);
}

// Mask of the valid bits of word `w` of a row of L sites.
__device__ __forceinline__ uint32_t valid_mask(int L, int w) {
  const int rem = L - 32 * w;
  return rem >= 32 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
}

// out[x] = in[x-1 mod L]  (the left neighbour of every site)
template <int W>
__device__ __forceinline__ void row_from_left(const uint32_t* in, uint32_t* out,
                                              int L) {
  const uint32_t top = (in[W - 1] >> ((L - 1) & 31)) & 1u;
#pragma unroll
  for (int w = W - 1; w >= 1; --w) out[w] = (in[w] << 1) | (in[w - 1] >> 31);
  out[0] = (in[0] << 1) | top;
  out[W - 1] &= valid_mask(L, W - 1);
}

// out[x] = in[x+1 mod L]  (the right neighbour of every site)
template <int W>
__device__ __forceinline__ void row_from_right(const uint32_t* in,
                                               uint32_t* out, int L) {
#pragma unroll
  for (int w = 0; w < W - 1; ++w) out[w] = (in[w] >> 1) | (in[w + 1] << 31);
  out[W - 1] = (in[W - 1] >> 1) | ((in[0] & 1u) << ((L - 1) & 31));
}

// Spread the 16 low bits of v to the even bit positions of a word.
__device__ __forceinline__ uint32_t spread_even(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// 4 int8 spins (+1 = 0x01, -1 = 0xFF) -> 4 bits, bit i = byte i is +1.
__device__ __forceinline__ uint32_t pack4(uint32_t w) {
  const uint32_t m = (~w >> 7) & 0x01010101u;
  return ((m * 0x01020408u) >> 24) & 0xFu;
}

// 4 bits -> 4 int8 spins.
__device__ __forceinline__ uint32_t unpack4(uint32_t nib) {
  const uint32_t b = (nib * 0x00204081u) & 0x01010101u;
  return 0xFFFFFFFFu - b * 0xFEu;
}

// Lane shuffle over the whole wave (ds_bpermute).
__device__ __forceinline__ uint32_t shfl(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

}  // namespace pa
