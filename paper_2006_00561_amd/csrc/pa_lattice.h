// Lattice pass of the population-annealing sweep for gfx950, shared by the
// single-population kernel and the persistent batched kernel.
//
// One replica's L x L lattice lives in the VGPRs of L/RPL lanes of one wave,
// bit packed: a lane holds RPL consecutive rows, 32 sites per register.
// Vertical neighbours come from the adjacent lanes through ds_bpermute,
// horizontal ones from in-register shifts, so the lattice is read from HBM
// once and written once per pass whatever the number of sweeps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa_device.h"
#include "pa_internal.h"

namespace pa {

template <int W, int RPL, bool INT8>
__device__ __forceinline__ void load_row(const uint8_t* rp, int L, int y,
                                         uint32_t* row) {
#pragma unroll
  for (int w = 0; w < W; ++w) row[w] = 0u;
  if (!INT8) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(rp) + (size_t)y * W;
#pragma unroll
    for (int w = 0; w < W; ++w) row[w] = src[w];
    return;
  }
  const uint8_t* src = rp + (size_t)y * L;
  if ((L & 15) == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int xo = 32 * w + 16 * q;
        if (xo < L) {
          const uint4 v = *reinterpret_cast<const uint4*>(src + xo);
          const uint32_t b = pack4(v.x) | (pack4(v.y) << 4) |
                             (pack4(v.z) << 8) | (pack4(v.w) << 12);
          row[w] |= b << (16 * q);
        }
      }
  } else if ((L & 3) == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int xo = 32 * w + 4 * q;
        if (xo < L)
          row[w] |= pack4(*reinterpret_cast<const uint32_t*>(src + xo))
                    << (4 * q);
      }
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int xo = 32 * w + 2 * q;
        if (xo < L) {
          const uint32_t v = *reinterpret_cast<const uint16_t*>(src + xo);
          row[w] |= (pack4(v | 0x01010000u) & 3u) << (2 * q);
        }
      }
  }
}

template <int W, int RPL, bool INT8>
__device__ __forceinline__ void store_row(uint8_t* rp, int L, int y,
                                          const uint32_t* row) {
  if (!INT8) {
    uint32_t* dst = reinterpret_cast<uint32_t*>(rp) + (size_t)y * W;
#pragma unroll
    for (int w = 0; w < W; ++w) dst[w] = row[w];
    return;
  }
  uint8_t* dst = rp + (size_t)y * L;
  if ((L & 15) == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int xo = 32 * w + 16 * q;
        if (xo < L) {
          const uint32_t b = row[w] >> (16 * q);
          uint4 v;
          v.x = unpack4(b & 0xFu);
          v.y = unpack4((b >> 4) & 0xFu);
          v.z = unpack4((b >> 8) & 0xFu);
          v.w = unpack4((b >> 12) & 0xFu);
          *reinterpret_cast<uint4*>(dst + xo) = v;
        }
      }
  } else if ((L & 3) == 0) {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int xo = 32 * w + 4 * q;
        if (xo < L)
          *reinterpret_cast<uint32_t*>(dst + xo) =
              unpack4((row[w] >> (4 * q)) & 0xFu);
      }
  } else {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int xo = 32 * w + 2 * q;
        if (xo < L)
          *reinterpret_cast<uint16_t*>(dst + xo) =
              (uint16_t)(unpack4((row[w] >> (2 * q)) & 3u) & 0xFFFFu);
      }
  }
}

// Acceptance by bit planes (the sweep's second random-number mode): the
// number a colour site compares with its threshold T is r = B 2^24 +
// floor(w / 2^8), with B a byte of bit planes and w the site's word of the
// default stream.  The block of domain MCMC_PLANES for row y, 32-site word
// `word` holds eight planes: plane m = 2i + h is bit 7 - m of B, taken for
// the site at bit position b of the word from bit b XOR h of output word i.
// All 16 colour sites of the word sit at positions of parity p, so planes
// 2i come from output word i as it is and planes 2i + 1 from it rotated by
// one place towards them.  r < T iff B < t, or B == t and floor(w / 2^8) <
// T - t 2^24, with t = min(T >> 24, 255): the comparison runs bit-sliced
// over the word, and only the ties need w.  (T = 2^32, which accepts every
// draw, becomes t = 255 with a low part of 2^24 that every tie passes.)
struct PlaneThr {
  uint32_t tm4[8], tm8[8];  // all ones where bit k of t is set
  uint32_t lo4, lo8;        // T - t 2^24, at most 2^24
};

__device__ __forceinline__ PlaneThr plane_thresholds(const LatticeArgs& a) {
  PlaneThr t;
  const uint64_t T4 = (1ull << 32) - a.K4, T8 = (1ull << 32) - a.K8;
  const uint64_t b4 = (T4 >> 24) < 255 ? (T4 >> 24) : 255;
  const uint64_t b8 = (T8 >> 24) < 255 ? (T8 >> 24) : 255;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    t.tm4[k] = 0u - (uint32_t)((b4 >> k) & 1u);
    t.tm8[k] = 0u - (uint32_t)((b8 >> k) & 1u);
  }
  t.lo4 = (uint32_t)(T4 - (b4 << 24));
  t.lo8 = (uint32_t)(T8 - (b8 << 24));
  return t;
}

// Rotation by one place that brings bit b XOR 1 to position b for the
// positions b of parity par: right by 1 for even b, left by 1 for odd b.
__device__ __forceinline__ uint32_t to_parity(uint32_t x, uint32_t par) {
  return __builtin_amdgcn_alignbit(x, x, par ? 31u : 1u);
}

// The plane block of one word: lt4/lt8 get B < t and e4/e8 B == t for the
// thresholds of dE = 4 and 8, per bit position (only positions of parity p
// are meaningful).
__device__ __forceinline__ void plane_decide(const uint4 o, uint32_t p,
                                             const PlaneThr& t, uint32_t& lt4,
                                             uint32_t& e4, uint32_t& lt8,
                                             uint32_t& e8) {
  uint32_t P[8];
  P[7] = o.x;
  P[6] = to_parity(o.x, p);
  P[5] = o.y;
  P[4] = to_parity(o.y, p);
  P[3] = o.z;
  P[2] = to_parity(o.z, p);
  P[1] = o.w;
  P[0] = to_parity(o.w, p);
  compare_byte(P, t.tm4, lt4, e4);
  compare_byte(P, t.tm8, lt8, e8);
}

// Two words of one row in one comparison: word A's colour sites keep their
// positions (parity p) and word B's colour site at position b moves to b
// XOR 1 (parity 1 - p), so all 32 positions are colour sites.  Results come
// back per word at the sites' own positions.
__device__ __forceinline__ void plane_decide2(const uint4 oA, const uint4 oB,
                                              uint32_t p, const PlaneThr& t,
                                              uint32_t* lt4, uint32_t* e4,
                                              uint32_t* lt8, uint32_t* e8) {
  const uint32_t cm = p ? 0xAAAAAAAAu : 0x55555555u;  // positions of parity p
  const uint32_t q = p ^ 1u;
  const uint32_t a[4] = {oA.x, oA.y, oA.z, oA.w};
  const uint32_t b[4] = {oB.x, oB.y, oB.z, oB.w};
  uint32_t P[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // plane 2i: A's bit at its site, B's bit at its site (now one over)
    P[7 - 2 * i] = (a[i] & cm) | (to_parity(b[i], q) & ~cm);
    // plane 2i + 1: A's bit next to its site, B's bit next to its site,
    // which is where B's site now sits
    P[6 - 2 * i] = (to_parity(a[i], p) & cm) | (b[i] & ~cm);
  }
  uint32_t l4, q4, l8, q8;
  compare_byte(P, t.tm4, l4, q4);
  compare_byte(P, t.tm8, l8, q8);
  lt4[0] = l4;
  e4[0] = q4;
  lt8[0] = l8;
  e8[0] = q8;
  lt4[1] = to_parity(l4, p);
  e4[1] = to_parity(q4, p);
  lt8[1] = to_parity(l8, p);
  e8[1] = to_parity(q8, p);
}

// An L = 64 int8 replica (4 KB, one row of 64 bytes per lane) moved as
// four contiguous kilobytes per wave: in load q, lane l reads bytes
// [1024 q + 16 l, +16), which hold columns 16 (l % 4) .. + 15 of row
// 16 q + l / 4; the 16 sites of each such piece are packed to 16 bits and
// sent to the lane of their row through ds_bpermute (lane y takes the
// pieces of lanes 4 (y % 16) + c of load y / 16).  Every load and store of
// the wave covers 1 KB of consecutive bytes instead of 16 bytes of 64 rows.
__device__ __forceinline__ void load_replica64_int8(const uint8_t* rp,
                                                    uint32_t row[2]) {
  const int lane = threadIdx.x & 63;
  uint32_t p[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 v =
        *reinterpret_cast<const uint4*>(rp + 1024 * q + 16 * lane);
    p[q] = pack4(v.x) | (pack4(v.y) << 4) | (pack4(v.z) << 8) |
           (pack4(v.w) << 12);
  }
  const uint32_t r01 = p[0] | (p[1] << 16), r23 = p[2] | (p[3] << 16);
  const int qy = lane >> 4;  // the load that holds this lane's row
  uint32_t piece[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int src = 4 * (lane & 15) + c;
    const uint32_t a = shfl(r01, src), b = shfl(r23, src);
    const uint32_t v = (qy & 2) ? b : a;
    piece[c] = (qy & 1) ? (v >> 16) : (v & 0xFFFFu);
  }
  row[0] = piece[0] | (piece[1] << 16);
  row[1] = piece[2] | (piece[3] << 16);
}

// The inverse: lane l writes bytes [1024 q + 16 l, +16) from the row
// 16 q + l / 4 of lane 16 q + l / 4.  Every lane takes part in the
// exchange; only `store` lanes write.
__device__ __forceinline__ void store_replica64_int8(uint8_t* rp,
                                                     const uint32_t row[2],
                                                     bool store) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int src = 16 * q + (lane >> 2);
    const uint32_t w0 = shfl(row[0], src), w1 = shfl(row[1], src);
    const uint32_t v = (lane & 2) ? w1 : w0;
    const uint32_t b = (lane & 1) ? (v >> 16) : (v & 0xFFFFu);
    uint4 out;
    out.x = unpack4(b & 0xFu);
    out.y = unpack4((b >> 4) & 0xFu);
    out.z = unpack4((b >> 8) & 0xFu);
    out.w = unpack4((b >> 12) & 0xFu);
    if (store) *reinterpret_cast<uint4*>(rp + 1024 * q + 16 * lane) = out;
  }
}

// One wave's share of a lattice pass: replicas wave*rpw .. wave*rpw+rpw-1.
// No workgroup barrier, so persistent kernels can call it per work item.
// PLANES selects the bit-plane random numbers, else one Philox word per
// site.
template <int W, int RPL, bool INT8, bool GLASS, bool PLANES = false>
__device__ __forceinline__ void lattice_pass(const LatticeArgs& a,
                                             int64_t wave) {
  const int lane = threadIdx.x & 63;
  const int L = a.L;
  const int g = lane / a.lpr;
  const int lr = lane - g * a.lpr;
  const int64_t R = a.Rdev ? min((int64_t)*a.Rdev, a.R) : a.R;
  // a wave past the population has nothing to do (the grid may be sized
  // for a bound of R); the pass has no workgroup barrier, so it may leave
  if (wave * a.rpw >= R) return;
  const int64_t rep = wave * a.rpw + g;
  const bool active = (g < a.rpw) && (rep < R);
  const int base = g * a.lpr;
  const int up_lane = active ? base + (lr == 0 ? a.lpr - 1 : lr - 1) : lane;
  const int dn_lane = active ? base + (lr == a.lpr - 1 ? 0 : lr + 1) : lane;
  const uint32_t slot = (uint32_t)(active ? rep : 0);
  uint8_t* rp = a.spins + (size_t)slot * (size_t)a.stride;
  // where the replica's spins come from: its own slot, or its parent's slot
  // of the other buffer when the resampling copy is fused into this pass
  const uint8_t* lp =
      a.parent ? a.src + (size_t)a.parent[slot] * (size_t)a.stride : rp;

  uint32_t s[RPL][W];
  // an int8 replica of L = 64 in one wave, one row per lane: loaded and
  // stored as whole kilobytes
  const bool T64 = INT8 && W == 2 && RPL == 1 && L == 64 && a.rpw == 1;
  // two such replicas per wave, two rows per lane: each replica moves as
  // four kilobytes through the same exchange (lane l taking its row l),
  // then lane 32 g + i takes rows 2i and 2i + 1 of replica g; a second
  // replica past the population is neither loaded nor stored
  const bool T64x2 = INT8 && W == 2 && RPL == 2 && L == 64 && a.rpw == 2;
  const int64_t rep0 = wave * a.rpw;
  const bool act1 = rep0 + 1 < R;
  // couplings: jr = bond to the right, jl = bond to the left (jr of x-1),
  // jd = bond below, ju = bond above (jd of row y-1); bit set = J < 0
  uint32_t jr[RPL][W], jl[RPL][W], jd[RPL][W], ju[RPL][W];

#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int y = lr * RPL + r;
    if (GLASS) {
      const int yu = (y == 0) ? L - 1 : y - 1;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        jr[r][w] = a.jbits[(size_t)y * W + w];
        jd[r][w] = a.jbits[(size_t)(L + y) * W + w];
        ju[r][w] = a.jbits[(size_t)(L + yu) * W + w];
      }
      row_from_left<W>(jr[r], jl[r], L);
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) jr[r][w] = jl[r][w] = jd[r][w] = ju[r][w] = 0u;
    }
    if (a.init == 2) {
      // ground state of the ferromagnet: every spin equals the replica's
      // INIT word of site (0,0)
      const uint4 b = philox10(make_uint4(kDomainInit << 28, 0u, slot, a.pop),
                               a.k0, a.k1);
#pragma unroll
      for (int w = 0; w < W; ++w) s[r][w] = (b.x >> 31) ? valid_mask(L, w) : 0u;
    } else if (a.init) {
      // INIT stream: site x of row y <- word x%4 of group y*ceil(L/4) + x/4
      const int G4 = (L + 3) >> 2;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint32_t v = 0u;
#pragma unroll
        for (int gq = 0; gq < 8; ++gq) {
          if (32 * w + 4 * gq < L) {
            const uint4 b = philox10(
                make_uint4((kDomainInit << 28) | (uint32_t)(y * G4 + 8 * w + gq),
                           0u, slot, a.pop),
                a.k0, a.k1);
            const uint32_t bits = (b.x >> 31) | ((b.y >> 31) << 1) |
                                  ((b.z >> 31) << 2) | ((b.w >> 31) << 3);
            v |= bits << (4 * gq);
          }
        }
        s[r][w] = v & valid_mask(L, w);
      }
    } else if (T64) {
      // the wave's one replica as four coalesced kilobytes (the branch is
      // uniform: the wave holds one replica, and a wave past the
      // population has left)
      uint32_t row2[2];
      load_replica64_int8(lp, row2);
#pragma unroll
      for (int w = 0; w < W; ++w) s[r][w] = row2[w < 2 ? w : 0];
    } else if (T64x2) {
      if (r == 0) {
        // both replicas of the wave (uniform branches: the first is in the
        // population, the second when act1)
        const uint32_t sl0 = (uint32_t)rep0, sl1 = act1 ? sl0 + 1u : sl0;
        const uint8_t* lp0 =
            a.parent ? a.src + (size_t)a.parent[sl0] * (size_t)a.stride
                     : a.spins + (size_t)sl0 * (size_t)a.stride;
        const uint8_t* lp1 =
            a.parent ? a.src + (size_t)a.parent[sl1] * (size_t)a.stride
                     : a.spins + (size_t)sl1 * (size_t)a.stride;
        uint32_t ra[2], rb[2] = {0u, 0u};
        load_replica64_int8(lp0, ra);
        if (act1) load_replica64_int8(lp1, rb);
        const int i2 = 2 * (lane & 31);
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          const uint32_t a0 = shfl(ra[w], i2), a1 = shfl(ra[w], i2 + 1);
          const uint32_t b0 = shfl(rb[w], i2), b1 = shfl(rb[w], i2 + 1);
          s[0][w < W ? w : 0] = (lane >> 5) ? b0 : a0;
          s[RPL > 1 ? 1 : 0][w < W ? w : 0] = (lane >> 5) ? b1 : a1;
        }
      }
    } else if (active) {
      load_row<W, RPL, INT8>(lp, L, y, s[r]);
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) s[r][w] = 0u;
    }
  }

  const int G8 = (L + 7) >> 3;
  // the 1 of the rejection multiplies in a vector register, so that each
  // v_mad_u64_u32 reads a single scalar operand (its threshold K) and K can
  // stay in scalar registers instead of being copied to vector registers
  // on every pass of the loop
  uint32_t one_v;
  asm("v_mov_b32 %0, %1" : "=v"(one_v) : "s"(a.one));
  PlaneThr pt;
  if (PLANES) pt = plane_thresholds(a);
  for (int t = 0; t < a.theta; ++t) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t up0[W], dnl[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        up0[w] = shfl(s[RPL - 1][w], up_lane);
        dnl[w] = shfl(s[0][w], dn_lane);
      }
      const uint32_t ctr1 = (a.step << 16) | (uint32_t)(2 * (a.t0 + t) + c);
      // bit-plane mode: flips decided by the planes, the sites whose byte
      // ties with the threshold's top byte, and their dE = +4 mask
      uint32_t flip[RPL][W], tie[RPL][W], cls4[RPL][W];
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int y = lr * RPL + r;
        const uint32_t p = (uint32_t)((c + y) & 1);
        const uint32_t rowbase = (kDomainMcmc << 28) | (uint32_t)(y * G8);
        const uint32_t* up = (r == 0) ? up0 : s[r > 0 ? r - 1 : 0];
        const uint32_t* dn = (r == RPL - 1) ? dnl : s[r < RPL - 1 ? r + 1 : 0];
        uint32_t lf[W], rt[W];
        row_from_left<W>(s[r], lf, L);
        row_from_right<W>(s[r], rt, L);
        uint32_t e0[W], e1[W], g2[W], cl[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint32_t sv = s[r][w];
          const uint32_t d1 = sv ^ lf[w] ^ jl[r][w];
          const uint32_t d2 = sv ^ rt[w] ^ jr[r][w];
          const uint32_t d3 = sv ^ up[w] ^ ju[r][w];
          const uint32_t d4 = sv ^ dn[w] ^ jd[r][w];
          const uint32_t x1 = d1 ^ d2, a1 = d1 & d2;
          const uint32_t x2 = d3 ^ d4, a2 = d3 & d4;
          e0[w] = ~(d1 | d2 | d3 | d4);        // dE = +8
          e1[w] = (x1 ^ x2) & ~(a1 | a2);      // dE = +4
          g2[w] = ~(e0[w] | e1[w]);            // dE <= 0
          cl[w] = (p ? 0xAAAAAAAAu : 0x55555555u) & valid_mask(L, w);
        }
        if (PLANES) {
          uint4 o[W];
#pragma unroll
          for (int w = 0; w < W; ++w)
            o[w] = philox10(
                make_uint4((kDomainMcmcPlanes << 28) | (uint32_t)(y * W + w),
                           ctr1, slot, a.pop),
                a.k0, a.k1);
          uint32_t lt4[W], e4[W], lt8[W], e8[W];
#pragma unroll
          for (int w = 0; w + 1 < W; w += 2)
            plane_decide2(o[w], o[w + 1], p, pt, &lt4[w], &e4[w], &lt8[w],
                          &e8[w]);
          if (W & 1)
            plane_decide(o[W - 1], p, pt, lt4[W - 1], e4[W - 1], lt8[W - 1],
                         e8[W - 1]);
          // lanes past the population hold no replica: no ties to resolve
          const uint32_t act = active ? ~0u : 0u;
#pragma unroll
          for (int w = 0; w < W; ++w) {
            flip[r][w] = cl[w] & (g2[w] | (e1[w] & lt4[w]) | (e0[w] & lt8[w]));
            tie[r][w] = cl[w] & act & ((e1[w] & e4[w]) | (e0[w] & e8[w]));
            cls4[r][w] = e1[w];
          }
          continue;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
          // The 16 colour sites of this word (k = 16w + j, x = 2k + p) draw
          // word j%4 of group 4w + j/4.  The rejection bit of a site is the
          // carry of r + (2^32 - T): hi(r * 1 + K) is 1 iff r >= T, one
          // v_mad_u64_u32 (the 1 comes from the arguments, so it is not
          // folded away); v_lshl_add then moves it to bit 2j, highest site
          // first.  T = 2^32 (K = 0) never rejects, T = 0 (K = 2^32) always.
          uint32_t rj4 = 0u, rj8 = 0u;
          const int ng = min(4, max(0, G8 - 4 * w));
          for (int gq = ng - 1; gq >= 0; --gq) {
            const uint4 b = philox10(
                make_uint4(rowbase + (uint32_t)(4 * w + gq), ctr1, slot, a.pop),
                a.k0, a.k1);
            rj4 = shl2_add(rj4, reject_bit(b.w, one_v, a.K4));
            rj8 = shl2_add(rj8, reject_bit(b.w, one_v, a.K8));
            rj4 = shl2_add(rj4, reject_bit(b.z, one_v, a.K4));
            rj8 = shl2_add(rj8, reject_bit(b.z, one_v, a.K8));
            rj4 = shl2_add(rj4, reject_bit(b.y, one_v, a.K4));
            rj8 = shl2_add(rj8, reject_bit(b.y, one_v, a.K8));
            rj4 = shl2_add(rj4, reject_bit(b.x, one_v, a.K4));
            rj8 = shl2_add(rj8, reject_bit(b.x, one_v, a.K8));
          }
          const uint32_t M4 = (~rj4 & 0x55555555u) << p;
          const uint32_t M8 = (~rj8 & 0x55555555u) << p;
          const uint32_t flp = cl[w] & (g2[w] | (e1[w] & M4) | (e0[w] & M8));
          s[r][w] ^= flp;
        }
      }
      if (PLANES) {
        // Ties: each pass takes the lowest pending tie of every lane that
        // has one, draws that site's default-stream word and decides it on
        // the low part of T.  The wave leaves when no lane has a tie left.
        // Every tie is decided by its own site's word, so the order of the
        // passes does not change the result.  With four words or more per
        // lane and an even number per row, a row's ties are merged two words
        // into one first (3.4 % faster at two rows of two words than one-hot
        // picks over the four words); with an odd number per row the pick is
        // a one-hot mask per word (pk), so that the site's row, class and
        // bookkeeping are plain mask operations, and with fewer than four
        // words an index of the picked word is cheaper (at one row of two
        // words the merged form was 0.5 % slower).
        constexpr int NW = RPL * W;
        if constexpr (W % 2 == 0 && NW >= 4) {
          // Words 2j and 2j + 1 of a row as one merged word j: the colour
          // sites of word 2j sit at positions of parity p and those of word
          // 2j + 1, moved by one place, at parity 1 - p, so the row's ties
          // and dE = +4 flags take W / 2 words.  A site at merged position
          // x of merged word j belongs to word 2j + ((x ^ p) & 1), and its
          // default-stream word is number (x >> 1) & 3 of group
          // y G8 + 4 word + (x >> 3).  Each pass takes the lowest pending
          // tie of every lane that has one (first by row and merged word,
          // then by position); the accepted ties go back to their words at
          // the end.
          constexpr int MW = W / 2, NM = RPL * MW;
          uint32_t tM[NM], cM[NM], aM[NM], pr[RPL], gb[RPL];
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const int y = lr * RPL + r;
            pr[r] = (uint32_t)((c + y) & 1);
            gb[r] = (uint32_t)(y * G8);
            const uint32_t cm = pr[r] ? 0xAAAAAAAAu : 0x55555555u;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
              tM[r * MW + j] = (tie[r][2 * j] & cm) |
                               (to_parity(tie[r][2 * j + 1], pr[r] ^ 1u) & ~cm);
              cM[r * MW + j] = (cls4[r][2 * j] & cm) |
                               (to_parity(cls4[r][2 * j + 1], pr[r] ^ 1u) & ~cm);
              aM[r * MW + j] = 0u;
            }
          }
          for (;;) {
            uint32_t pk[NM];
            uint32_t any = 0u;
#pragma unroll
            for (int i = 0; i < NM; ++i) {
              const uint32_t lowest = tM[i] & (0u - tM[i]);
              pk[i] = any ? 0u : lowest;
              any |= lowest;
            }
            if (!__any(any != 0u)) break;
            if (any) {
              // the picked site's merged word (the one nonzero pk): its row
              // parity and group base, its dE = +4 flag, and its position
              uint32_t par = pr[0], gbase = gb[0], c4 = cM[0] & pk[0];
              uint32_t bm = pk[0];
#pragma unroll
              for (int i = 1; i < NM; ++i) {
                par = pk[i] ? pr[i / MW] : par;
                gbase = pk[i] ? gb[i / MW] + 8u * (uint32_t)(i % MW) : gbase;
                c4 |= cM[i] & pk[i];
                bm |= pk[i];
              }
              const uint32_t x = (uint32_t)__builtin_ctz(bm);
              const uint32_t wd = (x ^ par) & 1u;
              const uint4 b = philox10(
                  make_uint4((kDomainMcmc << 28) | (gbase + 4u * wd + (x >> 3)),
                             ctr1, slot, a.pop),
                  a.k0, a.k1);
              const uint32_t sub = (x >> 1) & 3u;
              const uint32_t wv = (sub & 2u) ? ((sub & 1u) ? b.w : b.z)
                                             : ((sub & 1u) ? b.y : b.x);
              const uint32_t acc =
                  ((wv >> 8) < (c4 ? pt.lo4 : pt.lo8)) ? ~0u : 0u;
#pragma unroll
              for (int i = 0; i < NM; ++i) {
                tM[i] &= ~pk[i];
                aM[i] |= pk[i] & acc;
              }
            }
          }
#pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const uint32_t cm = pr[r] ? 0xAAAAAAAAu : 0x55555555u;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
              flip[r][2 * j] |= aM[r * MW + j] & cm;
              flip[r][2 * j + 1] |= to_parity(aM[r * MW + j], pr[r]) & cm;
            }
          }
        } else if constexpr (NW >= 4) {
          for (;;) {
            uint32_t pk[NW];
            uint32_t any = 0u;
#pragma unroll
            for (int i = 0; i < NW; ++i) {
              const uint32_t t = tie[i / W][i % W];
              const uint32_t lowest = t & (0u - t);
              pk[i] = any ? 0u : lowest;
              any |= lowest;
            }
            if (!__any(any != 0u)) break;
            if (any) {
              // the picked site: its bit, and from its word the MCMC group
              // base y G8 + 4 w and its dE = +4 flag
              uint32_t bm = 0u, base = 0u, c4 = 0u;
#pragma unroll
              for (int i = 0; i < NW; ++i) {
                bm |= pk[i];
                const uint32_t yb =
                    (uint32_t)((lr * RPL + i / W) * G8 + 4 * (i % W));
                base = pk[i] ? yb : base;
                c4 |= cls4[i / W][i % W] & pk[i];
              }
              const uint32_t bit = (uint32_t)__builtin_ctz(bm);
              const uint4 b = philox10(
                  make_uint4((kDomainMcmc << 28) | (base + (bit >> 3)), ctr1,
                             slot, a.pop),
                  a.k0, a.k1);
              const uint32_t sub = (bit >> 1) & 3u;
              const uint32_t wv = (sub & 2u) ? ((sub & 1u) ? b.w : b.z)
                                             : ((sub & 1u) ? b.y : b.x);
              const uint32_t acc =
                  ((wv >> 8) < (c4 ? pt.lo4 : pt.lo8)) ? ~0u : 0u;
#pragma unroll
              for (int i = 0; i < NW; ++i) {
                tie[i / W][i % W] &= ~pk[i];
                flip[i / W][i % W] |= pk[i] & acc;
              }
            }
          }
        } else {
          for (;;) {
            uint32_t tm = 0u;
            int sel = 0;
#pragma unroll
            for (int i = RPL * W - 1; i >= 0; --i) {
              const uint32_t ti = tie[i / W][i % W];
              if (ti) {
                tm = ti;
                sel = i;
              }
            }
            if (!__any(tm != 0u)) break;
            if (tm) {
              const uint32_t bit = (uint32_t)__builtin_ctz(tm);
              const uint32_t bm = 1u << bit;
              const int r = sel / W, w = sel - (sel / W) * W;
              const int y = lr * RPL + r;
              const uint32_t k = 16u * (uint32_t)w + (bit >> 1);
              const uint32_t grp = (uint32_t)(y * G8) + (k >> 2);
              const uint4 b = philox10(
                  make_uint4((kDomainMcmc << 28) | grp, ctr1, slot, a.pop),
                  a.k0, a.k1);
              const uint32_t sub = k & 3u;
              const uint32_t wv = (sub & 2u) ? ((sub & 1u) ? b.w : b.z)
                                             : ((sub & 1u) ? b.y : b.x);
              uint32_t is4 = 0u;
#pragma unroll
              for (int i = 0; i < RPL * W; ++i)
                if (sel == i) is4 = cls4[i / W][i % W] & bm;
              const uint32_t acc =
                  ((wv >> 8) < (is4 ? pt.lo4 : pt.lo8)) ? bm : 0u;
#pragma unroll
              for (int i = 0; i < RPL * W; ++i)
                if (sel == i) {
                  tie[i / W][i % W] &= ~bm;
                  flip[i / W][i % W] |= acc;
                }
            }
          }
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
          for (int w = 0; w < W; ++w) s[r][w] ^= flip[r][w];
      }
    }
  }

  // energy and magnetisation of the final state (Eq. Ham)
  uint32_t dnl[W];
#pragma unroll
  for (int w = 0; w < W; ++w) dnl[w] = shfl(s[0][w], dn_lane);
  int unsat = 0, ups = 0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const uint32_t* dn = (r == RPL - 1) ? dnl : s[r < RPL - 1 ? r + 1 : 0];
    uint32_t rt[W];
    row_from_right<W>(s[r], rt, L);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t vm = valid_mask(L, w);
      unsat += __popc((s[r][w] ^ rt[w] ^ jr[r][w]) & vm);
      unsat += __popc((s[r][w] ^ dn[w] ^ jd[r][w]) & vm);
      ups += __popc(s[r][w]);
    }
  }
  // segmented inclusive sum over the lpr consecutive lanes of a replica;
  // its last lane ends with the replica's totals
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int us = __shfl_up(unsat, off, 64);
    const int up = __shfl_up(ups, off, 64);
    if (lr >= off) {
      unsat += us;
      ups += up;
    }
  }
  if (T64) {
    uint32_t row2[2] = {s[0][0], s[0][W > 1 ? 1 : 0]};
    store_replica64_int8(rp, row2, active);
  }
  if (T64x2) {
    // lane l gathers row l of replica g (rows 2i, 2i + 1 sit in lane
    // 32 g + i), then the wave writes the replica as four kilobytes
    const int hl = lane >> 1;
#pragma unroll
    for (int g2 = 0; g2 < 2; ++g2) {
      uint32_t row2[2];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const uint32_t v0 = shfl(s[0][w < W ? w : 0], 32 * g2 + hl);
        const uint32_t v1 = shfl(s[RPL > 1 ? 1 : 0][w < W ? w : 0], 32 * g2 + hl);
        row2[w] = (lane & 1) ? v1 : v0;
      }
      if (g2 == 0 || act1)
        store_replica64_int8(a.spins + (size_t)(rep0 + g2) * (size_t)a.stride,
                             row2, true);
    }
  }
  if (active) {
    if (!T64 && !T64x2) {
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        store_row<W, RPL, INT8>(rp, L, lr * RPL + r, s[r]);
    }
    if (lr == a.lpr - 1) {
      const int N = L * L;
      a.E[rep] = 2 * unsat - 2 * N;
      a.M[rep] = 2 * ups - N;
    }
  }
}

}  // namespace pa
