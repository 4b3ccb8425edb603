// Device building blocks of the checkerboard sweep on colour-packed words.
//
// Layout: plane c holds the sites of colour c ((x + y) mod 2 == c); row y of
// a plane is W uint64 words; bit b of word w is the colour-local site
// k = 64*w + b, i.e. x = 2*k + ((y + c) & 1).  A set bit is spin +1
// (section 5.2 of the paper).  Padding bits past L/2 are always zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// Philox4x32-10 constants (Salmon et al., SC'11).
constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

// a ^ b ^ c in one VALU op (gfx950 BITOP3, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One Philox4x32-10 block.  Each round is two 32x32->64 multiplies
// (v_mad_u64_u32, full rate on gfx950) and two three-input XORs; the key
// schedule is wave-uniform.  With BUMP_SALU the round keys are bumped by a
// scalar add in every round instead of being precomputed, which keeps 18
// SGPRs free (the scalar adds issue beside the vector work).
template <bool BUMP_SALU = false>
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kM0 * x0;
    const uint64_t p1 = (uint64_t)kM1 * x2;
    const uint32_t y0 = xor3((uint32_t)(p1 >> 32), x1, k0);
    const uint32_t y2 = xor3((uint32_t)(p0 >> 32), x3, k1);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
    if (BUMP_SALU) {
      if (r < 9) {
        asm("s_add_u32 %0, %0, %1" : "+s"(k0) : "i"(kW0) : "scc");
        asm("s_add_u32 %0, %0, %1" : "+s"(k1) : "i"(kW1) : "scc");
      }
    } else {
      k0 += kW0;
      k1 += kW1;
    }
  }
}

// Geometry of one lattice as the kernels see it.
struct Geom {
  int64_t L;        // side
  int32_t W;        // words per colour-row
  int32_t nb_last;  // valid bits in the last word of a row (1..64)
  int64_t L8;       // L / 8 when L % 8 == 0 (Philox blocks per colour-row)
  int64_t half;     // L / 2
};

__device__ __forceinline__ uint64_t low_mask(int nbits) {
  return nbits >= 64 ? ~0ull : ((1ull << nbits) - 1ull);
}

// Neighbour words of word (y, w) of colour c, read from the other plane `o`
// (row stride W).  n0: same colour-local index in row y; n1: the horizontal
// partner (left if (y + c) even, right otherwise), with the periodic wrap
// of a possibly partial last word; n2/n3: rows y-1 and y+1 (periodic).
struct Nbr {
  uint64_t n0, n1, n2, n3;
};

template <typename Ptr>
__device__ __forceinline__ Nbr gather(Ptr o, const Geom& g, int c, int64_t y, int32_t w) {
  const int64_t W = g.W;
  const int64_t ym = (y == 0) ? g.L - 1 : y - 1;
  const int64_t yp = (y == g.L - 1) ? 0 : y + 1;
  const auto row = o + y * W;
  Nbr n;
  n.n0 = row[w];
  n.n2 = o[ym * W + w];
  n.n3 = o[yp * W + w];
  if (((y + c) & 1) == 0) {
    // left partner: site k-1; k = 0 wraps to the last valid site of the row
    const uint64_t carry =
        (w > 0) ? (row[w - 1] >> 63) : ((row[W - 1] >> (g.nb_last - 1)) & 1ull);
    n.n1 = (n.n0 << 1) | carry;
  } else {
    // right partner: site k+1; the last valid site wraps to k = 0
    if (w < g.W - 1)
      n.n1 = (n.n0 >> 1) | (row[w + 1] << 63);
    else
      n.n1 = (n.n0 >> 1) | ((row[0] & 1ull) << (g.nb_last - 1));
  }
  return n;
}

// Bit-sliced Metropolis decision for 64 sites (section 4, Eqs. (4)-(5)).
// a_i = s ^ n_i marks anti-aligned neighbours; with k = sum a_i the site
// flips iff k + [u < t4] + [u < t8] >= 2.  Since t8 <= t4, [u < t8] implies
// [u < t4], so flip = (k >= 2) | ((k >= 1) & r4) | r8.
// Truth-table immediate of a three-input bit function for v_bitop3: bit
// 4 a + 2 b + c of the table is f(a, b, c) (a, b, c the first, second and
// third operand).
template <typename F>
constexpr uint32_t bitop3_table(F f) {
  uint32_t t = 0;
  for (int i = 0; i < 8; ++i) t |= (uint32_t)(f((i >> 2) & 1, (i >> 1) & 1, i & 1) & 1) << i;
  return t;
}

__device__ __forceinline__ uint32_t flip_half(uint32_t s, uint32_t n0, uint32_t n1, uint32_t n2,
                                              uint32_t n3, uint32_t r4, uint32_t r8) {
  // both neighbours of a pair anti-aligned / at least one of them
  constexpr uint32_t kBoth = bitop3_table([](int a, int b, int c) { return (a ^ b) & (a ^ c); });
  constexpr uint32_t kEither = bitop3_table([](int a, int b, int c) { return (a ^ b) | (a ^ c); });
  constexpr uint32_t kOrAnd = bitop3_table([](int a, int b, int c) { return a | (b & c); });
  constexpr uint32_t kOrThenAnd = bitop3_table([](int a, int b, int c) { return (a | b) & c; });
  constexpr uint32_t kOr3 = bitop3_table([](int a, int b, int c) { return a | b | c; });
  const uint32_t p01 = __builtin_amdgcn_bitop3_b32(s, n0, n1, kBoth);
  const uint32_t p23 = __builtin_amdgcn_bitop3_b32(s, n2, n3, kBoth);
  const uint32_t o01 = __builtin_amdgcn_bitop3_b32(s, n0, n1, kEither);
  const uint32_t o23 = __builtin_amdgcn_bitop3_b32(s, n2, n3, kEither);
  // one anti-aligned neighbour in each pair: (a0 ^ a1) & (a2 ^ a3), where
  // a0 ^ a1 = n0 ^ n1 (s cancels)
  const uint32_t ge2 = __builtin_amdgcn_bitop3_b32(p01, n0 ^ n1, n2 ^ n3, kOrAnd);
  const uint32_t one = __builtin_amdgcn_bitop3_b32(o01, o23, r4, kOrThenAnd);
  return __builtin_amdgcn_bitop3_b32(ge2, p23, one, kOr3) | r8;
}

__device__ __forceinline__ uint64_t flip_mask(uint64_t s, const Nbr& n, uint64_t r4, uint64_t r8) {
  // k >= 2, or k >= 1 with r4, or r8 (r8 implies r4): the flip rule of
  // Eq. (5), evaluated per 32-bit half with three-input bit operations
  const uint32_t lo = flip_half((uint32_t)s, (uint32_t)n.n0, (uint32_t)n.n1, (uint32_t)n.n2,
                                (uint32_t)n.n3, (uint32_t)r4, (uint32_t)r8);
  const uint32_t hi = flip_half((uint32_t)(s >> 32), (uint32_t)(n.n0 >> 32),
                                (uint32_t)(n.n1 >> 32), (uint32_t)(n.n2 >> 32),
                                (uint32_t)(n.n3 >> 32), (uint32_t)(r4 >> 32),
                                (uint32_t)(r8 >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Insert the comparison results of one Philox block (4 consecutive sites,
// starting at bit 4q of a 32-bit half) into the r4/r8 halves.
__device__ __forceinline__ void insert4(uint32_t& r4, uint32_t& r8, int base, uint32_t x0,
                                        uint32_t x1, uint32_t x2, uint32_t x3, uint32_t t4,
                                        uint32_t t8) {
  r4 |= ((x0 < t4) ? (1u << base) : 0u) | ((x1 < t4) ? (2u << base) : 0u) |
        ((x2 < t4) ? (4u << base) : 0u) | ((x3 < t4) ? (8u << base) : 0u);
  r8 |= ((x0 < t8) ? (1u << base) : 0u) | ((x1 < t8) ? (2u << base) : 0u) |
        ((x2 < t8) ? (4u << base) : 0u) | ((x3 < t8) ? (8u << base) : 0u);
}

// Uniform comparison masks for word (y, w) when L % 8 == 0: the word's
// sites are Philox blocks g0 + q, q < nq, with g0 = y*L/8 + 16*w, and
// block q covers bits 4q..4q+3.  rA = [u < tA], rB = [u < tB] per site.
__device__ __forceinline__ void masks_aligned(const Geom& g, int64_t y, int32_t w, uint32_t k0,
                                              uint32_t k1, uint32_t t, uint32_t ctr3, uint32_t tA,
                                              uint32_t tB, uint64_t& rA, uint64_t& rB) {
  const int nq = (w == g.W - 1) ? (g.nb_last >> 2) : 16;
  const uint64_t g0 = (uint64_t)y * (uint64_t)g.L8 + 16ull * (uint64_t)w;
  uint32_t a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (q < nq) {
      const uint64_t gq = g0 + (uint64_t)q;
      uint32_t x0 = (uint32_t)gq, x1 = (uint32_t)(gq >> 32), x2 = t, x3 = ctr3;
      philox4x32_10(x0, x1, x2, x3, k0, k1);
      if (q < 8)
        insert4(a_lo, b_lo, 4 * q, x0, x1, x2, x3, tA, tB);
      else
        insert4(a_hi, b_hi, 4 * (q - 8), x0, x1, x2, x3, tA, tB);
    }
  }
  rA = ((uint64_t)a_hi << 32) | a_lo;
  rB = ((uint64_t)b_hi << 32) | b_lo;
}

// Same for any even L: the word's first site has colour-local index
// i0 = y*L/2 + 64*w, which need not be a multiple of 4, so its 64 sites may
// straddle 17 Philox blocks starting at i0/4.
__device__ __forceinline__ void masks_generic(const Geom& g, int64_t y, int32_t w, uint32_t k0,
                                              uint32_t k1, uint32_t t, uint32_t ctr3, uint32_t tA,
                                              uint32_t tB, uint64_t& rA, uint64_t& rB) {
  const int nbits = (w == g.W - 1) ? g.nb_last : 64;
  const uint64_t i0 = (uint64_t)y * (uint64_t)g.half + 64ull * (uint64_t)w;
  const int r = (int)(i0 & 3ull);
  const uint64_t gs = i0 >> 2;
  const int nc = (r + nbits + 3) >> 2;
  uint64_t a = 0, b = 0;
  for (int q = 0; q < nc; ++q) {
    const uint64_t gq = gs + (uint64_t)q;
    uint32_t x[4] = {(uint32_t)gq, (uint32_t)(gq >> 32), t, ctr3};
    philox4x32_10(x[0], x[1], x[2], x[3], k0, k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = 4 * q + j - r;
      if (o >= 0 && o < nbits) {
        a |= (uint64_t)(x[j] < tA) << o;
        b |= (uint64_t)(x[j] < tB) << o;
      }
    }
  }
  rA = a;
  rB = b;
}

// Compare the four outputs of one Philox block with t4 and t8 and shift the
// results into the 32-bit accumulators: acc = 2*acc + [x < t] for x3, x2,
// x1, x0 in that order, so that x0 lands in the lowest of the four new bit
// positions.  Each compare writes a lane mask into its own SGPR pair and
// each v_addc_co_u32 consumes one as carry-in; every mask is read at least
// three instructions after it is written (gfx950 needs two wait states
// between a VALU SGPR write and its use as a carry).
__device__ __forceinline__ void shift_in4(uint32_t& a4, uint32_t& a8, uint32_t x0, uint32_t x1,
                                          uint32_t x2, uint32_t x3, uint32_t t4, uint32_t t8) {
  uint64_t c0, c1, c2, c3, d;
  asm("v_cmp_gt_u32_e64 %[c0], %[t4], %[x3]\n\t"
      "v_cmp_gt_u32_e64 %[c1], %[t8], %[x3]\n\t"
      "v_cmp_gt_u32_e64 %[c2], %[t4], %[x2]\n\t"
      "v_cmp_gt_u32_e64 %[c3], %[t8], %[x2]\n\t"
      "v_addc_co_u32_e64 %[a4], %[d], %[a4], %[a4], %[c0]\n\t"
      "v_addc_co_u32_e64 %[a8], %[d], %[a8], %[a8], %[c1]\n\t"
      "v_cmp_gt_u32_e64 %[c0], %[t4], %[x1]\n\t"
      "v_cmp_gt_u32_e64 %[c1], %[t8], %[x1]\n\t"
      "v_addc_co_u32_e64 %[a4], %[d], %[a4], %[a4], %[c2]\n\t"
      "v_addc_co_u32_e64 %[a8], %[d], %[a8], %[a8], %[c3]\n\t"
      "v_cmp_gt_u32_e64 %[c2], %[t4], %[x0]\n\t"
      "v_cmp_gt_u32_e64 %[c3], %[t8], %[x0]\n\t"
      "v_addc_co_u32_e64 %[a4], %[d], %[a4], %[a4], %[c0]\n\t"
      "v_addc_co_u32_e64 %[a8], %[d], %[a8], %[a8], %[c1]\n\t"
      "v_addc_co_u32_e64 %[a4], %[d], %[a4], %[a4], %[c2]\n\t"
      "v_addc_co_u32_e64 %[a8], %[d], %[a8], %[a8], %[c3]"
      : [a4] "+v"(a4), [a8] "+v"(a8), [c0] "=&s"(c0), [c1] "=&s"(c1), [c2] "=&s"(c2),
        [c3] "=&s"(c3), [d] "=&s"(d)
      : [x0] "v"(x0), [x1] "v"(x1), [x2] "v"(x2), [x3] "v"(x3), [t4] "s"(t4), [t8] "s"(t8));
}

// Masks for one word whose Philox blocks are lo + q, q < nq, all with the
// same high counter word `hi` (no carry out of lo + q): block q covers bits
// 4q..4q+3.  Blocks are visited from q = 15 down to 0 so that the shift-in
// order leaves block 0 in the lowest bits; with FULL every word has 16
// blocks, otherwise blocks q >= nq are skipped and their bits stay zero.
template <bool FULL, bool BUMP_SALU = false>
__device__ __forceinline__ void masks_shift(uint32_t lo, uint32_t hi, int nq, uint32_t k0,
                                            uint32_t k1, uint32_t t, uint32_t ctr3, uint32_t t4,
                                            uint32_t t8, uint64_t& r4, uint64_t& r8) {
  uint32_t a4_hi = 0, a8_hi = 0, a4_lo = 0, a8_lo = 0;
#pragma unroll
  for (int q = 15; q >= 0; --q) {
    if (FULL || q < nq) {
      uint32_t x0 = lo + (uint32_t)q, x1 = hi, x2 = t, x3 = ctr3;
      philox4x32_10<BUMP_SALU>(x0, x1, x2, x3, k0, k1);
      if (q >= 8)
        shift_in4(a4_hi, a8_hi, x0, x1, x2, x3, t4, t8);
      else
        shift_in4(a4_lo, a8_lo, x0, x1, x2, x3, t4, t8);
    }
  }
  r4 = ((uint64_t)a4_hi << 32) | a4_lo;
  r8 = ((uint64_t)a8_hi << 32) | a8_lo;
}

// ---------------------------------------------------------------------
// The paper's per-thread linear congruential generator (section 5.3):
// x <- (1664525 x + 1013904223) mod 2^32 (Eq. (6)), one state per word of
// one colour.  The uniform of a value is |int32(x)| / 2^31, and an uphill
// move with threshold t' = floor(exp(-beta dE) 2^31) is accepted iff
// |int32(x)| < t'.  For integers that is x + (t' - 1) < 2 t' - 1 (mod 2^32)
// when t' >= 1, and never when t' = 0; with (d, m) = (t' - 1, 2 t' - 1), or
// (0, 0) for t' = 0, the test is (x + d) < m.
// ---------------------------------------------------------------------
constexpr uint32_t kLcgA = 1664525u;
constexpr uint32_t kLcgC = 1013904223u;

// The chain runs on z = x + d4 instead of x: z' = a z + (c + d4 - a d4), still
// one multiply-add, and the t4 test becomes the bare compare z < m4; the t8
// test is (z + e) < m8 with e = d8 - d4.  6 lane-operations per site.
__device__ __forceinline__ uint32_t lcg_next(uint32_t z, uint32_t c) {
  // one full-rate v_mad_u64_u32 per value (the low word is the next state;
  // the multiplier sits in a VGPR: one SGPR operand per VOP3 on gfx9);
  // written out so that the compiler keeps the chain instead of rewriting
  // it as independent jump-ahead products (v_mul_lo_u32 + v_add each)
  uint64_t r, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4"
      : "=v"(r), "=s"(carry)
      : "v"(z), "v"(kLcgA), "s"((uint64_t)c));
  return (uint32_t)r;
}

// Shift the decisions of four consecutive values (g1 first) into the
// accumulators: a4 = 2 a4 + [g < m4], a8 = 2 a8 + [g + e < m8], g1's bit
// ending highest.  Every compare writes its own SGPR pair, read as carry-in
// at least three instructions later (gfx950 needs two wait states).
__device__ __forceinline__ void shift_in4_lcg(uint32_t& a4, uint32_t& a8, uint32_t g1,
                                              uint32_t g2, uint32_t g3, uint32_t g4, uint32_t e,
                                              uint32_t m4, uint32_t m8) {
  uint64_t c0, c1, c2, c3, dd;
  uint32_t u0, u1, u2, u3;
  asm("v_add_u32_e32 %[u0], %[e], %[g1]\n\t"
      "v_add_u32_e32 %[u1], %[e], %[g2]\n\t"
      "v_cmp_gt_u32_e64 %[c0], %[m4], %[g1]\n\t"
      "v_cmp_gt_u32_e64 %[c1], %[m8], %[u0]\n\t"
      "v_cmp_gt_u32_e64 %[c2], %[m4], %[g2]\n\t"
      "v_cmp_gt_u32_e64 %[c3], %[m8], %[u1]\n\t"
      "v_add_u32_e32 %[u2], %[e], %[g3]\n\t"
      "v_addc_co_u32_e64 %[a4], %[dd], %[a4], %[a4], %[c0]\n\t"
      "v_addc_co_u32_e64 %[a8], %[dd], %[a8], %[a8], %[c1]\n\t"
      "v_add_u32_e32 %[u3], %[e], %[g4]\n\t"
      "v_addc_co_u32_e64 %[a4], %[dd], %[a4], %[a4], %[c2]\n\t"
      "v_addc_co_u32_e64 %[a8], %[dd], %[a8], %[a8], %[c3]\n\t"
      "v_cmp_gt_u32_e64 %[c0], %[m4], %[g3]\n\t"
      "v_cmp_gt_u32_e64 %[c1], %[m8], %[u2]\n\t"
      "v_cmp_gt_u32_e64 %[c2], %[m4], %[g4]\n\t"
      "v_cmp_gt_u32_e64 %[c3], %[m8], %[u3]\n\t"
      "v_addc_co_u32_e64 %[a4], %[dd], %[a4], %[a4], %[c0]\n\t"
      "v_addc_co_u32_e64 %[a8], %[dd], %[a8], %[a8], %[c1]\n\t"
      "v_addc_co_u32_e64 %[a4], %[dd], %[a4], %[a4], %[c2]\n\t"
      "v_addc_co_u32_e64 %[a8], %[dd], %[a8], %[a8], %[c3]"
      : [a4] "+v"(a4), [a8] "+v"(a8), [c0] "=&s"(c0), [c1] "=&s"(c1), [c2] "=&s"(c2),
        [c3] "=&s"(c3), [dd] "=&s"(dd), [u0] "=&v"(u0), [u1] "=&v"(u1), [u2] "=&v"(u2),
        [u3] "=&v"(u3)
      : [g1] "v"(g1), [g2] "v"(g2), [g3] "v"(g3), [g4] "v"(g4), [e] "s"(e), [m4] "s"(m4),
        [m8] "s"(m8));
}

// r4 / r8 of one word from its shifted LCG state z = x + d4 (advanced 64
// times): the k-th new value decides site 64 - k of the word (site 63
// first).  c = 1013904223 + d4 - 1664525 d4 (mod 2^32), e = d8 - d4.
__device__ __forceinline__ void masks_lcg(uint32_t& z, uint32_t c, uint32_t e, uint32_t m4,
                                          uint32_t m8, uint64_t& r4, uint64_t& r8) {
  uint32_t a4_hi = 0, a8_hi = 0, a4_lo = 0, a8_lo = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const uint32_t g1 = lcg_next(z, c);
    const uint32_t g2 = lcg_next(g1, c);
    const uint32_t g3 = lcg_next(g2, c);
    const uint32_t g4 = lcg_next(g3, c);
    z = g4;
    if (q < 8)
      shift_in4_lcg(a4_hi, a8_hi, g1, g2, g3, g4, e, m4, m8);
    else
      shift_in4_lcg(a4_lo, a8_lo, g1, g2, g3, g4, e, m4, m8);
  }
  r4 = ((uint64_t)a4_hi << 32) | a4_lo;
  r8 = ((uint64_t)a8_hi << 32) | a8_lo;
}

}  // namespace ising
