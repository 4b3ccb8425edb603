// HIP kernels (gfx950) of the checkerboard Metropolis sweep on
// colour-packed uint64 words: initialisation, half-sweeps with the energy
// and magnetisation reduction fused into the colour-1 pass, a measurement
// pass, and a single-workgroup LDS-resident multi-sweep kernel for small
// lattices.
#include <algorithm>

#include "ising_kernels.hpp"

#include "ising_device.hpp"

// Pointer qualifier for read-only tables: the AMDGPU constant address space
// in the device pass (scalar loads); the host pass never runs kernel code.
#if defined(__HIP_DEVICE_COMPILE__)
#define ISING_CONSTANT_AS __attribute__((address_space(4)))
#else
#define ISING_CONSTANT_AS
#endif

namespace ising {

// ---------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum (a, p) over the block in 64 bits (a block of a large lattice can
// count more than 2^32 bonds); thread 0 gets the totals.  `red` holds 2
// entries per wave.
__device__ __forceinline__ void block_sum2(uint32_t a32, uint32_t p32, uint64_t* red, uint64_t& a,
                                           uint64_t& p) {
  a = a32;
  p = p32;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    p += __shfl_xor(p, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wave] = a;
    red[2 * wave + 1] = p;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    uint64_t sa = 0, sp = 0;
    for (int i = 0; i < nw; ++i) {
      sa += red[2 * i];
      sp += red[2 * i + 1];
    }
    a = sa;
    p = sp;
  }
}

// Test hook: with a nonzero seed, this wave pauses for a pseudo-random
// 0 .. 31 short sleeps (hash of seed, call site, block and wave) before a
// block barrier.  Waves then reach the barrier in a shuffled order; a
// result that depends on that order (a missing barrier or fence) changes.
__device__ __forceinline__ void perturb_wave(uint32_t seed, uint32_t site) {
  if (seed == 0) return;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t h = seed ^ (site * 0x9E3779B9u) ^ (blockIdx.x * 0x85EBCA77u) ^ (wave * 0xC2B2AE3Du);
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  for (uint32_t i = 0, n = h & 31u; i < n; ++i) __builtin_amdgcn_s_sleep(8);
}

// Contribution of one updated colour-1 word to the bond and spin counts:
// every bond has exactly one colour-1 end, so summing the anti-aligned
// neighbours of all colour-1 sites counts each anti-aligned bond once;
// n0 is the colour-0 word with the same index, so each colour-0 word is
// counted once as well.  Padding bits are zero in s, n0, n2, n3; n1 may
// carry one stray bit past the last valid site and is masked.
__device__ __forceinline__ void count_word(uint64_t s, const Nbr& n, uint64_t valid, uint32_t& anti,
                                           uint32_t& up) {
  anti += __popcll(s ^ n.n0) + __popcll((s ^ n.n1) & valid) + __popcll(s ^ n.n2) +
          __popcll(s ^ n.n3);
  up += __popcll(s) + __popcll(n.n0);
}

// ---------------------------------------------------------------------
// Initialisation: cold (all +1 / all -1) or hot (phase 2 + colour).
// ---------------------------------------------------------------------
template <bool ALIGNED>
__global__ __launch_bounds__(256) void k_init(uint64_t* __restrict__ planes, Geom g, uint32_t k0,
                                              uint32_t k1, uint32_t sid4, int init) {
  const int64_t per_plane = g.L * (int64_t)g.W;
  const int64_t total = 2 * per_plane;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = idx >= per_plane ? 1 : 0;
    const int64_t r = idx - c * per_plane;
    const int64_t y = r / g.W;
    const int32_t w = (int32_t)(r - y * g.W);
    const uint64_t valid = (w == g.W - 1) ? low_mask(g.nb_last) : ~0ull;
    uint64_t word;
    if (init == 0) {
      word = valid;
    } else if (init == 1) {
      word = 0;
    } else {
      uint64_t m, unused;
      const uint32_t half = 0x80000000u;
      if (ALIGNED)
        masks_aligned(g, y, w, k0, k1, 0u, sid4 | (2u + c), half, half, m, unused);
      else
        masks_generic(g, y, w, k0, k1, 0u, sid4 | (2u + c), half, half, m, unused);
      word = m & valid;
    }
    planes[idx] = word;
  }
}

// ---------------------------------------------------------------------
// Half-sweep of colour C (section 3, step A for C = 0, step B for C = 1).
// One lane owns one word at a time (grid-stride).  With EM, the colour-1
// pass also accumulates 2*(anti-aligned bonds) and 2*(up spins) into
// EM[0], EM[1], which the colour-0 pass of the same sweep set to -2N, -N,
// so that EM = (E, M) exactly once the colour-1 pass has finished.
// ---------------------------------------------------------------------
template <int C, bool ALIGNED, bool EM>
__global__ __launch_bounds__(256) void k_half_sweep(SweepArgs a) {
  __shared__ uint64_t red[2 * 16];
  const Geom g = a.g;
  uint64_t* __restrict__ self = a.planes + (C ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (C ? 0 : a.plane_words);
  const int64_t total = a.plane_words;
  uint32_t anti = 0, up = 0;
  if (C == 0 && EM && blockIdx.x == 0 && threadIdx.x == 0) {
    a.EM[0] = -2 * g.L * g.L;
    a.EM[1] = -g.L * g.L;
  }
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = idx / g.W;
    const int32_t w = (int32_t)(idx - y * g.W);
    const uint64_t valid = (w == g.W - 1) ? low_mask(g.nb_last) : ~0ull;
    const uint64_t s = self[idx];
    const Nbr n = gather(other, g, C, y, w);
    uint64_t r4, r8;
    if (ALIGNED)
      masks_aligned(g, y, w, a.k0, a.k1, a.t, a.sid4 | C, a.t4, a.t8, r4, r8);
    else
      masks_generic(g, y, w, a.k0, a.k1, a.t, a.sid4 | C, a.t4, a.t8, r4, r8);
    const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
    self[idx] = s_new;
    if (C == 1 && EM) count_word(s_new, n, valid, anti, up);
  }
  if (C == 1 && EM) {
    uint64_t sa, sp;
    block_sum2(anti, up, red, sa, sp);
    if (threadIdx.x == 0) {
      atomicAdd((unsigned long long*)&a.EM[0], (unsigned long long)(2ull * sa));
      atomicAdd((unsigned long long*)&a.EM[1], (unsigned long long)(2ull * sp));
    }
  }
}

// ---------------------------------------------------------------------
// Measurement of the current state: EM[0] += 2A, EM[1] += 2P over all
// colour-1 words (EM must hold -2N, -N on entry).
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_measure(const uint64_t* __restrict__ planes, Geom g,
                                                 int64_t plane_words, int64_t* EM) {
  __shared__ uint64_t red[2 * 16];
  const uint64_t* self = planes + plane_words;
  const uint64_t* other = planes;
  uint32_t anti = 0, up = 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < plane_words;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = idx / g.W;
    const int32_t w = (int32_t)(idx - y * g.W);
    const uint64_t valid = (w == g.W - 1) ? low_mask(g.nb_last) : ~0ull;
    const Nbr n = gather(other, g, 1, y, w);
    count_word(self[idx], n, valid, anti, up);
  }
  uint64_t sa, sp;
  block_sum2(anti, up, red, sa, sp);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&EM[0], (unsigned long long)(2ull * sa));
    atomicAdd((unsigned long long*)&EM[1], (unsigned long long)(2ull * sp));
  }
}

__global__ void k_set_em(int64_t* EM, int64_t e, int64_t m) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    EM[0] = e;
    EM[1] = m;
  }
}

// ---------------------------------------------------------------------
// Small lattices: one workgroup keeps both planes in LDS and runs all n
// sweeps, with a block barrier between the colour steps (the barrier plays
// the role of the paper's second kernel launch, section 5.2).
// ---------------------------------------------------------------------
template <bool ALIGNED>
__global__ __launch_bounds__(1024) void k_small_sweeps(SmallArgs a) {
  extern __shared__ uint64_t lds[];
  __shared__ uint64_t red[2 * 16];
  const Geom g = a.g;
  const int64_t pw = a.plane_words;
  for (int64_t i = threadIdx.x; i < 2 * pw; i += blockDim.x) lds[i] = a.planes[i];
  __syncthreads();
  for (int64_t k = 0; k < a.n; ++k) {
    const uint32_t t = a.t0 + (uint32_t)k;
    uint32_t anti = 0, up = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t* self = lds + (c ? pw : 0);
      const uint64_t* other = lds + (c ? 0 : pw);
      for (int64_t idx = threadIdx.x; idx < pw; idx += blockDim.x) {
        const int64_t y = idx / g.W;
        const int32_t w = (int32_t)(idx - y * g.W);
        const uint64_t valid = (w == g.W - 1) ? low_mask(g.nb_last) : ~0ull;
        const uint64_t s = self[idx];
        const Nbr n = gather(other, g, c, y, w);
        uint64_t r4, r8;
        if (ALIGNED)
          masks_aligned(g, y, w, a.k0, a.k1, t, a.sid4 | c, a.t4, a.t8, r4, r8);
        else
          masks_generic(g, y, w, a.k0, a.k1, t, a.sid4 | c, a.t4, a.t8, r4, r8);
        const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
        self[idx] = s_new;
        if (c == 1) count_word(s_new, n, valid, anti, up);
      }
      perturb_wave(a.perturb, (uint32_t)(2 * k + c));
      __syncthreads();
    }
    if (a.EM) {
      uint64_t sa, sp;
      block_sum2(anti, up, red, sa, sp);
      if (threadIdx.x == 0) {
        a.EM[2 * k] = 2 * (int64_t)sa - 2 * g.L * g.L;
        a.EM[2 * k + 1] = 2 * (int64_t)sp - g.L * g.L;
      }
      __syncthreads();
    }
  }
  for (int64_t i = threadIdx.x; i < 2 * pw; i += blockDim.x) a.planes[i] = lds[i];
}

// Masks of one word split over LPW lanes (L % 8 == 0): lane `sub` of the
// word computes Philox blocks q = sub*NQ .. sub*NQ + NQ - 1 (NQ = 16 / LPW)
// of the word's 16 (blocks past a partial last word are computed too and
// later masked by `valid`), shifts their decisions into one 32-bit pair of
// accumulators and places them at bit 4*NQ*sub; the OR over the word's
// lanes (adjacent lanes, one DPP row) gives every lane the full masks.
template <int LPW>
__device__ __forceinline__ void masks_split(uint32_t lo, int sub, uint32_t k0, uint32_t k1,
                                            uint32_t t, uint32_t ctr3, uint32_t t4, uint32_t t8,
                                            uint64_t& r4, uint64_t& r8) {
  constexpr int NQ = 16 / LPW;
  uint32_t a4 = 0, a8 = 0;
  const uint32_t q0 = (uint32_t)(sub * NQ);
#pragma unroll
  for (int k = NQ - 1; k >= 0; --k) {
    uint32_t x0 = lo + q0 + (uint32_t)k, x1 = 0, x2 = t, x3 = ctr3;
    philox4x32_10<false>(x0, x1, x2, x3, k0, k1);
    shift_in4(a4, a8, x0, x1, x2, x3, t4, t8);
  }
  const int sh = 4 * NQ * sub;
  r4 = (uint64_t)a4 << sh;
  r8 = (uint64_t)a8 << sh;
#pragma unroll
  for (int off = 1; off < LPW; off <<= 1) {
    r4 |= __shfl_xor(r4, off, 64);
    r8 |= __shfl_xor(r8, off, 64);
  }
}

// All n sweeps of one lattice resident in LDS (one workgroup, L % 8 == 0,
// every Philox block index below 2^32), LPW lanes per word: for the
// smallest lattices the per-colour-step latency is the cost, and spreading
// a word's 16 Philox blocks over 2-16 lanes divides it.  Lane 0 of a word
// stores the update and counts E/M.
template <int LPW>
__global__ __launch_bounds__(1024) void k_small_sweeps_split(SmallArgs a) {
  extern __shared__ uint64_t lds[];
  __shared__ uint64_t red[32];
  const Geom g = a.g;
  const int64_t pw = a.plane_words;
  for (int64_t i = threadIdx.x; i < 2 * pw; i += blockDim.x) lds[i] = a.planes[i];
  __syncthreads();
  const int sub = threadIdx.x % LPW;
  for (int64_t k = 0; k < a.n; ++k) {
    const uint32_t t = a.t0 + (uint32_t)k;
    uint32_t anti = 0, up = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t* self = lds + (c ? pw : 0);
      const uint64_t* other = lds + (c ? 0 : pw);
      // the loop bound is uniform per word group, so the shuffles see
      // every lane of a word
      for (int64_t base = 0; base < pw * LPW; base += blockDim.x) {
        const int64_t idx = (base + threadIdx.x) / LPW;
        const bool ok = idx < pw;
        const int64_t ic = ok ? idx : pw - 1;
        const int64_t y = ic / g.W;
        const int32_t w = (int32_t)(ic - y * g.W);
        const uint32_t lo = (uint32_t)y * (uint32_t)g.L8 + 16u * (uint32_t)w;
        uint64_t r4, r8;
        masks_split<LPW>(lo, sub, a.k0, a.k1, t, a.sid4 | c, a.t4, a.t8, r4, r8);
        if (ok && sub == 0) {
          const uint64_t valid = (w == g.W - 1) ? low_mask(g.nb_last) : ~0ull;
          const uint64_t s = self[ic];
          const Nbr n = gather(other, g, c, y, w);
          const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
          self[ic] = s_new;
          if (c == 1) count_word(s_new, n, valid, anti, up);
        }
      }
      perturb_wave(a.perturb, (uint32_t)(2 * k + c));
      __syncthreads();
    }
    if (a.EM) {
      uint64_t sa, sp;
      block_sum2(anti, up, red, sa, sp);
      if (threadIdx.x == 0) {
        a.EM[2 * k] = 2 * (int64_t)sa - 2 * g.L * g.L;
        a.EM[2 * k + 1] = 2 * (int64_t)sp - g.L * g.L;
      }
      __syncthreads();
    }
  }
  for (int64_t i = threadIdx.x; i < 2 * pw; i += blockDim.x) a.planes[i] = lds[i];
}

// ---------------------------------------------------------------------
// Tiled half-sweep for L % 8 == 0.
//
// Work unit: a tile of TR = 4*R*RPW rows x TW words of colour C.  A wave
// processes RPW row groups of the tile one after the other, one word per
// lane per group (W >= kWideMinWords: a row group is one row of a 64-word segment;
// W < 64: a row group is R = floor(64/W) whole rows).  The plain and fused
// kernels read each word's four neighbour words directly
// (process_tile_direct: the rows that neighbouring lanes and tiles share
// hit in L1/L2, the loads are issued before the Philox stretch and used
// after it, and the waves of a workgroup never wait for each other).  The
// packed persistent kernel stages the other colour's rows y0-1 .. y0+TR
// and words w0-1 .. w0+TW (periodic) in LDS instead (process_tile), since
// it needs block barriers between colour steps anyway.  The Philox block index of word
// (y, w) is y*L/8 + 16*w + q; its high word is 0 (hi_mode 0) or uniform
// over the wave's row (hi_mode 1), so only the low word varies per lane.
//
// Workgroups walk the tiles with a grid stride; logical block numbers are
// grouped by XCD (hardware dispatches block b to XCD b mod 8), so that
// vertically adjacent tiles share one L2.
//
// E/M (colour 1): each block writes its (anti-aligned bond, up spin) counts
// to part[block]; block 0 of the next colour-0 pass (or launch_finalize_em)
// reduces them into (E, M) = (2A - 2N, 2P - N).
// ---------------------------------------------------------------------
__device__ __forceinline__ void finalize_partials(const uint64_t* part, int nblocks, int64_t L,
                                                  int64_t* EM, uint64_t* red64) {
  uint64_t a = 0, p = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
    a += part[2 * i];
    p += part[2 * i + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    p += __shfl_xor(p, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red64[2 * wave] = a;
    red64[2 * wave + 1] = p;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t sa = 0, sp = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      sa += red64[2 * i];
      sp += red64[2 * i + 1];
    }
    EM[0] = 2 * (int64_t)sa - 2 * L * L;
    EM[1] = 2 * (int64_t)sp - L * L;
  }
  __syncthreads();
}

__device__ __forceinline__ int64_t wrap_row(int64_t y, int64_t L) {
  return y < 0 ? y + L : (y >= L ? y - L : y);
}

// Lane-to-word and lane-to-staging maps of one lattice's tile shape.
struct TileLane {
  bool wide;
  int TR, SW, SR;    // rows per tile, staged row width, staged rows
  int r_off, w_l;    // position of this lane inside a row group
  bool lane_ok;
  int st_r, st_c, P; // staging: row/column of this lane within a pass of P rows
};

template <int WIDEM>
__device__ __forceinline__ TileLane tile_lane(const TileArgs& a) {
  TileLane t;
  // WIDEM: 0 / 1 fixes the row-group shape at compile time, 2 reads it from
  // the arguments (W >= kWideMinWords).
  const bool WIDE = WIDEM == 2 ? (a.g.W >= kWideMinWords) : (WIDEM == 1);
  t.wide = WIDE;
  const int lane = threadIdx.x & 63;
  const int TW = a.TW, R = a.R;
  t.TR = 4 * R * a.RPW;
  t.SW = TW + 2;
  t.SR = t.TR + 2;
  if (WIDE) {
    t.r_off = 0;
    t.w_l = lane;
    t.lane_ok = true;
    // a wave pass loads one staged row of 66 words (lanes 0 and 1 also
    // load words 64 and 65)
    t.P = 1;
    t.st_r = 0;
    t.st_c = lane;
  } else {
    t.r_off = lane / TW;
    t.w_l = lane - t.r_off * TW;
    t.lane_ok = t.r_off < R;
    t.P = 64 / t.SW;
    t.st_r = lane / t.SW;
    t.st_c = lane - t.st_r * t.SW;
    if (t.st_r >= t.P) t.st_r = -1;
    // hosts only build narrow shapes with SW <= 64; never let a pass be empty
    if (t.P < 1) t.P = 1;
  }
  return t;
}

// One tile of one colour step: stage the other colour's rows in LDS, then
// update this tile's words (RPW row groups per wave).  `colour` and `em`
// are uniform.  Contains two block barriers.
template <bool FULL, int WIDEM, bool BUMP_SALU = false>
__device__ __forceinline__ void process_tile(const TileArgs& a, const TileLane& tl, int colour,
                                             bool em, int64_t tidx, uint64_t* tile,
                                             uint32_t& anti, uint32_t& up) {
  const Geom& g = a.g;
  const bool WIDE = WIDEM == 2 ? tl.wide : (WIDEM == 1);
  uint64_t* __restrict__ self = a.planes + (colour ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (colour ? 0 : a.plane_words);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int R = a.R, RPW = a.RPW, TR = tl.TR, SW = tl.SW, SR = tl.SR;
  const int r_off = tl.r_off, w_l = tl.w_l, st_r = tl.st_r, st_c = tl.st_c, P = tl.P;
  const bool lane_ok = tl.lane_ok;
  const uint32_t ctr3 = a.sid4 | (uint32_t)colour;
  const int64_t y0 = (tidx / a.segs) * TR;
  const int32_t w0 = WIDE ? (int32_t)(tidx % a.segs) * 64 : 0;
  for (int rr0 = wave * P; rr0 < SR; rr0 += 4 * P) {
    const int rr = rr0 + st_r;
    if (st_r >= 0 && rr < SR) {
      // a tile may span more than L rows when L is small: full modulo
      int64_t yy = (y0 - 1 + rr) % g.L;
      yy = yy < 0 ? yy + g.L : yy;
      const int32_t ww = (int32_t)wrap_row(w0 - 1 + st_c, g.W);
      tile[rr * SW + st_c] = other[yy * g.W + ww];
      if (WIDE && lane < 2) {
        const int32_t w2 = (int32_t)wrap_row(w0 + 63 + lane, g.W);
        tile[rr * SW + 64 + lane] = other[yy * g.W + w2];
      }
    }
  }
  perturb_wave(a.perturb, (uint32_t)(4 * tidx + 2 * colour));
  __syncthreads();
  for (int j = 0; j < RPW; ++j) {
    const int r_l = (wave * RPW + j) * R + r_off;
    const int64_t y = y0 + r_l;
    const int32_t w = w0 + w_l;
    if (!(lane_ok && y < g.L && w < g.W)) continue;
    const uint64_t s = self[y * g.W + w];
    const int base = (r_l + 1) * SW + (w_l + 1);
    Nbr n;
    n.n0 = tile[base];
    n.n2 = tile[base - SW];
    n.n3 = tile[base + SW];
    if (((y + colour) & 1) == 0) {
      const uint64_t left = tile[base - 1];
      n.n1 = (n.n0 << 1) | ((w > 0) ? (left >> 63) : ((left >> (g.nb_last - 1)) & 1ull));
    } else {
      const uint64_t right = tile[base + 1];
      n.n1 = (w < g.W - 1) ? ((n.n0 >> 1) | (right << 63))
                           : ((n.n0 >> 1) | ((right & 1ull) << (g.nb_last - 1)));
    }
    uint32_t lo, hi;
    if (a.hi_mode == 0) {
      lo = (uint32_t)y * (uint32_t)g.L8 + 16u * (uint32_t)w;
      hi = 0;
    } else {
      const uint64_t gy =
          (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)y) * (uint64_t)g.L8;
      hi = (uint32_t)(gy >> 32);
      lo = (uint32_t)gy + 16u * (uint32_t)w;
    }
    const int nq = (FULL || w < g.W - 1) ? 16 : (g.nb_last >> 2);
    uint64_t r4, r8;
    masks_shift<FULL, BUMP_SALU>(lo, hi, nq, a.k0, a.k1, a.t, ctr3, a.t4, a.t8, r4, r8);
    const uint64_t valid = (FULL || w < g.W - 1) ? ~0ull : low_mask(g.nb_last);
    const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
    self[y * g.W + w] = s_new;
    if (colour == 1 && em) count_word(s_new, n, valid, anti, up);
  }
  perturb_wave(a.perturb, (uint32_t)(4 * tidx + 2 * colour + 1));
  __syncthreads();
}

// The same tile of one colour step without LDS staging: each lane loads its
// own word and its four neighbour words straight from memory (the rows
// shared by neighbouring lanes hit in L1/L2), issues the loads before the
// Philox stretch and uses them after it.  No block barrier: the four waves
// of a workgroup work independently.  Spin words are stored write-through.
template <bool FULL, int WIDEM, bool BUMP_SALU = false, bool LCG = false, bool FLAT = false>
__device__ __forceinline__ void process_tile_direct(const TileArgs& a, const TileLane& tl,
                                                    int colour, bool em, int64_t tidx,
                                                    uint32_t& anti, uint32_t& up) {
  const Geom& g = a.g;
  const bool WIDE = WIDEM == 2 ? tl.wide : (WIDEM == 1);
  uint64_t* __restrict__ self = a.planes + (colour ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (colour ? 0 : a.plane_words);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int R = a.R, RPW = a.RPW;
  const uint32_t ctr3 = a.sid4 | (uint32_t)colour;
  const int64_t y0 = (tidx / a.segs) * tl.TR;
  const int32_t w0 = WIDE ? (int32_t)(tidx % a.segs) * 64 : 0;
  const int64_t W = g.W;
  for (int j = 0; j < RPW; ++j) {
    int64_t y;
    int32_t w;
    uint32_t iu = 0;  // flat shapes: the word's index in its plane
    if (FLAT) {
      const int64_t i = ((tidx * 4 + wave) * RPW + j) * 64 + (threadIdx.x & 63);
      if (i >= a.plane_words) continue;
      iu = (uint32_t)i;  // plane_words < 2^32 for flat shapes
      if (W == 1) {  // floor(2^32 / 1) + 1 does not fit 32 bits
        y = iu;
        w = 0;
      } else {
        uint32_t q = (uint32_t)(((uint64_t)iu * a.wdiv_m) >> 32);
        int64_t r = (int64_t)iu - (int64_t)q * W;
        if (r < 0) {
          q -= 1u;
          r += W;
        }
        y = q;
        w = (int32_t)r;
      }
    } else {
      const int r_l = (wave * RPW + j) * R + tl.r_off;
      y = y0 + r_l;
      w = w0 + tl.w_l;
      if (!(tl.lane_ok && y < g.L && w < W)) continue;
    }
    // horizontal partner: left (site k-1) when (y + colour) is even, else right
    const bool left = ((y + colour) & 1) == 0;
    const int32_t ws = left ? (w > 0 ? w - 1 : (int32_t)W - 1) : (w < W - 1 ? w + 1 : 0);
    // word offsets in a plane of the word, its row neighbours (periodic) and
    // its horizontal partner; flat shapes have planes of < 2^32 words, so
    // they derive all four from the word's own index in 32-bit arithmetic
    uint64_t off, off_m, off_p, off_s;
    if (FLAT) {
      const uint32_t W32 = (uint32_t)W;
      const uint32_t wrap = (uint32_t)(a.plane_words - W);  // offset of the last row
      off = iu;
      off_m = y == 0 ? iu + wrap : iu - W32;
      off_p = y == g.L - 1 ? iu - wrap : iu + W32;
      off_s = iu + (uint32_t)(ws - w);
    } else {
      const int64_t ym = y == 0 ? g.L - 1 : y - 1;
      const int64_t yp = y == g.L - 1 ? 0 : y + 1;
      off = (uint64_t)(y * W + w);
      off_m = (uint64_t)(ym * W + w);
      off_p = (uint64_t)(yp * W + w);
      off_s = (uint64_t)(y * W + ws);
    }
    const uint64_t s = self[off];
    const uint64_t n0 = other[off];
    const uint64_t n2 = other[off_m];
    const uint64_t n3 = other[off_p];
    const uint64_t sd = other[off_s];
    uint64_t r4, r8;
    if (LCG) {
      // this word's generator: thread (colour L + y) W + w
      uint32_t* xs = a.lcg + (colour ? a.plane_words : 0) + off;
      uint32_t z = *xs + a.l4d;
      masks_lcg(z, a.lc, a.le, a.l4m, a.l8m, r4, r8);
      *xs = z - a.l4d;
    } else {
      uint32_t lo, hi;
      if (a.hi_mode == 0) {
        lo = (uint32_t)y * (uint32_t)g.L8 + 16u * (uint32_t)w;
        hi = 0;
      } else {
        const uint64_t gy =
            (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)y) * (uint64_t)g.L8;
        hi = (uint32_t)(gy >> 32);
        lo = (uint32_t)gy + 16u * (uint32_t)w;
      }
      const int nq = (FULL || w < W - 1) ? 16 : (g.nb_last >> 2);
      masks_shift<FULL, BUMP_SALU>(lo, hi, nq, a.k0, a.k1, a.t, ctr3, a.t4, a.t8, r4, r8);
    }
    __builtin_amdgcn_sched_barrier(0);
    Nbr n;
    n.n0 = n0;
    n.n2 = n2;
    n.n3 = n3;
    if (FULL) {
      n.n1 = left ? ((n0 << 1) | (sd >> 63)) : ((n0 >> 1) | (sd << 63));
    } else {
      const uint64_t bl = w > 0 ? (sd >> 63) : ((sd >> (g.nb_last - 1)) & 1ull);
      const uint64_t br = w < W - 1 ? (sd << 63) : ((sd & 1ull) << (g.nb_last - 1));
      n.n1 = left ? ((n0 << 1) | bl) : ((n0 >> 1) | br);
    }
    const uint64_t valid = (FULL || w < W - 1) ? ~0ull : low_mask(g.nb_last);
    const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
    // write-through at device scope (sc1): the XCD L2s then hold no dirty
    // lattice lines for the write-back at the end of the launch
    __hip_atomic_store(&self[off], s_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (colour == 1 && em) count_word(s_new, n, valid, anti, up);
  }
}

// Tiles read their neighbour words directly (process_tile_direct): no LDS
// staging and no barrier until the E/M reduction at the end.
template <int C, bool EM, bool FULL, bool WIDE, bool LCG, bool FLAT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_sweep(
    TileArgs a) {
  __shared__ uint64_t red64[8];
  __shared__ uint64_t red[8];
  if (C == 0 && a.prev_EM != nullptr && blockIdx.x == 0)
    finalize_partials(a.prev_part, a.prev_blocks, a.g.L, a.prev_EM, red64);
  // logical block number grouped by XCD
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  uint32_t anti = 0, up = 0;
  const TileLane tl = tile_lane<WIDE ? 1 : 0>(a);
  for (int64_t tidx = lb; tidx < a.tiles; tidx += G)
    process_tile_direct<FULL, WIDE ? 1 : 0, false, LCG, FLAT>(a, tl, C, EM, tidx, anti, up);
  if (C == 1 && EM) {
    uint64_t sa, sp;
    block_sum2(anti, up, red, sa, sp);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = sa;
      a.part[2 * blockIdx.x + 1] = sp;
    }
  }
}

// ---------------------------------------------------------------------
// Boltzmann-pattern pools (section 4's exp4/exp8 patterns, looked up at a
// random address per update instead of drawn per site; section 5.1 and
// Table 2 for the "unmodified" and "linear" GPU variants).  A pattern is a
// pair of words (r4, r8): bit b of pattern p is [u < t4], [u < t8] for the
// uniform u of index i = 64 p + b, Philox4x32-10 with the lattice's key and
// counter (lo32 i/4, hi32 i/4, 2^32 - 1, stream_id << 2 | 2).  The paper's
// encoding is exp8 = r8, exp4 = r4 & ~r8, and its flip rule k + 2 exp8 +
// exp4 >= 2 is flip_mask's.  In sweep t, colour c, word j = y W + w draws
// v = output 0 of Philox4x32-10 with counter (lo32 q, hi32 q, t,
// stream_id << 2 | c), q = j (random addresses) or q = j / 256 (linear
// reads), and reads pattern v >> (32 - m), plus j mod 256 for linear reads
// (mod 2^m).
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pool_fill(uint64_t* pool, int64_t P, uint32_t k0,
                                                   uint32_t k1, uint32_t sid4, uint32_t t4,
                                                   uint32_t t8) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    uint64_t r4, r8;
    masks_shift<true>(16u * (uint32_t)p, 0u, 16, k0, k1, 0xFFFFFFFFu, sid4 | 2u, t4, t8, r4,
                      r8);
    pool[2 * p] = r4;
    pool[2 * p + 1] = r8;
  }
}

hipError_t launch_pool_fill(hipStream_t st, uint64_t* pool, int m, uint32_t k0, uint32_t k1,
                            uint32_t sid4, uint32_t t4, uint32_t t8) {
  const int64_t P = (int64_t)1 << m;
  const int64_t blocks = std::min<int64_t>((P + 255) / 256, 8192);
  hipLaunchKernelGGL(k_pool_fill, dim3((unsigned)blocks), dim3(256), 0, st, pool, P, k0, k1,
                     sid4, t4, t8);
  return hipGetLastError();
}

// One tile of a pool colour step: 4 waves x 4 words per lane on the flat
// mapping (wave task k = words 256 k .. 256 k + 255, which is one linear
// group).  Every lane first draws the addresses of its 4 words and issues
// all their loads (own word, 4 neighbours, pattern), then updates them: the
// work per word is small, so the loads of the 4 words overlap.
template <int C, bool EM, bool FULL, bool LINEAR>
__device__ __forceinline__ void pool_tile(const TileArgs& a, int64_t tidx, uint32_t& anti,
                                          uint32_t& up) {
  constexpr int RPW = 4;
  const Geom& g = a.g;
  uint64_t* __restrict__ self = a.planes + (C ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (C ? 0 : a.plane_words);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t W = g.W;
  const uint32_t ctr3 = a.sid4 | (uint32_t)C;
  const int64_t task = tidx * 4 + wave;
  const ulonglong2* __restrict__ pool = (const ulonglong2*)a.pool;
  uint32_t lin = 0;
  if (LINEAR) {  // one draw per wave task (= 256-word group)
    uint32_t x0 = (uint32_t)task, x1 = 0, x2 = a.t, x3 = ctr3;
    philox4x32_10(x0, x1, x2, x3, a.k0, a.k1);
    lin = x0 >> a.pool_shift;
  }
  uint32_t iw[RPW];
  int32_t yv[RPW], wv[RPW];
  bool ok[RPW];
  uint64_t s[RPW], n0[RPW], n2[RPW], n3[RPW], sd[RPW];
  ulonglong2 pat[RPW];
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int64_t i = (task * RPW + j) * 64 + (threadIdx.x & 63);
    ok[j] = i < a.plane_words;
    const uint32_t iu = ok[j] ? (uint32_t)i : 0u;  // plane_words < 2^32 for pool lattices
    uint32_t y, w;
    if (W == 1) {
      y = iu;
      w = 0;
    } else {
      uint32_t q = (uint32_t)(((uint64_t)iu * a.wdiv_m) >> 32);
      int64_t r = (int64_t)iu - (int64_t)q * W;
      if (r < 0) {
        q -= 1u;
        r += W;
      }
      y = q;
      w = (uint32_t)r;
    }
    iw[j] = iu;
    yv[j] = (int32_t)y;
    wv[j] = (int32_t)w;
    uint32_t addr;
    if (LINEAR) {
      addr = (lin + (iu & 255u)) & a.pool_mask;
    } else {
      uint32_t x0 = iu, x1 = 0, x2 = a.t, x3 = ctr3;
      philox4x32_10(x0, x1, x2, x3, a.k0, a.k1);
      addr = x0 >> a.pool_shift;
    }
    const int64_t ym = y == 0 ? g.L - 1 : (int64_t)y - 1;
    const int64_t yp = (int64_t)y == g.L - 1 ? 0 : (int64_t)y + 1;
    const bool left = ((y + (uint32_t)C) & 1u) == 0;
    const int64_t ws = left ? (w > 0 ? w - 1 : W - 1) : ((int64_t)w < W - 1 ? w + 1 : 0);
    s[j] = self[iu];
    n0[j] = other[iu];
    n2[j] = other[ym * W + w];
    n3[j] = other[yp * W + w];
    sd[j] = other[(int64_t)y * W + ws];
    pat[j] = pool[addr];
  }
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    if (!ok[j]) continue;
    const int32_t y = yv[j], w = wv[j];
    const bool left = ((y + C) & 1) == 0;
    Nbr n;
    n.n0 = n0[j];
    n.n2 = n2[j];
    n.n3 = n3[j];
    if (FULL) {
      n.n1 = left ? ((n0[j] << 1) | (sd[j] >> 63)) : ((n0[j] >> 1) | (sd[j] << 63));
    } else {
      const uint64_t bl = w > 0 ? (sd[j] >> 63) : ((sd[j] >> (g.nb_last - 1)) & 1ull);
      const uint64_t br = w < W - 1 ? (sd[j] << 63) : ((sd[j] & 1ull) << (g.nb_last - 1));
      n.n1 = left ? ((n0[j] << 1) | bl) : ((n0[j] >> 1) | br);
    }
    const uint64_t valid = (FULL || w < W - 1) ? ~0ull : low_mask(g.nb_last);
    const uint64_t s_new = s[j] ^ (flip_mask(s[j], n, pat[j].x, pat[j].y) & valid);
    __hip_atomic_store(&self[iw[j]], s_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (C == 1 && EM) count_word(s_new, n, valid, anti, up);
  }
}

template <int C, bool EM, bool FULL, bool LINEAR>
__global__ __launch_bounds__(256) void k_pool_sweep(TileArgs a) {
  __shared__ uint64_t red64[8];
  __shared__ uint64_t red[8];
  if (C == 0 && a.prev_EM != nullptr && blockIdx.x == 0)
    finalize_partials(a.prev_part, a.prev_blocks, a.g.L, a.prev_EM, red64);
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  uint32_t anti = 0, up = 0;
  for (int64_t tidx = lb; tidx < a.tiles; tidx += G) pool_tile<C, EM, FULL, LINEAR>(a, tidx, anti, up);
  if (C == 1 && EM) {
    uint64_t sa, sp;
    block_sum2(anti, up, red, sa, sp);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = sa;
      a.part[2 * blockIdx.x + 1] = sp;
    }
  }
}

// ---------------------------------------------------------------------
// Strip shares (ShareArgs): the rows of one GPU's share of a row-strip
// decomposition, with halo rows supplied by the exchange.  Words are
// mapped flat over the strip's own rows, one word per lane per step of a
// grid-stride loop; the uniforms are keyed by global coordinates, so a set
// of strips advanced in step with halo exchanges reproduces the whole
// lattice bit for bit.
// ---------------------------------------------------------------------
__device__ __forceinline__ void share_word(const ShareArgs& a, uint32_t i, uint32_t& r,
                                           uint32_t& w) {
  if (a.W == 1) {
    r = i;
    w = 0;
    return;
  }
  uint32_t q = (uint32_t)(((uint64_t)i * a.wdiv_m) >> 32);
  int64_t rem = (int64_t)i - (int64_t)q * a.W;
  if (rem < 0) {
    q -= 1u;
    rem += a.W;
  }
  r = q;
  w = (uint32_t)rem;
}

__global__ __launch_bounds__(256) void k_share_init(ShareArgs a, int init) {
  const int64_t words = a.rows * a.W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * words;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = i >= words ? 1 : 0;
    const uint32_t j = (uint32_t)(i - c * words);
    uint32_t r, w;
    share_word(a, j, r, w);
    uint64_t word;
    if (init == 0) {
      word = ~0ull;
    } else if (init == 1) {
      word = 0;
    } else {
      const uint64_t g = (uint64_t)(a.y0 + r) * a.L8 + 16u * w;
      uint64_t m, unused;
      masks_shift<true>((uint32_t)g, (uint32_t)(g >> 32), 16, a.k0, a.k1, 0u,
                        a.sid4 | (2u + (uint32_t)c), 0x80000000u, 0x80000000u, m, unused);
      word = m;
    }
    a.planes[(int64_t)c * a.plane_words + ((int64_t)r + 1) * a.W + w] = word;
  }
}

template <int C, bool EM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_share_sweep(
    ShareArgs a) {
  __shared__ uint64_t red[8];
  uint64_t* __restrict__ self = a.planes + (C ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (C ? 0 : a.plane_words);
  const int64_t W = a.W;
  const uint32_t words = (uint32_t)(a.rows * W);  // < 2^32 (checked on the host)
  const uint32_t ctr3 = a.sid4 | (uint32_t)C;
  uint32_t anti = 0, up = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += gridDim.x * blockDim.x) {
    uint32_t r, w;
    share_word(a, i, r, w);
    const int64_t y = a.y0 + r;  // global row
    const int64_t row = (int64_t)r + 1;  // buffer row; rows 0 and rows + 1 are halos
    const bool left = ((y + C) & 1) == 0;
    const uint32_t ws = left ? (w > 0 ? w - 1 : (uint32_t)W - 1) : (w + 1 < (uint32_t)W ? w + 1 : 0);
    const uint64_t s = self[row * W + w];
    const uint64_t n0 = other[row * W + w];
    const uint64_t n2 = other[(row - 1) * W + w];
    const uint64_t n3 = other[(row + 1) * W + w];
    const uint64_t sd = other[row * W + ws];
    const uint64_t g = (uint64_t)y * a.L8 + 16u * w;
    uint64_t r4, r8;
    masks_shift<true>((uint32_t)g, (uint32_t)(g >> 32), 16, a.k0, a.k1, a.t, ctr3, a.t4, a.t8,
                      r4, r8);
    __builtin_amdgcn_sched_barrier(0);
    Nbr n;
    n.n0 = n0;
    n.n2 = n2;
    n.n3 = n3;
    n.n1 = left ? ((n0 << 1) | (sd >> 63)) : ((n0 >> 1) | (sd << 63));
    const uint64_t s_new = s ^ flip_mask(s, n, r4, r8);
    __hip_atomic_store(&self[row * W + w], s_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (C == 1 && EM) count_word(s_new, n, ~0ull, anti, up);
  }
  if (C == 1 && EM) {
    uint64_t sa, sp;
    block_sum2(anti, up, red, sa, sp);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = sa;
      a.part[2 * blockIdx.x + 1] = sp;
    }
  }
}

__global__ __launch_bounds__(256) void k_share_counts(const uint64_t* part, int blocks,
                                                      int64_t* counts) {
  __shared__ uint64_t red[8];
  uint64_t a = 0, p = 0;
  for (int i = threadIdx.x; i < blocks; i += blockDim.x) {
    a += part[2 * i];
    p += part[2 * i + 1];
  }
  uint64_t sa, sp;
  // per-thread sums fit 32 bits only per block, so reduce in 64 bits here
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    p += __shfl_xor(p, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wave] = a;
    red[2 * wave + 1] = p;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sa = sp = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      sa += red[2 * k];
      sp += red[2 * k + 1];
    }
    counts[0] = (int64_t)sa;
    counts[1] = (int64_t)sp;
  }
}

__global__ __launch_bounds__(256) void k_share_combine(const int64_t* counts, int32_t nstrips,
                                                       int64_t n, int64_t L, int64_t* EM) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    int64_t A = 0, P = 0;
    for (int32_t s = 0; s < nstrips; ++s) {
      A += counts[2 * (k * nstrips + s)];
      P += counts[2 * (k * nstrips + s) + 1];
    }
    EM[2 * k] = 2 * A - 2 * L * L;
    EM[2 * k + 1] = 2 * P - L * L;
  }
}

hipError_t launch_share_init(hipStream_t st, const ShareArgs& a, int init) {
  const int64_t blocks = std::min<int64_t>((2 * a.rows * a.W + 255) / 256, 4096);
  hipLaunchKernelGGL(k_share_init, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                     a, init);
  return hipGetLastError();
}

hipError_t launch_share_sweep(hipStream_t st, int colour, const ShareArgs& a, int blocks) {
  if (colour == 0)
    hipLaunchKernelGGL((k_share_sweep<0, false>), dim3(blocks), dim3(256), 0, st, a);
  else if (a.part)
    hipLaunchKernelGGL((k_share_sweep<1, true>), dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_share_sweep<1, false>), dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_share_counts(hipStream_t st, const uint64_t* part, int blocks, int64_t* counts) {
  hipLaunchKernelGGL(k_share_counts, dim3(1), dim3(256), 0, st, part, blocks, counts);
  return hipGetLastError();
}

hipError_t launch_share_combine(hipStream_t st, const int64_t* counts, int32_t nstrips, int64_t n,
                                int64_t L, int64_t* EM) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_share_combine, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0,
                     st, counts, nstrips, n, L, EM);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Strip form of the wide half-sweep: one wave owns 64 consecutive words of
// RPW consecutive rows (a "task") and walks down them, keeping the other
// colour's rows y-1, y, y+1 in registers and loading row y+2, the
// horizontal partner word and its own word of row y+1 while it computes
// row y.  No LDS staging and no barriers inside a task, so the waves of a
// workgroup run independently; the E/M partial is reduced once per
// workgroup at the end.  Tasks are numbered segment-fastest within a row
// strip: task = strip * segs + seg.
// ---------------------------------------------------------------------
template <int C, bool EM, bool FULL>
__device__ __forceinline__ void strip_task(const TileArgs& a, int64_t task, uint32_t& anti,
                                           uint32_t& up) {
  const Geom& g = a.g;
  const int64_t W = g.W, L = g.L;
  uint64_t* __restrict__ self = a.planes + (C ? a.plane_words : 0);
  const uint64_t* __restrict__ other = a.planes + (C ? 0 : a.plane_words);
  const int lane = threadIdx.x & 63;
  const int64_t strip = task / a.segs;
  const int32_t w = (int32_t)(task - strip * a.segs) * 64 + lane;
  const bool ok = w < W;
  const int32_t wc = ok ? w : (int32_t)W - 1;  // in-bounds column for idle lanes
  const int32_t wl = wc > 0 ? wc - 1 : (int32_t)W - 1;
  const int32_t wr = wc < W - 1 ? wc + 1 : 0;
  const int64_t y0 = strip * a.RPW;
  const int64_t y1 = (y0 + a.RPW < L) ? y0 + a.RPW : L;
  const uint32_t ctr3 = a.sid4 | (uint32_t)C;
  const uint64_t valid = (FULL || w < W - 1) ? ~0ull : low_mask(g.nb_last);
  const int nq = (FULL || w < W - 1) ? 16 : (g.nb_last >> 2);
  // Row y: the other colour's rows y-1, y, y+1 are in (om, oc, op), the
  // horizontal partner word in sd and the own word in s.  Before computing
  // it, the step loads row y+2 into `nx` and the partner and own words of
  // row y+1 into sd_n, s_n (rows modulo L).  The caller rotates the roles of the registers
  // (four-row cycle for the rows, two-row cycle for sd and s), so no value
  // is copied and no load is waited for before the next row needs it.
  auto step = [&](int64_t y, const uint64_t& om, const uint64_t& oc, const uint64_t& op,
                  uint64_t& nx, const uint64_t& sd, uint64_t& sd_n, const uint64_t& s,
                  uint64_t& s_n) {
    {
      // unconditional (the last row of a task loads values it never uses;
      // the rows wrap, so every address is inside the lattice)
      const int64_t yn = wrap_row(y + 1, L);
      nx = other[wrap_row(yn + 1, L) * W + wc];
      sd_n = other[yn * W + (((yn + C) & 1) == 0 ? wl : wr)];
      s_n = self[yn * W + wc];
    }
    if (!ok) return;
    uint32_t lo, hi;
    if (a.hi_mode == 0) {
      lo = (uint32_t)y * (uint32_t)g.L8 + 16u * (uint32_t)w;
      hi = 0;
    } else {
      const uint64_t gy = (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)y) * (uint64_t)g.L8;
      hi = (uint32_t)(gy >> 32);
      lo = (uint32_t)gy + 16u * (uint32_t)w;
    }
    uint64_t r4, r8;
    masks_shift<FULL>(lo, hi, nq, a.k0, a.k1, a.t, ctr3, a.t4, a.t8, r4, r8);
    // the uniforms need no lattice data: keep the gather below them so that
    // the row's loads have the whole Philox stretch to arrive
    __builtin_amdgcn_sched_barrier(0);
    Nbr n;
    n.n0 = oc;
    n.n2 = om;
    n.n3 = op;
    if (((y + C) & 1) == 0) {
      n.n1 = (oc << 1) | ((FULL || w > 0) ? (sd >> 63) : ((sd >> (g.nb_last - 1)) & 1ull));
    } else {
      n.n1 = (FULL || w < W - 1) ? ((oc >> 1) | (sd << 63))
                                 : ((oc >> 1) | ((sd & 1ull) << (g.nb_last - 1)));
    }
    const uint64_t s_new = s ^ (flip_mask(s, n, r4, r8) & valid);
    // written through to memory at device scope: the XCD L2s then hold no
    // dirty lattice lines for the kernel-boundary write-back
    __hip_atomic_store(&self[y * W + w], s_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (C == 1 && EM) count_word(s_new, n, valid, anti, up);
  };
  uint64_t o0 = other[wrap_row(y0 - 1, L) * W + wc];
  uint64_t o1 = other[y0 * W + wc];
  uint64_t o2 = other[wrap_row(y0 + 1, L) * W + wc];
  uint64_t o3 = 0;
  uint64_t sd0 = other[y0 * W + (((y0 + C) & 1) == 0 ? wl : wr)], sd1 = 0;
  uint64_t s0 = self[y0 * W + wc], s1 = 0;
  for (int64_t y = y0; y < y1; y += 4) {
    step(y, o0, o1, o2, o3, sd0, sd1, s0, s1);
    if (y + 1 >= y1) break;
    step(y + 1, o1, o2, o3, o0, sd1, sd0, s1, s0);
    if (y + 2 >= y1) break;
    step(y + 2, o2, o3, o0, o1, sd0, sd1, s0, s1);
    if (y + 3 >= y1) break;
    step(y + 3, o3, o0, o1, o2, sd1, sd0, s1, s0);
  }
}

// 8 waves per SIMD (the gfx950 maximum) need <= 100 SGPRs; without the
// hint the compiler takes 106 and a CU would hold only 7 workgroups.
template <int C, bool EM, bool FULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_strip_sweep(
    TileArgs a) {
  __shared__ uint64_t red64[8];
  __shared__ uint64_t red[8];
  if (C == 0 && a.prev_EM != nullptr && blockIdx.x == 0)
    finalize_partials(a.prev_part, a.prev_blocks, a.g.L, a.prev_EM, red64);
  // logical block number grouped by XCD, so that neighbouring tasks share an L2
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t anti = 0, up = 0;
  for (int64_t task = (int64_t)lb * 4 + wave; task < a.tiles; task += (int64_t)G * 4)
    strip_task<C, EM, FULL>(a, task, anti, up);
  if (C == 1 && EM) {
    uint64_t sa, sp;
    block_sum2(anti, up, red, sa, sp);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = sa;
      a.part[2 * blockIdx.x + 1] = sp;
    }
  }
}

__global__ __launch_bounds__(256) void k_finalize_em(const uint64_t* part, int nblocks, int64_t L,
                                                     int64_t* EM) {
  __shared__ uint64_t red64[8];
  finalize_partials(part, nblocks, L, EM, red64);
}

// ---------------------------------------------------------------------
// Batched sweeps over many lattices of uneven size and temperature.
//
// k_fused<C>: one launch advances colour C of every lattice of the batch by
// one sweep.  The tiles of all lattices form one flat list that the grid
// walks with a stride, so the work of a colour step is balanced over the
// whole GPU whatever the mix of sizes; the kernel boundary is the barrier
// between colour steps (a device-wide barrier inside a kernel would need
// an agent-scope release/acquire of the XCD L2s at every colour step).
// The sweep index is read from device memory (*kbase + klocal) so that a
// captured chunk of K sweeps can be replayed from a hipGraph, followed by
// k_advance (*kbase += K).  Colour 1 writes each tile's (anti-aligned
// bond, up spin) counts to part[(k & 1)][tile]; colour 0 of the next sweep
// (or k_fused_finalize after the last one) reduces them per lattice into
// (E, M) = (2A - 2N, 2P - N).
//
// k_batch: a persistent kernel for batches of small lattices that each fit
// one workgroup: every workgroup runs its packed list of lattices for all
// n sweeps with block barriers only (one launch in total).
// ---------------------------------------------------------------------
__device__ __forceinline__ void finalize_tiles(const FusedArgs& f, uint32_t k, uint64_t* red64) {
  // per-wave partials: 4 slots of (anti, up) per tile; lattice totals need
  // 64 bits (2 N reaches 2^32 at L = 46341)
  const uint32_t* part = f.part + (size_t)(k & 1u) * 8 * f.ntiles;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int l = blockIdx.x; l < f.nlat; l += gridDim.x) {
    const FusedLattice Lt = ((const FusedLattice ISING_CONSTANT_AS*)f.lat)[l];
    if (Lt.EM == nullptr || (int64_t)k >= Lt.nsweeps) continue;
    uint64_t a = 0, p = 0;
    for (int64_t i = threadIdx.x; i < 4 * Lt.ntiles; i += blockDim.x) {
      a += part[2 * (4 * Lt.first_tile + i)];
      p += part[2 * (4 * Lt.first_tile + i) + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      p += __shfl_xor(p, off, 64);
    }
    if (lane == 0) {
      red64[2 * wave] = a;
      red64[2 * wave + 1] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      a = p = 0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        a += red64[2 * i];
        p += red64[2 * i + 1];
      }
      const int64_t L = Lt.ta.g.L;
      Lt.EM[2 * (int64_t)k] = 2 * (int64_t)a - 2 * L * L;
      Lt.EM[2 * (int64_t)k + 1] = 2 * (int64_t)p - L * L;
    }
    __syncthreads();
  }
}

// 8 waves per SIMD need <= 100 SGPRs (the grid assumes 8 workgroups per CU)
template <int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_fused(
    FusedArgs f) {
  __shared__ uint64_t red64[8];
  const uint32_t k = *((const uint32_t ISING_CONSTANT_AS*)f.kbase) + (uint32_t)f.klocal;
  if (C == 0 && k > 0) finalize_tiles(f, k - 1, red64);
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* part = f.part + (size_t)(k & 1u) * 8 * f.ntiles;
  for (int64_t tidx = lb; tidx < f.ntiles; tidx += G) {
    const FusedTile ft = ((const FusedTile ISING_CONSTANT_AS*)f.tiles)[tidx];
    const FusedLattice Lt = ((const FusedLattice ISING_CONSTANT_AS*)f.lat)[ft.lattice];
    if ((int64_t)k >= Lt.nsweeps) continue;  // this lattice has finished its sweeps
    TileArgs a = Lt.ta;
    a.t = Lt.ta.t + k;
    const bool em = C == 1 && Lt.EM != nullptr;
    const TileLane tl = tile_lane<2>(a);
    uint32_t anti = 0, up = 0;
    // every fused lattice uses the flat mapping (run_fused sets it; for W
    // dividing 64 it is the narrow mapping itself)
    if (a.g.nb_last == 64)
      process_tile_direct<true, 2, false, false, true>(a, tl, C, em, ft.local, anti, up);
    else
      process_tile_direct<false, 2, false, false, true>(a, tl, C, em, ft.local, anti, up);
    if (em) {
      anti = wave_sum(anti);
      up = wave_sum(up);
      if ((threadIdx.x & 63) == 0) {
        part[2 * (4 * tidx + wave)] = anti;
        part[2 * (4 * tidx + wave) + 1] = up;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_fused_finalize(FusedArgs f) {
  __shared__ uint64_t red64[8];
  const uint32_t k = *((const uint32_t ISING_CONSTANT_AS*)f.kbase) + (uint32_t)f.klocal;
  finalize_tiles(f, k, red64);
}

__global__ void k_advance(uint32_t* kbase, uint32_t by) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *kbase += by;
}

__device__ __forceinline__ void run_packed_lattice(const BatchLattice& Lt, int64_t n,
                                                   uint64_t* tile, uint64_t* red) {
  TileArgs a = Lt.ta;
  const uint32_t t0 = Lt.ta.t;
  const bool em = Lt.EM != nullptr;
  const TileLane tl = tile_lane<2>(a);
  const int64_t nk = Lt.nsweeps < n ? Lt.nsweeps : n;
  for (int64_t k = 0; k < nk; ++k) {
    a.t = t0 + (uint32_t)k;
    uint32_t anti = 0, up = 0;
    for (int64_t tidx = 0; tidx < a.tiles; ++tidx)
      process_tile<false, 2, true>(a, tl, 0, false, tidx, tile, anti, up);
    for (int64_t tidx = 0; tidx < a.tiles; ++tidx)
      process_tile<false, 2, true>(a, tl, 1, em, tidx, tile, anti, up);
    if (em) {
      uint64_t sa, sp;
      block_sum2(anti, up, red, sa, sp);
      if (threadIdx.x == 0) {
        Lt.EM[2 * k] = 2 * (int64_t)sa - 2 * a.g.L * a.g.L;
        Lt.EM[2 * k + 1] = 2 * (int64_t)sp - a.g.L * a.g.L;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_batch(BatchArgs b) {
  __shared__ uint64_t tile[kTileLdsMaxWords];
  __shared__ uint64_t red[8];
  // The tables are read-only for the whole launch: read them through the
  // constant address space so that they land in SGPRs (scalar loads).
  typedef const BatchWG ISING_CONSTANT_AS* WgPtr;
  typedef const BatchItem ISING_CONSTANT_AS* ItemPtr;
  typedef const BatchLattice ISING_CONSTANT_AS* LatPtr;
  const BatchWG wg = ((WgPtr)b.wgs)[blockIdx.x];
  for (int it = 0; it < wg.n_items; ++it) {
    const BatchItem item = ((ItemPtr)b.items)[wg.first_item + it];
    const BatchLattice Lt = ((LatPtr)b.lat)[item.lattice];
    run_packed_lattice(Lt, b.n, tile, red);
  }
}

hipError_t launch_fused(hipStream_t st, int colour, const FusedArgs& f, int blocks) {
  if (colour == 0)
    hipLaunchKernelGGL(k_fused<0>, dim3(blocks), dim3(256), 0, st, f);
  else
    hipLaunchKernelGGL(k_fused<1>, dim3(blocks), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_fused_finalize(hipStream_t st, const FusedArgs& f, int blocks) {
  hipLaunchKernelGGL(k_fused_finalize, dim3(blocks), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_advance(hipStream_t st, uint32_t* kbase, uint32_t by) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, kbase, by);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------
template <bool LCG, bool FLAT>
static void launch_tile_sweep_rng(hipStream_t st, int colour, const TileArgs& a, int blocks) {
  const bool em = (colour == 1) ? (a.part != nullptr) : false;
  const bool full = a.g.nb_last == 64;
  // the flat mapping does not use the row-group shape: one instantiation
  const bool wide = !FLAT && a.g.W >= kWideMinWords;
#define ISING_TILE(C, E, F, WI) \
  hipLaunchKernelGGL((k_tile_sweep<C, E, F, WI, LCG, FLAT>), dim3(blocks), dim3(256), 0, st, a)
#define ISING_TILE_FW(C, E)                                   \
  do {                                                        \
    if (full) {                                               \
      if (wide) ISING_TILE(C, E, true, true);                 \
      else ISING_TILE(C, E, true, false);                     \
    } else {                                                  \
      if (wide) ISING_TILE(C, E, false, true);                \
      else ISING_TILE(C, E, false, false);                    \
    }                                                         \
  } while (0)
  if (colour == 0)
    ISING_TILE_FW(0, false);
  else if (em)
    ISING_TILE_FW(1, true);
  else
    ISING_TILE_FW(1, false);
#undef ISING_TILE_FW
#undef ISING_TILE
}

hipError_t launch_tile_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks) {
  if (a.lcg) {
    if (a.flat)
      launch_tile_sweep_rng<true, true>(st, colour, a, blocks);
    else
      launch_tile_sweep_rng<true, false>(st, colour, a, blocks);
  } else {
    if (a.flat)
      launch_tile_sweep_rng<false, true>(st, colour, a, blocks);
    else
      launch_tile_sweep_rng<false, false>(st, colour, a, blocks);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_lcg_seed(uint32_t* state, int64_t n, uint32_t s0) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    // 16807^j mod 2^32 by square and multiply
    uint32_t p = 1u, b = 16807u;
    for (uint64_t e = (uint64_t)j; e; e >>= 1) {
      if (e & 1u) p *= b;
      b *= b;
    }
    state[j] = s0 * p;
  }
}

hipError_t launch_lcg_seed(hipStream_t st, uint32_t* state, int64_t n, uint32_t s0) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lcg_seed, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                     state, n, s0);
  return hipGetLastError();
}

void make_flat(TileArgs& a, bool always) {
  const int64_t W = a.g.W;
  const int64_t words = a.plane_words;
  if (words >= (1ll << 32)) return;
  if (!always && (64 % W == 0 || W % 64 == 0)) return;
  a.flat = 1;
  a.wdiv_m = W == 1 ? 0u : (uint32_t)((1ull << 32) / (uint64_t)W + 1ull);
  const int64_t per_tile = 256 * (int64_t)a.RPW;
  a.tiles = (words + per_tile - 1) / per_tile;
}

template <bool LINEAR>
static void launch_pool_sweep_v(hipStream_t st, int colour, const TileArgs& a, int blocks) {
  const bool em = (colour == 1) ? (a.part != nullptr) : false;
  const bool full = a.g.nb_last == 64;
#define ISING_POOL(C, E, F) \
  hipLaunchKernelGGL((k_pool_sweep<C, E, F, LINEAR>), dim3(blocks), dim3(256), 0, st, a)
  if (colour == 0) {
    if (full) ISING_POOL(0, false, true);
    else ISING_POOL(0, false, false);
  } else if (em) {
    if (full) ISING_POOL(1, true, true);
    else ISING_POOL(1, true, false);
  } else {
    if (full) ISING_POOL(1, false, true);
    else ISING_POOL(1, false, false);
  }
#undef ISING_POOL
}

hipError_t launch_pool_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks) {
  if (a.pool_linear)
    launch_pool_sweep_v<true>(st, colour, a, blocks);
  else
    launch_pool_sweep_v<false>(st, colour, a, blocks);
  return hipGetLastError();
}

hipError_t launch_strip_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks) {
  const bool em = (colour == 1) ? (a.part != nullptr) : false;
  const bool full = a.g.nb_last == 64;
#define ISING_STRIP(C, E, F) \
  hipLaunchKernelGGL((k_strip_sweep<C, E, F>), dim3(blocks), dim3(256), 0, st, a)
  if (colour == 0) {
    if (full) ISING_STRIP(0, false, true);
    else ISING_STRIP(0, false, false);
  } else if (em) {
    if (full) ISING_STRIP(1, true, true);
    else ISING_STRIP(1, true, false);
  } else {
    if (full) ISING_STRIP(1, false, true);
    else ISING_STRIP(1, false, false);
  }
#undef ISING_STRIP
  return hipGetLastError();
}

hipError_t launch_finalize_em(hipStream_t st, const uint64_t* part, int blocks, int64_t L,
                              int64_t* EM) {
  hipLaunchKernelGGL(k_finalize_em, dim3(1), dim3(256), 0, st, part, blocks, L, EM);
  return hipGetLastError();
}
hipError_t launch_batch(hipStream_t st, const BatchArgs& a, int blocks) {
  hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_init(hipStream_t st, uint64_t* planes, const Geom& g, uint32_t k0, uint32_t k1,
                       uint32_t sid4, int init, int blocks) {
  const bool aligned = (g.L % 8) == 0;
  if (aligned)
    hipLaunchKernelGGL(k_init<true>, dim3(blocks), dim3(256), 0, st, planes, g, k0, k1, sid4,
                       init);
  else
    hipLaunchKernelGGL(k_init<false>, dim3(blocks), dim3(256), 0, st, planes, g, k0, k1, sid4,
                       init);
  return hipGetLastError();
}

hipError_t launch_half_sweep(hipStream_t st, int colour, const SweepArgs& a, int blocks) {
  const bool aligned = (a.g.L % 8) == 0;
  const bool em = a.EM != nullptr;
#define ISING_LAUNCH(C, AL, E) \
  hipLaunchKernelGGL((k_half_sweep<C, AL, E>), dim3(blocks), dim3(256), 0, st, a)
  if (colour == 0) {
    if (aligned) {
      if (em) ISING_LAUNCH(0, true, true); else ISING_LAUNCH(0, true, false);
    } else {
      if (em) ISING_LAUNCH(0, false, true); else ISING_LAUNCH(0, false, false);
    }
  } else {
    if (aligned) {
      if (em) ISING_LAUNCH(1, true, true); else ISING_LAUNCH(1, true, false);
    } else {
      if (em) ISING_LAUNCH(1, false, true); else ISING_LAUNCH(1, false, false);
    }
  }
#undef ISING_LAUNCH
  return hipGetLastError();
}

hipError_t launch_measure(hipStream_t st, const uint64_t* planes, const Geom& g,
                          int64_t plane_words, int64_t* EM, int blocks) {
  hipLaunchKernelGGL(k_set_em, dim3(1), dim3(64), 0, st, EM, -2 * g.L * g.L, -g.L * g.L);
  hipLaunchKernelGGL(k_measure, dim3(blocks), dim3(256), 0, st, planes, g, plane_words, EM);
  return hipGetLastError();
}

hipError_t launch_small_sweeps(hipStream_t st, const SmallArgs& a, int threads) {
  const size_t lds = (size_t)(2 * a.plane_words) * sizeof(uint64_t);
  const int64_t pw = a.plane_words;
  if ((a.g.L % 8) == 0 && pw >= 128 && pw <= 512) {
    // as many lanes per word as one workgroup of <= 1024 threads allows
    // (measured per sweep: 128^2 6.5 -> 5.2 us, 256^2 9.8 -> 9.3 us; at 64^2,
    // 16 lanes per word were slower than one, 4.5 against 4.1 us: there the
    // barriers and the per-sweep E/M reduction cost more than the Philox
    // stretch)
    int lpw = 16;
    while (lpw > 2 && pw * lpw > 1024) lpw >>= 1;
    const int th = (int)std::min<int64_t>(1024, (pw * lpw + 63) / 64 * 64);
#define ISING_SPLIT(N) hipLaunchKernelGGL(k_small_sweeps_split<N>, dim3(1), dim3(th), lds, st, a)
    switch (lpw) {
      case 16: ISING_SPLIT(16); break;
      case 8: ISING_SPLIT(8); break;
      case 4: ISING_SPLIT(4); break;
      default: ISING_SPLIT(2); break;
    }
#undef ISING_SPLIT
  } else if ((a.g.L % 8) == 0) {
    hipLaunchKernelGGL(k_small_sweeps<true>, dim3(1), dim3(threads), lds, st, a);
  } else {
    hipLaunchKernelGGL(k_small_sweeps<false>, dim3(1), dim3(threads), lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace ising
