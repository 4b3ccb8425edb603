// HIP kernels (gfx950) of the checkerboard Metropolis sweep on
// colour-packed uint64 words: initialisation, half-sweeps with the energy
// and magnetisation reduction fused into the colour-1 pass, a measurement
// pass, and a single-workgroup LDS-resident multi-sweep kernel for small
// lattices.
#include "ising_kernels.hpp"

#include "ising_device.hpp"

namespace ising {

// ---------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum (a, p) over the block; thread 0 gets the totals.  `red` holds 2
// entries per wave.
__device__ __forceinline__ void block_sum2(uint32_t& a, uint32_t& p, uint32_t* red) {
  a = wave_sum(a);
  p = wave_sum(p);
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
    a = (uint32_t)sa;
    p = (uint32_t)sp;
  }
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
  __shared__ uint32_t red[2 * 16];
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
    block_sum2(anti, up, red);
    if (threadIdx.x == 0) {
      atomicAdd((unsigned long long*)&a.EM[0], (unsigned long long)(2ull * anti));
      atomicAdd((unsigned long long*)&a.EM[1], (unsigned long long)(2ull * up));
    }
  }
}

// ---------------------------------------------------------------------
// Measurement of the current state: EM[0] += 2A, EM[1] += 2P over all
// colour-1 words (EM must hold -2N, -N on entry).
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_measure(const uint64_t* __restrict__ planes, Geom g,
                                                 int64_t plane_words, int64_t* EM) {
  __shared__ uint32_t red[2 * 16];
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
  block_sum2(anti, up, red);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&EM[0], (unsigned long long)(2ull * anti));
    atomicAdd((unsigned long long*)&EM[1], (unsigned long long)(2ull * up));
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
  __shared__ uint32_t red[2 * 16];
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
      __syncthreads();
    }
    if (a.EM) {
      block_sum2(anti, up, red);
      if (threadIdx.x == 0) {
        a.EM[2 * k] = 2 * (int64_t)anti - 2 * g.L * g.L;
        a.EM[2 * k + 1] = 2 * (int64_t)up - g.L * g.L;
      }
      __syncthreads();
    }
  }
  for (int64_t i = threadIdx.x; i < 2 * pw; i += blockDim.x) a.planes[i] = lds[i];
}

// ---------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------
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
  if ((a.g.L % 8) == 0)
    hipLaunchKernelGGL(k_small_sweeps<true>, dim3(1), dim3(threads), lds, st, a);
  else
    hipLaunchKernelGGL(k_small_sweeps<false>, dim3(1), dim3(threads), lds, st, a);
  return hipGetLastError();
}

}  // namespace ising
