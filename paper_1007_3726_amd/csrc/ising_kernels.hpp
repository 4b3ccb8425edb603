// Kernel argument blocks and launchers shared by the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

struct SweepArgs {
  uint64_t* planes;     // plane 0 then plane 1
  int64_t plane_words;  // L * W
  Geom g;
  uint32_t k0, k1;      // Philox key = (lo32, hi32) of the seed
  uint32_t sid4;        // stream_id << 2
  uint32_t t;           // sweep counter
  uint32_t t4, t8;      // Metropolis thresholds
  int64_t* EM;          // (E, M) of this sweep, or null
};

struct SmallArgs {
  uint64_t* planes;
  int64_t plane_words;
  Geom g;
  uint32_t k0, k1, sid4, t0, t4, t8;
  int64_t n;            // sweeps
  int64_t* EM;          // n x 2, or null
};

hipError_t launch_init(hipStream_t st, uint64_t* planes, const Geom& g, uint32_t k0, uint32_t k1,
                       uint32_t sid4, int init, int blocks);
hipError_t launch_half_sweep(hipStream_t st, int colour, const SweepArgs& a, int blocks);
hipError_t launch_measure(hipStream_t st, const uint64_t* planes, const Geom& g,
                          int64_t plane_words, int64_t* EM, int blocks);
hipError_t launch_small_sweeps(hipStream_t st, const SmallArgs& a, int threads);

}  // namespace ising
