// Internal host-side declarations of the runtime (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include "ising.h"
#include "ising_kernels.hpp"

namespace ising {

constexpr int64_t kMaxL = int64_t(1) << 21;
// scratch after the planes: [0, 256) measurement, then two slots of
// per-block E/M partials (2 x kMaxSweepBlocks x 16 bytes)
constexpr size_t kScratchBytes = 256 + 2 * (size_t)kMaxSweepBlocks * 16;

// Launch-shape choices for one lattice size (filled by default_tuning and
// refined by the autotuner).
struct Tuning {
  int64_t small_lds_bytes;  // lattices with both planes <= this run LDS-resident in one workgroup
  int max_blocks;           // grid cap of the grid-stride half-sweep kernels
  int rpw;                  // tile: row groups per wave; strip: rows per wave task (0: size rule)
  int form;                 // 0: tiles (default), 1: register-rolled strips (wide rows only)
};

// Shape for a lattice of side L: the autotuner's entry for L's size class
// if one is installed, else the defaults.
Tuning default_tuning(int64_t L);
// Row groups per wave the tile form uses for side L given the tuned value
// (0: the size rule).
int tile_rpw(int64_t L, int want);

ising_status fail(ising_status code, const char* fmt, ...);
ising_status hip_fail(hipError_t e, const char* what);
void clear_error();
int64_t words_per_row(int64_t L);
size_t lattice_bytes(int64_t L);
Geom make_geom(int64_t L);
uint32_t metropolis_threshold(double beta, int dE);
uint32_t lcg_threshold(double beta, int dE);
int grid_blocks(int64_t work_items, int threads, int max_blocks);
// Seed of the barrier-perturbation test hook (0: off; ising_debug_perturb).
uint32_t debug_perturb_seed();

}  // namespace ising

struct ising_lattice {
  int64_t L;
  ising::Geom g;
  int64_t plane_words;  // L * W
  uint64_t* planes;     // device: plane 0 then plane 1
  int64_t* scratch;     // device: scratch area after the planes
  uint64_t* part[2];    // device: E/M partial slots inside the scratch area
  size_t dev_bytes;
  uint64_t seed;
  uint32_t stream_id;
  int32_t init;
  double beta;
  uint32_t t4, t8;
  uint32_t l4, l8;      // LCG thresholds min(floor(exp(-beta dE) 2^31), 2^31)
  bool beta_set;
  uint32_t* lcg;        // device: per-thread LCG states [2][L][W] (caller's), or null
  uint64_t* pool;       // device: Boltzmann-pattern pool, 2^pool_m (r4, r8) pairs (caller's), or null
  int32_t pool_m;
  bool pool_linear;     // pool read linearly from one draw per 256-word group
  uint64_t sweep;       // counter of the next sweep
  hipStream_t stream;
  int device;
  ising::Tuning tune;
};

namespace ising {
ising::SweepArgs sweep_args(const ising_lattice* h, uint32_t t, int64_t* EM);
ising_status enqueue_sweeps(ising_lattice* h, int64_t n, int64_t* dev_EM);
bool tile_args(const ising_lattice* h, TileArgs* out);
}  // namespace ising
