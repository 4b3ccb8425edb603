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
  uint32_t perturb;     // test hook: nonzero seeds pauses before block barriers
};

// Tiled half-sweep (L % 8 == 0): a workgroup of four waves handles a tile
// of 4*R*RPW rows x TW words of one colour (the packed persistent kernel
// stages the neighbour rows of the other colour in LDS once per tile, and
// the tile shape is bounded by that staging area).
constexpr int kTileLdsMaxWords = 2048;
// Rows of at least this many words use the wide tile shape (64-word row
// segments).  A narrow tile stages whole rows of W + 2 words, and each such
// row must fit one 64-lane wave pass, so narrow tiles need W <= 62.
constexpr int kWideMinWords = 63;
constexpr int kMaxSweepBlocks = 2048;

struct TileArgs {
  uint64_t* planes;
  int64_t plane_words;
  Geom g;
  uint32_t k0, k1, sid4, t, t4, t8;
  int32_t TW;       // tile width in words: 64 when W >= kWideMinWords, else W
  int32_t R;        // rows per row group: 1 when W >= kWideMinWords, else floor(64 / W)
  int32_t RPW;      // row groups per wave in one tile
  int32_t segs;     // 64-word segments per row (1 when W < 64)
  int64_t tiles;    // ceil(L / (4 R RPW)) * segs
  int32_t hi_mode;  // 0: every Philox block index < 2^32; 1: high word uniform per row
  uint64_t* part;   // colour 1 with E/M: per-block (anti-aligned bonds, up spins)
  int64_t* prev_EM;           // colour 0: (E, M) slot of the previous sweep to finalise
  const uint64_t* prev_part;  // partials of the previous sweep
  int32_t prev_blocks;
  // per-thread LCG dynamics (plain tiles only): states [2][L][W], or null
  // for Philox; the chain runs on z = x + l4d with addend lc, the tests are
  // z < l4m and z + le < l8m (see ising_device.hpp)
  uint32_t* lcg;
  uint32_t l4d, lc, le, l4m, l8m;
  // flat lane mapping of the direct-load kernels (rows whose width W neither
  // divides 64 nor is a multiple of it): wave task k covers words
  // 64 k .. 64 k + 63 of the colour plane in row-major order, so every lane
  // has a word; tiles = ceil(plane_words / (256 RPW)).  Row of word i:
  // q = (i * wdiv_m) >> 32 with wdiv_m = floor(2^32 / W) + 1, minus one when
  // q W > i.
  int32_t flat;
  uint32_t wdiv_m;
  // Boltzmann-pattern-pool dynamics (plain tiles, flat mapping, RPW = 4):
  // 2^m patterns of (r4, r8) word pairs, or null; a word reads pattern
  // v >> pool_shift (pool_shift = 32 - m) of its own Philox draw, or, with
  // pool_linear, of its 256-word group's draw plus its offset in the group
  const uint64_t* pool;
  uint32_t pool_shift, pool_mask;
  int32_t pool_linear;
  // test hook of the LDS-staged tiles (packed persistent kernel): a nonzero
  // seed makes every wave pause a pseudo-random time before each block
  // barrier, so that a missing barrier shows up as a different result
  uint32_t perturb;
};

// Switch tile arguments of a lattice to the flat mapping (see
// TileArgs::flat) when its rows need it, or for any row width with
// `always`; keeps RPW.  Lattices of 2^32 or more words per plane keep the
// row-group mapping.
void make_flat(TileArgs& a, bool always = false);

hipError_t launch_tile_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks);
// Strip form (W >= kWideMinWords): TileArgs with TW = 64, R = 1, RPW = rows
// per wave task, tiles = number of wave tasks (segs x ceil(L / RPW)).
hipError_t launch_strip_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks);
hipError_t launch_finalize_em(hipStream_t st, const uint64_t* part, int blocks, int64_t L,
                              int64_t* EM);
// Thread seeds of the LCG dynamics: state[j] = s0 * 16807^j mod 2^32.
hipError_t launch_lcg_seed(hipStream_t st, uint32_t* state, int64_t n, uint32_t s0);
// Pattern pool: 2^m (r4, r8) pairs drawn for thresholds (t4, t8).
hipError_t launch_pool_fill(hipStream_t st, uint64_t* pool, int m, uint32_t k0, uint32_t k1,
                            uint32_t sid4, uint32_t t4, uint32_t t8);
// Colour step of the pool dynamics (TileArgs with flat = 1, RPW = 4, pool set).
hipError_t launch_pool_sweep(hipStream_t st, int colour, const TileArgs& a, int blocks);

// Batched sweeps (see ising_kernels.hip).
struct FusedLattice {
  TileArgs ta;          // tile shape; ta.t = sweep counter of the call's first sweep
  int64_t* EM;          // nsweeps x 2 per-sweep (E, M), or null
  int64_t first_tile;   // first entry of this lattice in the flat tile list
  int64_t ntiles;
  int64_t nsweeps;      // sweeps this lattice takes in the call (<= the call's n)
  int64_t rpw_cost;     // unused by the kernels (host bookkeeping)
};
struct FusedTile {
  int32_t lattice;
  int32_t local;        // tile index inside the lattice
};
struct FusedArgs {
  const FusedLattice* lat;
  int32_t nlat;
  int32_t klocal;       // sweep index inside a replayed chunk
  const FusedTile* tiles;
  int64_t ntiles;
  const uint32_t* kbase;  // device word: sweep index of the chunk's first sweep
  uint32_t* part;       // 2 slots x ntiles x (anti, up)
};

struct BatchLattice {
  TileArgs ta;          // tile shape, key, thresholds; ta.t is the first sweep counter
  int64_t* EM;          // nsweeps x 2 per-sweep (E, M), or null
  int64_t nsweeps;      // sweeps this lattice takes in the launch
};
struct BatchItem {
  int32_t lattice;
  int32_t rank;
};
struct BatchWG {
  int32_t first_item;
  int32_t n_items;
};
struct BatchArgs {
  const BatchLattice* lat;
  const BatchItem* items;
  const BatchWG* wgs;
  int64_t n;            // sweeps
};

hipError_t launch_fused(hipStream_t st, int colour, const FusedArgs& f, int blocks);
hipError_t launch_fused_finalize(hipStream_t st, const FusedArgs& f, int blocks);
hipError_t launch_advance(hipStream_t st, uint32_t* kbase, uint32_t by);
hipError_t launch_batch(hipStream_t st, const BatchArgs& a, int blocks);

// One GPU's share of a lattice split into row strips (the per-GPU part of
// a multi-GPU decomposition): global rows y0 .. y0 + rows - 1 of an L x L
// lattice (L % 128 == 0, so every word is full).  Each colour plane holds
// rows + 2 rows of W words: row 0 is the halo above (global row y0 - 1),
// rows 1 .. rows the strip, row rows + 1 the halo below (global row
// y0 + rows); the halos are written by the exchange, never by the kernels.
struct ShareArgs {
  uint64_t* planes;      // plane c at planes + c * plane_words
  int64_t plane_words;   // (rows + 2) * W
  int64_t rows, y0;      // strip rows, global row of the first one
  int32_t W;             // words per row (L / 128)
  uint32_t L8;           // L / 8: Philox blocks per colour row
  uint32_t wdiv_m;       // floor(2^32 / W) + 1 (flat word -> row), 0 for W == 1
  uint32_t k0, k1, sid4, t, t4, t8;
  uint64_t* part;        // colour 1 with counts: per-block (anti-aligned bonds, up spins)
};
hipError_t launch_share_init(hipStream_t st, const ShareArgs& a, int init);
hipError_t launch_share_sweep(hipStream_t st, int colour, const ShareArgs& a, int blocks);
// counts[0..1] = sums of part[0 .. 2 blocks) (anti-aligned bonds, up spins)
hipError_t launch_share_counts(hipStream_t st, const uint64_t* part, int blocks, int64_t* counts);
// EM[k] = (2 sum_s A[k][s] - 2 L^2, 2 sum_s P[k][s] - L^2) for k < n, from
// counts laid out [n][nstrips][2]
hipError_t launch_share_combine(hipStream_t st, const int64_t* counts, int32_t nstrips, int64_t n,
                                int64_t L, int64_t* EM);
hipError_t launch_init(hipStream_t st, uint64_t* planes, const Geom& g, uint32_t k0, uint32_t k1,
                       uint32_t sid4, int init, int blocks);
hipError_t launch_half_sweep(hipStream_t st, int colour, const SweepArgs& a, int blocks);
hipError_t launch_measure(hipStream_t st, const uint64_t* planes, const Geom& g,
                          int64_t plane_words, int64_t* EM, int blocks);
hipError_t launch_small_sweeps(hipStream_t st, const SmallArgs& a, int threads);

}  // namespace ising
