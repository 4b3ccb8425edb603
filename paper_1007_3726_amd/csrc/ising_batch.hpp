// Batched-sweep planning (internal).
#pragma once

#include <stdint.h>

#include <vector>

#include "ising_runtime.hpp"

namespace ising {

// Cost model of the batched launch forms (filled by the autotuner defaults).
struct PlanModel {
  int wg_per_cu;        // resident workgroups per CU for the tiled kernels
  double tile_s_full;   // seconds per tile per workgroup with every CU fully occupied
  double tile_s_alone;  // seconds per tile for a workgroup with its CU to itself
  double launch_gap_s;  // gap between dependent launches
};

// tile-steps (one word per lane) a lattice with these tile arguments costs per colour
inline int64_t tile_cost(int64_t tiles, int32_t rpw) { return tiles * (int64_t)rpw; }

struct BatchPlan {
  int fused_blocks = 0;                 // grid of the fused launches
  double fused_s = 0.0;                 // model: seconds per sweep, fused form
  std::vector<std::vector<int>> packs;  // packed form: lattices per workgroup
  double packed_s = 0.0;                // model: seconds per sweep, packed form
  bool packed = false;                  // the cheaper form
};

struct BatchOptions {
  PlanModel model;
  int force_form;   // -1: cost model, 0: fused, 1: packed
  int graph_chunk;  // sweeps per captured hipGraph chunk (0: no graph)
  // row groups per wave of a lattice's tiles: the largest r in {1, 2, 4},
  // r <= rpw_max, for which the lattice has at least 128 r tiles of one row
  // group per wave and the packed kernel's LDS staging still fits
  int rpw_max = 2;
  // when set (with graph_chunk 0): the table image is kept here, since it
  // must outlive its asynchronous upload, and the call returns without
  // waiting for the stream; the caller synchronises before it reuses the
  // image or the work buffer
  std::vector<char>* keep_image = nullptr;
};

PlanModel default_model();
// The built-in batched options, with the batched autotuner's installed
// fused shape (rpw_max, workgroups per CU, graph chunk) if there is one.
BatchOptions default_batch_options();
// Argument checks shared by the batched entry points (n: sweeps to come).
ising_status check_batch(ising_t* const* hs, int32_t count, int64_t n, const char* who);
BatchPlan plan_batch(const std::vector<int64_t>& tiles, int cus, const PlanModel& model);
// Device bytes of the work buffer batch_sweeps needs for these handles
// (0 when every lattice takes the plain path).
size_t batch_work_bytes(ising_lattice* const* hs, int32_t count, const BatchOptions& opt);
// An upper bound of one lattice's share of that buffer, whatever the form
// and the rest of the batch: batch_work_bytes of a set of lattices is at most
// kBatchWorkFixed plus the sum of their shares.
size_t batch_work_share(int64_t L);
constexpr size_t kBatchWorkFixed = 4 * 256;
// Advance hs[i] by nsw[i] sweeps (nsw may be null: n for all), n = max nsw,
// with the task tables in `work` (device, 256-byte aligned, work_bytes >=
// batch_work_bytes).  Does not change the handles' sweep counters.
ising_status batch_sweeps(ising_lattice* const* hs, int32_t count, int64_t n,
                          const int64_t* nsw, int64_t* const* dev_EM, const BatchOptions& opt,
                          void* work, size_t work_bytes, int* form_out);

}  // namespace ising
