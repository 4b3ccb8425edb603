// Batched-sweep planning (internal).
#pragma once

#include <stdint.h>

#include <vector>

#include "ising_runtime.hpp"

namespace ising {

// A lattice never gets more than this many workgroups in a batch.
constexpr int kMaxBatchLatticeBlocks = 2048;

struct PlanModel {
  double wg_rate;    // spins per second one workgroup updates
  double barrier_s;  // cost of one lattice barrier
};

struct BatchPlan {
  std::vector<int> nwg;                 // workgroups per lattice (1 = packed)
  std::vector<std::vector<int>> packs;  // single workgroups running several small lattices
  int blocks = 0;                       // grid size
  double est_seconds = 0.0;             // model estimate per sweep
};

struct BatchOptions {
  PlanModel model;
  int max_blocks;            // 0: occupancy-limited capacity of the device
  bool cooperative;          // cooperative launch (co-residency guaranteed)
  double barrier_timeout_s;  // a lattice barrier wait longer than this aborts the launch
};

PlanModel default_model();
BatchOptions default_batch_options();
int batch_capacity(int device);
BatchPlan plan_batch(const std::vector<int64_t>& work, const std::vector<int64_t>& max_wg,
                     int capacity, const PlanModel& model);
ising_status batch_sweeps(ising_lattice* const* hs, int32_t count, int64_t n,
                          int64_t* const* dev_EM, const BatchOptions& opt);

}  // namespace ising
