// Launch-shape defaults per lattice size.
#include "ising_batch.hpp"
#include "ising_runtime.hpp"

namespace ising {

Tuning default_tuning(int64_t L) {
  (void)L;
  Tuning t;
  t.small_lds_bytes = 4096;  // L <= 128 runs in one LDS-resident workgroup
  t.max_blocks = 2048;
  return t;
}

PlanModel default_model() {
  PlanModel m;
  m.wg_per_cu = 8;          // 16.4 KB LDS and <= 64 VGPRs per lane allow 8 per CU
  m.tile_s_full = 13e-6;    // ~1000 VALU instructions per lane, 8 waves per SIMD
  m.tile_s_alone = 4.5e-6;  // one wave per SIMD: issue plus memory latency (measured)
  m.launch_gap_s = 5e-6;    // dependent launches replayed from a graph (measured)
  return m;
}

BatchOptions default_batch_options() {
  BatchOptions o;
  o.model = default_model();
  o.force_form = -1;
  o.graph_chunk = 32;
  return o;
}

}  // namespace ising
