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

BatchOptions default_batch_options() {
  BatchOptions o;
  o.model = default_model();
  o.max_blocks = 0;
  o.cooperative = true;
  o.barrier_timeout_s = 2.0;
  return o;
}

}  // namespace ising
