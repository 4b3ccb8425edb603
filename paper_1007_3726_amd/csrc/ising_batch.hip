// Batched sweeps over many lattices (placeholder: sequential per handle).
#include "ising_runtime.hpp"

using namespace ising;

extern "C" ising_status ising_multi_sweep(ising_t* const* hs, int32_t count, int64_t n,
                                          int64_t* const* dev_EM) {
  clear_error();
  if (!hs || count < 0 || n < 0) return fail(ISING_EINVAL, "ising_multi_sweep: bad arguments");
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]) return fail(ISING_EINVAL, "ising_multi_sweep: NULL handle %d", i);
    if (!hs[i]->beta_set) return fail(ISING_EINVAL, "ising_multi_sweep: handle %d has no beta", i);
    if (hs[i]->sweep + (uint64_t)n > (1ull << 32))
      return fail(ISING_ERANGE, "ising_multi_sweep: counter overflow on handle %d", i);
  }
  for (int32_t i = 0; i < count; ++i) {
    ising_status st = enqueue_sweeps(hs[i], n, dev_EM ? dev_EM[i] : nullptr);
    if (st != ISING_OK) return st;
    hs[i]->sweep += (uint64_t)n;
  }
  return ISING_OK;
}
