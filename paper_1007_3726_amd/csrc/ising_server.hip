// Served mode (continuous batching).  Not built yet: every entry point
// reports EINVAL.
#include "ising_runtime.hpp"

using namespace ising;

extern "C" {
ising_status ising_server_create(void*, size_t, void*, int32_t, ising_server_t** out) {
  if (out) *out = nullptr;
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_batch_submit(ising_server_t*, const ising_request*, int32_t, uint64_t*) {
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_server_step(ising_server_t*) {
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_poll(ising_server_t*, uint64_t, ising_result*) {
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_server_inject_fault(ising_server_t*, int64_t) {
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_server_stats(const ising_server_t*, int64_t*) {
  return fail(ISING_EINVAL, "served mode is not available in this build");
}
ising_status ising_server_destroy(ising_server_t*) { return ISING_OK; }
}
