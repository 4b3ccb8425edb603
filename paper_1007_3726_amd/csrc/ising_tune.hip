// Launch shapes: defaults, the autotuner, and the installed tuning table.
//
// The autotuner times candidate shapes of the plain sweep (tiles with their
// row groups per wave, register-rolled strips with their rows per wave task,
// the grid cap, and for small lattices the single-workgroup LDS-resident
// kernel) on the current device for one lattice side, and
// installs the fastest for that side's size class (L in [2^k, 2^(k+1))).
// The table can be read and written so that callers keep a cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ising_batch.hpp"
#include "ising_runtime.hpp"

namespace ising {
namespace {

std::mutex g_tune_mutex;
std::vector<ising_tuning> g_table;

int64_t class_lo(int64_t L) {
  int64_t c = 1;
  while (c * 2 <= L) c *= 2;
  return c;
}

}  // namespace

Tuning default_tuning(int64_t L) {
  Tuning t;
  t.small_lds_bytes = 4096;  // L <= 128 runs in one LDS-resident workgroup
  t.max_blocks = 2048;
  t.rpw = 0;
  // tiles with direct neighbour loads: measured faster than strips at every
  // size from 1024^2 to 262144^2 (strips stay an autotuner candidate)
  t.form = ISING_FORM_TILE;
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  for (const ising_tuning& e : g_table)
    if (L >= e.L_min && L <= e.L_max) {
      t.form = e.form;
      t.rpw = e.rpw;
      t.max_blocks = e.max_blocks;
      t.small_lds_bytes = e.small_lds_bytes;
    }
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

static void install(const ising_tuning& e) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  for (ising_tuning& x : g_table)
    if (x.L_min == e.L_min && x.L_max == e.L_max) {
      x = e;
      return;
    }
  g_table.push_back(e);
}

}  // namespace ising

using namespace ising;

extern "C" {

ising_status ising_autotune(int64_t L, void* dev_buf, size_t dev_bytes, void* hip_stream,
                            int32_t trial_sweeps, ising_tuning* out) {
  clear_error();
  if (trial_sweeps < 1 || !out) return fail(ISING_EINVAL, "ising_autotune: bad arguments");
  ising_t* h = nullptr;
  ising_status st = ising_create(L, 12345, 0, ISING_INIT_HOT, dev_buf, dev_bytes, hip_stream, &h);
  if (st != ISING_OK) return st;
  // trials record their per-sweep (E, M) as a caller's run would, when the
  // buffer has room for the series after the lattice
  const size_t lat_bytes = (lattice_bytes(L) + 255) / 256 * 256;
  const int64_t em_sweeps = std::max<int64_t>(trial_sweeps, 2);
  int64_t* dev_EM = nullptr;
  if (dev_bytes >= lat_bytes + 16 * (size_t)em_sweeps)
    dev_EM = (int64_t*)((char*)dev_buf + lat_bytes);
  st = ising_set_beta(h, 1.0 / 2.269185);
  struct Cand {
    Tuning t;
  };
  std::vector<Cand> cands;
  const int64_t plane_bytes = 2 * h->plane_words * (int64_t)sizeof(uint64_t);
  if (plane_bytes <= 65536)  // LDS-resident
    cands.push_back({Tuning{plane_bytes, 2048, 0, ISING_FORM_TILE}});
  for (int rpw : {1, 2, 4})
    for (int mb : {512, 1024, 2048}) cands.push_back({Tuning{0, mb, rpw, ISING_FORM_TILE}});
  if (h->g.W >= kWideMinWords)
    for (int rows : {0, 4, 8, 16, 32})
      for (int mb : {1024, 2048}) cands.push_back({Tuning{0, mb, rows, ISING_FORM_STRIP}});
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  double best = -1.0;
  Tuning best_t = default_tuning(L);
  const hipStream_t stream = (hipStream_t)hip_stream;
  for (size_t i = 0; i < cands.size() && st == ISING_OK && e == hipSuccess; ++i) {
    h->tune = cands[i].t;
    TileArgs ta;
    // skip shapes the tiled layout would not honour
    if (h->tune.small_lds_bytes == 0 && h->tune.form == ISING_FORM_TILE && tile_args(h, &ta) &&
        ta.RPW != h->tune.rpw)
      continue;
    h->sweep = 0;
    st = enqueue_sweeps(h, 2, dev_EM);  // warm-up
    if (st != ISING_OK) break;
    e = hipEventRecord(a, stream);
    if (e == hipSuccess) st = enqueue_sweeps(h, trial_sweeps, dev_EM);
    if (e == hipSuccess && st == ISING_OK) e = hipEventRecord(b, stream);
    if (e == hipSuccess && st == ISING_OK) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess && st == ISING_OK) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess || st != ISING_OK) break;
    const double rate = (double)L * (double)L * trial_sweeps / (ms * 1e6);
    if (rate > best) {
      best = rate;
      best_t = cands[i].t;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  ising_destroy(h);
  if (st != ISING_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "ising_autotune: timing");
  ising_tuning r;
  r.L_min = class_lo(L);
  r.L_max = 2 * r.L_min - 1;
  r.form = best_t.form;
  r.rpw = best_t.rpw;
  r.max_blocks = best_t.max_blocks;
  r.reserved = 0;
  r.small_lds_bytes = best_t.small_lds_bytes;
  r.updates_per_ns = best;
  install(r);
  *out = r;
  return ISING_OK;
}

ising_status ising_tuning_set(const ising_tuning* entries, int32_t count) {
  clear_error();
  if (count < 0 || (count > 0 && !entries)) return fail(ISING_EINVAL, "ising_tuning_set: bad args");
  for (int32_t i = 0; i < count; ++i) {
    const ising_tuning& e = entries[i];
    const int32_t rpw_max = e.form == ISING_FORM_STRIP ? (1 << 21) : 16;
    if (e.L_min < 4 || e.L_max < e.L_min || (e.form != ISING_FORM_TILE &&
        e.form != ISING_FORM_STRIP) || e.rpw < 0 || e.rpw > rpw_max || e.max_blocks < 1 ||
        e.max_blocks > kMaxSweepBlocks || e.small_lds_bytes < 0 || e.small_lds_bytes > 65536)
      return fail(ISING_EINVAL, "ising_tuning_set: entry %d out of range", i);
  }
  for (int32_t i = 0; i < count; ++i) install(entries[i]);
  return ISING_OK;
}

ising_status ising_tuning_get(ising_tuning* entries, int32_t capacity, int32_t* count) {
  clear_error();
  if (!count || capacity < 0 || (capacity > 0 && !entries))
    return fail(ISING_EINVAL, "ising_tuning_get: bad args");
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  *count = (int32_t)g_table.size();
  for (int32_t i = 0; i < capacity && i < (int32_t)g_table.size(); ++i) entries[i] = g_table[i];
  return ISING_OK;
}

ising_status ising_tuning_lookup(int64_t L, ising_tuning* out) {
  clear_error();
  if (!out || L < 4) return fail(ISING_EINVAL, "ising_tuning_lookup: bad args");
  const Tuning t = default_tuning(L);
  ising_tuning r;
  r.L_min = L;
  r.L_max = L;
  r.updates_per_ns = 0.0;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const ising_tuning& e : g_table)
      if (L >= e.L_min && L <= e.L_max) r = e;
  }
  r.form = t.form;
  // the tile form's size rule (rpw 0) resolved to the value it uses
  r.rpw = (t.form == ISING_FORM_TILE && L % 8 == 0) ? tile_rpw(L, t.rpw) : t.rpw;
  r.max_blocks = t.max_blocks;
  r.reserved = 0;
  r.small_lds_bytes = t.small_lds_bytes;
  *out = r;
  return ISING_OK;
}

ising_status ising_tuning_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_table.clear();
  return ISING_OK;
}

}  // extern "C"
