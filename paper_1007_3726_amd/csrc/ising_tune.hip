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
#include <chrono>
#include <mutex>
#include <vector>

#include "ising_batch.hpp"
#include "ising_runtime.hpp"

namespace ising {
namespace {

std::mutex g_tune_mutex;
std::vector<ising_tuning> g_table;
// the batched autotuner's installed fused shape
bool g_batch_set = false;
ising_batch_tuning g_batch;

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
  o.rpw_max = 2;
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  if (g_batch_set) {
    o.rpw_max = g_batch.rpw_max;
    o.model.wg_per_cu = g_batch.wg_per_cu;
    o.graph_chunk = g_batch.graph_chunk;
  }
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

// ---------------------------------------------------------------------
// Batched autotuner
// ---------------------------------------------------------------------
namespace ising {
namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bool valid_batch_shape(const ising_batch_tuning& t) {
  return (t.rpw_max == 1 || t.rpw_max == 2 || t.rpw_max == 4) && t.wg_per_cu >= 1 &&
         t.wg_per_cu <= 8 && t.graph_chunk >= 0 && t.graph_chunk <= 4096;
}

// Layout of the autotuner's buffer: lattice copies, then their (E, M)
// series of 2 m sweeps, then the work buffer.
struct TuneLayout {
  std::vector<size_t> lat, em;
  size_t work = 0, work_bytes = 0, bytes = 0;
};

TuneLayout tune_layout(ising_t* const* hs, int32_t count, int64_t m) {
  TuneLayout t;
  size_t off = 0;
  for (int32_t i = 0; i < count; ++i) {
    t.lat.push_back(off);
    off += align256(lattice_bytes(hs[i]->L));
  }
  for (int32_t i = 0; i < count; ++i) {
    t.em.push_back(off);
    off += align256((size_t)(2 * m) * 2 * sizeof(int64_t));
  }
  BatchOptions opt = default_batch_options();
  opt.force_form = 0;
  opt.rpw_max = 1;  // the finest tiles need the most table space
  t.work = off;
  t.work_bytes = batch_work_bytes(hs, count, opt);
  t.bytes = off + align256(t.work_bytes);
  return t;
}

}  // namespace
}  // namespace ising

extern "C" {

ising_status ising_multi_autotune_bytes(ising_t* const* hs, int32_t count, int32_t trial_sweeps,
                                        size_t* bytes) {
  clear_error();
  if (!bytes || trial_sweeps < 1) return fail(ISING_EINVAL, "ising_multi_autotune_bytes: bad args");
  *bytes = 0;
  ising_status st = check_batch(hs, count, 0, "ising_multi_autotune_bytes");
  if (st != ISING_OK) return st;
  *bytes = tune_layout(hs, count, trial_sweeps).bytes;
  return ISING_OK;
}

ising_status ising_multi_autotune(ising_t* const* hs, int32_t count, int32_t trial_sweeps,
                                  void* dev_buf, size_t dev_bytes, ising_batch_tuning* out) {
  clear_error();
  if (!out || trial_sweeps < 1 || count < 1)
    return fail(ISING_EINVAL, "ising_multi_autotune: bad arguments");
  ising_status st = check_batch(hs, count, 0, "ising_multi_autotune");
  if (st != ISING_OK) return st;
  const int64_t m = trial_sweeps;
  const TuneLayout lay = tune_layout(hs, count, m);
  if (!dev_buf || ((uintptr_t)dev_buf & 255) || dev_bytes < lay.bytes)
    return fail(ISING_ENOMEM,
                "ising_multi_autotune: needs a 256-byte aligned buffer of %zu bytes (got %zu)",
                lay.bytes, dev_buf ? dev_bytes : (size_t)0);
  char* base = (char*)dev_buf;
  const hipStream_t stream = hs[0]->stream;
  // copies of the lattices, each at the start of its own sweep counter
  std::vector<ising_t*> tmp(count, nullptr);
  std::vector<int64_t*> ems(count);
  for (int32_t i = 0; i < count && st == ISING_OK; ++i) {
    const ising_lattice* h = hs[i];
    st = ising_create(h->L, h->seed, h->stream_id, h->init, base + lay.lat[i],
                      align256(lattice_bytes(h->L)), stream, &tmp[i]);
    if (st == ISING_OK) st = ising_set_beta(tmp[i], h->beta);
    ems[i] = (int64_t*)(base + lay.em[i]);
  }
  void* work = base + lay.work;
  int64_t updates = 0;  // spin updates of one sweep of the batch
  for (int32_t i = 0; i < count; ++i) updates += hs[i]->L * hs[i]->L;

  // seconds of a synchronous batched call of n sweeps
  auto run = [&](const BatchOptions& opt, int64_t n, double* sec) -> ising_status {
    const auto t0 = std::chrono::steady_clock::now();
    ising_status s2 = batch_sweeps(tmp.data(), count, n, nullptr, ems.data(), opt, work,
                                   lay.work_bytes, nullptr);
    if (s2 != ISING_OK) return s2;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "ising_multi_autotune: synchronize");
    *sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (ising_t* h : tmp) h->sweep += (uint64_t)n;
    return ISING_OK;
  };
  // updates/ns of one candidate: m sweeps over t(2 m) - t(m)
  auto rate = [&](const BatchOptions& opt, double* r) -> ising_status {
    double t1 = 0.0, t2 = 0.0;
    ising_status s2 = run(opt, m, &t1);
    if (s2 == ISING_OK) s2 = run(opt, 2 * m, &t2);
    if (s2 != ISING_OK) return s2;
    const double dt = t2 > t1 ? t2 - t1 : t2 / 2.0;
    *r = (double)updates * (double)m / (dt * 1e9);
    return ISING_OK;
  };
  auto shape = [](int rpw_max, int wg, int chunk) {
    BatchOptions o = default_batch_options();
    o.force_form = 0;
    o.rpw_max = rpw_max;
    o.model = default_model();
    o.model.wg_per_cu = wg;
    o.graph_chunk = chunk;
    return o;
  };

  ising_batch_tuning best;
  best.form = 0;
  best.rpw_max = 2;
  best.wg_per_cu = 8;
  best.graph_chunk = 32;
  best.updates_per_ns = -1.0;
  best.default_updates_per_ns = 0.0;
  best.packed_updates_per_ns = 0.0;
  if (st == ISING_OK) {  // warm-up: first launches of the kernels
    double t = 0.0;
    st = run(shape(2, 8, 32), m, &t);
  }
  for (int rpw : {1, 2, 4})
    for (int wg : {8, 6, 4}) {
      if (st != ISING_OK) break;
      double r = 0.0;
      st = rate(shape(rpw, wg, 32), &r);
      if (st != ISING_OK) break;
      if (rpw == 2 && wg == 8) best.default_updates_per_ns = r;
      if (r > best.updates_per_ns) {
        best.rpw_max = rpw;
        best.wg_per_cu = wg;
        best.updates_per_ns = r;
      }
    }
  for (int chunk : {8, 16, 64}) {
    if (st != ISING_OK) break;
    double r = 0.0;
    st = rate(shape(best.rpw_max, best.wg_per_cu, chunk), &r);
    if (st != ISING_OK) break;
    if (r > best.updates_per_ns) {
      best.graph_chunk = chunk;
      best.updates_per_ns = r;
    }
  }
  if (st == ISING_OK) {
    // the packed form, unless the cost model puts it far behind (one
    // workgroup per lattice: a large lattice alone would take seconds)
    std::vector<int64_t> tiles;
    BatchOptions o = shape(best.rpw_max, best.wg_per_cu, best.graph_chunk);
    for (int32_t i = 0; i < count; ++i) {
      TileArgs ta;
      if (tile_args(hs[i], &ta)) tiles.push_back(tile_cost(ta.tiles, ta.RPW));
    }
    int dev_cus = 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hs[0]->device) == hipSuccess)
      dev_cus = prop.multiProcessorCount;
    if (!tiles.empty() && dev_cus > 0) {
      const BatchPlan plan = plan_batch(tiles, dev_cus, o.model);
      if (plan.packed_s <= 4.0 * plan.fused_s) {
        o.force_form = 1;
        double r = 0.0;
        st = rate(o, &r);
        if (st == ISING_OK) {
          best.packed_updates_per_ns = r;
          if (r > best.updates_per_ns) best.form = 1;
        }
      }
    }
  }
  for (ising_t* h : tmp)
    if (h) ising_destroy(h);
  if (st != ISING_OK) return st;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_batch = best;
    g_batch_set = true;
  }
  *out = best;
  return ISING_OK;
}

ising_status ising_batch_tuning_set(const ising_batch_tuning* t) {
  clear_error();
  if (!t || !valid_batch_shape(*t)) return fail(ISING_EINVAL, "ising_batch_tuning_set: bad shape");
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_batch = *t;
  g_batch_set = true;
  return ISING_OK;
}

ising_status ising_batch_tuning_get(ising_batch_tuning* out, int32_t* installed) {
  clear_error();
  if (!out || !installed) return fail(ISING_EINVAL, "ising_batch_tuning_get: bad args");
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  *installed = g_batch_set ? 1 : 0;
  if (g_batch_set) {
    *out = g_batch;
  } else {
    out->form = 0;
    out->rpw_max = 2;
    out->wg_per_cu = 8;
    out->graph_chunk = 32;
    out->updates_per_ns = 0.0;
    out->default_updates_per_ns = 0.0;
    out->packed_updates_per_ns = 0.0;
  }
  return ISING_OK;
}

ising_status ising_batch_tuning_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_batch_set = false;
  return ISING_OK;
}

}  // extern "C"
