// Batched sweeps: many lattices of uneven size and temperature.
//
// Two launch forms, chosen per call by the cost model of the autotuner
// (ising_tune.hip):
//   * fused: the tiles of all lattices form one flat list; each sweep is
//     two launches of k_fused (colour 0, colour 1) that walk the whole list,
//     so every colour step is balanced over the whole GPU.  Long runs are
//     replayed from a captured hipGraph chunk of K sweeps (a device-side
//     sweep counter advanced by the last node keeps the chunk reusable);
//   * packed: when every lattice is small, lattices are packed (longest
//     first) onto workgroups of one persistent launch (k_batch) that runs all
//     n sweeps with block barriers only.
// Lattices the tiled layout does not cover (L % 8 != 0, or Philox block
// indices crossing 2^32 inside a row) are advanced with the plain path.
// The task tables live in a library-owned device buffer per device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "ising_batch.hpp"
#include "ising_runtime.hpp"

namespace ising {

bool tile_args(const ising_lattice* h, TileArgs* out);

namespace {

struct DeviceTable {
  std::mutex m;
  void* ptr = nullptr;
  size_t cap = 0;
  int cus = 0;
  hipStream_t capture = nullptr;  // private stream for graph capture
};

DeviceTable& table_for(int device) {
  static DeviceTable tables[64];
  return tables[device & 63];
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

ising_status ensure_table(DeviceTable& T, size_t bytes) {
  if (T.cap >= bytes) return ISING_OK;
  if (T.ptr) (void)hipFree(T.ptr);
  T.ptr = nullptr;
  T.cap = 0;
  const size_t want = std::max<size_t>(bytes * 2, 1 << 20);
  hipError_t e = hipMalloc(&T.ptr, want);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table allocation");
  T.cap = want;
  return ISING_OK;
}

int cu_count(DeviceTable& T, int device) {
  if (T.cus == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) == hipSuccess) T.cus = p.multiProcessorCount;
  }
  return T.cus;
}

}  // namespace

// Pack single-workgroup lattices onto `bins` workgroups, longest first.
std::vector<std::vector<int>> pack_lpt(const std::vector<double>& cost, int bins) {
  std::vector<int> order(cost.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  bins = std::max(1, std::min<int>(bins, (int)cost.size()));
  std::vector<std::vector<int>> packs(bins);
  std::vector<double> load(bins, 0.0);
  for (int i : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[b] += cost[i];
    packs[b].push_back(i);
  }
  return packs;
}

BatchPlan plan_batch(const std::vector<int64_t>& tiles, int cus, const PlanModel& m) {
  BatchPlan p;
  const int count = (int)tiles.size();
  const int64_t total = std::accumulate(tiles.begin(), tiles.end(), (int64_t)0);
  // fused: two launches per sweep, each walking all tiles with the full grid
  p.fused_blocks = (int)std::min<int64_t>(std::max<int64_t>(total, 1), (int64_t)m.wg_per_cu * cus);
  const double rounds = std::ceil((double)total / p.fused_blocks);
  p.fused_s = 2.0 * (m.launch_gap_s + rounds * m.tile_s_full);
  // packed: one workgroup per bin, all sweeps in one launch
  const int bins = std::min<int>(count, m.wg_per_cu * cus);
  std::vector<double> cost(count);
  for (int i = 0; i < count; ++i) cost[i] = (double)tiles[i];
  p.packs = pack_lpt(cost, bins);
  double worst = 0.0;
  for (const auto& pk : p.packs) {
    double s = 0.0;
    for (int i : pk) s += cost[i];
    worst = std::max(worst, s);
  }
  const double per_cu = std::ceil((double)p.packs.size() / std::max(cus, 1));
  const double tile_s = std::max(m.tile_s_alone, m.tile_s_full * per_cu / m.wg_per_cu);
  p.packed_s = 2.0 * worst * tile_s;
  p.packed = p.packed_s < p.fused_s;
  return p;
}

static ising_status run_fused(ising_lattice* const* hs, const std::vector<int>& idx,
                              const std::vector<TileArgs>& targs, int64_t n, const int64_t* nsw,
                              int64_t* const* dev_EM, const BatchOptions& opt, DeviceTable& T,
                              int blocks) {
  hipStream_t stream = hs[idx[0]]->stream;
  const int nl = (int)idx.size();
  std::vector<FusedLattice> lat(nl);
  std::vector<FusedTile> tiles;
  bool any_em = false;
  // Every lattice keeps the tile shape of the plan (coarser tiles for the
  // largest lattices helped a batch made mostly of them, +1.9 % on the
  // 224-lattice grid, but unbalanced served mixes: p50 latency 1.7 -> 3.0 s).
  for (int j = 0; j < nl; ++j) {
    const int i = idx[j];
    FusedLattice& F = lat[j];
    std::memset(&F, 0, sizeof(F));
    F.ta = targs[i];
    make_flat(F.ta, true);  // the fused kernel uses the flat mapping for every lattice
    F.ta.t = (uint32_t)hs[i]->sweep;
    F.EM = dev_EM ? dev_EM[i] : nullptr;
    any_em = any_em || F.EM != nullptr;
    F.ntiles = F.ta.tiles;
    F.nsweeps = nsw ? nsw[i] : n;
  }
  // The grid deals the tile list out with a static stride.  Listing the
  // larger tiles first (two row groups per wave before one), and within a
  // size the lattices that run the most sweeps of this launch first, gives
  // every workgroup about the same work per round (longest first), and the
  // tiles of lattices that finish early in a chunk drop out of the end of
  // the list.  Results do not depend on the order.
  std::vector<int> order(nl);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (lat[a].ta.RPW != lat[b].ta.RPW) return lat[a].ta.RPW > lat[b].ta.RPW;
    return lat[a].nsweeps > lat[b].nsweeps;
  });
  for (int j : order) {
    lat[j].first_tile = (int64_t)tiles.size();
    for (int64_t t = 0; t < lat[j].ntiles; ++t) tiles.push_back(FusedTile{j, (int32_t)t});
  }
  const int64_t ntiles = (int64_t)tiles.size();
  blocks = (int)std::min<int64_t>(blocks, std::max<int64_t>(ntiles, 1));
  const size_t off_k = 0;
  const size_t off_lat = 256;
  const size_t off_tiles = align_up(off_lat + nl * sizeof(FusedLattice), 256);
  const size_t off_part = align_up(off_tiles + ntiles * sizeof(FusedTile), 256);
  // per-wave E/M partials: 2 sweep slots x 4 waves x (anti, up) per tile
  const size_t bytes = align_up(off_part + 2 * 4 * 2 * (size_t)ntiles * sizeof(uint32_t), 256);
  ising_status st = ensure_table(T, bytes);
  if (st != ISING_OK) return st;
  char* d = (char*)T.ptr;
  std::vector<char> img(off_part, 0);
  std::memcpy(img.data() + off_lat, lat.data(), nl * sizeof(FusedLattice));
  std::memcpy(img.data() + off_tiles, tiles.data(), ntiles * sizeof(FusedTile));
  hipError_t e = hipMemcpyAsync(d, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table upload");

  FusedArgs f;
  f.lat = (const FusedLattice*)(d + off_lat);
  f.nlat = nl;
  f.klocal = 0;
  f.tiles = (const FusedTile*)(d + off_tiles);
  f.ntiles = ntiles;
  f.kbase = (const uint32_t*)(d + off_k);
  f.part = (uint32_t*)(d + off_part);
  uint32_t* kbase = (uint32_t*)(d + off_k);

  int64_t done = 0;
  const int K = opt.graph_chunk;
  if (K > 0 && n >= 2 * (int64_t)K) {
    // capture K sweeps (+ the counter advance) once on a private stream,
    // then replay the chunk n / K times on the caller's stream
    if (!T.capture) {
      e = hipStreamCreateWithFlags(&T.capture, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "batched sweeps: capture stream");
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(T.capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int k = 0; k < K && e == hipSuccess; ++k) {
        f.klocal = k;
        e = launch_fused(T.capture, 0, f, blocks);
        if (e == hipSuccess) e = launch_fused(T.capture, 1, f, blocks);
      }
      if (e == hipSuccess) e = launch_advance(T.capture, kbase, (uint32_t)K);
      hipError_t e2 = hipStreamEndCapture(T.capture, &graph);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    const int64_t reps = n / K;
    for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, stream);
    // the executable graph may be destroyed once its launches are enqueued
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "batched sweeps: graph capture/replay");
    done = reps * K;
  }
  // remaining sweeps: direct launches at kbase + klocal
  for (int64_t k = 0; k < n - done; ++k) {
    f.klocal = (int32_t)k;
    e = launch_fused(stream, 0, f, blocks);
    if (e == hipSuccess) e = launch_fused(stream, 1, f, blocks);
    if (e != hipSuccess) return hip_fail(e, "batched sweeps: fused launch");
  }
  if (any_em) {
    f.klocal = (int32_t)(n - done) - 1;  // the last sweep: kbase + klocal = n - 1
    e = launch_fused_finalize(stream, f, std::min(nl, 1024));
    if (e != hipSuccess) return hip_fail(e, "batched sweeps: finalize launch");
  }
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: synchronize");
  return ISING_OK;
}

static ising_status run_packed(ising_lattice* const* hs, const std::vector<int>& idx,
                               const std::vector<TileArgs>& targs, int64_t n, const int64_t* nsw,
                               int64_t* const* dev_EM, const BatchPlan& plan, DeviceTable& T) {
  hipStream_t stream = hs[idx[0]]->stream;
  const int nl = (int)idx.size();
  std::vector<BatchLattice> lat(nl);
  for (int j = 0; j < nl; ++j) {
    const int i = idx[j];
    std::memset(&lat[j], 0, sizeof(BatchLattice));
    lat[j].ta = targs[i];
    lat[j].ta.t = (uint32_t)hs[i]->sweep;
    lat[j].ta.perturb = debug_perturb_seed();
    lat[j].EM = dev_EM ? dev_EM[i] : nullptr;
    lat[j].nsweeps = nsw ? nsw[i] : n;
  }
  std::vector<BatchWG> wgs(plan.packs.size());
  std::vector<BatchItem> items;
  for (size_t b = 0; b < plan.packs.size(); ++b) {
    wgs[b].first_item = (int32_t)items.size();
    wgs[b].n_items = (int32_t)plan.packs[b].size();
    for (int j : plan.packs[b]) items.push_back(BatchItem{j, 0});
  }
  const size_t off_lat = 0;
  const size_t off_items = align_up(nl * sizeof(BatchLattice), 256);
  const size_t off_wgs = align_up(off_items + items.size() * sizeof(BatchItem), 256);
  const size_t bytes = align_up(off_wgs + wgs.size() * sizeof(BatchWG), 256);
  ising_status st = ensure_table(T, bytes);
  if (st != ISING_OK) return st;
  std::vector<char> img(bytes, 0);
  std::memcpy(img.data() + off_lat, lat.data(), nl * sizeof(BatchLattice));
  std::memcpy(img.data() + off_items, items.data(), items.size() * sizeof(BatchItem));
  std::memcpy(img.data() + off_wgs, wgs.data(), wgs.size() * sizeof(BatchWG));
  char* d = (char*)T.ptr;
  hipError_t e = hipMemcpyAsync(d, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table upload");
  BatchArgs a;
  a.lat = (const BatchLattice*)(d + off_lat);
  a.items = (const BatchItem*)(d + off_items);
  a.wgs = (const BatchWG*)(d + off_wgs);
  a.n = n;
  e = launch_batch(stream, a, (int)wgs.size());
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: packed launch");
  return ISING_OK;
}

ising_status batch_sweeps(ising_lattice* const* hs, int32_t count, int64_t n,
                          const int64_t* nsw, int64_t* const* dev_EM, const BatchOptions& opt,
                          int* form_out) {
  if (form_out) *form_out = -1;
  if (count == 0 || n == 0) return ISING_OK;
  const int device = hs[0]->device;
  std::vector<int> tiled, other;
  std::vector<TileArgs> targs(count);
  for (int i = 0; i < count; ++i) {
    TileArgs ta;
    // the fused kernel indexes a plane with 32-bit word numbers: planes of
    // 2^32 words or more (L >= 741456) take the plain path
    if (tile_args(hs[i], &ta) && hs[i]->plane_words < (1ll << 32)) {
      // fine tiles balance best across the flat list; lattices with many
      // tiles take two row groups per wave (the packed kernel's LDS
      // staging bounds the shape)
      ta.RPW = 1;
      int64_t TR = 4 * (int64_t)ta.R;
      if (((hs[i]->L + TR - 1) / TR) * ta.segs >= 256 &&
          (2 * TR + 2) * (ta.TW + 2) <= kTileLdsMaxWords) {
        ta.RPW = 2;
        TR *= 2;
      }
      ta.tiles = ((hs[i]->L + TR - 1) / TR) * ta.segs;
      targs[i] = ta;
      tiled.push_back(i);
    } else {
      other.push_back(i);
    }
  }
  // one large lattice alone runs faster on the plain path (its own tuned
  // shape, no tile table): 4096^2 1345-1366 against 1140 updates/ns fused
  if (opt.force_form < 0 && tiled.size() == 1 && hs[tiled[0]]->plane_words >= (int64_t)1 << 16) {
    other.push_back(tiled[0]);
    tiled.clear();
  }
  for (int i : other) {
    // the plain path reads the handle's counter: advance a copy of it
    ising_lattice tmp = *hs[i];
    ising_status st = enqueue_sweeps(&tmp, nsw ? nsw[i] : n, dev_EM ? dev_EM[i] : nullptr);
    if (st != ISING_OK) return st;
  }
  if (tiled.empty()) {
    hipError_t e = hipStreamSynchronize(hs[0]->stream);
    return e == hipSuccess ? ISING_OK : hip_fail(e, "batched sweeps: synchronize");
  }
  DeviceTable& T = table_for(device);
  std::lock_guard<std::mutex> lock(T.m);
  const int cus = cu_count(T, device);
  if (cus <= 0) return fail(ISING_EDEVICE, "batched sweeps: no device properties");
  std::vector<int64_t> tiles;
  for (int i : tiled) tiles.push_back(tile_cost(targs[i].tiles, targs[i].RPW));
  const BatchPlan plan = plan_batch(tiles, cus, opt.model);
  bool packed = plan.packed;
  if (opt.force_form == 0) packed = false;
  if (opt.force_form == 1) packed = true;
  if (form_out) *form_out = packed ? 1 : 0;
  if (packed) return run_packed(hs, tiled, targs, n, nsw, dev_EM, plan, T);
  // the fused grid walks actual tiles; size it for them
  int64_t ntiles = 0;
  for (int i : tiled) ntiles += targs[i].tiles;
  const int blocks = (int)std::min<int64_t>(std::max<int64_t>(ntiles, 1), plan.fused_blocks);
  return run_fused(hs, tiled, targs, n, nsw, dev_EM, opt, T, blocks);
}

}  // namespace ising

using namespace ising;

extern "C" ising_status ising_batch_plan(const int64_t* Ls, int32_t count, int32_t cus,
                                         int32_t* form_out, int32_t* blocks_out,
                                         double* est_seconds_out) {
  clear_error();
  if (!Ls || count < 1 || cus < 1 || !form_out || !blocks_out)
    return fail(ISING_EINVAL, "ising_batch_plan: bad arguments");
  std::vector<int64_t> tiles(count);
  for (int32_t i = 0; i < count; ++i) {
    const int64_t L = Ls[i];
    if (L < 8 || L % 8 || L > kMaxL)
      return fail(ISING_EINVAL, "ising_batch_plan: L=%lld is not a tiled size", (long long)L);
    const int64_t W = words_per_row(L);
    const int64_t R = W >= kWideMinWords ? 1 : 64 / W;
    const int64_t segs = W >= kWideMinWords ? (W + 63) / 64 : 1;
    tiles[i] = ((L + 4 * R - 1) / (4 * R)) * segs;
  }
  const BatchPlan plan = plan_batch(tiles, cus, default_model());
  *form_out = plan.packed ? 1 : 0;
  *blocks_out = plan.packed ? (int32_t)plan.packs.size() : plan.fused_blocks;
  if (est_seconds_out) *est_seconds_out = plan.packed ? plan.packed_s : plan.fused_s;
  return ISING_OK;
}

static ising_status check_batch(ising_t* const* hs, int32_t count, int64_t n, const char* who) {
  if (!hs || count < 0 || n < 0) return fail(ISING_EINVAL, "%s: bad arguments", who);
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]) return fail(ISING_EINVAL, "%s: NULL handle %d", who, i);
    if (!hs[i]->beta_set) return fail(ISING_EINVAL, "%s: handle %d has no beta", who, i);
    if (hs[i]->lcg || hs[i]->pool)
      return fail(ISING_EINVAL,
                  "%s: handle %d uses the LCG or pattern-pool dynamics (plain sweeps only)", who,
                  i);
    if (hs[i]->sweep + (uint64_t)n > (1ull << 32))
      return fail(ISING_ERANGE, "%s: counter overflow on handle %d", who, i);
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device)
      return fail(ISING_EINVAL, "%s: handles must share one device and stream", who);
    for (int32_t j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(ISING_EINVAL, "%s: handle %d repeated", who, i);
  }
  return ISING_OK;
}

extern "C" ising_status ising_multi_sweep(ising_t* const* hs, int32_t count, int64_t n,
                                          int64_t* const* dev_EM) {
  return ising_multi_sweep_form(hs, count, n, dev_EM, -1, -1);
}

extern "C" ising_status ising_multi_sweep_form(ising_t* const* hs, int32_t count, int64_t n,
                                               int64_t* const* dev_EM, int32_t form,
                                               int32_t graph_chunk) {
  clear_error();
  ising_status st = check_batch(hs, count, n, "ising_multi_sweep");
  if (st != ISING_OK) return st;
  if (form < -1 || form > 1 || graph_chunk < -1)
    return fail(ISING_EINVAL, "ising_multi_sweep: bad form or graph chunk");
  BatchOptions opt = default_batch_options();
  opt.force_form = form;
  if (graph_chunk >= 0) opt.graph_chunk = graph_chunk;
  st = batch_sweeps(hs, count, n, nullptr, dev_EM, opt, nullptr);
  if (st != ISING_OK) return st;
  for (int32_t i = 0; i < count; ++i) hs[i]->sweep += (uint64_t)n;
  return ISING_OK;
}
