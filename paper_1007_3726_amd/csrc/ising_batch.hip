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
// The task tables live in a work buffer the caller provides (device
// memory, batch_work_bytes of it); the library allocates no device memory.
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

// Per-device host state: the compute-unit count and a private stream for
// graph capture (the caller's stream may be the null stream, which cannot
// be captured).  The mutex serialises captures on that stream.
struct DeviceState {
  std::mutex m;
  int cus = 0;
  hipStream_t capture = nullptr;
};

DeviceState& state_for(int device) {
  static DeviceState states[64];
  return states[device & 63];
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int cu_count(DeviceState& D, int device) {
  std::lock_guard<std::mutex> lock(D.m);
  if (D.cus == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) == hipSuccess) D.cus = p.multiProcessorCount;
  }
  return D.cus;
}

// Byte offsets of the fused form's tables in the work buffer.
struct FusedLayout {
  size_t off_k = 0, off_lat = 256, off_tiles = 0, off_part = 0, bytes = 0;
};

FusedLayout fused_layout(size_t nl, size_t ntiles) {
  FusedLayout f;
  f.off_tiles = align_up(f.off_lat + nl * sizeof(FusedLattice), 256);
  f.off_part = align_up(f.off_tiles + ntiles * sizeof(FusedTile), 256);
  // per-wave E/M partials: 2 sweep slots x 4 waves x (anti, up) per tile
  f.bytes = align_up(f.off_part + 2 * 4 * 2 * ntiles * sizeof(uint32_t), 256);
  return f;
}

// Byte offsets of the packed form's tables (one item per lattice, at most
// one workgroup per lattice).
struct PackedLayout {
  size_t off_lat = 0, off_items = 0, off_wgs = 0, bytes = 0;
};

PackedLayout packed_layout(size_t nl, size_t nitems, size_t nwgs) {
  PackedLayout p;
  p.off_items = align_up(nl * sizeof(BatchLattice), 256);
  p.off_wgs = align_up(p.off_items + nitems * sizeof(BatchItem), 256);
  p.bytes = align_up(p.off_wgs + nwgs * sizeof(BatchWG), 256);
  return p;
}

// Tiles of the fused form's flat mapping for one lattice (RPW row groups per wave).
int64_t fused_tiles(int64_t plane_words, int32_t rpw) {
  const int64_t per_tile = 256 * (int64_t)rpw;
  return (plane_words + per_tile - 1) / per_tile;
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
                              int64_t* const* dev_EM, const BatchOptions& opt, char* work,
                              size_t work_bytes, int blocks) {
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
  const FusedLayout fl = fused_layout(nl, ntiles);
  if (fl.bytes > work_bytes)
    return fail(ISING_ENOMEM, "batched sweeps: work buffer of %zu bytes < %zu needed", work_bytes,
                fl.bytes);
  // the image covers the sweep counter (zero) and the tables; the partials
  // are written before they are read
  const bool async = opt.keep_image != nullptr && opt.graph_chunk == 0;
  std::vector<char> local;
  std::vector<char>& img = async ? *opt.keep_image : local;
  img.assign(fl.off_part, 0);
  std::memcpy(img.data() + fl.off_lat, lat.data(), nl * sizeof(FusedLattice));
  std::memcpy(img.data() + fl.off_tiles, tiles.data(), ntiles * sizeof(FusedTile));
  hipError_t e = hipMemcpyAsync(work, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table upload");
  // a local image ends with this call: wait for its upload
  if (!async) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table upload");

  FusedArgs f;
  f.lat = (const FusedLattice*)(work + fl.off_lat);
  f.nlat = nl;
  f.klocal = 0;
  f.tiles = (const FusedTile*)(work + fl.off_tiles);
  f.ntiles = ntiles;
  f.kbase = (const uint32_t*)(work + fl.off_k);
  f.part = (uint32_t*)(work + fl.off_part);
  uint32_t* kbase = (uint32_t*)(work + fl.off_k);

  int64_t done = 0;
  const int K = opt.graph_chunk;
  if (K > 0 && n >= 2 * (int64_t)K) {
    // capture K sweeps (+ the counter advance) once on a private stream,
    // then replay the chunk n / K times on the caller's stream
    DeviceState& D = state_for(hs[idx[0]]->device);
    std::lock_guard<std::mutex> lock(D.m);
    if (!D.capture) {
      e = hipStreamCreateWithFlags(&D.capture, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "batched sweeps: capture stream");
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(D.capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int k = 0; k < K && e == hipSuccess; ++k) {
        f.klocal = k;
        e = launch_fused(D.capture, 0, f, blocks);
        if (e == hipSuccess) e = launch_fused(D.capture, 1, f, blocks);
      }
      if (e == hipSuccess) e = launch_advance(D.capture, kbase, (uint32_t)K);
      hipError_t e2 = hipStreamEndCapture(D.capture, &graph);
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
  // remaining sweeps: direct launches at kbase + klocal; the device counter
  // moves on every 2^20 sweeps so that klocal stays small
  const int64_t kStep = int64_t(1) << 20;
  int64_t base = 0;
  for (int64_t k = 0; k < n - done; ++k) {
    if (k - base == kStep) {
      e = launch_advance(stream, kbase, (uint32_t)kStep);
      if (e != hipSuccess) return hip_fail(e, "batched sweeps: counter advance");
      base = k;
    }
    f.klocal = (int32_t)(k - base);
    e = launch_fused(stream, 0, f, blocks);
    if (e == hipSuccess) e = launch_fused(stream, 1, f, blocks);
    if (e != hipSuccess) return hip_fail(e, "batched sweeps: fused launch");
  }
  if (any_em) {
    // the last sweep: kbase + klocal = n - 1
    f.klocal = n - done > 0 ? (int32_t)(n - done - 1 - base) : -1;
    e = launch_fused_finalize(stream, f, std::min(nl, 1024));
    if (e != hipSuccess) return hip_fail(e, "batched sweeps: finalize launch");
  }
  if (async) return ISING_OK;
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: synchronize");
  return ISING_OK;
}

static ising_status run_packed(ising_lattice* const* hs, const std::vector<int>& idx,
                               const std::vector<TileArgs>& targs, int64_t n, const int64_t* nsw,
                               int64_t* const* dev_EM, const BatchPlan& plan, char* work,
                               size_t work_bytes, std::vector<char>* keep_image) {
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
  const PackedLayout pl = packed_layout(nl, items.size(), wgs.size());
  if (pl.bytes > work_bytes)
    return fail(ISING_ENOMEM, "batched sweeps: work buffer of %zu bytes < %zu needed", work_bytes,
                pl.bytes);
  std::vector<char> local;
  std::vector<char>& img = keep_image ? *keep_image : local;
  img.assign(pl.bytes, 0);
  std::memcpy(img.data() + pl.off_lat, lat.data(), nl * sizeof(BatchLattice));
  std::memcpy(img.data() + pl.off_items, items.data(), items.size() * sizeof(BatchItem));
  std::memcpy(img.data() + pl.off_wgs, wgs.data(), wgs.size() * sizeof(BatchWG));
  hipError_t e = hipMemcpyAsync(work, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: table upload");
  BatchArgs a;
  a.lat = (const BatchLattice*)(work + pl.off_lat);
  a.items = (const BatchItem*)(work + pl.off_items);
  a.wgs = (const BatchWG*)(work + pl.off_wgs);
  a.n = n;
  e = launch_batch(stream, a, (int)wgs.size());
  // the host image must outlive the upload: wait before it goes, unless the
  // caller keeps it
  if (e == hipSuccess && !keep_image) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "batched sweeps: packed launch");
  return ISING_OK;
}

// Which lattices take the tiled batched kernels (their tile arguments in
// targs) and which the plain path.
static void classify(ising_lattice* const* hs, int32_t count, const BatchOptions& opt,
                     std::vector<int>& tiled, std::vector<int>& other,
                     std::vector<TileArgs>& targs) {
  targs.assign(count, TileArgs{});
  for (int i = 0; i < count; ++i) {
    TileArgs ta;
    // the fused kernel indexes a plane with 32-bit word numbers: planes of
    // 2^32 words or more (L >= 741456) take the plain path
    if (tile_args(hs[i], &ta) && hs[i]->plane_words < (1ll << 32)) {
      // fine tiles balance best across the flat list; lattices with many
      // tiles take up to rpw_max row groups per wave (the packed kernel's
      // LDS staging bounds the shape)
      const int64_t TR1 = 4 * (int64_t)ta.R;
      const int64_t tiles1 = ((hs[i]->L + TR1 - 1) / TR1) * ta.segs;
      int rpw = 1;
      for (int r = 2; r <= opt.rpw_max; r *= 2) {
        if (tiles1 < 128 * (int64_t)r || (r * TR1 + 2) * (ta.TW + 2) > kTileLdsMaxWords) break;
        rpw = r;
      }
      ta.RPW = rpw;
      const int64_t TR = TR1 * rpw;
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
}

// Work-buffer bytes for the tiled lattices: the larger of the two forms.
static size_t work_bytes_for(ising_lattice* const* hs, const std::vector<int>& tiled,
                             const std::vector<TileArgs>& targs) {
  if (tiled.empty()) return 0;
  size_t ntiles = 0;
  for (int i : tiled) ntiles += (size_t)fused_tiles(hs[i]->plane_words, targs[i].RPW);
  const size_t nl = tiled.size();
  return std::max(fused_layout(nl, ntiles).bytes, packed_layout(nl, nl, nl).bytes);
}

size_t batch_work_bytes(ising_lattice* const* hs, int32_t count, const BatchOptions& opt) {
  std::vector<int> tiled, other;
  std::vector<TileArgs> targs;
  classify(hs, count, opt, tiled, other, targs);
  return work_bytes_for(hs, tiled, targs);
}

size_t batch_work_share(int64_t L) {
  const int64_t plane_words = L * words_per_row(L);
  const size_t fused = sizeof(FusedLattice) +
                       (size_t)fused_tiles(plane_words, 1) * (sizeof(FusedTile) + 64);
  const size_t packed = sizeof(BatchLattice) + sizeof(BatchItem) + sizeof(BatchWG);
  return std::max(fused, packed);
}

ising_status batch_sweeps(ising_lattice* const* hs, int32_t count, int64_t n,
                          const int64_t* nsw, int64_t* const* dev_EM, const BatchOptions& opt,
                          void* work, size_t work_bytes, int* form_out) {
  if (form_out) *form_out = -1;
  if (count == 0 || n == 0) return ISING_OK;
  const int device = hs[0]->device;
  std::vector<int> tiled, other;
  std::vector<TileArgs> targs;
  classify(hs, count, opt, tiled, other, targs);
  if (!tiled.empty()) {
    const size_t need = work_bytes_for(hs, tiled, targs);
    if (!work || need > work_bytes || ((uintptr_t)work & 255))
      return fail(ISING_ENOMEM,
                  "batched sweeps: needs a 256-byte aligned work buffer of %zu bytes (got %zu)",
                  need, work ? work_bytes : (size_t)0);
  }
  for (int i : other) {
    // the plain path reads the handle's counter: advance a copy of it
    ising_lattice tmp = *hs[i];
    ising_status st = enqueue_sweeps(&tmp, nsw ? nsw[i] : n, dev_EM ? dev_EM[i] : nullptr);
    if (st != ISING_OK) return st;
  }
  if (tiled.empty()) {
    if (opt.keep_image) return ISING_OK;
    hipError_t e = hipStreamSynchronize(hs[0]->stream);
    return e == hipSuccess ? ISING_OK : hip_fail(e, "batched sweeps: synchronize");
  }
  const int cus = cu_count(state_for(device), device);
  if (cus <= 0) return fail(ISING_EDEVICE, "batched sweeps: no device properties");
  std::vector<int64_t> tiles;
  for (int i : tiled) tiles.push_back(tile_cost(targs[i].tiles, targs[i].RPW));
  const BatchPlan plan = plan_batch(tiles, cus, opt.model);
  bool packed = plan.packed;
  if (opt.force_form == 0) packed = false;
  if (opt.force_form == 1) packed = true;
  if (form_out) *form_out = packed ? 1 : 0;
  if (packed)
    return run_packed(hs, tiled, targs, n, nsw, dev_EM, plan, (char*)work, work_bytes,
                      opt.keep_image);
  // the fused grid walks actual tiles; size it for them
  int64_t ntiles = 0;
  for (int i : tiled) ntiles += targs[i].tiles;
  const int blocks = (int)std::min<int64_t>(std::max<int64_t>(ntiles, 1), plan.fused_blocks);
  return run_fused(hs, tiled, targs, n, nsw, dev_EM, opt, (char*)work, work_bytes, blocks);
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

namespace ising {
ising_status check_batch(ising_t* const* hs, int32_t count, int64_t n, const char* who) {
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
}  // namespace ising

// ---------------------------------------------------------------------
// The allocation-free variant (ising_multi_sweep_static): the task tables
// live in this file-scope device array instead of a caller work buffer.
// Each GPU holds its own copy of the array for the life of the process; its
// device address is looked up once per device (hipGetSymbolAddress) and
// used from then on, never the array's host-side name.  Calls on one device
// are serialised by a per-device mutex (each call waits for its stream
// before it returns), so calls from several threads of a process do not
// overlap on the array.
// ---------------------------------------------------------------------
constexpr size_t kStaticWorkBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

namespace {
struct StaticScratch {
  std::mutex m;
  void* ptr = nullptr;  // device address of `scratch` on this device
};
StaticScratch& static_scratch(int device) {
  static StaticScratch s[64];
  return s[device & 63];
}
}  // namespace

extern "C" ising_status ising_multi_sweep_static(ising_t* const* hs, int32_t count, int64_t n,
                                                 int64_t* const* dev_EM) {
  clear_error();
  ising_status st = check_batch(hs, count, n, "ising_multi_sweep_static");
  if (st != ISING_OK) return st;
  if (count == 0 || n == 0) return ISING_OK;
  BatchOptions opt = default_batch_options();
  opt.graph_chunk = 0;  // no hipGraph: instantiating one allocates
  const size_t need = batch_work_bytes(hs, count, opt);
  if (need > kStaticWorkBytes)
    return fail(ISING_ENOMEM,
                "ising_multi_sweep_static: the batch needs %zu bytes of tables, more than the "
                "%zu-byte static scratch",
                need, kStaticWorkBytes);
  const int device = hs[0]->device;
  if (device < 0 || device >= 64) return fail(ISING_EINVAL, "ising_multi_sweep_static: device");
  StaticScratch& S = static_scratch(device);
  std::lock_guard<std::mutex> lock(S.m);
  if (!S.ptr) {
    int current = 0;
    hipError_t e = hipGetDevice(&current);
    if (e == hipSuccess && current != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (current != device) (void)hipSetDevice(current);
    if (e != hipSuccess || !p) return hip_fail(e, "ising_multi_sweep_static: scratch address");
    S.ptr = p;
  }
  st = batch_sweeps(hs, count, n, nullptr, dev_EM, opt, S.ptr, kStaticWorkBytes, nullptr);
  if (st != ISING_OK) return st;
  for (int32_t i = 0; i < count; ++i) hs[i]->sweep += (uint64_t)n;
  return ISING_OK;
}

extern "C" ising_status ising_multi_sweep_work_bytes(ising_t* const* hs, int32_t count,
                                                     size_t* bytes) {
  clear_error();
  if (!bytes) return fail(ISING_EINVAL, "ising_multi_sweep_work_bytes: bytes is NULL");
  *bytes = 0;
  ising_status st = check_batch(hs, count, 0, "ising_multi_sweep_work_bytes");
  if (st != ISING_OK) return st;
  // every form the caller may force and every fused shape the batched
  // autotuner may install: count each tiled lattice (a lone large lattice
  // takes the plain path only when the cost model chooses) with its finest
  // tiles
  BatchOptions opt = default_batch_options();
  opt.force_form = 0;
  opt.rpw_max = 1;
  *bytes = batch_work_bytes(hs, count, opt);
  return ISING_OK;
}

extern "C" ising_status ising_multi_sweep(ising_t* const* hs, int32_t count, int64_t n,
                                          int64_t* const* dev_EM, void* dev_work,
                                          size_t work_bytes) {
  return ising_multi_sweep_form(hs, count, n, dev_EM, -1, -1, dev_work, work_bytes);
}

extern "C" ising_status ising_multi_sweep_form(ising_t* const* hs, int32_t count, int64_t n,
                                               int64_t* const* dev_EM, int32_t form,
                                               int32_t graph_chunk, void* dev_work,
                                               size_t work_bytes) {
  clear_error();
  ising_status st = check_batch(hs, count, n, "ising_multi_sweep");
  if (st != ISING_OK) return st;
  if (form < -1 || form > 1 || graph_chunk < -1)
    return fail(ISING_EINVAL, "ising_multi_sweep: bad form or graph chunk");
  BatchOptions opt = default_batch_options();
  opt.force_form = form;
  if (graph_chunk >= 0) opt.graph_chunk = graph_chunk;
  st = batch_sweeps(hs, count, n, nullptr, dev_EM, opt, dev_work, work_bytes, nullptr);
  if (st != ISING_OK) return st;
  for (int32_t i = 0; i < count; ++i) hs[i]->sweep += (uint64_t)n;
  return ISING_OK;
}
