// Batched sweeps: many lattices of uneven size and temperature advanced by
// one persistent fused kernel launch (k_batch).
//
// Host side:
//   * plan_batch (the autotuner's cost model) assigns workgroups to
//     lattices: a lattice whose work per sweep exceeds the per-workgroup
//     share gets k workgroups (tile shares rank, rank + k, ... and an atomic
//     barrier between colour steps); smaller lattices are packed, longest
//     first, onto single workgroups that run them one after the other;
//   * the workgroups of one lattice are placed on one XCD where possible
//     (block b runs on XCD b mod 8), so the lattice stays in one L2;
//   * the task tables are uploaded into a library-owned device buffer and
//     the kernel is launched cooperatively (all workgroups co-resident).
// Lattices the tiled layout does not cover (L % 8 != 0, or Philox block
// indices crossing 2^32 inside a row) are advanced with the plain path.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  int capacity_blocks = 0;  // co-resident k_batch workgroups
};

DeviceTable& table_for(int device) {
  static DeviceTable tables[64];
  return tables[device & 63];
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

int batch_capacity(int device) {
  DeviceTable& t = table_for(device);
  if (t.capacity_blocks == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return 0;
    const int per_cu = batch_max_blocks_per_cu();
    t.capacity_blocks = per_cu * p.multiProcessorCount;
  }
  return t.capacity_blocks;
}

// Cost model (seconds per sweep) used to compare plans: a workgroup
// updates about `wg_rate` spins per second; a multi-workgroup lattice pays
// two barriers per sweep.
BatchPlan plan_batch(const std::vector<int64_t>& work, const std::vector<int64_t>& max_wg,
                     int capacity, const PlanModel& model) {
  const int count = (int)work.size();
  const double total = std::accumulate(work.begin(), work.end(), 0.0);
  BatchPlan best;
  best.est_seconds = 1e300;
  if (count == 0 || capacity <= 0) return best;
  const double scales[] = {0.7, 0.85, 1.0, 1.2, 1.5, 2.0, 3.0};
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  for (double sc : scales) {
    const int target_wg = std::max(1, (int)(capacity / sc));
    const double share = total / target_wg;
    BatchPlan p;
    p.nwg.assign(count, 1);
    std::vector<int> small;
    int used = 0;
    for (int i : order) {
      int k = 1;
      if ((double)work[i] > 1.5 * share) {
        k = (int)std::llround((double)work[i] / share);
        k = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)k, max_wg[i], capacity}));
      }
      if (k > 1) {
        p.nwg[i] = k;
        used += k;
      } else {
        small.push_back(i);  // one workgroup: packed with the other small lattices
      }
    }
    int bins = capacity - used;
    if (bins < 1 && !small.empty()) continue;
    // pack small lattices onto single workgroups, longest first
    bins = std::min<int>(bins, (int)small.size());
    std::vector<double> load(bins, 0.0);
    p.packs.assign(bins, {});
    for (int i : small) {
      int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[b] += (double)work[i];
      p.packs[b].push_back(i);
    }
    double est = 0.0;
    for (int i = 0; i < count; ++i)
      if (p.nwg[i] > 1)
        est = std::max(est, (double)work[i] / p.nwg[i] / model.wg_rate + 2 * model.barrier_s);
    for (double l : load) est = std::max(est, l / model.wg_rate);
    p.blocks = used + bins;
    p.est_seconds = est;
    if (est < best.est_seconds) best = p;
  }
  return best;
}

// Block indices for the plan: the workgroups of a multi-workgroup lattice
// go to one XCD (block b -> XCD b mod 8) when they fit.  Returns, per block,
// the list of (lattice, rank) items.
static std::vector<std::vector<BatchItem>> place_blocks(const BatchPlan& p, int count) {
  const int G = p.blocks;
  const int nx = 8;
  std::vector<std::vector<int>> free_slots(nx);  // block indices per XCD
  for (int b = 0; b < G; ++b) free_slots[b % nx].push_back(b);
  for (auto& v : free_slots) std::reverse(v.begin(), v.end());
  std::vector<std::vector<BatchItem>> blocks(G);
  std::vector<int> big;
  for (int i = 0; i < count; ++i)
    if (p.nwg[i] > 1) big.push_back(i);
  std::sort(big.begin(), big.end(), [&](int a, int b) { return p.nwg[a] > p.nwg[b]; });
  for (int i : big) {
    int rank = 0;
    while (rank < p.nwg[i]) {
      int x = 0;
      for (int j = 1; j < nx; ++j)
        if (free_slots[j].size() > free_slots[x].size()) x = j;
      while (rank < p.nwg[i] && !free_slots[x].empty()) {
        const int b = free_slots[x].back();
        free_slots[x].pop_back();
        blocks[b].push_back(BatchItem{i, rank++});
      }
    }
  }
  int x = 0;
  for (const auto& pack : p.packs) {
    for (int j = 0; j < nx && free_slots[x].empty(); ++j) x = (x + 1) % nx;
    const int b = free_slots[x].back();
    free_slots[x].pop_back();
    for (int i : pack) blocks[b].push_back(BatchItem{i, 0});
    x = (x + 1) % nx;
  }
  return blocks;
}

PlanModel default_model() {
  PlanModel m;
  m.wg_rate = 1.1e9;     // spins per second per workgroup at 8 workgroups per CU
  m.barrier_s = 6e-6;    // one lattice barrier
  return m;
}

ising_status batch_sweeps(ising_lattice* const* hs, int32_t count, int64_t n,
                          int64_t* const* dev_EM, const BatchOptions& opt) {
  if (count == 0 || n == 0) return ISING_OK;
  hipStream_t stream = hs[0]->stream;
  const int device = hs[0]->device;
  // split off lattices the tiled layout does not cover
  std::vector<int> tiled, other;
  std::vector<TileArgs> targs(count);
  for (int i = 0; i < count; ++i) {
    TileArgs ta;
    if (tile_args(hs[i], &ta)) {
      ta.RPW = 1;  // finest tiles: most workgroups can share a lattice
      const int64_t TR = 4 * (int64_t)ta.R;
      ta.tiles = ((hs[i]->L + TR - 1) / TR) * ta.segs;
      targs[i] = ta;
      tiled.push_back(i);
    } else {
      other.push_back(i);
    }
  }
  for (int i : other) {
    ising_status st = enqueue_sweeps(hs[i], n, dev_EM ? dev_EM[i] : nullptr);
    if (st != ISING_OK) return st;
  }
  if (tiled.empty()) return ISING_OK;

  const int cap = opt.max_blocks > 0 ? std::min(opt.max_blocks, batch_capacity(device))
                                     : batch_capacity(device);
  if (cap <= 0) return fail(ISING_EDEVICE, "ising_multi_sweep: cannot size the persistent grid");
  std::vector<int64_t> work, max_wg;
  for (int i : tiled) {
    work.push_back(hs[i]->L * hs[i]->L);
    max_wg.push_back(std::min<int64_t>(targs[i].tiles, kMaxBatchLatticeBlocks));
  }
  const BatchPlan plan = plan_batch(work, max_wg, cap, opt.model);
  if (plan.blocks <= 0) return fail(ISING_EDEVICE, "ising_multi_sweep: no feasible plan");
  const auto blocks = place_blocks(plan, (int)tiled.size());

  // host image of the device tables
  const int nl = (int)tiled.size();
  size_t n_items = 0;
  for (const auto& b : blocks) n_items += b.size();
  size_t n_part = 0;
  for (int j = 0; j < nl; ++j) n_part += (plan.nwg[j] > 1) ? 2 * (size_t)plan.nwg[j] : 0;
  const size_t off_err = 0;
  const size_t off_lat = 256;
  const size_t off_items = align_up(off_lat + nl * sizeof(BatchLattice), 256);
  const size_t off_wgs = align_up(off_items + n_items * sizeof(BatchItem), 256);
  const size_t off_bar = align_up(off_wgs + blocks.size() * sizeof(BatchWG), 256);
  const size_t off_part = align_up(off_bar + nl * sizeof(uint32_t), 256);
  const size_t bytes = align_up(off_part + n_part * sizeof(uint64_t), 256);

  DeviceTable& T = table_for(device);
  std::lock_guard<std::mutex> lock(T.m);
  if (T.cap < bytes) {
    if (T.ptr) hipFree(T.ptr);
    T.ptr = nullptr;
    T.cap = 0;
    hipError_t e = hipMalloc(&T.ptr, bytes * 2);
    if (e != hipSuccess) return hip_fail(e, "ising_multi_sweep: table allocation");
    T.cap = bytes * 2;
  }
  char* dbase = (char*)T.ptr;
  std::vector<char> img(off_part, 0);  // partials need no initial value
  std::vector<BatchLattice> lat(nl);
  size_t part_at = 0;
  for (int j = 0; j < nl; ++j) {
    const int i = tiled[j];
    BatchLattice& B = lat[j];
    std::memset(&B, 0, sizeof(B));
    B.ta = targs[i];
    B.ta.t = (uint32_t)hs[i]->sweep;
    B.EM = dev_EM ? dev_EM[i] : nullptr;
    B.nwg = plan.nwg[j];
    B.bar = (uint32_t*)(dbase + off_bar) + j;
    if (B.nwg > 1) {
      B.part = (uint64_t*)(dbase + off_part) + part_at;
      part_at += 2 * (size_t)B.nwg;
    }
    B.full = hs[i]->g.nb_last == 64;
    B.wide = hs[i]->g.W >= 64;
  }
  std::memcpy(img.data() + off_lat, lat.data(), nl * sizeof(BatchLattice));
  std::vector<BatchWG> wgs(blocks.size());
  {
    size_t at = 0;
    BatchItem* items = (BatchItem*)(img.data() + off_items);
    for (size_t b = 0; b < blocks.size(); ++b) {
      wgs[b].first_item = (int32_t)at;
      wgs[b].n_items = (int32_t)blocks[b].size();
      for (const BatchItem& it : blocks[b]) items[at++] = it;
    }
  }
  std::memcpy(img.data() + off_wgs, wgs.data(), wgs.size() * sizeof(BatchWG));
  hipError_t e = hipMemcpyAsync(T.ptr, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "ising_multi_sweep: table upload");

  BatchArgs a;
  a.lat = (const BatchLattice*)(dbase + off_lat);
  a.items = (const BatchItem*)(dbase + off_items);
  a.wgs = (const BatchWG*)(dbase + off_wgs);
  a.n = n;
  a.err = (uint32_t*)(dbase + off_err);
  a.spin_limit = (uint64_t)(opt.barrier_timeout_s * 1e8);
  e = launch_batch(stream, a, (int)blocks.size(), opt.cooperative);
  if (e != hipSuccess) return hip_fail(e, "ising_multi_sweep: persistent kernel launch");
  uint32_t err = 0;
  e = hipMemcpyAsync(&err, a.err, sizeof(err), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "ising_multi_sweep: synchronize");
  if (err)
    return fail(ISING_EDEVICE,
                "ising_multi_sweep: a lattice barrier timed out (workgroups not co-resident)");
  return ISING_OK;
}

}  // namespace ising

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
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device)
      return fail(ISING_EINVAL, "ising_multi_sweep: handles must share one device and stream");
    for (int32_t j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(ISING_EINVAL, "ising_multi_sweep: handle %d repeated", i);
  }
  BatchOptions opt = default_batch_options();
  ising_status st = batch_sweeps(hs, count, n, dev_EM, opt);
  if (st != ISING_OK) return st;
  for (int32_t i = 0; i < count; ++i) hs[i]->sweep += (uint64_t)n;
  return ISING_OK;
}
