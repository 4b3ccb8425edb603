// Host runtime of the C ABI declared in include/ising.h: handle lifecycle,
// argument validation, Metropolis thresholds, launch selection, and the
// conversion between the packed device layout and int8 host spins.
#include <atomic>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ising.h"
#include "ising_kernels.hpp"
#include "ising_runtime.hpp"

namespace ising {

static thread_local std::string g_last_error;

ising_status fail(ising_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

ising_status hip_fail(hipError_t e, const char* what) {
  return fail(ISING_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

int64_t words_per_row(int64_t L) { return ((L / 2) + 63) / 64; }

size_t plane_bytes(int64_t L) { return (size_t)L * (size_t)words_per_row(L) * sizeof(uint64_t); }

size_t lattice_bytes(int64_t L) {
  if (L < 4 || L > kMaxL || (L & 1)) return 0;
  size_t b = 2 * plane_bytes(L);
  b = (b + 255) & ~(size_t)255;
  return b + kScratchBytes;
}

Geom make_geom(int64_t L) {
  Geom g;
  g.L = L;
  g.W = (int32_t)words_per_row(L);
  g.half = L / 2;
  g.nb_last = (int32_t)(g.half - 64 * (int64_t)(g.W - 1));
  g.L8 = L / 8;
  return g;
}

// Section 3: the Boltzmann factor of an uphill move dE, precomputed on the
// host once per temperature; section 4, Eq. (3): accept iff r < factor.
// With r = u / 2^32 for a 32-bit uniform u this is u < floor(factor 2^32),
// clamped to 2^32 - 1 (beta = 0 then accepts with probability 1 - 2^-32).
uint32_t metropolis_threshold(double beta, int dE) {
  const double factor = std::exp(-beta * (double)dE);
  const double scaled = std::floor(std::ldexp(factor, 32));
  if (scaled >= 4294967295.0) return 0xFFFFFFFFu;
  if (scaled <= 0.0) return 0u;
  return (uint32_t)scaled;
}

// Threshold of the per-thread LCG dynamics (uniform |int32(x)| / 2^31):
// floor(exp(-beta dE) 2^31), clamped to 2^31.
uint32_t lcg_threshold(double beta, int dE) {
  const double factor = std::exp(-beta * (double)dE);
  const double scaled = std::floor(std::ldexp(factor, 31));
  if (scaled >= 2147483648.0) return 0x80000000u;
  if (scaled <= 0.0) return 0u;
  return (uint32_t)scaled;
}

int grid_blocks(int64_t work_items, int threads, int max_blocks) {
  int64_t b = (work_items + threads - 1) / threads;
  if (b > max_blocks) b = max_blocks;
  if (b < 1) b = 1;
  return (int)b;
}

SweepArgs sweep_args(const ising_lattice* h, uint32_t t, int64_t* EM) {
  SweepArgs a;
  a.planes = h->planes;
  a.plane_words = h->plane_words;
  a.g = h->g;
  a.k0 = (uint32_t)h->seed;
  a.k1 = (uint32_t)(h->seed >> 32);
  a.sid4 = h->stream_id << 2;
  a.t = t;
  a.t4 = h->t4;
  a.t8 = h->t8;
  a.EM = EM;
  return a;
}

bool strip_form(const ising_lattice* h) {
  return h->tune.form == 1 && h->g.W >= kWideMinWords && h->lcg == nullptr && h->pool == nullptr;
}

// Shape of the tiled half-sweep for this lattice; false when it does not
// apply (L % 8 != 0, or Philox block indices that cross 2^32 inside a row).
// Row groups per wave of the tile form for side L: the tuned value `want`
// if it fits in LDS, else as many as keep >= 2048 tiles (8 per CU) and fit.
int tile_rpw(int64_t L, int want) {
  const int64_t W = words_per_row(L);
  const bool wide = W >= kWideMinWords;
  const int64_t TW = wide ? 64 : W, R = wide ? 1 : 64 / W, segs = wide ? (W + 63) / 64 : 1;
  if (want > 0 && (4 * R * want + 2) * (TW + 2) <= kTileLdsMaxWords) return want;
  for (int rpw = 4; rpw > 1; rpw >>= 1) {
    const int64_t TR = 4 * R * rpw;
    const int64_t tiles = ((L + TR - 1) / TR) * segs;
    if (tiles >= 2048 && (TR + 2) * (TW + 2) <= kTileLdsMaxWords) return rpw;
  }
  return 1;
}

bool tile_args(const ising_lattice* h, TileArgs* out) {
  const int64_t L = h->L, W = h->g.W;
  if (L % 8 != 0) return false;
  TileArgs a;
  std::memset(&a, 0, sizeof(a));
  const bool wide = W >= kWideMinWords;
  a.TW = wide ? 64 : (int32_t)W;
  a.R = wide ? 1 : (int32_t)(64 / W);
  a.segs = wide ? (int32_t)((W + 63) / 64) : 1;
  a.RPW = tile_rpw(L, h->tune.rpw);
  const int64_t TR = 4 * (int64_t)a.R * a.RPW;
  a.tiles = ((L + TR - 1) / TR) * a.segs;
  if ((TR + 2) * (a.TW + 2) > kTileLdsMaxWords) return false;
  // a narrow staged row (W + 2 words) must fit one 64-lane wave pass
  if (!wide && a.TW + 2 > 64) return false;
  const bool pow2 = (L & (L - 1)) == 0;
  if ((uint64_t)L * (uint64_t)L / 8 <= (1ull << 32))
    a.hi_mode = 0;
  else if (wide && pow2)
    a.hi_mode = 1;
  else
    return false;
  a.planes = h->planes;
  a.plane_words = h->plane_words;
  a.g = h->g;
  a.k0 = (uint32_t)h->seed;
  a.k1 = (uint32_t)(h->seed >> 32);
  a.sid4 = h->stream_id << 2;
  a.t4 = h->t4;
  a.t8 = h->t8;
  *out = a;
  return true;
}

// Strip form of the same lattice (wide rows only): RPW = rows per wave
// task, tiles = number of wave tasks.
bool strip_args(const ising_lattice* h, TileArgs* out) {
  TileArgs a;
  if (!strip_form(h) || !tile_args(h, &a) || a.TW != 64) return false;
  const int64_t L = h->L;
  // rows per wave task: the tuned value, else about one task per resident
  // wave (8 waves on each of 1024 SIMDs)
  int64_t rows = h->tune.rpw > 0 ? h->tune.rpw : (L * a.segs + 8191) / 8192;
  if (rows < 1) rows = 1;
  if (rows > L) rows = L;
  a.R = 1;
  a.RPW = (int32_t)rows;
  a.tiles = ((L + rows - 1) / rows) * a.segs;
  *out = a;
  return true;
}

bool use_small_path(const ising_lattice* h) {
  return h->lcg == nullptr && h->pool == nullptr &&
         2 * h->plane_words * (int64_t)sizeof(uint64_t) <= h->tune.small_lds_bytes;
}

// (d, m) of the LCG decision (x + d) < m for threshold t' (ising_device.hpp)
static void lcg_decision(uint32_t t, uint32_t* d, uint32_t* m) {
  *d = t ? t - 1u : 0u;
  *m = t ? (uint32_t)(2ull * t - 1ull) : 0u;
}

// Tile arguments of the pool dynamics: flat mapping with 4 words per lane.
static bool pool_tile_args(const ising_lattice* h, TileArgs* out) {
  TileArgs ta;
  if (!tile_args(h, &ta) || h->plane_words >= (1ll << 32)) return false;
  ta.RPW = 4;
  make_flat(ta, true);
  *out = ta;
  return true;
}

static ising_status enqueue_pool_sweeps(ising_lattice* h, int64_t n, int64_t* dev_EM) {
  TileArgs ta;
  if (!pool_tile_args(h, &ta))
    return fail(ISING_EINVAL, "pattern-pool dynamics need L %% 8 == 0 and < 2^32 words per plane");
  ta.pool = h->pool;
  ta.pool_shift = (uint32_t)(32 - h->pool_m);
  ta.pool_mask = (uint32_t)((1ull << h->pool_m) - 1);
  ta.pool_linear = h->pool_linear ? 1 : 0;
  const int blocks = (int)std::min<int64_t>(ta.tiles, kMaxSweepBlocks);
  for (int64_t k = 0; k < n; ++k) {
    ta.t = (uint32_t)(h->sweep + (uint64_t)k);
    ta.prev_EM = (dev_EM && k > 0) ? dev_EM + 2 * (k - 1) : nullptr;
    ta.prev_part = h->part[(k + 1) & 1];
    ta.prev_blocks = blocks;
    ta.part = nullptr;
    hipError_t e = launch_pool_sweep(h->stream, 0, ta, blocks);
    if (e != hipSuccess) return hip_fail(e, "colour-0 pool half-sweep launch");
    ta.prev_EM = nullptr;
    ta.part = dev_EM ? h->part[k & 1] : nullptr;
    e = launch_pool_sweep(h->stream, 1, ta, blocks);
    if (e != hipSuccess) return hip_fail(e, "colour-1 pool half-sweep launch");
  }
  if (dev_EM) {
    hipError_t e = launch_finalize_em(h->stream, h->part[(n - 1) & 1], blocks, h->L,
                                      dev_EM + 2 * (n - 1));
    if (e != hipSuccess) return hip_fail(e, "E/M finalisation launch");
  }
  return ISING_OK;
}

static ising_status fill_pool(ising_lattice* h) {
  hipError_t e = launch_pool_fill(h->stream, h->pool, h->pool_m, (uint32_t)h->seed,
                                  (uint32_t)(h->seed >> 32), h->stream_id << 2, h->t4, h->t8);
  return e == hipSuccess ? ISING_OK : hip_fail(e, "pattern pool fill");
}

ising_status enqueue_sweeps(ising_lattice* h, int64_t n, int64_t* dev_EM) {
  if (n == 0) return ISING_OK;
  if (use_small_path(h)) {
    SmallArgs a;
    a.planes = h->planes;
    a.plane_words = h->plane_words;
    a.g = h->g;
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    a.sid4 = h->stream_id << 2;
    a.t0 = (uint32_t)h->sweep;
    a.t4 = h->t4;
    a.t8 = h->t8;
    a.n = n;
    a.EM = dev_EM;
    a.perturb = debug_perturb_seed();
    int threads = (int)std::min<int64_t>(1024, ((h->plane_words + 63) / 64) * 64);
    hipError_t e = launch_small_sweeps(h->stream, a, threads);
    if (e != hipSuccess) return hip_fail(e, "small-lattice sweep launch");
    return ISING_OK;
  }
  TileArgs ta;
  if (h->pool) return enqueue_pool_sweeps(h, n, dev_EM);
  const bool strip = strip_args(h, &ta);
  if (strip || tile_args(h, &ta)) {
    if (!strip) make_flat(ta);  // direct-load tiles: every lane busy at any W
    const int64_t units = strip ? (ta.tiles + 3) / 4 : ta.tiles;  // 4 wave tasks per block
    const int blocks = (int)std::min<int64_t>(units, std::min(h->tune.max_blocks,
                                                              kMaxSweepBlocks));
    auto launch = strip ? launch_strip_sweep : launch_tile_sweep;
    ta.lcg = h->lcg;
    uint32_t l8d = 0;
    lcg_decision(h->l4, &ta.l4d, &ta.l4m);
    lcg_decision(h->l8, &l8d, &ta.l8m);
    ta.lc = kLcgC + ta.l4d - kLcgA * ta.l4d;  // addend of the chain on z = x + l4d
    ta.le = l8d - ta.l4d;
    for (int64_t k = 0; k < n; ++k) {
      ta.t = (uint32_t)(h->sweep + (uint64_t)k);
      ta.prev_EM = (dev_EM && k > 0) ? dev_EM + 2 * (k - 1) : nullptr;
      ta.prev_part = h->part[(k + 1) & 1];
      ta.prev_blocks = blocks;
      ta.part = nullptr;
      hipError_t e = launch(h->stream, 0, ta, blocks);
      if (e != hipSuccess) return hip_fail(e, "colour-0 tiled half-sweep launch");
      ta.prev_EM = nullptr;
      ta.part = dev_EM ? h->part[k & 1] : nullptr;
      e = launch(h->stream, 1, ta, blocks);
      if (e != hipSuccess) return hip_fail(e, "colour-1 tiled half-sweep launch");
    }
    if (dev_EM) {
      hipError_t e = launch_finalize_em(h->stream, h->part[(n - 1) & 1], blocks, h->L,
                                        dev_EM + 2 * (n - 1));
      if (e != hipSuccess) return hip_fail(e, "E/M finalisation launch");
    }
    return ISING_OK;
  }
  if (h->lcg) return fail(ISING_EINVAL, "LCG dynamics need the tiled layout (L %% 8 == 0)");
  const int blocks = grid_blocks(h->plane_words, 256, h->tune.max_blocks);
  for (int64_t k = 0; k < n; ++k) {
    const uint32_t t = (uint32_t)(h->sweep + (uint64_t)k);
    SweepArgs a = sweep_args(h, t, dev_EM ? dev_EM + 2 * k : nullptr);
    hipError_t e = launch_half_sweep(h->stream, 0, a, blocks);
    if (e != hipSuccess) return hip_fail(e, "colour-0 half-sweep launch");
    e = launch_half_sweep(h->stream, 1, a, blocks);
    if (e != hipSuccess) return hip_fail(e, "colour-1 half-sweep launch");
  }
  return ISING_OK;
}

// Host-side unpacking of one packed row pair into int8 spins for the
// columns [x0, x0 + w) (periodic).
static void unpack_row(const uint64_t* p0, const uint64_t* p1, int64_t L, int64_t y, int64_t x0,
                       int64_t w, int8_t* out) {
  for (int64_t i = 0; i < w; ++i) {
    const int64_t x = (x0 + i) % L;
    const int c = (int)((x + y) & 1);
    const int64_t k = x >> 1;
    const uint64_t word = (c ? p1 : p0)[k >> 6];
    out[i] = ((word >> (k & 63)) & 1ull) ? (int8_t)1 : (int8_t)-1;
  }
}

}  // namespace ising

using namespace ising;

static std::atomic<uint32_t> g_perturb_seed{0};

namespace ising {
uint32_t debug_perturb_seed() { return g_perturb_seed.load(std::memory_order_relaxed); }
}  // namespace ising

extern "C" {

const char* ising_last_error(void) { return g_last_error.c_str(); }

const char* ising_version(void) { return "ising-mi355x 0.1 (gfx950)"; }

size_t ising_lattice_bytes(int64_t L) { return lattice_bytes(L); }

ising_status ising_create(int64_t L, uint64_t seed, uint32_t stream_id, int32_t init,
                          void* dev_buf, size_t dev_bytes, void* hip_stream, ising_t** out) {
  clear_error();
  if (!out) return fail(ISING_EINVAL, "ising_create: out is NULL");
  *out = nullptr;
  if (L < 4 || (L & 1) || L > kMaxL)
    return fail(ISING_EINVAL, "ising_create: L=%lld must be even and in [4, %lld]", (long long)L,
                (long long)kMaxL);
  if (init < 0 || init > 2) return fail(ISING_EINVAL, "ising_create: init=%d invalid", init);
  if (stream_id >= (1u << 30))
    return fail(ISING_EINVAL, "ising_create: stream_id must be < 2^30");
  if (!dev_buf) return fail(ISING_EINVAL, "ising_create: dev_buf is NULL");
  if (((uintptr_t)dev_buf) & 255)
    return fail(ISING_EINVAL, "ising_create: dev_buf must be 256-byte aligned");
  const size_t need = lattice_bytes(L);
  if (dev_bytes < need)
    return fail(ISING_ENOMEM, "ising_create: dev_bytes=%zu < %zu needed for L=%lld", dev_bytes,
                need, (long long)L);
  ising_lattice* h = new (std::nothrow) ising_lattice();
  if (!h) return fail(ISING_ENOMEM, "ising_create: host allocation failed");
  h->L = L;
  h->g = make_geom(L);
  h->plane_words = L * (int64_t)h->g.W;
  h->planes = (uint64_t*)dev_buf;
  h->scratch = (int64_t*)((char*)dev_buf + (need - kScratchBytes));
  h->part[0] = (uint64_t*)((char*)h->scratch + 256);
  h->part[1] = h->part[0] + 2 * kMaxSweepBlocks;
  h->dev_bytes = dev_bytes;
  h->seed = seed;
  h->stream_id = stream_id;
  h->init = init;
  h->stream = (hipStream_t)hip_stream;
  h->sweep = 0;
  h->beta_set = false;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "ising_create: hipGetDevice");
  }
  h->tune = default_tuning(L);
  e = launch_init(h->stream, h->planes, h->g, (uint32_t)seed, (uint32_t)(seed >> 32),
                  stream_id << 2, init, grid_blocks(2 * h->plane_words, 256, 8192));
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "ising_create: init launch");
  }
  *out = h;
  return ISING_OK;
}

ising_status ising_destroy(ising_t* h) {
  clear_error();
  delete h;
  return ISING_OK;
}

ising_status ising_set_beta(ising_t* h, double beta) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_set_beta: NULL handle");
  if (std::isnan(beta) || beta < 0.0)
    return fail(ISING_EINVAL, "ising_set_beta: beta must be >= 0 or +inf");
  h->beta = beta;
  h->t4 = metropolis_threshold(beta, 4);
  h->t8 = metropolis_threshold(beta, 8);
  h->l4 = lcg_threshold(beta, 4);
  h->l8 = lcg_threshold(beta, 8);
  h->beta_set = true;
  if (h->pool) return fill_pool(h);  // the patterns encode this temperature
  return ISING_OK;
}

ising_status ising_debug_perturb(uint32_t seed) {
  clear_error();
  g_perturb_seed.store(seed, std::memory_order_relaxed);
  return ISING_OK;
}

size_t ising_pool_bytes(int32_t log2_patterns) {
  if (log2_patterns < 10 || log2_patterns > 28) return 0;
  return (size_t)16 << log2_patterns;
}

size_t ising_lcg_bytes(int64_t L) {
  if (L < 4 || (L & 1) || L > kMaxL) return 0;
  return (size_t)2 * (size_t)L * (size_t)words_per_row(L) * sizeof(uint32_t);
}

ising_status ising_set_rng(ising_t* h, int32_t kind, void* dev_state, size_t state_bytes) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_set_rng: NULL handle");
  if (kind == ISING_RNG_PHILOX) {
    h->lcg = nullptr;
    h->pool = nullptr;
    return ISING_OK;
  }
  if (kind == ISING_RNG_POOL || kind == ISING_RNG_POOL_LINEAR) {
    TileArgs pa;
    if (!pool_tile_args(h, &pa))
      return fail(ISING_EINVAL,
                  "ising_set_rng: pattern pools need L %% 8 == 0 and < 2^32 words per plane");
    int m = 10;
    while (m <= 28 && ising_pool_bytes(m) != state_bytes) ++m;
    if (m > 28)
      return fail(ISING_EINVAL, "ising_set_rng: pool bytes must be ising_pool_bytes(m), 10 <= m <= 28");
    if (!dev_state) return fail(ISING_EINVAL, "ising_set_rng: NULL pool buffer");
    if (((uintptr_t)dev_state & 15u) != 0)
      return fail(ISING_EINVAL, "ising_set_rng: pool buffer must be 16-byte aligned");
    h->lcg = nullptr;
    h->pool = (uint64_t*)dev_state;
    h->pool_m = m;
    h->pool_linear = kind == ISING_RNG_POOL_LINEAR;
    return h->beta_set ? fill_pool(h) : ISING_OK;
  }
  if (kind != ISING_RNG_LCG) return fail(ISING_EINVAL, "ising_set_rng: unknown kind %d", kind);
  TileArgs ta;
  if (!tile_args(h, &ta))
    return fail(ISING_EINVAL, "ising_set_rng: LCG dynamics need L %% 8 == 0 (tiled layout)");
  const size_t need = ising_lcg_bytes(h->L);
  if (!dev_state || state_bytes < need)
    return fail(ISING_ENOMEM, "ising_set_rng: state buffer of %zu bytes needed", need);
  if (((uintptr_t)dev_state & 3u) != 0)
    return fail(ISING_EINVAL, "ising_set_rng: state buffer must be 4-byte aligned");
  hipError_t e = launch_lcg_seed(h->stream, (uint32_t*)dev_state, (int64_t)(need / 4),
                                 (uint32_t)h->seed);
  if (e != hipSuccess) return hip_fail(e, "ising_set_rng: seeding");
  h->lcg = (uint32_t*)dev_state;
  h->pool = nullptr;
  return ISING_OK;
}

ising_status ising_get_thresholds(const ising_t* h, uint32_t t[2]) {
  clear_error();
  if (!h || !t) return fail(ISING_EINVAL, "ising_get_thresholds: NULL argument");
  if (!h->beta_set) return fail(ISING_EINVAL, "ising_get_thresholds: no beta set");
  t[0] = h->t4;
  t[1] = h->t8;
  return ISING_OK;
}

ising_status ising_sweep(ising_t* h, int64_t n, int64_t* dev_EM) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_sweep: NULL handle");
  if (n < 0) return fail(ISING_EINVAL, "ising_sweep: n < 0");
  if (!h->beta_set) return fail(ISING_EINVAL, "ising_sweep: set beta first");
  if (h->sweep + (uint64_t)n > (1ull << 32))
    return fail(ISING_ERANGE, "ising_sweep: sweep counter would pass 2^32 - 1");
  ising_status st = enqueue_sweeps(h, n, dev_EM);
  if (st != ISING_OK) return st;
  h->sweep += (uint64_t)n;
  return ISING_OK;
}

ising_status ising_measure(ising_t* h, int64_t* E, int64_t* M) {
  clear_error();
  if (!h || !E || !M) return fail(ISING_EINVAL, "ising_measure: NULL argument");
  hipError_t e = launch_measure(h->stream, h->planes, h->g, h->plane_words, h->scratch,
                                grid_blocks(h->plane_words, 256, h->tune.max_blocks));
  if (e != hipSuccess) return hip_fail(e, "ising_measure: launch");
  int64_t em[2];
  e = hipMemcpyAsync(em, h->scratch, sizeof(em), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(e, "ising_measure: copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "ising_measure: synchronize");
  *E = em[0];
  *M = em[1];
  return ISING_OK;
}

ising_status ising_get_window(ising_t* h, int64_t x0, int64_t y0, int64_t w, int64_t hgt,
                              int8_t* host) {
  clear_error();
  if (!h || !host) return fail(ISING_EINVAL, "ising_get_window: NULL argument");
  const int64_t L = h->L;
  if (x0 < 0 || y0 < 0 || x0 >= L || y0 >= L || w < 1 || hgt < 1 || w > L || hgt > L)
    return fail(ISING_EINVAL, "ising_get_window: window out of range");
  const int64_t W = h->g.W;
  std::vector<uint64_t> rows(2 * (size_t)hgt * (size_t)W);
  // rows y0 .. y0+hgt-1 (mod L) of both planes: at most two contiguous chunks each
  for (int c = 0; c < 2; ++c) {
    int64_t done = 0;
    while (done < hgt) {
      const int64_t y = (y0 + done) % L;
      const int64_t chunk = std::min<int64_t>(hgt - done, L - y);
      hipError_t e = hipMemcpyAsync(rows.data() + ((size_t)c * hgt + done) * W,
                                    h->planes + (size_t)c * h->plane_words + (size_t)y * W,
                                    (size_t)chunk * W * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                    h->stream);
      if (e != hipSuccess) return hip_fail(e, "ising_get_window: copy");
      done += chunk;
    }
  }
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "ising_get_window: synchronize");
  for (int64_t j = 0; j < hgt; ++j) {
    const int64_t y = (y0 + j) % L;
    unpack_row(rows.data() + (size_t)j * W, rows.data() + ((size_t)hgt + j) * W, L, y, x0, w,
               host + j * w);
  }
  return ISING_OK;
}

ising_status ising_get_spins(ising_t* h, int8_t* host) {
  if (!h) {
    clear_error();
    return fail(ISING_EINVAL, "ising_get_spins: NULL handle");
  }
  return ising_get_window(h, 0, 0, h->L, h->L, host);
}

ising_status ising_set_spins(ising_t* h, const int8_t* host) {
  clear_error();
  if (!h || !host) return fail(ISING_EINVAL, "ising_set_spins: NULL argument");
  const int64_t L = h->L, W = h->g.W;
  std::vector<uint64_t> packed(2 * (size_t)h->plane_words, 0ull);
  for (int64_t y = 0; y < L; ++y)
    for (int64_t x = 0; x < L; ++x) {
      const int8_t v = host[y * L + x];
      if (v != 1 && v != -1)
        return fail(ISING_EINVAL, "ising_set_spins: spin at (%lld, %lld) is %d, not +-1",
                    (long long)x, (long long)y, (int)v);
      if (v == 1) {
        const int c = (int)((x + y) & 1);
        const int64_t k = x >> 1;
        packed[(size_t)c * h->plane_words + (size_t)y * W + (k >> 6)] |= 1ull << (k & 63);
      }
    }
  hipError_t e = hipMemcpyAsync(h->planes, packed.data(), packed.size() * sizeof(uint64_t),
                                hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "ising_set_spins: copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "ising_set_spins: synchronize");
  return ISING_OK;
}

ising_status ising_get_sweep(const ising_t* h, uint64_t* t) {
  clear_error();
  if (!h || !t) return fail(ISING_EINVAL, "ising_get_sweep: NULL argument");
  *t = h->sweep;
  return ISING_OK;
}

ising_status ising_set_sweep(ising_t* h, uint64_t t) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_set_sweep: NULL handle");
  if (t >= (1ull << 32)) return fail(ISING_ERANGE, "ising_set_sweep: t must be < 2^32");
  h->sweep = t;
  return ISING_OK;
}

ising_status ising_get_info(const ising_t* h, int64_t* L, int64_t* words_per_row_out,
                            void** planes) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_get_info: NULL handle");
  if (L) *L = h->L;
  if (words_per_row_out) *words_per_row_out = h->g.W;
  if (planes) *planes = h->planes;
  return ISING_OK;
}

}  // extern "C"
