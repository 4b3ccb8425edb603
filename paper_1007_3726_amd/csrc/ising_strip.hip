// Row-strip shares of one lattice (C ABI in include/ising.h): the part of
// a multi-GPU row-strip decomposition that one GPU runs.  A strip holds
// global rows y0 .. y0 + rows - 1 of an L x L lattice plus one halo row
// above and below per colour plane; a colour step updates the strip's own
// rows from the other colour's rows and halos, and between colour steps
// the halos of the colour just updated are refreshed from the neighbouring
// strips (ising_strip_exchange here; RCCL send/recv of the same rows
// across GPUs).  The uniforms are keyed by global (x, y), so any split
// reproduces the whole lattice bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "ising.h"
#include "ising_kernels.hpp"
#include "ising_runtime.hpp"

using namespace ising;

struct ising_strip {
  int64_t L, rows, y0;
  int32_t W;
  uint64_t* planes;     // device: plane 0 then plane 1, (rows + 2) x W words each
  int64_t plane_words;  // (rows + 2) * W
  uint64_t* part;       // device: per-block (A, P) partials after the planes
  uint64_t seed;
  uint32_t stream_id;
  hipStream_t stream;
  uint32_t t4, t8;
  bool beta_set;
};

namespace {

constexpr int kStripBlocks = 2048;

bool strip_shape_ok(int64_t L, int64_t rows) {
  if (L < 128 || L % 128 != 0 || L > kMaxL || rows < 1 || rows > L) return false;
  return rows * (L / 128) <= (int64_t)1 << 31;  // 32-bit word numbers, no wrap in the loop
}

ShareArgs share_args(const ising_strip* h, uint32_t t) {
  ShareArgs a;
  a.planes = h->planes;
  a.plane_words = h->plane_words;
  a.rows = h->rows;
  a.y0 = h->y0;
  a.W = h->W;
  a.L8 = (uint32_t)(h->L / 8);
  a.wdiv_m = h->W == 1 ? 0u : (uint32_t)((1ull << 32) / (uint64_t)h->W + 1ull);
  a.k0 = (uint32_t)h->seed;
  a.k1 = (uint32_t)(h->seed >> 32);
  a.sid4 = h->stream_id << 2;
  a.t = t;
  a.t4 = h->t4;
  a.t8 = h->t8;
  a.part = nullptr;
  return a;
}

int strip_blocks(const ising_strip* h) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((h->rows * h->W + 255) / 256, kStripBlocks));
}

}  // namespace

extern "C" {

size_t ising_strip_bytes(int64_t L, int64_t rows) {
  if (!strip_shape_ok(L, rows)) return 0;
  const int64_t W = L / 128;
  return (size_t)(2 * (rows + 2) * W) * sizeof(uint64_t) +
         (size_t)2 * kStripBlocks * sizeof(uint64_t);
}

ising_status ising_strip_create(int64_t L, int64_t y0, int64_t rows, uint64_t seed,
                                uint32_t stream_id, int32_t init, void* dev_buf,
                                size_t dev_bytes, void* hip_stream, ising_strip_t** out) {
  clear_error();
  if (!out) return fail(ISING_EINVAL, "ising_strip_create: NULL output");
  *out = nullptr;
  if (!strip_shape_ok(L, rows))
    return fail(ISING_EINVAL,
                "ising_strip_create: need L %% 128 == 0, 128 <= L <= 2^21, 1 <= rows <= L and "
                "rows * L / 128 <= 2^31 (L=%lld rows=%lld)",
                (long long)L, (long long)rows);
  if (y0 < 0 || y0 + rows > L) return fail(ISING_EINVAL, "ising_strip_create: rows outside 0..L");
  if (init < 0 || init > 2) return fail(ISING_EINVAL, "ising_strip_create: init %d", init);
  if (stream_id >= (1u << 30)) return fail(ISING_EINVAL, "ising_strip_create: stream_id >= 2^30");
  const size_t need = ising_strip_bytes(L, rows);
  if (!dev_buf || dev_bytes < need)
    return fail(ISING_ENOMEM, "ising_strip_create: device buffer of %zu bytes needed", need);
  if (((uintptr_t)dev_buf & 7u) != 0)
    return fail(ISING_EINVAL, "ising_strip_create: device buffer must be 8-byte aligned");
  ising_strip* h = new (std::nothrow) ising_strip();
  if (!h) return fail(ISING_ENOMEM, "ising_strip_create: host allocation");
  h->L = L;
  h->rows = rows;
  h->y0 = y0;
  h->W = (int32_t)(L / 128);
  h->planes = (uint64_t*)dev_buf;
  h->plane_words = (rows + 2) * h->W;
  h->part = h->planes + 2 * h->plane_words;
  h->seed = seed;
  h->stream_id = stream_id;
  h->stream = (hipStream_t)hip_stream;
  h->beta_set = false;
  hipError_t e = launch_share_init(h->stream, share_args(h, 0), init);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "ising_strip_create: init launch");
  }
  *out = h;
  return ISING_OK;
}

ising_status ising_strip_destroy(ising_strip_t* h) {
  clear_error();
  delete h;
  return ISING_OK;
}

ising_status ising_strip_set_beta(ising_strip_t* h, double beta) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_strip_set_beta: NULL handle");
  if (std::isnan(beta) || beta < 0.0)
    return fail(ISING_EINVAL, "ising_strip_set_beta: beta must be >= 0 or +inf");
  h->t4 = metropolis_threshold(beta, 4);
  h->t8 = metropolis_threshold(beta, 8);
  h->beta_set = true;
  return ISING_OK;
}

ising_status ising_strip_step(ising_strip_t* h, int32_t colour, uint32_t sweep,
                              int64_t* dev_counts) {
  clear_error();
  if (!h) return fail(ISING_EINVAL, "ising_strip_step: NULL handle");
  if (colour != 0 && colour != 1) return fail(ISING_EINVAL, "ising_strip_step: colour %d", colour);
  if (!h->beta_set) return fail(ISING_EINVAL, "ising_strip_step: no beta set");
  ShareArgs a = share_args(h, sweep);
  const int blocks = strip_blocks(h);
  if (colour == 1 && dev_counts) a.part = h->part;
  hipError_t e = launch_share_sweep(h->stream, colour, a, blocks);
  if (e != hipSuccess) return hip_fail(e, "ising_strip_step: launch");
  if (a.part) {
    e = launch_share_counts(h->stream, h->part, blocks, dev_counts);
    if (e != hipSuccess) return hip_fail(e, "ising_strip_step: counts launch");
  }
  return ISING_OK;
}

ising_status ising_strip_exchange(ising_strip_t* const* hs, int32_t count, int32_t colour) {
  clear_error();
  if (!hs || count < 1 || (colour != 0 && colour != 1))
    return fail(ISING_EINVAL, "ising_strip_exchange: bad arguments");
  int64_t next_row = 0;
  for (int32_t k = 0; k < count; ++k) {
    if (!hs[k]) return fail(ISING_EINVAL, "ising_strip_exchange: NULL handle %d", k);
    if (hs[k]->L != hs[0]->L || hs[k]->stream != hs[0]->stream)
      return fail(ISING_EINVAL, "ising_strip_exchange: strips must share L and the stream");
    if (hs[k]->y0 != next_row)
      return fail(ISING_EINVAL, "ising_strip_exchange: strip %d starts at row %lld, not %lld", k,
                  (long long)hs[k]->y0, (long long)next_row);
    next_row += hs[k]->rows;
  }
  if (next_row != hs[0]->L)
    return fail(ISING_EINVAL, "ising_strip_exchange: strips cover %lld of %lld rows",
                (long long)next_row, (long long)hs[0]->L);
  const size_t row_bytes = (size_t)hs[0]->W * sizeof(uint64_t);
  for (int32_t k = 0; k < count; ++k) {
    const ising_strip* up = hs[(k + count - 1) % count];
    const ising_strip* dn = hs[(k + 1) % count];
    const ising_strip* me = hs[k];
    uint64_t* mine = me->planes + (int64_t)colour * me->plane_words;
    const uint64_t* up_p = up->planes + (int64_t)colour * up->plane_words;
    const uint64_t* dn_p = dn->planes + (int64_t)colour * dn->plane_words;
    // halo above <- last row of the strip above; halo below <- first row of the strip below
    hipError_t e = hipMemcpyAsync(mine, up_p + up->rows * up->W, row_bytes,
                                  hipMemcpyDeviceToDevice, me->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(mine + (me->rows + 1) * me->W, dn_p + dn->W, row_bytes,
                         hipMemcpyDeviceToDevice, me->stream);
    if (e != hipSuccess) return hip_fail(e, "ising_strip_exchange: copy");
  }
  return ISING_OK;
}

ising_status ising_strip_row(const ising_strip_t* h, int32_t colour, int32_t which, void** ptr,
                             size_t* bytes) {
  clear_error();
  if (!h || !ptr || !bytes || (colour != 0 && colour != 1) || which < 0 || which > 3)
    return fail(ISING_EINVAL, "ising_strip_row: bad arguments");
  const int64_t row = which == 0 ? 0 : which == 1 ? 1 : which == 2 ? h->rows : h->rows + 1;
  *ptr = h->planes + (int64_t)colour * h->plane_words + row * h->W;
  *bytes = (size_t)h->W * sizeof(uint64_t);
  return ISING_OK;
}

ising_status ising_strip_get_rows(ising_strip_t* h, int8_t* host) {
  clear_error();
  if (!h || !host) return fail(ISING_EINVAL, "ising_strip_get_rows: NULL argument");
  std::vector<uint64_t> p((size_t)(2 * h->plane_words));
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess)
    e = hipMemcpy(p.data(), h->planes, p.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "ising_strip_get_rows: copy");
  const int64_t L = h->L, W = h->W;
  for (int64_t r = 0; r < h->rows; ++r) {
    const int64_t y = h->y0 + r;
    for (int64_t x = 0; x < L; ++x) {
      const int c = (int)((x + y) & 1);
      const int64_t k = x >> 1;
      const uint64_t word = p[(size_t)(c * h->plane_words + (r + 1) * W + (k >> 6))];
      host[r * L + x] = (int8_t)(((word >> (k & 63)) & 1ull) ? 1 : -1);
    }
  }
  return ISING_OK;
}

ising_status ising_strip_combine(const int64_t* dev_counts, int32_t nstrips, int64_t n, int64_t L,
                                 int64_t* dev_EM, void* hip_stream) {
  clear_error();
  if (!dev_counts || !dev_EM || nstrips < 1 || n < 0 || L < 4)
    return fail(ISING_EINVAL, "ising_strip_combine: bad arguments");
  if (n == 0) return ISING_OK;
  hipError_t e = launch_share_combine((hipStream_t)hip_stream, dev_counts, nstrips, n, L, dev_EM);
  return e == hipSuccess ? ISING_OK : hip_fail(e, "ising_strip_combine: launch");
}

}  // extern "C"
