// Served mode: continuous batching of independent Ising simulations.
//
// A server owns a device arena given by the caller (the HBM budget) and a
// FIFO of submitted requests.  Each ising_server_step is one quantum:
//   1. admission: queued requests are admitted in submission order while
//      their lattice and per-sweep (E, M) series fit in the free arena
//      (first-fit allocator, 256-byte aligned); a request larger than the
//      whole arena is rejected at submission;
//   2. one batched call advances every active lattice by up to
//      quantum_sweeps sweeps (fewer for a request that has fewer left), all
//      lattices together in fused launches or one packed launch, with the
//      task tables in a region reserved at the end of the arena (1/32 of
//      it; every admitted lattice also reserves its share of that region,
//      so the tables of any active set fit);
//   3. retirement: finished requests copy their series/spins to the
//      caller's host buffers, get exact moment sums, a completion time, and
//      free their arena space, so the next step can admit more.
// A request's result is a pure function of its own parameters: its
// uniforms are keyed by (seed, stream_id, sweep), never by arena slot or
// by the mix it ran in.
//
// Fault injection (tests): a quantum armed with ising_server_inject_fault
// snapshots the active lattices to host memory, runs, is declared failed,
// restores the snapshot and runs again; the final results are unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <vector>

#include "ising_batch.hpp"
#include "ising_runtime.hpp"

namespace ising {
namespace {

double now_s() {
  using clock = std::chrono::steady_clock;
  return std::chrono::duration<double>(clock::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

enum class State { Queued, Active, Done };

struct Job {
  uint64_t ticket;
  ising_request req;
  State state = State::Queued;
  size_t off = 0, bytes = 0;   // arena slice: lattice then series
  size_t share = 0;            // reserved bytes of the task-table region
  ising_lattice* h = nullptr;
  int64_t* dev_series = nullptr;
  int64_t done = 0;            // sweeps completed
  ising_result res;
};

size_t job_bytes(const ising_request& r) {
  return align256(lattice_bytes(r.L)) + align256((size_t)r.n_sweeps * 2 * sizeof(int64_t));
}

}  // namespace
}  // namespace ising

using namespace ising;

struct ising_server {
  char* arena_base;
  size_t arena_bytes;   // lattice and series space: [0, arena_bytes)
  char* table;          // task-table region: [arena_bytes, arena_bytes + table_bytes)
  size_t table_bytes;
  size_t table_used = kBatchWorkFixed;  // the fixed part plus the active shares
  hipStream_t stream;
  int32_t quantum;
  Arena arena;
  uint64_t next_ticket = 1;
  std::map<uint64_t, Job> jobs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;
  std::set<int64_t> faults;
  int64_t quanta = 0, admitted = 0, finished = 0, peak = 0, recovered = 0;
  // the quantum in flight: its tickets and sweeps, and its table image
  bool inflight = false;
  std::vector<uint64_t> ran;
  std::vector<int64_t> took;
  std::vector<char> image;
  // retirement in progress: tickets whose series are being copied to the
  // pinned staging buffer (offsets in int64 words), and the copies' event
  std::vector<std::pair<uint64_t, size_t>> leaving;
  int64_t* staging = nullptr;
  size_t staging_words = 0;
  hipEvent_t copied = nullptr;
  explicit ising_server(size_t bytes) : arena(bytes) {}
};

namespace ising {
namespace {

ising_status admit(ising_server* s) {
  while (!s->queue.empty()) {
    Job& j = s->jobs.at(s->queue.front());
    size_t off;
    // strict FIFO: wait for space in the arena and in the table region
    if (s->table_used + j.share > s->table_bytes) break;
    if (!s->arena.alloc(j.bytes, &off)) break;
    j.off = off;
    ising_t* h = nullptr;
    const size_t lb = align256(lattice_bytes(j.req.L));
    ising_status st = ising_create(j.req.L, j.req.seed, j.req.stream_id, j.req.init,
                                   s->arena_base + off, lb, s->stream, &h);
    if (st == ISING_OK) st = ising_set_beta(h, j.req.beta);
    if (st != ISING_OK) {
      s->arena.release(off, j.bytes);
      if (h) ising_destroy(h);
      return st;
    }
    j.h = h;
    s->table_used += j.share;
    j.dev_series = (int64_t*)(s->arena_base + off + lb);
    j.state = State::Active;
    j.res.t_admit = now_s();
    s->active.push_back(j.ticket);
    s->queue.pop_front();
    ++s->admitted;
    s->peak = std::max<int64_t>(s->peak, (int64_t)s->arena.used());
  }
  return ISING_OK;
}

}  // namespace

// 256-bit unsigned accumulator for sums of M^4: |M| <= L^2 <= 2^42, so one
// term is below 2^168 and 2^32 of them below 2^200.
struct U256 {
  unsigned __int128 lo = 0, hi = 0;
  void add_square(unsigned __int128 q) {  // += q * q for q < 2^85
    const uint64_t b = (uint64_t)q;
    const unsigned __int128 a = q >> 64;  // < 2^21
    const unsigned __int128 bb = (unsigned __int128)b * b;
    const unsigned __int128 cross = 2 * a * b;  // < 2^86
    unsigned __int128 carry = 0;
    unsigned __int128 t = lo + bb;
    carry += t < lo;
    const unsigned __int128 u = t + (cross << 64);
    carry += u < t;
    lo = u;
    hi += a * a + (cross >> 64) + carry;
  }
  // Rounded once to the nearest double: the bits below the top 128 only
  // matter as a sticky bit, which is folded into bit 0 of the shifted value.
  double to_double() const {
    if (hi == 0) return (double)lo;
    int s = 0;
    for (unsigned __int128 h = hi; h != 0; h >>= 1) ++s;  // bit length of hi, 1..128
    unsigned __int128 top;
    bool sticky;
    if (s == 128) {
      top = hi;
      sticky = lo != 0;
    } else {
      top = (hi << (128 - s)) | (lo >> s);
      sticky = (lo & ((((unsigned __int128)1) << s) - 1)) != 0;
    }
    return std::ldexp((double)(top | (unsigned __int128)sticky), s);
  }
};

// Exact sums of M^2 and M^4 over sweeps discard .. n - 1 of an interleaved
// (E, M) series, each rounded once to double.
void exact_moments(const int64_t* series, int64_t n, int64_t discard, double* sum_M2,
                   double* sum_M4, int64_t* kept) {
  unsigned __int128 s2 = 0;  // < 2^84 per term, 2^32 terms
  U256 s4;
  int64_t k0 = std::max<int64_t>(discard, 0), cnt = 0;
  for (int64_t k = k0; k < n; ++k) {
    const int64_t m = series[2 * k + 1];
    const unsigned __int128 am = (unsigned __int128)(m < 0 ? -(__int128)m : (__int128)m);
    const unsigned __int128 m2 = am * am;
    s2 += m2;
    s4.add_square(m2);
    ++cnt;
  }
  *sum_M2 = (double)s2;
  *sum_M4 = s4.to_double();
  *kept = cnt;
}

namespace {

void moments(const int64_t* series, int64_t n, int64_t discard, ising_result* r) {
  exact_moments(series, n, discard, &r->sum_M2, &r->sum_M4, &r->n_kept);
}

// Retirement, first half: the finished requests' series are copied to the
// pinned staging buffer on the stream (spins, if asked for, synchronously),
// and their arena space is released at once: anything that reuses it is
// enqueued later on the same stream.
ising_status begin_retire(ising_server* s, const std::vector<uint64_t>& done) {
  s->leaving.clear();
  if (done.empty()) return ISING_OK;
  size_t words = 0;
  for (uint64_t t : done) words += 2 * (size_t)s->jobs.at(t).req.n_sweeps;
  if (words > s->staging_words) {
    if (s->staging) (void)hipHostFree(s->staging);
    s->staging = nullptr;
    s->staging_words = 0;
    const size_t want = std::max<size_t>(words, size_t(1) << 20);
    hipError_t e = hipHostMalloc((void**)&s->staging, want * sizeof(int64_t), 0);
    if (e != hipSuccess) return hip_fail(e, "server: staging buffer");
    s->staging_words = want;
  }
  if (!s->copied) {
    hipError_t e = hipEventCreateWithFlags(&s->copied, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "server: event");
  }
  size_t off = 0;
  for (uint64_t t : done) {
    Job& j = s->jobs.at(t);
    const size_t n = 2 * (size_t)j.req.n_sweeps;
    hipError_t e = hipMemcpyAsync(s->staging + off, j.dev_series, n * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "server: series copy");
    if ((j.req.flags & ISING_REQ_RETURN_SPINS) && j.req.spins_out) {
      ising_status st = ising_get_spins(j.h, j.req.spins_out);
      if (st != ISING_OK) return st;
    }
    s->leaving.emplace_back(t, off);
    off += n;
    s->arena.release(j.off, j.bytes);
    s->table_used -= j.share;
  }
  hipError_t e = hipEventRecord(s->copied, s->stream);
  return e == hipSuccess ? ISING_OK : hip_fail(e, "server: event");
}

// Retirement, second half (on the host, while the next quantum runs):
// results, exact moment sums, completion time.
ising_status end_retire(ising_server* s) {
  if (s->leaving.empty()) return ISING_OK;
  hipError_t e = hipEventSynchronize(s->copied);
  if (e != hipSuccess) return hip_fail(e, "server: series copy");
  for (const auto& lv : s->leaving) {
    Job& j = s->jobs.at(lv.first);
    const int64_t* series = s->staging + lv.second;
    const size_t n = 2 * (size_t)j.req.n_sweeps;
    if ((j.req.flags & ISING_REQ_RECORD_SERIES) && j.req.EM_series)
      std::memcpy(j.req.EM_series, series, n * sizeof(int64_t));
    j.res.E_final = series[n - 2];
    j.res.M_final = series[n - 1];
    j.res.sweeps_done = (uint64_t)j.done;
    moments(series, j.req.n_sweeps, j.req.n_discard, &j.res);
    j.res.status = ISING_OK;
    j.res.t_done = now_s();
    ising_destroy(j.h);
    j.h = nullptr;
    j.state = State::Done;
    ++s->finished;
  }
  s->leaving.clear();
  return ISING_OK;
}

// Wait for the quantum in flight and count its sweeps; `done` receives the
// tickets that have finished (removed from the active set).
ising_status finish_quantum(ising_server* s, std::vector<uint64_t>& done) {
  if (!s->inflight) return ISING_OK;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(e, "server: quantum");
  s->inflight = false;
  for (size_t i = 0; i < s->ran.size(); ++i) {
    Job& j = s->jobs.at(s->ran[i]);
    j.h->sweep += (uint64_t)s->took[i];
    j.done += s->took[i];
  }
  std::vector<uint64_t> still;
  for (uint64_t t : s->active) {
    Job& j = s->jobs.at(t);
    if (j.done >= j.req.n_sweeps)
      done.push_back(t);
    else
      still.push_back(t);
  }
  s->active.swap(still);
  return ISING_OK;
}

// Enqueue one quantum of up to Q sweeps on every active lattice (direct
// launches, no waiting); `wait` makes it synchronous and leaves nothing in
// flight (the failed run of a fault-injected quantum).
ising_status enqueue_quantum(ising_server* s, bool wait) {
  std::vector<ising_lattice*> hs;
  std::vector<int64_t> nsw;
  std::vector<int64_t*> ems;
  s->ran.clear();
  s->took.clear();
  int64_t n = 0;
  for (uint64_t t : s->active) {
    Job& j = s->jobs.at(t);
    const int64_t take = std::min<int64_t>(s->quantum, j.req.n_sweeps - j.done);
    hs.push_back(j.h);
    nsw.push_back(take);
    ems.push_back(j.dev_series + 2 * j.done);
    s->ran.push_back(t);
    s->took.push_back(take);
    n = std::max(n, take);
  }
  if (hs.empty()) return ISING_OK;
  BatchOptions opt = default_batch_options();
  opt.graph_chunk = 0;  // direct launches: nothing to keep alive but the image
  opt.keep_image = &s->image;
  ising_status st = batch_sweeps(hs.data(), (int32_t)hs.size(), n, nsw.data(), ems.data(), opt,
                                 s->table, s->table_bytes, nullptr);
  if (st != ISING_OK) {
    (void)hipStreamSynchronize(s->stream);
    return st;
  }
  if (wait) {
    hipError_t e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? ISING_OK : hip_fail(e, "server: quantum");
  }
  s->inflight = true;
  return ISING_OK;
}

// One step: finish the quantum in flight, start retiring what it finished,
// admit, enqueue the next quantum, and only then finish the retirement on
// the host, so the GPU does not wait for the host's bookkeeping.
ising_status step(ising_server* s) {
  std::vector<uint64_t> done;
  ising_status st = finish_quantum(s, done);
  if (st == ISING_OK) st = begin_retire(s, done);
  if (st == ISING_OK) st = admit(s);
  if (st != ISING_OK) return st;
  const int64_t q = s->quanta;
  if (!s->active.empty()) {
    ++s->quanta;
    if (s->faults.count(q)) {
      // snapshot, run, declare the quantum failed, restore; the quantum is
      // then enqueued again below
      st = end_retire(s);
      if (st != ISING_OK) return st;
      std::vector<std::vector<char>> snap(s->active.size());
      for (size_t i = 0; i < s->active.size(); ++i) {
        const ising_lattice* h = s->jobs.at(s->active[i]).h;
        snap[i].resize(2 * (size_t)h->plane_words * sizeof(uint64_t));
        hipError_t e = hipMemcpyAsync(snap[i].data(), h->planes, snap[i].size(),
                                      hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return hip_fail(e, "server: snapshot");
      }
      st = enqueue_quantum(s, true);
      if (st != ISING_OK) return st;
      for (size_t i = 0; i < s->active.size(); ++i) {
        const ising_lattice* h = s->jobs.at(s->active[i]).h;
        hipError_t e = hipMemcpyAsync(h->planes, snap[i].data(), snap[i].size(),
                                      hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return hip_fail(e, "server: restore");
      }
      // the restore reads host memory that ends with this block
      hipError_t e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(e, "server: restore");
      s->faults.erase(q);
      ++s->recovered;
    }
    st = enqueue_quantum(s, false);
    if (st != ISING_OK) return st;
  }
  st = end_retire(s);
  if (st != ISING_OK) return st;
  return (s->active.empty() && s->queue.empty() && !s->inflight) ? ISING_OK : ISING_AGAIN;
}

}  // namespace
}  // namespace ising

extern "C" {

ising_status ising_server_create(void* dev_arena, size_t arena_bytes, void* hip_stream,
                                 int32_t quantum_sweeps, ising_server_t** out) {
  clear_error();
  if (!out) return fail(ISING_EINVAL, "ising_server_create: out is NULL");
  *out = nullptr;
  if (!dev_arena || arena_bytes < 256 || ((uintptr_t)dev_arena & 255))
    return fail(ISING_EINVAL, "ising_server_create: arena must be non-NULL, 256-B aligned");
  if (quantum_sweeps < 1)
    return fail(ISING_EINVAL, "ising_server_create: quantum_sweeps must be >= 1");
  // the last 1/32 of the arena (at least 4 KiB) holds the batched task tables
  const size_t total = arena_bytes & ~(size_t)255;
  const size_t table = std::max<size_t>((total / 32) & ~(size_t)255, 4096);
  if (total < 2 * table)
    return fail(ISING_EINVAL, "ising_server_create: arena of %zu bytes is too small", total);
  ising_server* s = new (std::nothrow) ising_server(total - table);
  if (!s) return fail(ISING_ENOMEM, "ising_server_create: host allocation failed");
  s->arena_base = (char*)dev_arena;
  s->arena_bytes = total - table;
  s->table = (char*)dev_arena + (total - table);
  s->table_bytes = table;
  s->stream = (hipStream_t)hip_stream;
  s->quantum = quantum_sweeps;
  *out = s;
  return ISING_OK;
}

ising_status ising_batch_submit(ising_server_t* s, const ising_request* reqs, int32_t n,
                                uint64_t* tickets_out) {
  clear_error();
  if (!s || (n > 0 && (!reqs || !tickets_out)) || n < 0)
    return fail(ISING_EINVAL, "ising_batch_submit: bad arguments");
  // validate all first: nothing is queued if any request is invalid
  for (int32_t i = 0; i < n; ++i) {
    const ising_request& r = reqs[i];
    if (lattice_bytes(r.L) == 0)
      return fail(ISING_EINVAL, "ising_batch_submit: request %d: bad L=%lld", i, (long long)r.L);
    if (std::isnan(r.beta) || r.beta < 0)
      return fail(ISING_EINVAL, "ising_batch_submit: request %d: bad beta", i);
    if (r.init < 0 || r.init > 2 || r.stream_id >= (1u << 30) || r.n_sweeps < 1 ||
        r.n_sweeps >= (int64_t(1) << 32) || r.n_discard < 0)
      return fail(ISING_EINVAL, "ising_batch_submit: request %d: bad init/stream/sweeps", i);
    if ((r.flags & ISING_REQ_RECORD_SERIES) && !r.EM_series)
      return fail(ISING_EINVAL, "ising_batch_submit: request %d: series buffer missing", i);
    if ((r.flags & ISING_REQ_RETURN_SPINS) && !r.spins_out)
      return fail(ISING_EINVAL, "ising_batch_submit: request %d: spins buffer missing", i);
    if (job_bytes(r) > s->arena_bytes || kBatchWorkFixed + batch_work_share(r.L) > s->table_bytes)
      return fail(ISING_ENOMEM, "ising_batch_submit: request %d needs %zu bytes > arena %zu", i,
                  job_bytes(r), s->arena_bytes);
  }
  const double t = now_s();
  for (int32_t i = 0; i < n; ++i) {
    Job j;
    j.ticket = s->next_ticket++;
    j.req = reqs[i];
    j.bytes = job_bytes(reqs[i]);
    j.share = batch_work_share(reqs[i].L);
    std::memset(&j.res, 0, sizeof(j.res));
    j.res.ticket = j.ticket;
    j.res.status = ISING_AGAIN;
    j.res.t_arrive = t;
    s->jobs.emplace(j.ticket, j);
    s->queue.push_back(j.ticket);
    tickets_out[i] = j.ticket;
  }
  return ISING_OK;
}

ising_status ising_server_step(ising_server_t* s) {
  clear_error();
  if (!s) return fail(ISING_EINVAL, "ising_server_step: NULL server");
  return step(s);
}

ising_status ising_poll(ising_server_t* s, uint64_t ticket, ising_result* out) {
  clear_error();
  if (!s || !out) return fail(ISING_EINVAL, "ising_poll: NULL argument");
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(ISING_ENOTFOUND, "ising_poll: unknown ticket %llu",
                                       (unsigned long long)ticket);
  *out = it->second.res;
  if (it->second.state != State::Done) {
    out->status = ISING_AGAIN;
    out->sweeps_done = (uint64_t)it->second.done;
    return ISING_AGAIN;
  }
  s->jobs.erase(it);
  return ISING_OK;
}

ising_status ising_series_moments(const int64_t* series, int64_t n, int64_t discard,
                                  double* sum_M2, double* sum_M4, int64_t* n_kept) {
  clear_error();
  if ((n > 0 && !series) || n < 0 || discard < 0 || !sum_M2 || !sum_M4 || !n_kept)
    return fail(ISING_EINVAL, "ising_series_moments: bad arguments");
  for (int64_t k = 0; k < n; ++k) {
    const int64_t m = series[2 * k + 1];
    if (m > ((int64_t)1 << 42) || m < -((int64_t)1 << 42))
      return fail(ISING_EINVAL, "ising_series_moments: |M| > 2^42 at sweep %lld", (long long)k);
  }
  exact_moments(series, n, discard, sum_M2, sum_M4, n_kept);
  return ISING_OK;
}

ising_status ising_server_inject_fault(ising_server_t* s, int64_t quantum_index) {
  clear_error();
  if (!s || quantum_index < 0) return fail(ISING_EINVAL, "ising_server_inject_fault: bad args");
  s->faults.insert(quantum_index);
  return ISING_OK;
}

ising_status ising_server_stats(const ising_server_t* s, int64_t out[6]) {
  clear_error();
  if (!s || !out) return fail(ISING_EINVAL, "ising_server_stats: NULL argument");
  out[0] = s->quanta;
  out[1] = s->admitted;
  out[2] = s->finished;
  out[3] = (int64_t)s->arena.used();
  out[4] = s->peak;
  out[5] = s->recovered;
  return ISING_OK;
}

ising_status ising_server_destroy(ising_server_t* s) {
  clear_error();
  if (!s) return ISING_OK;
  // a quantum or a series copy may still be in flight
  (void)hipStreamSynchronize(s->stream);
  if (s->staging) (void)hipHostFree(s->staging);
  if (s->copied) (void)hipEventDestroy(s->copied);
  for (auto& kv : s->jobs)
    if (kv.second.h) ising_destroy(kv.second.h);
  delete s;
  return ISING_OK;
}

}  // extern "C"
