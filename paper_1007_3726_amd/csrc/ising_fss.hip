// Finite-size-scaling analysis of per-sweep (E, M) series.
//
// The paper locates T_C where the Binder cumulants U4 = 1 - <M^4>/(3<M^2>^2)
// (section 2, Eq. (2)) of different lattice sizes cross.  Turning the
// batched simulations' series into those curves takes three steps:
//
//  * k_reweight (device, fp64): single-histogram reweighting (Ferrenberg and
//    Swendsen, PRL 61, 2635 (1988)) of each series sampled at beta0 to a
//    target beta, accumulated as five sums per block of consecutive kept
//    sweeps.  The series stay where the sweeps wrote them.
//  * ising_fss_moments (host): U4, <E>/N and <|M|>/N from the totals and
//    their delete-one-block jackknife errors (B sets of a few numbers).
//  * ising_binder_crossing (host): where two U4 curves on a common grid
//    cross, with the jackknife error from the replica curves.
//
// Definitions (the same in the test oracle, written separately):
//   kept sweeps t = discard .. n-1, count = n - discard; sample j = t -
//   discard is in block floor(j B / count);
//   x_t = -(beta - beta0)(E_t - E_ref), E_ref = E of the first kept sweep;
//   w_t = exp(x_t - max x); sums per block: w, w|M|, w M^2, w M^4, w E with
//   m = double(M), m2 = m m, m4 = m2 m2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <vector>

#include "ising.h"
#include "ising_runtime.hpp"

namespace ising {
namespace {

constexpr int kRwThreads = 256;
constexpr int kRwMaxBlocks = 4096;

struct RwLattice {
  const int64_t* EM;  // n x (E, M)
  int64_t n;
  int64_t discard;
  double beta0;
};
struct RwTask {
  int32_t lattice;
  int32_t pad;
  double beta;
};

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_add(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One workgroup per task (lattice, target beta): the maximum exponent over
// the kept sweeps, then the five sums of every block.
__global__ __launch_bounds__(kRwThreads) void k_reweight(const RwLattice* lat, const RwTask* task,
                                                         int nblocks, double* sums,
                                                         double* shift) {
  // every product and sum rounds on its own, as in the definition above (a
  // fused multiply-add would move the exponent by an ulp of |x|, which is
  // then amplified by exp)
#pragma clang fp contract(off)
  __shared__ double red[kRwThreads / 64][5];
  const RwTask tk = task[blockIdx.x];
  const RwLattice lt = lat[tk.lattice];
  const int64_t* EM = lt.EM;
  const int64_t t0 = lt.discard;
  const int64_t count = lt.n - t0;
  const int64_t E_ref = EM[2 * t0];
  const double db = tk.beta - lt.beta0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  double xm = -std::numeric_limits<double>::infinity();
  for (int64_t j = threadIdx.x; j < count; j += kRwThreads)
    xm = fmax(xm, -db * (double)(EM[2 * (t0 + j)] - E_ref));
  xm = wave_max(xm);
  if (lane == 0) red[wave][0] = xm;
  __syncthreads();
  xm = red[0][0];
  for (int i = 1; i < kRwThreads / 64; ++i) xm = fmax(xm, red[i][0]);
  __syncthreads();

  for (int b = 0; b < nblocks; ++b) {
    const int64_t j0 = ((int64_t)b * count + nblocks - 1) / nblocks;
    const int64_t j1 = ((int64_t)(b + 1) * count + nblocks - 1) / nblocks;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kRwThreads) {
      const int64_t E = EM[2 * (t0 + j)];
      const double m = (double)EM[2 * (t0 + j) + 1];
      const double x = -db * (double)(E - E_ref);
      const double w = exp(x - xm);
      const double m2 = m * m;
      s[0] += w;
      s[1] += w * fabs(m);
      s[2] += w * m2;
      s[3] += w * (m2 * m2);
      s[4] += w * (double)E;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) s[i] = wave_add(s[i]);
    if (lane == 0)
      for (int i = 0; i < 5; ++i) red[wave][i] = s[i];
    __syncthreads();
    if (threadIdx.x < 5) {
      double v = 0.0;
      for (int k = 0; k < kRwThreads / 64; ++k) v += red[k][threadIdx.x];
      sums[((int64_t)blockIdx.x * nblocks + b) * 5 + threadIdx.x] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && shift) shift[blockIdx.x] = xm;
}

// Layout of the task tables in the caller's work buffer: the series
// table, then (256-byte aligned) the task list.
size_t rw_task_offset(int32_t nlat) { return ((size_t)nlat * sizeof(RwLattice) + 255) / 256 * 256; }
size_t rw_work_bytes(int32_t nlat, int32_t ntask) {
  return rw_task_offset(nlat) + (size_t)ntask * sizeof(RwTask);
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// (U4, <E>/N, <|M|>/N) from one set of the five sums.
void quantities(const double* S, double N, double* q) {
  const double m2 = S[2] / S[0];
  const double m4 = S[3] / S[0];
  q[0] = 1.0 - m4 / (3.0 * m2 * m2);
  q[1] = S[4] / (S[0] * N);
  q[2] = S[1] / (S[0] * N);
}

// First k with d_k < 0 <= d_{k+1}, d = Ua - Ub; (T*, U*) or NaNs.
void crossing(const double* T, int K, const double* Ua, const double* Ub, double* Tx,
              double* Ux) {
  *Tx = *Ux = std::numeric_limits<double>::quiet_NaN();
  for (int k = 0; k + 1 < K; ++k) {
    const double d0 = Ua[k] - Ub[k], d1 = Ua[k + 1] - Ub[k + 1];
    if (d0 < 0.0 && 0.0 <= d1) {
      const double f = d0 / (d0 - d1);
      *Tx = T[k] + (T[k + 1] - T[k]) * f;
      *Ux = Ua[k] + (Ua[k + 1] - Ua[k]) * f;
      return;
    }
  }
}

// In-place radix-2 FFT of a (size a power of two) with the twiddles
// exp(-2 pi i k / n) taken from a table computed directly (no accumulated
// rotation), sign +1 for the inverse transform (unscaled).
void fft(std::vector<std::complex<double>>& a, int sign) {
  const size_t n = a.size();
  std::vector<std::complex<double>> tw(n / 2);
  for (size_t k = 0; k < n / 2; ++k) {
    const double ang = sign * 2.0 * M_PI * (double)k / (double)n;
    tw[k] = std::complex<double>(std::cos(ang), std::sin(ang));
  }
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t half = len / 2, step = n / len;
    for (size_t i = 0; i < n; i += len)
      for (size_t j = 0; j < half; ++j) {
        const std::complex<double> u = a[i + j], v = a[i + j + half] * tw[j * step];
        a[i + j] = u + v;
        a[i + j + half] = u - v;
      }
  }
}

}  // namespace
}  // namespace ising

using namespace ising;

extern "C" {

size_t ising_reweight_work_bytes(int32_t nlat, int32_t ntask) {
  if (nlat < 1 || ntask < 1) return 0;
  return rw_work_bytes(nlat, ntask);
}

ising_status ising_reweight(int32_t nlat, const int64_t* const* dev_EM, const int64_t* n_sweeps,
                            const int64_t* discard, const double* beta0, int32_t ntask,
                            const int32_t* task_lattice, const double* task_beta,
                            int32_t nblocks, double* dev_sums, double* dev_shift,
                            void* dev_work, size_t work_bytes, void* hip_stream) {
  clear_error();
  if (nlat < 1 || ntask < 1 || !dev_EM || !n_sweeps || !discard || !beta0 || !task_lattice ||
      !task_beta || !dev_sums)
    return fail(ISING_EINVAL, "ising_reweight: bad arguments");
  if (!dev_work || ((uintptr_t)dev_work & 255) || work_bytes < rw_work_bytes(nlat, ntask))
    return fail(ISING_ENOMEM,
                "ising_reweight: needs a 256-byte aligned work buffer of %zu bytes (got %zu)",
                rw_work_bytes(nlat, ntask), dev_work ? work_bytes : (size_t)0);
  if (nblocks < 1 || nblocks > kRwMaxBlocks)
    return fail(ISING_EINVAL, "ising_reweight: nblocks must be in 1..%d", kRwMaxBlocks);
  std::vector<RwLattice> lat((size_t)nlat);
  for (int32_t i = 0; i < nlat; ++i) {
    if (!dev_EM[i] || discard[i] < 0 || n_sweeps[i] - discard[i] < nblocks ||
        !finite_nonneg(beta0[i]))
      return fail(ISING_EINVAL,
                  "ising_reweight: series %d needs a device pointer, 0 <= discard and at least "
                  "nblocks kept sweeps, and a finite beta0 >= 0",
                  i);
    lat[i] = RwLattice{dev_EM[i], n_sweeps[i], discard[i], beta0[i]};
  }
  std::vector<RwTask> tasks((size_t)ntask);
  for (int32_t k = 0; k < ntask; ++k) {
    if (task_lattice[k] < 0 || task_lattice[k] >= nlat || !finite_nonneg(task_beta[k]))
      return fail(ISING_EINVAL, "ising_reweight: task %d has a bad series index or beta", k);
    tasks[k] = RwTask{task_lattice[k], 0, task_beta[k]};
  }
  const size_t off_task = rw_task_offset(nlat);
  const size_t bytes = rw_work_bytes(nlat, ntask);
  std::vector<char> img(bytes, 0);
  std::memcpy(img.data(), lat.data(), nlat * sizeof(RwLattice));
  std::memcpy(img.data() + off_task, tasks.data(), ntask * sizeof(RwTask));
  const hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = hipMemcpyAsync(dev_work, img.data(), bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "ising_reweight: table upload");
  // the host image must outlive the copy
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "ising_reweight: table upload");
  hipLaunchKernelGGL(k_reweight, dim3(ntask), dim3(kRwThreads), 0, st, (const RwLattice*)dev_work,
                     (const RwTask*)((char*)dev_work + off_task), nblocks, dev_sums, dev_shift);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ising_reweight: launch");
  return ISING_OK;
}

ising_status ising_fss_moments(const double* sums, int32_t ntask, int32_t nblocks,
                               const int64_t* sites, double* est, double* err, double* u4_rep) {
  clear_error();
  if (!sums || !sites || !est || !err || ntask < 1 || nblocks < 2)
    return fail(ISING_EINVAL, "ising_fss_moments: bad arguments (nblocks >= 2)");
  std::vector<double> reps((size_t)nblocks * 3);
  for (int32_t k = 0; k < ntask; ++k) {
    const double* S = sums + (size_t)k * nblocks * 5;
    if (sites[k] < 1) return fail(ISING_EINVAL, "ising_fss_moments: sites[%d] < 1", k);
    const double N = (double)sites[k];
    double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t b = 0; b < nblocks; ++b)
      for (int i = 0; i < 5; ++i) tot[i] += S[b * 5 + i];
    quantities(tot, N, est + 3 * (size_t)k);
    double mean[3] = {0.0, 0.0, 0.0};
    for (int32_t b = 0; b < nblocks; ++b) {
      double R[5];
      for (int i = 0; i < 5; ++i) R[i] = tot[i] - S[b * 5 + i];
      quantities(R, N, &reps[3 * (size_t)b]);
      for (int i = 0; i < 3; ++i) mean[i] += reps[3 * (size_t)b + i];
    }
    for (int i = 0; i < 3; ++i) mean[i] /= nblocks;
    for (int i = 0; i < 3; ++i) {
      double ss = 0.0;
      for (int32_t b = 0; b < nblocks; ++b) {
        const double dv = reps[3 * (size_t)b + i] - mean[i];
        ss += dv * dv;
      }
      err[3 * (size_t)k + i] = std::sqrt((double)(nblocks - 1) / nblocks * ss);
    }
    if (u4_rep)
      for (int32_t b = 0; b < nblocks; ++b) u4_rep[(size_t)k * nblocks + b] = reps[3 * (size_t)b];
  }
  return ISING_OK;
}

ising_status ising_autocorr_time(const double* x, int64_t n, double c, double* tau,
                                 int64_t* window) {
  clear_error();
  if (!x || n < 2 || !tau || !window || !(c > 0.0) || !std::isfinite(c))
    return fail(ISING_EINVAL, "ising_autocorr_time: bad arguments (n >= 2, c > 0)");
  if (n > (int64_t(1) << 28)) return fail(ISING_EINVAL, "ising_autocorr_time: n > 2^28");
  double mean = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(x[i])) return fail(ISING_EINVAL, "ising_autocorr_time: x[%lld] not finite",
                                          (long long)i);
    mean += x[i];
  }
  mean /= (double)n;
  // sums S(t) = sum_{i < n - t} y_i y_{i+t} for all t at once: the inverse
  // transform of |FFT(y)|^2, zero-padded to avoid wrap-around
  size_t m = 1;
  while (m < 2 * (size_t)n) m <<= 1;
  std::vector<std::complex<double>> a(m, std::complex<double>(0.0, 0.0));
  double c0 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double y = x[i] - mean;
    a[i] = y;
    c0 += y * y;
  }
  c0 /= (double)n;
  if (c0 == 0.0) {
    *tau = 0.5;
    *window = 0;
    return ISING_OK;
  }
  fft(a, -1);
  for (size_t k = 0; k < m; ++k) a[k] = std::complex<double>(std::norm(a[k]), 0.0);
  fft(a, +1);
  double t = 0.5;
  for (int64_t W = 1; W <= n / 2; ++W) {
    t += a[W].real() / (double)m / (double)(n - W) / c0;
    if ((double)W >= c * t) {
      *tau = t;
      *window = W;
      return ISING_OK;
    }
  }
  *tau = t;
  *window = -1;
  return ISING_OK;
}

ising_status ising_binder_crossing(const double* T, int32_t K, const double* Ua,
                                   const double* Ub, const double* Ua_rep, const double* Ub_rep,
                                   int32_t nblocks, double* out) {
  clear_error();
  if (!T || !Ua || !Ub || !out || K < 2 || ((Ua_rep || Ub_rep) && (!Ua_rep || !Ub_rep)) ||
      ((Ua_rep != nullptr) && nblocks < 2))
    return fail(ISING_EINVAL, "ising_binder_crossing: bad arguments");
  for (int32_t k = 0; k + 1 < K; ++k)
    if (!(T[k] < T[k + 1])) return fail(ISING_EINVAL, "ising_binder_crossing: T not ascending");
  crossing(T, K, Ua, Ub, &out[0], &out[1]);
  const double nan = std::numeric_limits<double>::quiet_NaN();
  out[2] = out[3] = nan;
  if (!Ua_rep) return ISING_OK;
  std::vector<double> tx((size_t)nblocks), ux((size_t)nblocks);
  double mt = 0.0, mu = 0.0;
  for (int32_t b = 0; b < nblocks; ++b) {
    crossing(T, K, Ua_rep + (size_t)b * K, Ub_rep + (size_t)b * K, &tx[b], &ux[b]);
    if (std::isnan(tx[b])) return ISING_OK;
    mt += tx[b];
    mu += ux[b];
  }
  mt /= nblocks;
  mu /= nblocks;
  double st = 0.0, su = 0.0;
  for (int32_t b = 0; b < nblocks; ++b) {
    st += (tx[b] - mt) * (tx[b] - mt);
    su += (ux[b] - mu) * (ux[b] - mu);
  }
  out[2] = std::sqrt((double)(nblocks - 1) / nblocks * st);
  out[3] = std::sqrt((double)(nblocks - 1) / nblocks * su);
  return ISING_OK;
}

}  // extern "C"
