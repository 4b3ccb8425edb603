/*
 * Multi-spin-coded CPU baseline of the checkerboard Metropolis sweep of the
 * 2D Ising model (J = 1, no field, periodic L x L lattice).
 *
 * The paper measures its GPU speed-ups against an optimised multi-spin-coded
 * CPU program (section 4 for the coding, section 5.4 for the comparison), not
 * against a byte-per-spin code.  This file is that kind of CPU program, so
 * that the GPU's throughput can be stated against a fair CPU reference on the
 * same host.  It is a measurement baseline only: the GPU library never calls
 * it, and it shares no code with the GPU library or with the oracle.
 *
 * It computes exactly the same Markov chain as the GPU library and the
 * oracle (tested bit for bit against the oracle):
 *   - storage: one bit per spin (set = +1), 64 spins per word, the two
 *     checkerboard colours in separate planes (section 4); colour-c row y
 *     holds the sites x = 2k + ((y + c) & 1), k = 0 .. L/2 - 1, bit k % 64
 *     of word k / 64; padding bits of a row's last word stay zero;
 *   - a sweep updates colour 0 (x + y even) and then colour 1 (section 3);
 *   - a site with k anti-aligned neighbours has dE = 8 - 4k (Eq. 1); it flips
 *     if k >= 2, else if u < t(dE) with t(dE) = min(floor(exp(-beta dE) 2^32),
 *     2^32 - 1) (Eq. 3 with a 32-bit uniform u);
 *   - u for the site with colour-local index i = y L/2 + floor(x/2) in sweep
 *     t is output i mod 4 of Philox4x32-10 (Salmon et al., SC'11) with key
 *     (lo32 seed, hi32 seed) and counter (lo32 i/4, hi32 i/4, t,
 *     4 stream_id + colour); the hot start draws with phase 2 + colour at
 *     t = 0 and sets the spin iff u < 2^31;
 *   - after each sweep E = 2A - 2N and M = 2P - N, with A the anti-aligned
 *     bonds (counted from the colour-1 end of every bond) and P the up spins.
 *
 * Philox blocks are evaluated 16 at a time in AVX-512 registers (one word's
 * 64 sites) when the CPU has AVX-512 and L is a multiple of 8; otherwise a
 * scalar Philox is used.  Rows of one colour are independent and are shared
 * among OpenMP threads.
 */
#include <immintrin.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

typedef struct {
  int64_t L, W;         /* side; words per colour row */
  int nb_last;          /* sites in the last word of a row (1 .. 64) */
  uint64_t last_valid;  /* mask of those sites */
  uint32_t k0, k1;      /* Philox key */
  uint32_t sid4;        /* stream_id << 2 */
  int vector;           /* 1: AVX-512 Philox (L % 8 == 0 and the CPU has it) */
} msc_ctx;

static int g_scalar_only = 0; /* set by msc_scalar_only(): tests of the scalar Philox */

static void ctx_make(msc_ctx* x, int64_t L, uint64_t seed, uint32_t stream_id) {
  x->L = L;
  x->W = (L / 2 + 63) / 64;
  x->nb_last = (int)(L / 2 - 64 * (x->W - 1));
  x->last_valid = x->nb_last == 64 ? ~0ull : ((1ull << x->nb_last) - 1);
  x->k0 = (uint32_t)seed;
  x->k1 = (uint32_t)(seed >> 32);
  x->sid4 = stream_id << 2;
  x->vector = !g_scalar_only && (L % 8 == 0) && __builtin_cpu_supports("avx512f") &&
              __builtin_cpu_supports("avx512dq") && __builtin_cpu_supports("bmi2");
}

/* threshold of Eq. (3) for energy change dE, as a 32-bit integer */
static uint32_t threshold(double beta, int dE) {
  if (isinf(beta)) return 0;
  const double p = exp(-(double)dE * beta);
  if (!(p < 1.0)) return 0xFFFFFFFFu;
  return (uint32_t)floor(p * 4294967296.0);
}

/* ---- scalar Philox4x32-10 ---- */
static inline void philox_block(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    const uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    const uint32_t x0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t x2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = x0;
    c[2] = x2;
  }
}

/* Comparison masks of word (y, w): bit s of *ra is [u < ta] for the word's
 * site s, likewise *rb with tb (any L). */
static void masks_scalar(const msc_ctx* x, int64_t y, int64_t w, uint32_t t, uint32_t phase,
                         uint32_t ta, uint32_t tb, uint64_t* ra, uint64_t* rb) {
  const uint64_t i0 = (uint64_t)y * (uint64_t)(x->L / 2) + 64u * (uint64_t)w;
  const int n = (w == x->W - 1) ? x->nb_last : 64;
  uint64_t a = 0, b = 0, have = ~0ull;
  uint32_t blk[4] = {0, 0, 0, 0};
  for (int s = 0; s < n; ++s) {
    const uint64_t i = i0 + (uint64_t)s;
    const uint64_t g = i >> 2;
    if (g != have) {
      blk[0] = (uint32_t)g;
      blk[1] = (uint32_t)(g >> 32);
      blk[2] = t;
      blk[3] = x->sid4 | phase;
      philox_block(blk, x->k0, x->k1);
      have = g;
    }
    const uint32_t u = blk[i & 3];
    a |= (uint64_t)(u < ta) << s;
    b |= (uint64_t)(u < tb) << s;
  }
  *ra = a;
  *rb = b;
}

/* ---- 16 Philox blocks in AVX-512 registers ---- */
#define MSC_AVX512 __attribute__((target("avx512f,avx512dq,bmi2")))

/* 32 x 32 -> 64-bit products of 16 lanes: low and high halves */
static inline MSC_AVX512 void mul16(__m512i m, __m512i c, __m512i* lo, __m512i* hi) {
  const __m512i pe = _mm512_mul_epu32(c, m);                         /* lanes 0, 2, .. */
  const __m512i po = _mm512_mul_epu32(_mm512_srli_epi64(c, 32), m);  /* lanes 1, 3, .. */
  *lo = _mm512_mask_blend_epi32((__mmask16)0xAAAA, pe, _mm512_slli_epi64(po, 32));
  *hi = _mm512_mask_blend_epi32((__mmask16)0xAAAA, _mm512_srli_epi64(pe, 32), po);
}

/* L % 8 == 0: the word's sites 4q + j (q < 16, j < 4) take output j of
 * block g0 + q. */
static MSC_AVX512 void masks_avx512(const msc_ctx* x, uint64_t g0, uint32_t t, uint32_t phase,
                                    uint32_t ta, uint32_t tb, uint64_t* ra, uint64_t* rb) {
  const __m512i q = _mm512_setr_epi32(0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
  __m512i c0 = _mm512_add_epi32(_mm512_set1_epi32((int)(uint32_t)g0), q);
  const __mmask16 wrapped = _mm512_cmplt_epu32_mask(c0, q); /* low word passed 2^32 */
  const __m512i hi = _mm512_set1_epi32((int)(uint32_t)(g0 >> 32));
  __m512i c1 = _mm512_mask_add_epi32(hi, wrapped, hi, _mm512_set1_epi32(1));
  __m512i c2 = _mm512_set1_epi32((int)t);
  __m512i c3 = _mm512_set1_epi32((int)(x->sid4 | phase));
  const __m512i m0 = _mm512_set1_epi32((int)PHILOX_M0);
  const __m512i m1 = _mm512_set1_epi32((int)PHILOX_M1);
  uint32_t k0 = x->k0, k1 = x->k1;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    __m512i lo0, hi0, lo1, hi1;
    mul16(m0, c0, &lo0, &hi0);
    mul16(m1, c2, &lo1, &hi1);
    /* 0x96: three-way exclusive or */
    c0 = _mm512_ternarylogic_epi32(hi1, c1, _mm512_set1_epi32((int)k0), 0x96);
    c2 = _mm512_ternarylogic_epi32(hi0, c3, _mm512_set1_epi32((int)k1), 0x96);
    c1 = lo1;
    c3 = lo0;
  }
  const __m512i A = _mm512_set1_epi32((int)ta), B = _mm512_set1_epi32((int)tb);
  const uint64_t sel = 0x1111111111111111ull; /* bit 4q of each nibble */
  *ra = _pdep_u64(_mm512_cmplt_epu32_mask(c0, A), sel) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c1, A), sel << 1) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c2, A), sel << 2) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c3, A), sel << 3);
  *rb = _pdep_u64(_mm512_cmplt_epu32_mask(c0, B), sel) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c1, B), sel << 1) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c2, B), sel << 2) |
        _pdep_u64(_mm512_cmplt_epu32_mask(c3, B), sel << 3);
}

static inline void word_masks(const msc_ctx* x, int64_t y, int64_t w, uint32_t t, uint32_t phase,
                              uint32_t ta, uint32_t tb, uint64_t* ra, uint64_t* rb) {
  if (x->vector)
    masks_avx512(x, (uint64_t)y * (uint64_t)(x->L / 8) + 16u * (uint64_t)w, t, phase, ta, tb, ra,
                 rb);
  else
    masks_scalar(x, y, w, t, phase, ta, tb, ra, rb);
}

/* One row of one colour step.  Adds the row's anti-aligned bonds and up
 * spins to *A, *P when `count` (colour 1 only). */
static void row_step(const msc_ctx* x, uint64_t* planes, int64_t y, int c, uint32_t t,
                     uint32_t t4, uint32_t t8, int count, int64_t* A, int64_t* P) {
  const int64_t L = x->L, W = x->W;
  uint64_t* self = planes + (int64_t)c * L * W + y * W;
  const uint64_t* other = planes + (int64_t)(1 - c) * L * W;
  const uint64_t* o0 = other + y * W;
  const uint64_t* up = other + (y == 0 ? L - 1 : y - 1) * W;
  const uint64_t* dn = other + (y == L - 1 ? 0 : y + 1) * W;
  /* the horizontal partner of site k is the other colour's site k - 1 when
   * (y + c) is even, else site k + 1 (periodic in k) */
  const int left = ((y + c) & 1) == 0;
  int64_t a_sum = 0, p_sum = 0;
  for (int64_t w = 0; w < W; ++w) {
    const int last = w == W - 1;
    const uint64_t valid = last ? x->last_valid : ~0ull;
    const uint64_t s = self[w], n0 = o0[w], n2 = up[w], n3 = dn[w];
    uint64_t n1;
    if (left) {
      const uint64_t in = w > 0 ? (o0[w - 1] >> 63) : ((o0[W - 1] >> (x->nb_last - 1)) & 1u);
      n1 = (n0 << 1) | in;
    } else {
      const uint64_t in = (last ? o0[0] : o0[w + 1]) & 1u;
      n1 = (n0 >> 1) | (in << (last ? x->nb_last - 1 : 63));
    }
    uint64_t r4, r8;
    word_masks(x, y, w, t, (uint32_t)c, t4, t8, &r4, &r8);
    /* anti-aligned neighbour count k, bit-sliced over the 64 sites */
    const uint64_t a0 = s ^ n0, a1 = s ^ n1, a2 = s ^ n2, a3 = s ^ n3;
    const uint64_t two_plus = (a0 & a1) | (a2 & a3) | ((a0 ^ a1) & (a2 ^ a3));
    const uint64_t some = a0 | a1 | a2 | a3;
    const uint64_t exactly_one = some & ~two_plus;
    const uint64_t none = ~some;
    const uint64_t flip = (two_plus | (exactly_one & r4) | (none & r8)) & valid;
    const uint64_t sn = s ^ flip;
    self[w] = sn;
    if (count) {
      a_sum += __builtin_popcountll(sn ^ n0) + __builtin_popcountll((sn ^ n1) & valid) +
               __builtin_popcountll(sn ^ n2) + __builtin_popcountll(sn ^ n3);
      p_sum += __builtin_popcountll(sn) + __builtin_popcountll(n0);
    }
  }
  *A += a_sum;
  *P += p_sum;
}

/* ---- Boltzmann-pattern pools (section 4: the paper's own CPU program
 * reads exp4 / exp8 patterns from a pool at a random address) ----
 * The pool holds P = 2^m patterns of 64 sites, each stored here as the
 * pair (r4, r8) = (exp4 | exp8, exp8): bit b of pattern p compares the
 * uniform of index 64 p + b (counter (lo32, hi32 of (64 p + b) / 4,
 * 2^32 - 1, stream_id << 2 | 2)) with t4 and t8.  In sweep t, colour c,
 * word j = y W + w reads pattern v >> (32 - m), v = output 0 of the block
 * with counter (lo32 j, hi32 j, t, stream_id << 2 | c); with linear reads
 * v comes from the block of q = j / 256 and the word reads pattern
 * ((v >> (32 - m)) + j mod 256) mod P.  The same dynamics as the GPU
 * library's ISING_RNG_POOL / ISING_RNG_POOL_LINEAR. */

/* Output 0 of the Philox block with counter (lo32 q, hi32 q, t, word3). */
static inline uint32_t philox_x0(const msc_ctx* x, uint64_t q, uint32_t t, uint32_t word3) {
  uint32_t c[4] = {(uint32_t)q, (uint32_t)(q >> 32), t, word3};
  philox_block(c, x->k0, x->k1);
  return c[0];
}

/* 2^m patterns into pool[2 p] = r4, pool[2 p + 1] = r8.  Returns 0, or -1
 * for m outside [1, 28]. */
int msc_pool_fill(uint64_t* pool, int m, uint64_t seed, uint32_t stream_id, double beta,
                  int threads) {
  if (!pool || m < 1 || m > 28 || beta < 0 || isnan(beta)) return -1;
  msc_ctx x;
  ctx_make(&x, 128, seed, stream_id);  /* L only sets the word geometry, unused here */
  const uint32_t t4 = threshold(beta, 4), t8 = threshold(beta, 8);
  const int64_t P = (int64_t)1 << m;
  const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t p = 0; p < P; ++p) {
    uint64_t r4 = 0, r8 = 0;
    if (x.vector) {
      masks_avx512(&x, 16u * (uint64_t)p, 0xFFFFFFFFu, 2u, t4, t8, &r4, &r8);
    } else {
      for (int q = 0; q < 16; ++q) {
        uint32_t c[4] = {(uint32_t)(16 * p + q), 0u, 0xFFFFFFFFu, x.sid4 | 2u};
        philox_block(c, x.k0, x.k1);
        for (int j = 0; j < 4; ++j) {
          r4 |= (uint64_t)(c[j] < t4) << (4 * q + j);
          r8 |= (uint64_t)(c[j] < t8) << (4 * q + j);
        }
      }
    }
    pool[2 * p] = r4;
    pool[2 * p + 1] = r8;
  }
  return 0;
}

static void row_step_pool(const msc_ctx* x, uint64_t* planes, int64_t y, int c, uint32_t t,
                          const uint64_t* pool, int m, int linear, int count, int64_t* A,
                          int64_t* P) {
  const int64_t L = x->L, W = x->W;
  uint64_t* self = planes + (int64_t)c * L * W + y * W;
  const uint64_t* other = planes + (int64_t)(1 - c) * L * W;
  const uint64_t* o0 = other + y * W;
  const uint64_t* up = other + (y == 0 ? L - 1 : y - 1) * W;
  const uint64_t* dn = other + (y == L - 1 ? 0 : y + 1) * W;
  const int left = ((y + c) & 1) == 0;
  const uint32_t word3 = x->sid4 | (uint32_t)c, mask = (uint32_t)(((uint64_t)1 << m) - 1);
  uint64_t have_q = ~0ull;
  uint32_t start = 0;
  int64_t a_sum = 0, p_sum = 0;
  for (int64_t w = 0; w < W; ++w) {
    const int last = w == W - 1;
    const uint64_t valid = last ? x->last_valid : ~0ull;
    const uint64_t s = self[w], n0 = o0[w], n2 = up[w], n3 = dn[w];
    uint64_t n1;
    if (left) {
      const uint64_t in = w > 0 ? (o0[w - 1] >> 63) : ((o0[W - 1] >> (x->nb_last - 1)) & 1u);
      n1 = (n0 << 1) | in;
    } else {
      const uint64_t in = (last ? o0[0] : o0[w + 1]) & 1u;
      n1 = (n0 >> 1) | (in << (last ? x->nb_last - 1 : 63));
    }
    const uint64_t j = (uint64_t)(y * W + w);
    uint32_t a;
    if (linear) {
      if ((j >> 8) != have_q) {
        have_q = j >> 8;
        start = philox_x0(x, have_q, t, word3) >> (32 - m);
      }
      a = (start + (uint32_t)(j & 255u)) & mask;
    } else {
      a = philox_x0(x, j, t, word3) >> (32 - m);
    }
    const uint64_t r4 = pool[2 * (uint64_t)a], r8 = pool[2 * (uint64_t)a + 1];
    const uint64_t a0 = s ^ n0, a1 = s ^ n1, a2 = s ^ n2, a3 = s ^ n3;
    const uint64_t two_plus = (a0 & a1) | (a2 & a3) | ((a0 ^ a1) & (a2 ^ a3));
    const uint64_t some = a0 | a1 | a2 | a3;
    const uint64_t flip = (two_plus | (some & ~two_plus & r4) | (~some & r8)) & valid;
    const uint64_t sn = s ^ flip;
    self[w] = sn;
    if (count) {
      a_sum += __builtin_popcountll(sn ^ n0) + __builtin_popcountll((sn ^ n1) & valid) +
               __builtin_popcountll(sn ^ n2) + __builtin_popcountll(sn ^ n3);
      p_sum += __builtin_popcountll(sn) + __builtin_popcountll(n0);
    }
  }
  *A += a_sum;
  *P += p_sum;
}

/* n sweeps with a pool of 2^m patterns (msc_pool_fill for this beta);
 * linear 0: an address per word, 1: linear reads per 256-word group.
 * Returns 0, or -1 for bad arguments. */
int msc_pool_sweeps(uint64_t* planes, int64_t L, uint64_t seed, uint32_t stream_id,
                    const uint64_t* pool, int m, int linear, uint32_t t0, int64_t n, int64_t* EM,
                    int threads) {
  if (L < 4 || L % 2 || !planes || !pool || m < 1 || m > 28 || n < 0) return -1;
  msc_ctx x;
  ctx_make(&x, L, seed, stream_id);
  const int nt = threads > 0 ? threads : omp_get_max_threads();
  const int64_t N = L * L;
  for (int64_t k = 0; k < n; ++k) {
    const uint32_t t = t0 + (uint32_t)k;
    for (int c = 0; c < 2; ++c) {
      const int count = c == 1 && EM != NULL;
      int64_t A = 0, P = 0;
#pragma omp parallel for schedule(static) num_threads(nt) reduction(+ : A, P)
      for (int64_t y = 0; y < L; ++y)
        row_step_pool(&x, planes, y, c, t, pool, m, linear, count, &A, &P);
      if (count) {
        EM[2 * k] = 2 * A - 2 * N;
        EM[2 * k + 1] = 2 * P - N;
      }
    }
  }
  return 0;
}

/* Bytes of the two colour planes of an L x L lattice. */
int64_t msc_bytes(int64_t L) {
  if (L < 4 || L % 2) return 0;
  return 2 * L * ((L / 2 + 63) / 64) * 8;
}

/* Reports 1 when the AVX-512 Philox serves lattices with L % 8 == 0. */
int msc_vector_available(void) {
  return __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq") &&
         __builtin_cpu_supports("bmi2");
}

/* 1: use the scalar Philox even where the AVX-512 one could serve. */
void msc_scalar_only(int on) { g_scalar_only = on != 0; }

/* Initial state: init 0 all +1, 1 all -1, 2 hot start from (seed,
 * stream_id).  Returns 0, or -1 for bad arguments. */
int msc_init(uint64_t* planes, int64_t L, uint64_t seed, uint32_t stream_id, int init,
             int threads) {
  if (L < 4 || L % 2 || !planes || init < 0 || init > 2) return -1;
  msc_ctx x;
  ctx_make(&x, L, seed, stream_id);
  const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t r = 0; r < 2 * L; ++r) {
    const int c = r >= L;
    const int64_t y = r - c * L;
    uint64_t* row = planes + r * x.W;
    for (int64_t w = 0; w < x.W; ++w) {
      const uint64_t valid = w == x.W - 1 ? x.last_valid : ~0ull;
      if (init == 0) {
        row[w] = valid;
      } else if (init == 1) {
        row[w] = 0;
      } else {
        uint64_t m, unused;
        word_masks(&x, y, w, 0u, 2u + (uint32_t)c, 0x80000000u, 0x80000000u, &m, &unused);
        row[w] = m & valid;
      }
    }
  }
  return 0;
}

/* n sweeps starting at sweep counter t0 at inverse temperature beta; EM (if
 * not NULL) receives (E, M) after each sweep, 2 int64 per sweep.  Returns 0,
 * or -1 for bad arguments. */
int msc_sweeps(uint64_t* planes, int64_t L, uint64_t seed, uint32_t stream_id, double beta,
               uint32_t t0, int64_t n, int64_t* EM, int threads) {
  if (L < 4 || L % 2 || !planes || n < 0 || beta < 0 || isnan(beta)) return -1;
  msc_ctx x;
  ctx_make(&x, L, seed, stream_id);
  const uint32_t t4 = threshold(beta, 4), t8 = threshold(beta, 8);
  const int nt = threads > 0 ? threads : omp_get_max_threads();
  const int64_t N = L * L;
  for (int64_t k = 0; k < n; ++k) {
    const uint32_t t = t0 + (uint32_t)k;
    for (int c = 0; c < 2; ++c) {
      const int count = c == 1 && EM != NULL;
      int64_t A = 0, P = 0;
#pragma omp parallel for schedule(static) num_threads(nt) reduction(+ : A, P)
      for (int64_t y = 0; y < L; ++y) row_step(&x, planes, y, c, t, t4, t8, count, &A, &P);
      if (count) {
        EM[2 * k] = 2 * A - 2 * N;
        EM[2 * k + 1] = 2 * P - N;
      }
    }
  }
  return 0;
}

/* The comparison masks of one word as the sweeps compute them (tests):
 * out[0] bit s = [u < ta], out[1] bit s = [u < tb] for site s of colour
 * `phase & 1`, row y, word w. */
void msc_word_masks(int64_t L, uint64_t seed, uint32_t stream_id, int64_t y, int64_t w,
                    uint32_t t, uint32_t phase, uint32_t ta, uint32_t tb, uint64_t* out) {
  msc_ctx x;
  ctx_make(&x, L, seed, stream_id);
  word_masks(&x, y, w, t, phase, ta, tb, &out[0], &out[1]);
}

/* Unpack to one int8 (+1 / -1) per site, row-major [y][x]. */
void msc_get_spins(const uint64_t* planes, int64_t L, int8_t* out) {
  const int64_t W = (L / 2 + 63) / 64;
  for (int64_t y = 0; y < L; ++y)
    for (int64_t xx = 0; xx < L; ++xx) {
      const int c = (int)((xx + y) & 1);
      const int64_t k = xx / 2;
      const uint64_t word = planes[(int64_t)c * L * W + y * W + k / 64];
      out[y * L + xx] = (int8_t)(((word >> (k % 64)) & 1u) ? 1 : -1);
    }
}
