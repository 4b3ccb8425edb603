/*
 * Oracle for the checkerboard Metropolis sweep of the 2D Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, byte-per-spin
 * reference that the HIP path is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, loads or calls it, and it shares no code,
 * header, table or helper with the HIP sources.
 *
 * What it computes (B. Block, P. Virnau, T. Preis, "Multi-GPU accelerated
 * multi-spin Monte Carlo simulations of the 2D Ising model"):
 *   - Section 3, Eq. (1): H = -J sum_<ij> S_i S_j - H sum_i S_i on an L x L
 *     square lattice with periodic boundaries; here J = 1, k_B = 1, field 0.
 *   - Section 3: Metropolis acceptance W = exp(-dH/T) for dH > 0, else 1;
 *     the two possible factors (dH = 4J and 8J) are computed on the host
 *     once per temperature.
 *   - Section 3: checkerboard update, all sites of one colour (step A),
 *     then all sites of the other colour (step B), B strictly after A.
 *   - Section 4, Eq. (3): a move is accepted when a uniform r in [0,1) is
 *     strictly below the Boltzmann factor.  Here r is a 32-bit integer u and
 *     the factor is the integer threshold floor(exp(-dH/T) * 2^32), clamped
 *     to 2^32 - 1, so "r < exp(-dH/T)" becomes "u < threshold".
 *
 * Readings of points the paper leaves open:
 *   - colour of site (x, y) is (x + y) mod 2; colour 0 is updated first;
 *   - the uniforms come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by
 *     (seed, stream id, sweep, phase, site) as in oracle_uniform() below;
 *     the paper's own generator is a per-thread LCG (section 5.3);
 *   - L even and >= 4; spins are +1/-1 stored one int8 per site, row-major
 *     [y][x]; a set bit in a packed layout means +1 (section 5.2);
 *   - energy E and magnetisation M are exact int64 sums measured after each
 *     full sweep.
 *
 * Every function is written for clarity, not speed: one site at a time.
 * The only parallelism is OpenMP over rows inside one colour step, which is
 * legal because sites of one colour do not interact (section 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of                 */
/*   (hi0,lo0) = M0 * x0, (hi1,lo1) = M1 * x2,                          */
/*   x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0),                     */
/* with the key bumped by the Weyl constants between rounds.           */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Integer Metropolis threshold for an uphill move of size dE          */
/* (section 3: W = exp(-dE/T), precomputed on the host per T;         */
/*  section 4, Eq. (3): accept when r < W).                            */
/* Returns floor(exp(-beta*dE) * 2^32), clamped to 2^32 - 1.          */
/* beta must be >= 0 (may be +inf); the caller checks this.            */
/* ------------------------------------------------------------------ */
uint32_t oracle_threshold(double beta, int dE)
{
    double w = exp(-beta * (double)dE);
    double scaled = floor(ldexp(w, 32));
    if (scaled >= 4294967295.0)
        return 0xFFFFFFFFu;
    if (scaled <= 0.0)
        return 0u;
    return (uint32_t)scaled;
}

/* ------------------------------------------------------------------ */
/* The uniform used at site (x, y) in sweep t for a given phase.       */
/* Keying (the build's reading; the paper's LCG is replaced):          */
/*   colour-local index i = y * (L/2) + floor(x/2),                    */
/*   group g = floor(i / 4), lane j = i mod 4,                          */
/*   key = (lo32(seed), hi32(seed)),                                    */
/*   counter = (lo32(g), hi32(g), t, (stream_id << 2) | phase),         */
/*   u = Philox4x32-10(key, counter)[j].                                */
/* phase 0/1: update of colour 0/1 in sweep t; phase 2/3: hot start    */
/* of colour 0/1 sites (t = 0).                                        */
/* ------------------------------------------------------------------ */
uint32_t oracle_uniform(uint64_t seed, uint32_t stream_id, uint32_t phase,
                        uint32_t t, int64_t L, int64_t x, int64_t y)
{
    uint64_t i = (uint64_t)y * (uint64_t)(L / 2) + (uint64_t)(x / 2);
    uint64_t g = i >> 2;
    uint32_t j = (uint32_t)(i & 3u);
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), t, (stream_id << 2) | phase};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[j];
}

/* ------------------------------------------------------------------ */
/* Metropolis decision for one site (section 3), written with the      */
/* energy change of Eq. (1): flipping s changes H by                    */
/*   dE = 2 J s (n1 + n2 + n3 + n4),  J = 1.                            */
/* dE <= 0: always accepted; dE = 4: accepted iff u < t4;              */
/* dE = 8: accepted iff u < t8.  Returns 1 to flip, 0 to keep.         */
/* ------------------------------------------------------------------ */
int oracle_accept(int s, int n1, int n2, int n3, int n4,
                  uint32_t u, uint32_t t4, uint32_t t8)
{
    int dE = 2 * s * (n1 + n2 + n3 + n4);
    if (dE <= 0)
        return 1;
    if (dE == 4)
        return u < t4;
    /* dE == 8 */
    return u < t8;
}

static inline int64_t wrap(int64_t a, int64_t L)
{
    a %= L;
    return a < 0 ? a + L : a;
}

/* ------------------------------------------------------------------ */
/* Initial state.  init 0: all +1; init 1: all -1; init 2: hot start,  */
/* s = +1 iff the site's phase-(2 + colour) uniform at t = 0 is below  */
/* 2^31 (probability 1/2).                                              */
/* ------------------------------------------------------------------ */
void oracle_init(int64_t L, uint64_t seed, uint32_t stream_id, int init, int8_t *s)
{
    for (int64_t y = 0; y < L; ++y)
        for (int64_t x = 0; x < L; ++x) {
            int8_t v;
            if (init == 0)
                v = 1;
            else if (init == 1)
                v = -1;
            else {
                uint32_t colour = (uint32_t)((x + y) & 1);
                uint32_t u = oracle_uniform(seed, stream_id, 2u + colour, 0u, L, x, y);
                v = (u < 0x80000000u) ? 1 : -1;
            }
            s[y * L + x] = v;
        }
}

/* ------------------------------------------------------------------ */
/* Energy and magnetisation of a configuration, Eq. (1) with J = 1 and  */
/* no field: E = -sum_{x,y} s(x,y) [s(x+1,y) + s(x,y+1)] (each of the  */
/* 2 L^2 bonds once), M = sum s.                                         */
/* ------------------------------------------------------------------ */
void oracle_measure(int64_t L, const int8_t *s, int64_t *E, int64_t *M)
{
    int64_t e = 0, m = 0;
    for (int64_t y = 0; y < L; ++y)
        for (int64_t x = 0; x < L; ++x) {
            int64_t v = s[y * L + x];
            int64_t right = s[y * L + wrap(x + 1, L)];
            int64_t down = s[wrap(y + 1, L) * L + x];
            e -= v * (right + down);
            m += v;
        }
    *E = e;
    *M = m;
}

/* One colour step (section 3, step A or B) over the sites of `colour`. */
static void colour_step(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed,
                        uint32_t stream_id, uint32_t t, int colour, int8_t *s)
{
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < L; ++y) {
        for (int64_t x = (y + colour) & 1; x < L; x += 2) {
            int v = s[y * L + x];
            int n1 = s[y * L + wrap(x - 1, L)];
            int n2 = s[y * L + wrap(x + 1, L)];
            int n3 = s[wrap(y - 1, L) * L + x];
            int n4 = s[wrap(y + 1, L) * L + x];
            uint32_t u = oracle_uniform(seed, stream_id, (uint32_t)colour, t, L, x, y);
            if (oracle_accept(v, n1, n2, n3, n4, u, t4, t8))
                s[y * L + x] = (int8_t)(-v);
        }
    }
}

/* ------------------------------------------------------------------ */
/* n full sweeps starting at sweep counter t0: for each sweep t, colour */
/* 0 then colour 1 (section 3), then (E_t, M_t) into EM[2k], EM[2k+1]  */
/* (EM may be NULL).                                                    */
/* ------------------------------------------------------------------ */
void oracle_sweeps(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                   uint32_t t0, int64_t n, int8_t *s, int64_t *EM)
{
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        colour_step(L, t4, t8, seed, stream_id, t, 0, s);
        colour_step(L, t4, t8, seed, stream_id, t, 1, s);
        if (EM)
            oracle_measure(L, s, &EM[2 * k], &EM[2 * k + 1]);
    }
}

/* ================================================================== */
/* The paper's own random numbers (section 5.3), as an alternative     */
/* dynamics: one linear congruential generator per update thread,      */
/*   x_{i+1} = (1664525 x_i + 1013904223) mod 2^32            (Eq. (6)) */
/* normalised as y = |x / 2^31| with x read as a signed 32-bit integer, */
/* and thread seeds x_{0,j+1} = 16807 x_{0,j} mod 2^32       (Eq. (7)). */
/* Readings (the paper leaves the thread layout to its CUDA code):      */
/*   - a "thread" is one 64-site word of one colour: word w of row y of */
/*     colour c is thread j = (c L + y) W + w, W = ceil((L/2) / 64);    */
/*   - x_{0,0} = lo32(seed) (seed 1 gives the paper's x_{0,0} = 1);     */
/*   - each colour step advances every thread 64 times; the k-th new    */
/*     value (k = 1..64) decides colour-local site 64 w + 64 - k of its */
/*     row (site 63 of the word first); sites past L/2 use no value     */
/*     but still advance the generator;                                 */
/*   - accept an uphill move dE iff |int32(x)| < t'(dE) with            */
/*     t'(dE) = min(floor(exp(-beta dE) 2^31), 2^31).                   */
/* ================================================================== */

uint32_t oracle_lcg_threshold(double beta, int dE)
{
    double w = exp(-beta * (double)dE);
    double scaled = floor(ldexp(w, 31));
    if (scaled >= 2147483648.0)
        return 0x80000000u;
    if (scaled <= 0.0)
        return 0u;
    return (uint32_t)scaled;
}

/* Thread seeds by the recurrence of Eq. (7): state[j] for j = 0 .. 2 L W - 1. */
void oracle_lcg_seed(int64_t L, uint64_t seed, uint32_t *state)
{
    int64_t W = (L / 2 + 63) / 64;
    uint32_t x = (uint32_t)seed;
    for (int64_t j = 0; j < 2 * L * W; ++j) {
        state[j] = x;
        x = (uint32_t)((uint64_t)16807u * x);
    }
}

static void lcg_colour_step(int64_t L, uint32_t t4, uint32_t t8, int colour, int8_t *s,
                            uint32_t *state)
{
    int64_t half = L / 2, W = (L / 2 + 63) / 64;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < L; ++y) {
        for (int64_t w = 0; w < W; ++w) {
            uint32_t x = state[(colour * L + y) * W + w];
            for (int k = 1; k <= 64; ++k) {
                x = (uint32_t)((uint64_t)1664525u * x + 1013904223u);
                int64_t site = 64 * w + 64 - k;       /* colour-local index in the row */
                if (site >= half)
                    continue;
                int64_t px = 2 * site + ((y + colour) & 1);
                int32_t sx = (int32_t)x;
                uint32_t u = (uint32_t)(sx < 0 ? -(int64_t)sx : (int64_t)sx);
                int v = s[y * L + px];
                int n1 = s[y * L + wrap(px - 1, L)];
                int n2 = s[y * L + wrap(px + 1, L)];
                int n3 = s[wrap(y - 1, L) * L + px];
                int n4 = s[wrap(y + 1, L) * L + px];
                if (oracle_accept(v, n1, n2, n3, n4, u, t4, t8))
                    s[y * L + px] = (int8_t)(-v);
            }
            state[(colour * L + y) * W + w] = x;
        }
    }
}

/* n sweeps with the per-thread LCG: colour 0 then colour 1, then       */
/* (E, M) into EM (may be NULL).  t4, t8 from oracle_lcg_threshold.     */
void oracle_lcg_sweeps(int64_t L, uint32_t t4, uint32_t t8, int64_t n, int8_t *s,
                       uint32_t *state, int64_t *EM)
{
    for (int64_t k = 0; k < n; ++k) {
        lcg_colour_step(L, t4, t8, 0, s, state);
        lcg_colour_step(L, t4, t8, 1, s, state);
        if (EM)
            oracle_measure(L, s, &EM[2 * k], &EM[2 * k + 1]);
    }
}

/* ================================================================== */
/* Boltzmann-pattern pools (section 4, and the "unmodified" and        */
/* "linear" GPU variants of section 5.1 / Table 2): instead of one     */
/* uniform per site, an update reads two precomputed bit patterns from */
/* a pool at a random address.  Pattern bit b is, for its own uniform  */
/* r, exp8 = [r < exp(-8 beta)] and exp4 = [exp(-8 beta) <= r <        */
/* exp(-4 beta)], and a site with k anti-aligned neighbours flips iff   */
/* k + 2 exp8 + exp4 >= 2 (Eq. (5)).                                    */
/* Readings (the paper leaves these to its code):                       */
/*   - one pattern covers one 64-site word of a colour row: word w of   */
/*     row y is j = y W + w, W = ceil((L/2) / 64), and site 64 w + b of */
/*     the row reads bit b;                                             */
/*   - the pool holds P = 2^m patterns; pattern p's bit b takes the      */
/*     uniform u of index i = 64 p + b: Philox4x32-10 with the lattice's */
/*     key and counter (lo32 i/4, hi32 i/4, 2^32 - 1, (stream_id << 2)  */
/*     | 2), output i mod 4 (a counter no sweep or start uses); exp8 =  */
/*     [u < t8], exp4 = [t8 <= u < t4] with the integer thresholds of   */
/*     oracle_threshold; the pool is drawn again when beta changes;     */
/*   - "random" (each update draws its own address): in sweep t,        */
/*     colour c, word j reads pattern v >> (32 - m), v = output 0 of     */
/*     Philox4x32-10 with counter (lo32 j, hi32 j, t, (stream_id << 2)  */
/*     | c);                                                             */
/*   - "linear" (one random start per block of threads, which then read */
/*     consecutive patterns): words are grouped by q = floor(j / 256);  */
/*     the group draws v as above with counter (lo32 q, hi32 q, t,      */
/*     (stream_id << 2) | c), and word j reads pattern                  */
/*     ((v >> (32 - m)) + j mod 256) mod P.                             */
/* ================================================================== */

/* Pool of 2^m patterns: bit b of e8[p] / e4[p] is exp8 / exp4 of pattern p. */
void oracle_pool_fill(uint64_t seed, uint32_t stream_id, uint32_t t4, uint32_t t8, int m,
                      uint64_t *e4, uint64_t *e8)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t P = (int64_t)1 << m;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        uint64_t a4 = 0, a8 = 0;
        for (int b = 0; b < 64; ++b) {
            uint64_t i = 64 * (uint64_t)p + (uint64_t)b, g = i / 4;
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), 0xFFFFFFFFu,
                               (stream_id << 2) | 2u};
            uint32_t out[4];
            oracle_philox4x32_10(ctr, key, out);
            uint32_t u = out[i % 4];
            if (u < t8)
                a8 |= 1ull << b;
            else if (u < t4)
                a4 |= 1ull << b;
        }
        e4[p] = a4;
        e8[p] = a8;
    }
}

/* Pool address read by word j in sweep t, colour c (see above). */
uint32_t oracle_pool_address(uint64_t seed, uint32_t stream_id, uint32_t t, int colour, int m,
                             int linear, uint64_t j)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t q = linear ? j / 256 : j;
    uint32_t ctr[4] = {(uint32_t)q, (uint32_t)(q >> 32), t, (stream_id << 2) | (uint32_t)colour};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    uint32_t a = out[0] >> (32 - m);
    if (linear)
        a = (uint32_t)((a + j % 256) & (((uint64_t)1 << m) - 1));
    return a;
}

static void pool_colour_step(int64_t L, const uint64_t *e4, const uint64_t *e8, int m,
                             int linear, uint64_t seed, uint32_t stream_id, uint32_t t,
                             int colour, int8_t *s)
{
    int64_t W = (L / 2 + 63) / 64;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < L; ++y) {
        for (int64_t x = (y + colour) & 1; x < L; x += 2) {
            int64_t k = x / 2;                          /* colour-local site of the row */
            uint64_t j = (uint64_t)(y * W + k / 64);
            uint32_t a = oracle_pool_address(seed, stream_id, t, colour, m, linear, j);
            int exp8 = (int)((e8[a] >> (k % 64)) & 1u);
            int exp4 = (int)((e4[a] >> (k % 64)) & 1u);
            int v = s[y * L + x];
            int anti = (s[y * L + wrap(x - 1, L)] != v) + (s[y * L + wrap(x + 1, L)] != v) +
                       (s[wrap(y - 1, L) * L + x] != v) + (s[wrap(y + 1, L) * L + x] != v);
            if (anti + 2 * exp8 + exp4 >= 2)            /* Eq. (5) */
                s[y * L + x] = (int8_t)(-v);
        }
    }
}

/* n sweeps from sweep counter t0 with a pool of 2^m patterns drawn for  */
/* (t4, t8); linear 0: an address per word, 1: per 256-word group.      */
/* (E, M) into EM after each sweep (may be NULL).  Returns 0, or -1 if  */
/* m is outside [1, 30] or the pool cannot be allocated.                */
int oracle_pool_sweeps(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                       uint32_t t0, int64_t n, int m, int linear, int8_t *s, int64_t *EM)
{
    if (m < 1 || m > 30)
        return -1;
    int64_t P = (int64_t)1 << m;
    uint64_t *e4 = (uint64_t *)malloc((size_t)P * sizeof(uint64_t));
    uint64_t *e8 = (uint64_t *)malloc((size_t)P * sizeof(uint64_t));
    if (!e4 || !e8) {
        free(e4);
        free(e8);
        return -1;
    }
    oracle_pool_fill(seed, stream_id, t4, t8, m, e4, e8);
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        pool_colour_step(L, e4, e8, m, linear, seed, stream_id, t, 0, s);
        pool_colour_step(L, e4, e8, m, linear, seed, stream_id, t, 1, s);
        if (EM)
            oracle_measure(L, s, &EM[2 * k], &EM[2 * k + 1]);
    }
    free(e4);
    free(e8);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Light-cone window.  After n sweeps a site depends only on the       */
/* initial spins and uniforms within Manhattan distance 2n (one site   */
/* per colour step).  This simulates the patch of global coordinates   */
/* [x0 - m, x0 + w + m) x [y0 - m, y0 + h + m) (periodic in L) with     */
/* m = 2n + 1, keeping the outermost ring frozen, and returns the inner */
/* w x h window, which then equals the full-lattice result exactly.     */
/* The uniforms are keyed by global coordinates.  Requires w + 2m <= L  */
/* and h + 2m <= L (otherwise run oracle_sweeps on the whole lattice).  */
/* Returns 0 on success, -1 on a size error.                            */
/* ------------------------------------------------------------------ */
int oracle_window(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                  int init, uint32_t t0, int64_t n, int64_t x0, int64_t y0,
                  int64_t w, int64_t h, int8_t *out)
{
    int64_t m = 2 * n + 1;
    int64_t pw = w + 2 * m, ph = h + 2 * m;
    if (pw > L || ph > L || w <= 0 || h <= 0)
        return -1;
    int8_t *p = (int8_t *)malloc((size_t)(pw * ph));
    if (!p)
        return -1;
    /* initial state at global coordinates */
    for (int64_t j = 0; j < ph; ++j)
        for (int64_t i = 0; i < pw; ++i) {
            int64_t gx = wrap(x0 - m + i, L), gy = wrap(y0 - m + j, L);
            int8_t v;
            if (init == 0)
                v = 1;
            else if (init == 1)
                v = -1;
            else {
                uint32_t colour = (uint32_t)((gx + gy) & 1);
                uint32_t u = oracle_uniform(seed, stream_id, 2u + colour, 0u, L, gx, gy);
                v = (u < 0x80000000u) ? 1 : -1;
            }
            p[j * pw + i] = v;
        }
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 1; j < ph - 1; ++j) {
                for (int64_t i = 1; i < pw - 1; ++i) {
                    int64_t gx = wrap(x0 - m + i, L), gy = wrap(y0 - m + j, L);
                    if (((gx + gy) & 1) != colour)
                        continue;
                    int v = p[j * pw + i];
                    int n1 = p[j * pw + i - 1];
                    int n2 = p[j * pw + i + 1];
                    int n3 = p[(j - 1) * pw + i];
                    int n4 = p[(j + 1) * pw + i];
                    uint32_t u = oracle_uniform(seed, stream_id, (uint32_t)colour, t, L, gx, gy);
                    if (oracle_accept(v, n1, n2, n3, n4, u, t4, t8))
                        p[j * pw + i] = (int8_t)(-v);
                }
            }
        }
    }
    for (int64_t j = 0; j < h; ++j)
        memcpy(out + j * w, p + (j + m) * pw + m, (size_t)w);
    free(p);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Band of rows: energy and magnetisation contributions of the rows    */
/* [y0, y0 + h) (periodic in L) after each of n sweeps from a fresh     */
/* start, without holding the whole lattice.  It is the light-cone      */
/* argument of oracle_window applied to full rows: the band is          */
/* simulated with m = 2n + 1 extra rows above and below (x is periodic  */
/* over the full width, so no column margin is needed), the outermost   */
/* row at each end stays frozen, and after sweep k (k = 1 .. n) rows   */
/* more than 2k rows from a frozen row equal the full-lattice result.   */
/* The inner rows and the row just below them are such rows for every  */
/* k <= n.  EM[2(k-1)] receives the band's share of Eq. (1),            */
/*   -sum_{y in band} sum_x s(x,y) [s(x+1,y) + s(x,y+1)],               */
/* (each bond counted at its left or upper end, as oracle_measure       */
/* does), and EM[2(k-1)+1] the band's sum of spins.  Bands that         */
/* partition the rows of the lattice therefore sum to the (E, M) of     */
/* oracle_measure.  Requires h + 2m <= L.  Returns 0, or -1 on a size    */
/* or allocation error.                                                 */
/* ------------------------------------------------------------------ */
int oracle_band_em(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                   int init, uint32_t t0, int64_t n, int64_t y0, int64_t h, int64_t *EM)
{
    int64_t m = 2 * n + 1;
    int64_t ph = h + 2 * m;
    if (ph > L || h <= 0 || n < 0 || L < 4 || (L & 1))
        return -1;
    int8_t *p = (int8_t *)malloc((size_t)(ph * L));
    if (!p)
        return -1;
    /* initial state of the patch rows, at global coordinates */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ph; ++j) {
        int64_t gy = wrap(y0 - m + j, L);
        for (int64_t x = 0; x < L; ++x) {
            int8_t v;
            if (init == 0)
                v = 1;
            else if (init == 1)
                v = -1;
            else {
                uint32_t colour = (uint32_t)((x + gy) & 1);
                uint32_t u = oracle_uniform(seed, stream_id, 2u + colour, 0u, L, x, gy);
                v = (u < 0x80000000u) ? 1 : -1;
            }
            p[j * L + x] = v;
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 1; j < ph - 1; ++j) {
                int64_t gy = wrap(y0 - m + j, L);
                for (int64_t x = (gy + colour) & 1; x < L; x += 2) {
                    int v = p[j * L + x];
                    int n1 = p[j * L + wrap(x - 1, L)];
                    int n2 = p[j * L + wrap(x + 1, L)];
                    int n3 = p[(j - 1) * L + x];
                    int n4 = p[(j + 1) * L + x];
                    uint32_t u = oracle_uniform(seed, stream_id, (uint32_t)colour, t, L, x, gy);
                    if (oracle_accept(v, n1, n2, n3, n4, u, t4, t8))
                        p[j * L + x] = (int8_t)(-v);
                }
            }
        }
        int64_t e = 0, s = 0;
#pragma omp parallel for schedule(static) reduction(+ : e, s)
        for (int64_t j = m; j < m + h; ++j)
            for (int64_t x = 0; x < L; ++x) {
                int64_t v = p[j * L + x];
                e -= v * (p[j * L + wrap(x + 1, L)] + p[(j + 1) * L + x]);
                s += v;
            }
        EM[2 * k] = e;
        EM[2 * k + 1] = s;
    }
    free(p);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Light-cone windows of the two alternative dynamics.  The argument of */
/* oracle_window holds for them too: a site's update reads its four    */
/* neighbours and a random decision that does not depend on any spin   */
/* (a pool pattern at an address keyed by the global word index and    */
/* the sweep, or the next draw of its word's generator), so after n     */
/* sweeps the inner window of a patch with margin m = 2n + 1 (outer     */
/* ring frozen) equals the whole lattice exactly.  Requires w + 2m <= L */
/* and h + 2m <= L; 0 on success, -1 on a size or memory error.         */
/* ------------------------------------------------------------------ */

/* initial spins of the patch [x0 - m, x0 - m + pw) x [y0 - m, y0 - m + ph) */
static void patch_init(int64_t L, uint64_t seed, uint32_t stream_id, int init, int64_t x0,
                       int64_t y0, int64_t m, int64_t pw, int64_t ph, int8_t *p)
{
    for (int64_t j = 0; j < ph; ++j)
        for (int64_t i = 0; i < pw; ++i) {
            int64_t gx = wrap(x0 - m + i, L), gy = wrap(y0 - m + j, L);
            int8_t v;
            if (init == 0)
                v = 1;
            else if (init == 1)
                v = -1;
            else {
                uint32_t colour = (uint32_t)((gx + gy) & 1);
                uint32_t u = oracle_uniform(seed, stream_id, 2u + colour, 0u, L, gx, gy);
                v = (u < 0x80000000u) ? 1 : -1;
            }
            p[j * pw + i] = v;
        }
}

static int anti_aligned(const int8_t *p, int64_t pw, int64_t i, int64_t j)
{
    int v = p[j * pw + i];
    return (p[j * pw + i - 1] != v) + (p[j * pw + i + 1] != v) + (p[(j - 1) * pw + i] != v) +
           (p[(j + 1) * pw + i] != v);
}

/* Pattern-pool dynamics (see oracle_pool_sweeps): n sweeps from sweep     */
/* counter t0 with the pool (e4, e8) of 2^m patterns.                     */
int oracle_pool_window(int64_t L, uint64_t seed, uint32_t stream_id, int init, uint32_t t0,
                       int64_t n, int m_pool, int linear, const uint64_t *e4,
                       const uint64_t *e8, int64_t x0, int64_t y0, int64_t w, int64_t h,
                       int8_t *out)
{
    int64_t m = 2 * n + 1;
    int64_t pw = w + 2 * m, ph = h + 2 * m;
    int64_t W = (L / 2 + 63) / 64;
    if (pw > L || ph > L || w <= 0 || h <= 0 || m_pool < 1 || m_pool > 30)
        return -1;
    int8_t *p = (int8_t *)malloc((size_t)(pw * ph));
    if (!p)
        return -1;
    patch_init(L, seed, stream_id, init, x0, y0, m, pw, ph, p);
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t j = 1; j < ph - 1; ++j)
                for (int64_t i = 1; i < pw - 1; ++i) {
                    int64_t gx = wrap(x0 - m + i, L), gy = wrap(y0 - m + j, L);
                    if (((gx + gy) & 1) != colour)
                        continue;
                    int64_t site = gx / 2;                /* colour-local index in the row */
                    uint64_t word = (uint64_t)(gy * W + site / 64);
                    uint32_t a = oracle_pool_address(seed, stream_id, t, colour, m_pool, linear,
                                                     word);
                    int exp8 = (int)((e8[a] >> (site % 64)) & 1u);
                    int exp4 = (int)((e4[a] >> (site % 64)) & 1u);
                    if (anti_aligned(p, pw, i, j) + 2 * exp8 + exp4 >= 2)  /* Eq. (5) */
                        p[j * pw + i] = (int8_t)(-p[j * pw + i]);
                }
        }
    }
    for (int64_t j = 0; j < h; ++j)
        memcpy(out + j * w, p + (j + m) * pw + m, (size_t)w);
    free(p);
    return 0;
}

/* 16807^e mod 2^32 by square and multiply (thread seeds of Eq. (7)). */
static uint32_t pow16807(uint64_t e)
{
    uint32_t r = 1u, b = 16807u;
    while (e) {
        if (e & 1u)
            r = (uint32_t)((uint64_t)r * b);
        b = (uint32_t)((uint64_t)b * b);
        e >>= 1;
    }
    return r;
}

/* Per-thread-LCG dynamics (see oracle_lcg_sweeps), n sweeps from the     */
/* thread seeds of oracle_lcg_seed (sweep 0).  Every word a patch row     */
/* touches keeps its own generator: state (colour L + y) W + w starts at  */
/* seed 16807^((colour L + y) W + w) and makes its 64 draws per colour    */
/* step whether or not its sites lie in the patch.                        */
int oracle_lcg_window(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                      int init, int64_t n, int64_t x0, int64_t y0, int64_t w, int64_t h,
                      int8_t *out)
{
    int64_t m = 2 * n + 1;
    int64_t pw = w + 2 * m, ph = h + 2 * m;
    int64_t half = L / 2, W = (L / 2 + 63) / 64;
    if (pw > L || ph > L || w <= 0 || h <= 0)
        return -1;
    int8_t *p = (int8_t *)malloc((size_t)(pw * ph));
    /* words of each (colour, patch row): at most pw / 128 + 2 per row */
    int64_t per = pw / 128 + 3;
    int64_t *wid = (int64_t *)malloc((size_t)(2 * ph * per) * sizeof(int64_t));
    uint32_t *st = (uint32_t *)malloc((size_t)(2 * ph * per) * sizeof(uint32_t));
    int64_t *cnt = (int64_t *)calloc((size_t)(2 * ph), sizeof(int64_t));
    if (!p || !wid || !st || !cnt) {
        free(p);
        free(wid);
        free(st);
        free(cnt);
        return -1;
    }
    patch_init(L, seed, stream_id, init, x0, y0, m, pw, ph, p);
    for (int colour = 0; colour < 2; ++colour)
        for (int64_t j = 1; j < ph - 1; ++j) {
            int64_t gy = wrap(y0 - m + j, L), r = colour * ph + j;
            for (int64_t i = 1; i < pw - 1; ++i) {
                int64_t gx = wrap(x0 - m + i, L);
                if (((gx + gy) & 1) != colour)
                    continue;
                int64_t word = (gx / 2) / 64, seen = 0;
                for (int64_t q = 0; q < cnt[r]; ++q)
                    seen |= wid[r * per + q] == word;
                if (!seen) {
                    wid[r * per + cnt[r]] = word;
                    st[r * per + cnt[r]] =
                        (uint32_t)((uint64_t)(uint32_t)seed *
                                   pow16807((uint64_t)((colour * L + gy) * W + word)));
                    ++cnt[r];
                }
            }
        }
    for (int64_t k = 0; k < n; ++k)
        for (int colour = 0; colour < 2; ++colour)
            for (int64_t j = 1; j < ph - 1; ++j) {
                int64_t gy = wrap(y0 - m + j, L), r = colour * ph + j;
                for (int64_t q = 0; q < cnt[r]; ++q) {
                    int64_t word = wid[r * per + q];
                    uint32_t x = st[r * per + q];
                    for (int d = 1; d <= 64; ++d) {
                        x = (uint32_t)((uint64_t)1664525u * x + 1013904223u);
                        int64_t site = 64 * word + 64 - d;
                        if (site >= half)
                            continue;
                        int64_t gx = 2 * site + ((gy + colour) & 1);
                        int64_t i = wrap(gx - (x0 - m), L);  /* patch column */
                        if (i < 1 || i > pw - 2)
                            continue;
                        int32_t sx = (int32_t)x;
                        uint32_t u = (uint32_t)(sx < 0 ? -(int64_t)sx : (int64_t)sx);
                        int v = p[j * pw + i];
                        if (oracle_accept(v, p[j * pw + i - 1], p[j * pw + i + 1],
                                          p[(j - 1) * pw + i], p[(j + 1) * pw + i], u, t4, t8))
                            p[j * pw + i] = (int8_t)(-v);
                    }
                    st[r * per + q] = x;
                }
            }
    for (int64_t j = 0; j < h; ++j)
        memcpy(out + j * w, p + (j + m) * pw + m, (size_t)w);
    free(p);
    free(wid);
    free(st);
    free(cnt);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Bands of rows for the two alternative dynamics: oracle_band_em's     */
/* light-cone argument (a band with m = 2n + 1 extra rows above and     */
/* below, outermost rows frozen, x periodic over the full width) with   */
/* the LCG or pool decisions of oracle_lcg_window / oracle_pool_window. */
/* EM[2k], EM[2k + 1] receive the rows [y0, y0 + h)'s shares of E      */
/* (bonds to the right and downwards) and M after sweep k + 1.          */
/* ------------------------------------------------------------------ */

static int8_t *band_init(int64_t L, uint64_t seed, uint32_t stream_id, int init, int64_t y0,
                         int64_t m, int64_t ph)
{
    int8_t *p = (int8_t *)malloc((size_t)(ph * L));
    if (!p)
        return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ph; ++j) {
        int64_t gy = wrap(y0 - m + j, L);
        for (int64_t x = 0; x < L; ++x) {
            int8_t v;
            if (init == 0)
                v = 1;
            else if (init == 1)
                v = -1;
            else {
                uint32_t colour = (uint32_t)((x + gy) & 1);
                uint32_t u = oracle_uniform(seed, stream_id, 2u + colour, 0u, L, x, gy);
                v = (u < 0x80000000u) ? 1 : -1;
            }
            p[j * L + x] = v;
        }
    }
    return p;
}

static void band_measure(int64_t L, const int8_t *p, int64_t m, int64_t h, int64_t *E,
                         int64_t *M)
{
    int64_t e = 0, s = 0;
#pragma omp parallel for schedule(static) reduction(+ : e, s)
    for (int64_t j = m; j < m + h; ++j)
        for (int64_t x = 0; x < L; ++x) {
            int64_t v = p[j * L + x];
            e -= v * (p[j * L + wrap(x + 1, L)] + p[(j + 1) * L + x]);
            s += v;
        }
    *E = e;
    *M = s;
}

int oracle_pool_band_em(int64_t L, uint64_t seed, uint32_t stream_id, int init, uint32_t t0,
                        int64_t n, int m_pool, int linear, const uint64_t *e4,
                        const uint64_t *e8, int64_t y0, int64_t h, int64_t *EM)
{
    int64_t m = 2 * n + 1, ph = h + 2 * m, W = (L / 2 + 63) / 64;
    if (ph > L || h <= 0 || n < 0 || L < 4 || (L & 1) || m_pool < 1 || m_pool > 30)
        return -1;
    int8_t *p = band_init(L, seed, stream_id, init, y0, m, ph);
    if (!p)
        return -1;
    for (int64_t k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 1; j < ph - 1; ++j) {
                int64_t gy = wrap(y0 - m + j, L);
                for (int64_t x = (gy + colour) & 1; x < L; x += 2) {
                    int64_t site = x / 2;
                    uint64_t word = (uint64_t)(gy * W + site / 64);
                    uint32_t a = oracle_pool_address(seed, stream_id, t, colour, m_pool, linear,
                                                     word);
                    int exp8 = (int)((e8[a] >> (site % 64)) & 1u);
                    int exp4 = (int)((e4[a] >> (site % 64)) & 1u);
                    int v = p[j * L + x];
                    int anti = (p[j * L + wrap(x - 1, L)] != v) + (p[j * L + wrap(x + 1, L)] != v) +
                               (p[(j - 1) * L + x] != v) + (p[(j + 1) * L + x] != v);
                    if (anti + 2 * exp8 + exp4 >= 2)    /* Eq. (5) */
                        p[j * L + x] = (int8_t)(-v);
                }
            }
        }
        band_measure(L, p, m, h, &EM[2 * k], &EM[2 * k + 1]);
    }
    free(p);
    return 0;
}

int oracle_lcg_band_em(int64_t L, uint32_t t4, uint32_t t8, uint64_t seed, uint32_t stream_id,
                       int init, int64_t n, int64_t y0, int64_t h, int64_t *EM)
{
    int64_t m = 2 * n + 1, ph = h + 2 * m;
    int64_t half = L / 2, W = (L / 2 + 63) / 64;
    if (ph > L || h <= 0 || n < 0 || L < 4 || (L & 1))
        return -1;
    int8_t *p = band_init(L, seed, stream_id, init, y0, m, ph);
    uint32_t *st = (uint32_t *)malloc((size_t)(2 * ph * W) * sizeof(uint32_t));
    if (!p || !st) {
        free(p);
        free(st);
        return -1;
    }
    /* generator of word w of colour c in patch row j: thread (c L + gy) W + w */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ph; ++j) {
        int64_t gy = wrap(y0 - m + j, L);
        for (int c = 0; c < 2; ++c)
            for (int64_t w = 0; w < W; ++w)
                st[(c * ph + j) * W + w] =
                    (uint32_t)((uint64_t)(uint32_t)seed * pow16807((uint64_t)((c * L + gy) * W + w)));
    }
    for (int64_t k = 0; k < n; ++k) {
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 1; j < ph - 1; ++j) {
                int64_t gy = wrap(y0 - m + j, L);
                for (int64_t w = 0; w < W; ++w) {
                    uint32_t x = st[(colour * ph + j) * W + w];
                    for (int d = 1; d <= 64; ++d) {
                        x = (uint32_t)((uint64_t)1664525u * x + 1013904223u);
                        int64_t site = 64 * w + 64 - d;
                        if (site >= half)
                            continue;
                        int64_t px = 2 * site + ((gy + colour) & 1);
                        int32_t sx = (int32_t)x;
                        uint32_t u = (uint32_t)(sx < 0 ? -(int64_t)sx : (int64_t)sx);
                        int v = p[j * L + px];
                        if (oracle_accept(v, p[j * L + wrap(px - 1, L)], p[j * L + wrap(px + 1, L)],
                                          p[(j - 1) * L + px], p[(j + 1) * L + px], u, t4, t8))
                            p[j * L + px] = (int8_t)(-v);
                    }
                    st[(colour * ph + j) * W + w] = x;
                }
            }
        }
        band_measure(L, p, m, h, &EM[2 * k], &EM[2 * k + 1]);
    }
    free(p);
    free(st);
    return 0;
}

/* Number of OpenMP threads the oracle uses (1 when built without it). */
int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
