/*
 * ising.h - C ABI of the MI355X (gfx950) multi-spin-coded checkerboard
 * Metropolis sweep of the 2D ferromagnetic Ising model.
 *
 * Model (B. Block, P. Virnau, T. Preis, "Multi-GPU accelerated multi-spin
 * Monte Carlo simulations of the 2D Ising model"):
 *   - Section 3, Eq. (1): H = -J sum_<ij> S_i S_j on an L x L square lattice
 *     with periodic boundaries, J = 1, k_B = 1, no field.
 *   - Section 3: Metropolis acceptance exp(-dH/T) for dH > 0, else 1; the two
 *     possible factors (dH = 4 and 8) are precomputed on the host per
 *     temperature (ising_set_beta).
 *   - Section 3: checkerboard sweep; all sites of colour 0 ((x + y) even),
 *     then all sites of colour 1.
 *   - Section 4, Eqs. (3)-(5): multi-spin coding; a site flips when
 *     (number of anti-aligned neighbours) + [u < t4] + [u < t8] >= 2, with
 *     u a 32-bit uniform and t4, t8 the integer thresholds below.
 *   - Section 5.2: one bit per spin, a set bit meaning +1.
 *
 * Uniforms: Philox4x32-10 (Salmon et al., SC'11).  For site (x, y) the
 * colour-local index is i = y*(L/2) + x/2, the block is g = i/4 and the
 * output word is i mod 4; key = (lo32(seed), hi32(seed)); counter =
 * (lo32(g), hi32(g), sweep, (stream_id << 2) | phase) with phase 0/1 for
 * the colour-0/1 update and 2/3 for the hot start of colour-0/1 sites.
 * Results are therefore independent of the device layout, the launch shape,
 * batching and co-scheduling: a lattice is a pure function of
 * (L, beta history, seed, stream_id, init, sweep count).
 *
 * Conventions for every entry point:
 *   - Returns an ising_status (int32).  No C++ exception crosses the ABI.
 *     On failure ising_last_error() gives a thread-local message.
 *   - Device memory is always owned by the caller (e.g. a torch uint8 tensor
 *     on the GPU); the library never frees it.  Host buffers are owned by
 *     the caller.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Work is enqueued asynchronously on the HIP stream given at creation
 *     (NULL = the legacy default stream) unless the function says it
 *     synchronises.
 *
 * Device layout of a lattice (ising_lattice_bytes bytes, 256-B aligned):
 *   plane 0 (colour 0) then plane 1 (colour 1), each L rows of W uint64
 *   words, W = ceil((L/2)/64).  Bit b of word w in row y of plane c holds
 *   the site x = 2*(64*w + b) + ((y + c) & 1); padding bits are zero.
 *   A scratch area of 256 + 65536 bytes follows the planes (E/M partials).
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define ISING_API __attribute__((visibility("default")))
#else
#define ISING_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ising_status;
#define ISING_OK 0
#define ISING_AGAIN 1         /* ising_poll: request not finished yet */
#define ISING_EINVAL (-1)     /* bad argument (null pointer, bad size, bad beta, ...) */
#define ISING_ENOMEM (-2)     /* caller buffer or arena too small */
#define ISING_EDEVICE (-3)    /* a HIP call failed */
#define ISING_ENOTFOUND (-4)  /* unknown ticket */
#define ISING_ERANGE (-5)     /* the sweep counter would pass 2^32 - 1 */

#define ISING_INIT_COLD_UP 0   /* all spins +1 */
#define ISING_INIT_COLD_DOWN 1 /* all spins -1 */
#define ISING_INIT_HOT 2       /* each spin +1 iff its phase-(2+colour) uniform < 2^31 */

typedef struct ising_lattice ising_t;
typedef struct ising_server ising_server_t;
typedef struct ising_strip ising_strip_t;

/* Thread-local text of the last failure in this thread ("" if none). */
ISING_API const char *ising_last_error(void);

/* Library version string. */
ISING_API const char *ising_version(void);

/* Device bytes a lattice of side L needs (planes + scratch); 0 if L
 * is invalid (odd, < 4 or > 2^21). */
ISING_API size_t ising_lattice_bytes(int64_t L);

/*
 * Create a lattice of side L (even, 4 <= L <= 2^21) in the caller's device
 * buffer dev_buf (at least ising_lattice_bytes(L) bytes, 256-B aligned) and
 * enqueue its initialisation (init = ISING_INIT_*) on hip_stream.  seed is
 * the Philox key; stream_id (< 2^30) separates independent chains with the
 * same seed.  The sweep counter starts at 0.  No beta is set yet.
 * Errors: EINVAL (bad L, init, stream_id, alignment or null pointer),
 * ENOMEM (dev_bytes too small), EDEVICE.
 */
ISING_API ising_status ising_create(int64_t L, uint64_t seed, uint32_t stream_id, int32_t init,
                          void *dev_buf, size_t dev_bytes, void *hip_stream, ising_t **out);

/* Release the handle (never frees dev_buf).  NULL is accepted. */
ISING_API ising_status ising_destroy(ising_t *h);

/*
 * Set the inverse temperature (section 3: Boltzmann factors precomputed on
 * the host per temperature).  beta >= 0, finite or +inf; NaN or negative
 * gives EINVAL.  Thresholds: t4 = min(floor(exp(-4 beta) 2^32), 2^32 - 1),
 * t8 = min(floor(exp(-8 beta) 2^32), 2^32 - 1) (binary64 exp).
 */
ISING_API ising_status ising_set_beta(ising_t *h, double beta);

/* t[0] = t4, t[1] = t8 for the current beta (EINVAL before set_beta). */
ISING_API ising_status ising_get_thresholds(const ising_t *h, uint32_t t[2]);

/*
 * Enqueue n >= 0 full sweeps (colour 0 then colour 1, section 3) with sweep
 * counters h.sweep ... h.sweep + n - 1, then advance h.sweep by n.
 * If dev_EM is not NULL it is a device array of n x 2 int64: after sweep k
 * it holds E_k = -sum_<ij> S_i S_j (Eq. (1) with J = 1, no field) and
 * M_k = sum_i S_i (the magnetisation section 5.2 reduces), both exact.
 * Errors: EINVAL (no beta set, n < 0), ERANGE (counter overflow), EDEVICE.
 */
ISING_API ising_status ising_sweep(ising_t *h, int64_t n, int64_t *dev_EM);

/* E (Eq. (1), J = 1, no field) and M (sum of the spins, section 5.2) of
 * the current state into host *E, *M, exact.  Synchronises the stream. */
ISING_API ising_status ising_measure(ising_t *h, int64_t *E, int64_t *M);

/* Copy all spins to host (L*L int8, +1/-1, row-major [y][x]; on the device
 * a set bit is a +1 spin, section 5.2's one bit per spin).  Synchronises. */
ISING_API ising_status ising_get_spins(ising_t *h, int8_t *host);

/* Overwrite all spins from host (L*L int8, each +1 or -1, else EINVAL).
 * Synchronises.  The sweep counter is unchanged. */
ISING_API ising_status ising_set_spins(ising_t *h, const int8_t *host);

/* Copy the w x h window with top-left (x0, y0) (periodic, 0 <= x0, y0 < L,
 * 1 <= w, h <= L) to host (h rows of w int8).  Synchronises. */
ISING_API ising_status ising_get_window(ising_t *h, int64_t x0, int64_t y0, int64_t w, int64_t hgt,
                              int8_t *host);

/* Checkpoint/resume of the sweep counter (< 2^32). */
ISING_API ising_status ising_get_sweep(const ising_t *h, uint64_t *t);
ISING_API ising_status ising_set_sweep(ising_t *h, uint64_t t);

/* Side L and device address of the lattice planes (for tests). */
ISING_API ising_status ising_get_info(const ising_t *h, int64_t *L, int64_t *words_per_row, void **planes);

/*
 * Device bytes of the work buffer ising_multi_sweep (and
 * ising_multi_sweep_form, whatever form it forces) needs for these handles
 * (same conditions on the handles as there; 0 when no lattice can take the
 * batched kernels).  The bytes depend only on the lattice sides.  Host only.
 */
ISING_API ising_status ising_multi_sweep_work_bytes(ising_t *const *hs, int32_t count,
                                                    size_t *bytes);

/*
 * Batched sweeps: n sweeps on each of the `count` handles (all created on
 * the same device and stream, each with a beta set, no handle twice),
 * equivalent bit for bit to calling ising_sweep(hs[i], n, dev_EM[i]) on
 * each (section 3's checkerboard sweep, Eqs. (1), (3)-(5), per lattice).
 * All lattices advance together in fused launches (or, for batches of small
 * lattices, one persistent launch); see ising_multi_sweep_form.  dev_EM may
 * be NULL or hold NULL entries.  The task tables go to dev_work (device,
 * caller-owned, 256-byte aligned, at least ising_multi_sweep_work_bytes
 * bytes; may be NULL when that is 0); the library allocates no device
 * memory.  Each handle's counter advances by n.  Synchronises the stream,
 * so dev_work is free again on return.  Errors: EINVAL, ERANGE, EDEVICE,
 * ENOMEM (work buffer missing, misaligned or too small).
 */
ISING_API ising_status ising_multi_sweep(ising_t *const *hs, int32_t count, int64_t n,
                                         int64_t *const *dev_EM, void *dev_work,
                                         size_t work_bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched sweeps as ising_multi_sweep, bit for bit, with no work buffer.
 * The task tables go to a static device array of 4 MiB inside the library
 * (one per GPU, held until the process ends); a batch whose tables need
 * more is rejected with ENOMEM before any device work.  No hipGraph is
 * built (instantiation allocates): two kernel launches per sweep, enqueued
 * directly on the handles' stream.  The call allocates no device memory,
 * waits for the stream before it returns, and is serialised with other
 * calls on the same GPU in this process (they share the array).  Errors:
 * EINVAL, ERANGE, ENOMEM, EDEVICE.
 */
ISING_API ising_status ising_multi_sweep_static(ising_t *const *hs, int32_t count, int64_t n,
                                                int64_t *const *dev_EM);

/*
 * Same as ising_multi_sweep with the launch form chosen by the caller:
 * form -1 lets the cost model choose, 0 forces the fused form (two launches
 * per sweep over the flattened tiles of all lattices, replayed from captured
 * hipGraph chunks of graph_chunk sweeps; 0 disables graphs, -1 keeps the
 * default), 1 forces the packed persistent form (each lattice on one
 * workgroup, one launch for all n sweeps).  Results are bit-identical for
 * every form.  For tests and tuning.
 */
ISING_API ising_status ising_multi_sweep_form(ising_t *const *hs, int32_t count, int64_t n,
                                              int64_t *const *dev_EM, int32_t form,
                                              int32_t graph_chunk, void *dev_work,
                                              size_t work_bytes);

/*
 * Launch form the batched path would choose for lattices of sides Ls[i]
 * (each a multiple of 8) on a device with `cus` compute units: *form_out
 * 0 (fused) or 1 (packed), *blocks_out its grid size, *est_seconds_out
 * (may be NULL) the cost model's seconds per sweep.  Host-only; for
 * inspection and tests.
 */
ISING_API ising_status ising_batch_plan(const int64_t *Ls, int32_t count, int32_t cus,
                                        int32_t *form_out, int32_t *blocks_out,
                                        double *est_seconds_out);

/* ---------------------------------------------------------------- */
/* Autotuner: launch shapes of the plain sweep per lattice size class. */
/* ---------------------------------------------------------------- */

#define ISING_FORM_TILE 0  /* workgroup tiles of 4 independent waves, neighbour words
                              loaded directly (the default) */
#define ISING_FORM_STRIP 1 /* one wave per 64-word x rpw-row strip, rows rolled in
                              registers (rows of >= 63 words only; others use tiles) */

typedef struct {
    int64_t L_min, L_max;    /* size class the entry applies to */
    int32_t form;            /* ISING_FORM_* */
    int32_t rpw;             /* tile: row groups per wave, 0..16; strip: rows per wave
                                task, 0..2^21 (0: size rule) */
    int32_t max_blocks;      /* grid cap, 1..2048 */
    int32_t reserved;        /* 0 */
    int64_t small_lds_bytes; /* lattices with both planes <= this run in one LDS-resident
                                workgroup (0: never) */
    double updates_per_ns;   /* rate measured by the autotuner (informational) */
} ising_tuning;

/*
 * Time candidate shapes of the plain sweep for a lattice of side L: the
 * LDS-resident single workgroup for small lattices; tiles with rpw in
 * {1, 2, 4} x grid cap in {512, 1024, 2048}; for rows of >= 63 words, strips
 * of {rule, 4, 8, 16, 32} rows x grid cap in {1024, 2048}.  It uses the
 * caller's device buffer as scratch: at least ising_lattice_bytes(L) bytes
 * (rounded up to 256); with 16 * max(trial_sweeps, 2) bytes more, every
 * trial also records its per-sweep (E, M) there, as a run with a series
 * does, and is timed with that cost.  It times trial_sweeps sweeps per
 * shape, installs the fastest for L's size class [2^k, 2^(k+1)) and returns
 * it in *out.  Handles created afterwards use it; results are bit-identical
 * for every shape.  Synchronises the stream.
 */
ISING_API ising_status ising_autotune(int64_t L, void *dev_buf, size_t dev_bytes, void *hip_stream,
                                      int32_t trial_sweeps, ising_tuning *out);

/* Install tuning entries (for example a cache written by an earlier run). */
ISING_API ising_status ising_tuning_set(const ising_tuning *entries, int32_t count);

/* Copy up to `capacity` installed entries; *count receives how many exist. */
ISING_API ising_status ising_tuning_get(ising_tuning *entries, int32_t capacity, int32_t *count);

/* The launch shape a handle of side L created now would use (the installed
 * entry of L's size class, else the built-in default); updates_per_ns is 0
 * for a default. */
ISING_API ising_status ising_tuning_lookup(int64_t L, ising_tuning *out);

/* Remove all installed entries (back to the defaults). */
ISING_API ising_status ising_tuning_clear(void);

/* ---------------------------------------------------------------- */
/* Batched autotuner: the fused kernel's tile shape, grid and graph   */
/* chunk for ising_multi_sweep.                                       */
/* ---------------------------------------------------------------- */

typedef struct {
    int32_t form;           /* the faster form on the timed batch: 0 fused, 1 packed
                               (informational: the cost model still chooses per call) */
    int32_t rpw_max;        /* fused tiles: a lattice takes the largest of 1, 2, 4 row
                               groups per wave up to this that leaves it >= 128 r tiles
                               of one row group (built-in: 2); 1, 2 or 4 */
    int32_t wg_per_cu;      /* fused grid: workgroups per compute unit, 1..8 (built-in 8) */
    int32_t graph_chunk;    /* sweeps per captured hipGraph chunk, 0..4096 (0: no graph;
                               built-in 32) */
    double updates_per_ns;          /* rate of this fused shape on the timed batch */
    double default_updates_per_ns;  /* the built-in fused shape on the same batch */
    double packed_updates_per_ns;   /* the packed form on the same batch (0: not timed,
                                       the cost model puts it far behind) */
} ising_batch_tuning;

/* Device bytes ising_multi_autotune needs for these handles and
 * trial_sweeps (>= 1): copies of every lattice, their per-sweep (E, M) for
 * 2 trial_sweeps sweeps, and the largest work buffer of any candidate.
 * Host only. */
ISING_API ising_status ising_multi_autotune_bytes(ising_t *const *hs, int32_t count,
                                                  int32_t trial_sweeps, size_t *bytes);

/*
 * Time the batched sweep's fused shapes on copies of these lattices (same
 * sides, seeds, stream ids, starts and betas, made in dev_buf: device,
 * 256-byte aligned, at least ising_multi_autotune_bytes; the handles
 * themselves are not touched): rpw_max in {1, 2, 4} x workgroups per CU in
 * {8, 6, 4} with graph chunk 32, then chunks {8, 16, 64} at the best of
 * those, and the packed form when the cost model does not put it far
 * behind.  A candidate's rate is trial_sweeps sweeps of updates over the
 * time of a 2 trial_sweeps call less that of a trial_sweeps call (the
 * table upload and graph capture cancel), with per-sweep (E, M) recorded.
 * Installs the fastest fused shape for every later batched call
 * (ising_multi_sweep, _form, _static and the server) and returns it in
 * *out.  Results are bit-identical for every shape.  Runs on the handles'
 * stream and synchronises it.  Errors: EINVAL, ENOMEM (buffer too small or
 * misaligned), EDEVICE.
 */
ISING_API ising_status ising_multi_autotune(ising_t *const *hs, int32_t count,
                                            int32_t trial_sweeps, void *dev_buf,
                                            size_t dev_bytes, ising_batch_tuning *out);

/* Install a fused shape (rpw_max, wg_per_cu, graph_chunk of *t; the other
 * fields are ignored), for example one an earlier run measured. */
ISING_API ising_status ising_batch_tuning_set(const ising_batch_tuning *t);

/* The fused shape batched calls use now; *installed is 1 if it was
 * installed (rates as measured), 0 for the built-in one (rates 0). */
ISING_API ising_status ising_batch_tuning_get(ising_batch_tuning *out, int32_t *installed);

/* Back to the built-in fused shape. */
ISING_API ising_status ising_batch_tuning_clear(void);

/* ---------------------------------------------------------------- */
/* The paper's own random numbers (alternative dynamics).            */
/* ---------------------------------------------------------------- */

#define ISING_RNG_PHILOX 0      /* counter-based Philox4x32-10 per site (the default) */
#define ISING_RNG_LCG 1         /* per-thread linear congruential generators */
#define ISING_RNG_POOL 2        /* Boltzmann-pattern pool, a random address per word */
#define ISING_RNG_POOL_LINEAR 3 /* Boltzmann-pattern pool read linearly from one random
                                   start per group of 256 words */

/* Device bytes of the per-thread LCG states of a lattice of side L
 * (2 * L * W uint32, W = ceil((L/2)/64)); 0 for an invalid L. */
ISING_API size_t ising_lcg_bytes(int64_t L);

/* Device bytes of a Boltzmann-pattern pool of 2^log2_patterns patterns (16
 * bytes each) for 10 <= log2_patterns <= 28; 0 otherwise. */
ISING_API size_t ising_pool_bytes(int32_t log2_patterns);

/*
 * Choose the random numbers of the Metropolis decisions (section 5.3).
 * ISING_RNG_LCG uses one generator per 64-site word of each colour
 * ("thread" j = (c L + y) W + w): x <- (1664525 x + 1013904223) mod 2^32
 * (Eq. (6)), seeds x_{0,j} = lo32(seed) * 16807^j mod 2^32 (Eq. (7); seed 1
 * gives the paper's x_{0,0} = 1).  Each colour step advances a word's
 * generator 64 times; the k-th value decides site 64 - k of the word (site
 * 63 first), and an uphill move dE is accepted iff |int32(x)| <
 * min(floor(exp(-beta dE) 2^31), 2^31), i.e. y = |x / 2^31| < exp(-beta dE).
 * The states live in dev_state (caller-owned device memory of
 * ising_lcg_bytes(L) bytes, 4-byte aligned, kept for the handle's life); the
 * call seeds them asynchronously on the handle's stream.  Needs L % 8 == 0
 * (tiled layout); plain sweeps only (ising_multi_sweep rejects such
 * handles); the hot start is unchanged.
 *
 * ISING_RNG_POOL and ISING_RNG_POOL_LINEAR use a pool of Boltzmann patterns
 * (section 4: bit patterns exp4, exp8 with the flip rule k + 2 exp8 + exp4
 * >= 2 of Eq. (5); section 5.1 and Table 2 for the two GPU variants).  The
 * pool holds P = 2^m patterns of 64 sites; bit b of pattern p is drawn from
 * the uniform u of index i = 64 p + b (Philox4x32-10, the lattice's key,
 * counter (lo32 i/4, hi32 i/4, 2^32 - 1, stream_id << 2 | 2), output
 * i mod 4): exp8 = [u < t8], exp4 = [t8 <= u < t4].  In sweep t, colour c,
 * word j = y W + w of the colour plane reads pattern v >> (32 - m), with v
 * output 0 of Philox4x32-10 at counter (lo32 j, 0, t, stream_id << 2 | c)
 * (POOL), or pattern ((v >> (32 - m)) + j mod 256) mod P with v drawn at
 * counter (lo32 (j / 256), 0, t, stream_id << 2 | c) (POOL_LINEAR: one draw
 * per group of 256 consecutive words, read linearly).  dev_state is the
 * pool (caller-owned device memory of exactly ising_pool_bytes(m) bytes,
 * which fixes m, 16-byte aligned, kept for the handle's life); it is drawn
 * on the handle's stream now (if beta is set) and again at every
 * ising_set_beta.  A small pool biases the dynamics (each bit position's
 * acceptance rate is an empirical fraction over P patterns; the paper
 * suggests 2^22 to 2^24).  Needs L % 8 == 0 and fewer than 2^32 words per
 * colour plane; plain sweeps only.
 *
 * ISING_RNG_PHILOX (dev_state ignored) returns to the default.  EINVAL /
 * ENOMEM on bad arguments.
 */
ISING_API ising_status ising_set_rng(ising_t *h, int32_t kind, void *dev_state,
                                     size_t state_bytes);

/* ---------------------------------------------------------------- */
/* Row-strip shares: one GPU's part of a multi-GPU decomposition.      */
/* ---------------------------------------------------------------- */

/*
 * Section 6 splits one lattice over several GPUs; each updates its own
 * part and exchanges border rows with its neighbours between the two
 * colour steps of a sweep (B only after all of A, section 3).  A strip is
 * the rows y0 .. y0 + rows - 1 of an L x L lattice (L % 128 == 0) held with
 * one halo row above (global row y0 - 1 mod L) and below (y0 + rows mod L)
 * in each colour plane.  Uniforms are keyed by global (x, y) exactly as in
 * ising_sweep, so strips that tile the lattice, stepped colour by colour
 * with a halo exchange after each step, reproduce the whole lattice's
 * spins and (E, M) bit for bit.
 *
 * Device bytes of a strip of `rows` rows (planes of (rows + 2) x L/128
 * words plus per-block partials); 0 for an unsupported shape (L % 128 != 0,
 * L outside [128, 2^21], rows outside [1, L], rows * L / 128 > 2^31).
 */
ISING_API size_t ising_strip_bytes(int64_t L, int64_t rows);

/*
 * Create a strip in dev_buf (caller-owned, >= ising_strip_bytes, 8-byte
 * aligned) and initialise its own rows (init as in ising_create, keyed by
 * global coordinates) on hip_stream.  The halos are undefined until the
 * first exchange of each colour.  EINVAL / ENOMEM / EDEVICE.
 */
ISING_API ising_status ising_strip_create(int64_t L, int64_t y0, int64_t rows, uint64_t seed,
                                          uint32_t stream_id, int32_t init, void *dev_buf,
                                          size_t dev_bytes, void *hip_stream,
                                          ising_strip_t **out);
ISING_API ising_status ising_strip_destroy(ising_strip_t *h);
/* Thresholds as ising_set_beta. */
ISING_API ising_status ising_strip_set_beta(ising_strip_t *h, double beta);

/*
 * One colour step (0 or 1) of sweep `sweep` on the strip's own rows,
 * reading the other colour's halos (which must hold the neighbours' rows
 * of that colour as they are after the previous colour step).  For colour
 * 1, dev_counts (2 int64 on the device, or NULL) receives the strip's
 * anti-aligned bonds A (each bond counted at its colour-1 end, halo
 * neighbours included) and up spins P; the lattice's E = 2 sum A - 2 L^2,
 * M = 2 sum P - L^2 (ising_strip_combine).  Asynchronous on the strip's
 * stream.
 */
ISING_API ising_status ising_strip_step(ising_strip_t *h, int32_t colour, uint32_t sweep,
                                        int64_t *dev_counts);

/*
 * In-process halo exchange of colour `colour` among strips that tile the
 * lattice in order (strip k starts where strip k-1 ends, the first at row
 * 0, the last ending at row L; one stream): each strip's halo above
 * receives the last row of the strip above, its halo below the first row
 * of the strip below (periodically).  Call after every colour step with
 * that colour, and once per colour after creation.  Across GPUs the same
 * rows move by RCCL send/recv (ising_strip_row gives their addresses).
 */
ISING_API ising_status ising_strip_exchange(ising_strip_t *const *hs, int32_t count,
                                            int32_t colour);

/* Device address and size of one row of colour `colour`: which 0 = halo
 * above, 1 = first own row, 2 = last own row, 3 = halo below. */
ISING_API ising_status ising_strip_row(const ising_strip_t *h, int32_t colour, int32_t which,
                                       void **ptr, size_t *bytes);

/* The strip's own rows as int8 (+1 / -1), rows x L row-major (synchronous). */
ISING_API ising_status ising_strip_get_rows(ising_strip_t *h, int8_t *host);

/* EM[k] = (2 sum_s A - 2 L^2, 2 sum_s P - L^2) for k < n from dev_counts laid
 * out [n][nstrips][2] (the per-sweep all-reduce of the strips' counts), on
 * hip_stream. */
ISING_API ising_status ising_strip_combine(const int64_t *dev_counts, int32_t nstrips, int64_t n,
                                           int64_t L, int64_t *dev_EM, void *hip_stream);

/* ---------------------------------------------------------------- */
/* Test hook.                                                         */
/* ---------------------------------------------------------------- */

/*
 * Barrier perturbation for race tests (process-wide; 0 turns it off, the
 * default).  With a nonzero seed, the kernels that rely on block barriers
 * inside a launch (the LDS-resident small-lattice sweeps and the packed
 * persistent batched kernel) make every wave pause a pseudo-random time,
 * drawn from the seed, before each such barrier.  Results must not change;
 * a difference points at a missing barrier.  Applies to launches enqueued
 * after the call.  Always ISING_OK.
 */
ISING_API ising_status ising_debug_perturb(uint32_t seed);

/* ---------------------------------------------------------------- */
/* Finite-size-scaling analysis of per-sweep (E, M) series.           */
/* ---------------------------------------------------------------- */

/*
 * Single-histogram reweighting (Ferrenberg and Swendsen, PRL 61, 2635
 * (1988)) of device-resident per-sweep series, the input of the Binder
 * cumulant crossing by which the paper locates T_C (section 2, Eq. (2)).
 *
 * Series i is n_sweeps[i] rows of int64 (E, M) at dev_EM[i] (device, as
 * written by ising_sweep / ising_multi_sweep), simulated at beta0[i]
 * (finite, >= 0).  Sweeps discard[i] .. n_sweeps[i]-1 are kept (at least
 * nblocks of them); kept sweep j belongs to block floor(j * nblocks / count).
 * Task k reweights series task_lattice[k] to task_beta[k] (finite, >= 0):
 * with x_t = -(beta - beta0)(E_t - E_ref), E_ref = E of the first kept sweep,
 * and w_t = exp(x_t - max x), it writes for every block b the five fp64
 * sums  w, w|M|, w M^2, w M^4, w E  to dev_sums[(k * nblocks + b) * 5 + i]
 * (device, ntask * nblocks * 5 doubles, caller-owned) and max x to
 * dev_shift[k] (device, may be NULL).  1 <= nblocks <= 4096.  The task
 * tables go to dev_work (device, caller-owned, 256-byte aligned, at least
 * ising_reweight_work_bytes(nlat, ntask) bytes).  The host arrays are read
 * before the call returns: they are copied to dev_work on hip_stream, the
 * call waits for that copy, and the kernel then runs asynchronously on
 * hip_stream, reading dev_work; the caller must not reuse dev_work (or
 * free it) until the stream has passed the kernel.  Calls on different
 * streams with different work buffers are independent.  Errors: EINVAL,
 * ENOMEM (work buffer missing, misaligned or too small), EDEVICE.
 */
ISING_API ising_status ising_reweight(int32_t nlat, const int64_t *const *dev_EM,
                                      const int64_t *n_sweeps, const int64_t *discard,
                                      const double *beta0, int32_t ntask,
                                      const int32_t *task_lattice, const double *task_beta,
                                      int32_t nblocks, double *dev_sums, double *dev_shift,
                                      void *dev_work, size_t work_bytes, void *hip_stream);

/* Device bytes of ising_reweight's work buffer for nlat series and ntask
 * tasks (0 if either is < 1).  Host only. */
ISING_API size_t ising_reweight_work_bytes(int32_t nlat, int32_t ntask);

/*
 * From the per-block sums of ising_reweight (host copy, ntask * nblocks * 5
 * doubles) and the number of sites N of each task's lattice: est[3k..3k+2] =
 * (U4, <E>/N, <|M|>/N) of the totals, U4 = 1 - <M^4> / (3 <M^2>^2) (Eq. (2)),
 * err[3k..] their delete-one-block jackknife errors
 * sqrt((B-1)/B sum_b (q_b - mean q)^2), and, if u4_rep is not NULL,
 * u4_rep[k * nblocks + b] = U4 without block b.  nblocks >= 2.  Host only.
 */
ISING_API ising_status ising_fss_moments(const double *sums, int32_t ntask, int32_t nblocks,
                                         const int64_t *sites, double *est, double *err,
                                         double *u4_rep);

/*
 * Crossing of two Binder-cumulant curves on an ascending grid T[0..K-1]: Ua
 * of the smaller lattice, Ub of the larger.  With d = Ua - Ub, the first k
 * with d[k] < 0 <= d[k+1] gives T* by linear interpolation and U* = Ua at
 * T* (below T_C the larger lattice has the larger U4).  out[0..3] = T*, U*,
 * and their jackknife errors from the replica curves Ua_rep / Ub_rep
 * (nblocks x K each, may both be NULL).  NaN where there is no such k (in
 * the full curves, or in any replica for the errors).  Host only.
 */
ISING_API ising_status ising_binder_crossing(const double *T, int32_t K, const double *Ua,
                                             const double *Ub, const double *Ua_rep,
                                             const double *Ub_rep, int32_t nblocks,
                                             double *out);

/*
 * Integrated autocorrelation time of a series x[0 .. n-1] (host, n >= 2),
 * the measure of how many sweeps separate independent samples, which the
 * errors of the Binder-cumulant analysis (section 2, Eq. (2)) need: kept
 * blocks must be long against it.  With y = x - mean,
 * C(t) = sum_{i < n-t} y_i y_{i+t} / (n - t), rho(t) = C(t) / C(0) and
 * tau(W) = 1/2 + sum_{t=1..W} rho(t), the window W is the smallest in
 * 1 .. floor(n/2) with W >= c tau(W) (A. D. Sokal's automatic window;
 * c = 5 is usual).  *tau = tau(W), *window = W; *window = -1 when no
 * window qualifies (*tau is then tau(floor(n/2)): the series is too short
 * for its correlations); a constant series gives 0.5 and 0.  The sums
 * C(t) are formed by FFT in fp64.  n <= 2^28.  Errors: EINVAL (NULL
 * pointers, n < 2, c <= 0, a non-finite sample).
 */
ISING_API ising_status ising_autocorr_time(const double *x, int64_t n, double c, double *tau,
                                           int64_t *window);

/* ---------------------------------------------------------------- */
/* Served mode: continuous batching of independent simulations.      */
/* ---------------------------------------------------------------- */

#define ISING_REQ_RECORD_SERIES 1u /* copy the per-sweep (E, M) series to EM_series */
#define ISING_REQ_RETURN_SPINS 2u  /* copy the final spins to spins_out */

typedef struct {
    int64_t L;           /* even, >= 4 */
    double beta;         /* >= 0 or +inf */
    uint64_t seed;
    uint32_t stream_id;  /* < 2^30 */
    int32_t init;        /* ISING_INIT_* */
    int64_t n_sweeps;    /* >= 1 */
    int64_t n_discard;   /* sweeps excluded from the moment sums */
    uint32_t flags;      /* ISING_REQ_* */
    int64_t *EM_series;  /* caller-owned host buffer of n_sweeps x 2, or NULL */
    int8_t *spins_out;   /* caller-owned host buffer of L*L, or NULL */
} ising_request;

typedef struct {
    uint64_t ticket;
    int32_t status;       /* ISING_OK when done, ISING_AGAIN while running */
    int64_t E_final, M_final;
    uint64_t sweeps_done;
    double sum_M2, sum_M4; /* exact integer sums over kept sweeps, each rounded once to double */
    int64_t n_kept;
    double t_arrive, t_admit, t_done; /* seconds on the host monotonic clock */
} ising_result;

/*
 * A server owns nothing on the device except what it carves from the
 * caller's arena (dev_arena, 256-byte aligned, arena_bytes = the HBM
 * budget, caller-owned until ising_server_destroy).  The last 1/32 of the
 * arena (at least 4 KiB) holds the batched task tables; the rest holds the
 * lattices and their per-sweep series.  Requests are admitted in FIFO order
 * whenever their lattice, series and share of the table region fit;
 * every quantum runs quantum_sweeps sweeps on all admitted lattices in
 * fused launches (continuous batching).  Results do not depend on the mix:
 * each lattice's uniforms are keyed by its own (seed, stream_id, sweep).
 * Errors: EINVAL (NULL or misaligned arena, arena under 8 KiB, quantum < 1).
 */
ISING_API ising_status ising_server_create(void *dev_arena, size_t arena_bytes, void *hip_stream,
                                 int32_t quantum_sweeps, ising_server_t **out);

/* Queue n requests; tickets_out[i] receives each ticket.  Requests larger
 * than the whole arena are rejected (ENOMEM) without queueing any. */
ISING_API ising_status ising_batch_submit(ising_server_t *s, const ising_request *reqs, int32_t n,
                                uint64_t *tickets_out);

/* Advance the server by one quantum: wait for the quantum in flight, start
 * copying the series of the requests it finished, admit, enqueue the next
 * quantum on the stream without waiting for it, then finish the finished
 * requests' results on the host (so the GPU runs while the host retires).
 * Returns AGAIN while work remains or a quantum is in flight, OK when idle
 * (nothing queued, active or in flight).  The server creates one pinned
 * host staging buffer for the series copies. */
ISING_API ising_status ising_server_step(ising_server_t *s);

/* Result of a ticket: OK (done, *out filled, ticket released), AGAIN
 * (queued or running; out->status = AGAIN), ENOTFOUND. */
ISING_API ising_status ising_poll(ising_server_t *s, uint64_t ticket, ising_result *out);

/* Fail the given quantum index (host-side fault injection for tests): the
 * quantum's work is discarded and re-run from the last committed state. */
ISING_API ising_status ising_server_inject_fault(ising_server_t *s, int64_t quantum_index);

/* Counters: [0] quanta run, [1] requests admitted, [2] requests done,
 * [3] bytes in use, [4] peak bytes in use, [5] faults recovered. */
ISING_API ising_status ising_server_stats(const ising_server_t *s, int64_t out[6]);

ISING_API ising_status ising_server_destroy(ising_server_t *s);

/*
 * The moments a served request reports, for any host series: sum_M2 and
 * sum_M4 are the exact integer sums of M^2 and M^4 over sweeps
 * discard .. n - 1 of `series` (n x 2 int64, interleaved E, M, host
 * memory), each rounded once to the nearest double (M^4 is summed in 256
 * bits); n_kept = max(n - discard, 0).  These feed the Binder cumulant
 * U4 = 1 - <M^4> / (3 <M^2>^2) of Eq. (2).  Host only, no device call.
 * EINVAL for NULL outputs, n < 0, discard < 0, or |M| > 2^42 (no lattice
 * has more sites).
 */
ISING_API ising_status ising_series_moments(const int64_t *series, int64_t n, int64_t discard,
                                            double *sum_M2, double *sum_M4, int64_t *n_kept);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
