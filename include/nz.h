/*
 * nz.h -- C ABI of libnz: the Newman-Ziff first-spanning sweep for random site
 * percolation on the five-dimensional simple hypercubic lattice sc(5) with
 * complex neighbourhoods, on one AMD Instinct MI355X (gfx950).
 *
 * The method (Malarz & Woloszyn, "Random site percolation with complex
 * neighborhoods in five dimension"):
 *   - Sec. I: sites of an L^5 lattice are occupied at random; a cluster that
 *     connects opposite borders "spans"; under free boundaries the borders are
 *     the faces x0 = 0 and x0 = L-1; under periodic boundaries (every
 *     coordinate mod L) a cluster "spans" when it wraps around axis 0, i.e.
 *     holds a loop whose unwrapped x0 displacement is a non-zero multiple of
 *     L (Newman & Ziff 2001, Sec. III);
 *   - Sec. II.A.2, eqs. (7)-(8), Table I: a neighbourhood is any non-empty set
 *     of coordination zones 1..7, zone k being the shell r^2 = k (10, 40, 80,
 *     90, 112, 240, 320 sites); bit k-1 of zone_mask selects zone k;
 *   - Sec. II.B: the Newman-Ziff construction adds occupied sites one at a time
 *     in a random order and merges clusters with union-find; a binomial
 *     convolution turns per-n results into functions of p.
 *
 * Conventions shared by every entry point:
 *   - site i has coordinates x_j = floor(i / L^j) mod L (x0 fastest);
 *   - the occupation order of sample s under seed is the sites sorted by
 *     (K(i), i), where (w0..w3) = Philox4x32-10 of counter (floor(i / 2),
 *     lo32(s), hi32(s), 0) under key (lo32(seed), hi32(seed)) and
 *     K(i) = (w1 << 32) | w0 for even i, (w3 << 32) | w2 for odd i;
 *   - n* (1-based) is the number of occupied sites when a spanning cluster first
 *     exists, mass its size at that moment; n* = mass = 0 when even the full
 *     lattice does not span (only L = 2 with zones 6 and/or 7 alone).
 *
 * Every function returns an int status (NZ_OK or a negative NZ_E* code); on
 * failure nz_last_error() describes the cause and output buffers are left
 * unspecified.  No exception crosses the ABI.  Functions are thread-compatible:
 * calls from different host threads must not share a workspace.
 */
#ifndef NZ_H
#define NZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NZ_OK 0
#define NZ_EINVAL (-1)        /* an argument is out of range or a pointer is NULL */
#define NZ_EUNSUPPORTED (-2)  /* valid request this library does not implement */
#define NZ_ENOMEM (-3)        /* a host or device allocation failed */
#define NZ_EDEVICE (-4)       /* a HIP runtime call or kernel launch failed */
#define NZ_EWORKSPACE (-5)    /* the caller's workspace is too small */

#define NZ_FREE 0             /* free boundaries */
#define NZ_PERIODIC 1         /* periodic boundaries (coordinates mod L, L >= 5): n* and mass refer
                                 to the first cluster that wraps around axis 0; L < 5 gives
                                 NZ_EUNSUPPORTED (two offsets could then reach one site) */

/* Message describing the last failure on the calling thread (never NULL). */
const char *nz_last_error(void);

/* ABI version of this header. */
#define NZ_ABI_VERSION 2
int nz_abi_version(void);

/* Number of sites z = |D(zone_mask)| of a neighbourhood (eq. (7)); -1 when
 * zone_mask is outside [1, 127]. */
int nz_coordination(uint32_t zone_mask);

/*
 * nz_sweep -- n* and spanning mass of samples 0 .. nsamples-1 (Sec. II.B).
 *   L          lattice side, 1 <= L <= 55 (N = L^5 < 2^29);
 *   zone_mask  1..127;  boundary  NZ_FREE or NZ_PERIODIC (L >= 5);
 *   seed  any 64-bit value;
 *   nstar      HOST array of nsamples int32, written;
 *   mass       HOST array of nsamples int32, written; may be NULL.
 * Synchronous; allocates and frees its own device memory; runs on the current
 * HIP device and its default stream.  Plain sweep (no prefill).
 */
int nz_sweep(int32_t L, uint32_t zone_mask, int32_t boundary, int64_t nsamples, uint64_t seed,
             int32_t *nstar, int32_t *mass);

/*
 * nz_canonical -- R_L(p) = sum_n C(N,n) p^n (1-p)^(N-n) F_n (Sec. II.B, the
 * binomial convolution), F_n = sum_{1<=m<=n} hist[m] / sum_{m>=0} hist[m].
 *   hist    HOST, hist_len = N + 1 counts; hist[0] = samples that never span;
 *   p_grid  HOST, np values in [0, 1];  R  HOST, np doubles, written.
 * FP64 on the host; binomial weights built outward from the mode by their
 * ratio recurrence, so no factorial or log-gamma is formed.
 */
int nz_canonical(const uint64_t *hist, int64_t hist_len, const double *p_grid, int64_t np,
                 double *R);

/*
 * nz_smax_window -- the largest cluster S_max(n) after n occupied sites, summed
 * over samples sample0 .. sample0+nsamples-1, for n in [n_lo, n_hi): the
 * observable of eqs. (5)-(6) (P_max = S_max / L^5 before the convolution).
 * The sweep runs on past n* through the window, one site per step.
 *   boundary   NZ_FREE or NZ_PERIODIC (L >= 5);
 *   n0         -1: plain sweep; else 0 <= n0 < n_lo: the sites whose keys lie
 *              below floor(n0 / N * 2^64), rounded down to a multiple of 2^32
 *              (about the n0 lowest-ranked sites) are labelled in bulk first
 *              (if that count reaches the window, n0 is halved and the sample
 *              redone);
 *   1 <= n_lo < n_hi <= N;
 *   smax_sum   HOST array of n_hi - n_lo uint64, written (sum over samples of
 *              S_max(n_lo + k) in entry k).
 * Synchronous; allocates and frees its own device memory; current device,
 * default stream.
 */
int nz_smax_window(int32_t L, uint32_t zone_mask, int32_t boundary, uint64_t seed, int64_t sample0,
                   int64_t nsamples, int64_t n0, int64_t n_lo, int64_t n_hi, uint64_t *smax_sum);

/*
 * nz_convolve_window -- binomial convolution of an observable known on a
 * window of n (eqs. (5)-(6): P_max(p) from <S_max(n)> / N):
 *   out[j]   = sum_{n_lo <= n < n_hi} C(N,n) p_j^n (1-p_j)^(N-n) Q[n - n_lo],
 *   cover[j] = sum of the same weights (1 when the window holds the whole
 *              binomial mass at p_j); cover may be NULL.
 *   0 <= n_lo < n_hi <= N + 1; HOST arrays; FP64, weights built outward from
 * the mode like nz_canonical.
 */
int nz_convolve_window(const double *Q, int64_t n_lo, int64_t n_hi, int64_t N, const double *p_grid,
                       int64_t np, double *out, double *cover);

/*
 * Batched device API.  One nz_job describes nsamples consecutive samples
 * (Philox sample indices sample0 ..) of one (L, zone_mask) lattice.
 *   n0        -1: plain sweep from the empty lattice.
 *             >= 0: learned prefill (Sec. II.B construction started from a
 *             bulk state): every site whose key lies below
 *             floor(n0 / N * 2^64), rounded down to a multiple of 2^32
 *             (about n0 sites), is occupied at once and its clusters are
 *             labelled by parallel connected components; the sequential sweep
 *             continues from there.  If that bulk state already spans, the
 *             sample backs off to n0 - backoff, then n0 - 3 backoff,
 *             n0 - 7 backoff, ... (the step doubling each time), then to 0
 *             (plain sweep), and is redone, so n* and mass never depend on n0.
 *   backoff   sites to back off by on the first span at n0 (0: halve n0 on
 *             every span, down to 0 below 64 sites).
 *   band_hi   expected upper bound on n* used to size the key band (sites;
 *             0: library default).  Never changes results, only work.
 *   prio      relative expected cost of a sample, for longest-first
 *             scheduling (0: library estimate).  Never changes results.
 */
typedef struct {
    int32_t L;
    uint32_t zone_mask;
    int32_t boundary;
    int32_t reserved;
    uint64_t seed;
    int64_t sample0;
    int64_t nsamples;
    int64_t n0;
    int64_t backoff;
    int64_t band_hi;
    double prio;
} nz_job;

/*
 * Tuning knobs (all 0 = automatic).  None of them changes any output.
 *   residency       1: occupancy bitset in LDS (L^5 / 8 bytes must fit);
 *                   2: everything in HBM; 3: bitset and parents in LDS.
 *   wg_waves        waves per workgroup of the sweep (1..4).
 *   waves_per_simd  resident sweep waves per SIMD of the persistent launch.
 *   bucket_log2     log2 of the mean number of keys per sort bucket (4..10; 0: 7).
 *   sweep_mode      1: one site per wave step (z lanes check the neighbours);
 *                   2: 64 sites per wave step (one site per lane; the block's
 *                   unions are merged by a connected-components pass in LDS;
 *                   the block in which spanning first occurs, and a block
 *                   that does not fit the LDS tables, is redone one site at a
 *                   time); 0: 64 sites per step for z <= 512, one site per
 *                   step for wider neighbourhoods.
 *   summary         the HBM-resident sweep reads, before each occupancy load,
 *                   a one-bit-per-block summary of the bitset held in LDS and
 *                   skips loads of all-empty words.  1: on; 2: off; 0: on when
 *                   the chunk has at least 2 samples per compute unit (with
 *                   fewer resident waves the extra LDS read is not repaid).
 *   split_z         when a batch runs as two groups side by side (see
 *                   nz_sweep_batch), jobs with z <= split_z form the first
 *                   group and the rest the second (10..892; 0: 64).
 */
typedef struct {
    int32_t residency;
    int32_t wg_waves;
    int32_t waves_per_simd;
    int32_t bucket_log2;
    int32_t sweep_mode;
    int32_t summary;
    int32_t split_z;
} nz_tuning;

/* Device workspace bytes that lets nz_sweep_batch run the jobs with all their
 * samples resident at once.  Smaller workspaces (down to the size needed by one
 * sample of the largest L) are accepted and processed in chunks. */
int nz_batch_workspace_bytes(const nz_job *jobs, int32_t njobs, const nz_tuning *tune,
                             size_t *bytes);

/*
 * nz_sweep_batch -- all samples of all jobs, scheduled longest-first over one
 * persistent sweep launch per chunk of the workspace.
 *   jobs, njobs    HOST array;
 *   d_ws, ws_bytes DEVICE workspace owned by the caller (256-byte aligned);
 *   d_nstar        DEVICE int32 array, sum of nsamples entries, written in job
 *                  order (job 0's samples first);
 *   d_mass         DEVICE int32 array like d_nstar; may be NULL;
 *   h_backoffs     HOST int32 array of njobs, backoff count per job; may be NULL;
 *   tune           may be NULL;  stream  hipStream_t (NULL: default stream).
 * Returns after the results are in d_nstar / d_mass (the call synchronises the
 * stream, because samples whose key band or bucket ran short are redone).
 * A batch with at least 256 samples of narrow neighbourhoods (z <= 64, or
 * z <= tune->split_z) and 256 of wider ones runs the two groups side by side
 * when the workspace holds both resident (nz_batch_workspace_bytes sizes it
 * so): the wider group on a second
 * host thread and a library-owned stream that first waits for the work already
 * queued on `stream`.  Results, backoff counts and statistics are the same as
 * for one group; the environment variable NZ_DEBUG_NO_SPLIT keeps one group.
 * Jobs with NZ_PERIODIC run in chunks of their own, one site per step with
 * their state in HBM whatever the tuning says: each site keeps its x0
 * displacement from its parent beside the parent (8 bytes a site instead of
 * 4), and their bulk prefill backs off when its state already wraps.
 */
int nz_sweep_batch(const nz_job *jobs, int32_t njobs, void *d_ws, size_t ws_bytes,
                   int32_t *d_nstar, int32_t *d_mass, int32_t *h_backoffs,
                   const nz_tuning *tune, void *stream);

/*
 * nz_sweep_batch_static -- nz_sweep_batch for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation calls).  The caller passes jobs and outputs only; the
 * workspace is a device buffer of NZ_STATIC_SCRATCH_BYTES that the library
 * holds on every device it has run on until the process ends.  No device or
 * host memory is allocated by the call: no hipMalloc or hipFree, no stream,
 * event or thread is created (the batch runs as one group on `stream`, and
 * nz_set_timing has no effect on it).
 *   jobs, njobs, d_nstar, d_mass, h_backoffs, tune, stream: as for
 *                  nz_sweep_batch (d_nstar, d_mass DEVICE, written in job
 *                  order; results are in place when the call returns);
 * Errors: NZ_EWORKSPACE, before any device call, when one sample of some job
 * (with the chunk header) does not fit the buffer: at the default key band
 * every L <= 24 fits; a sample whose band must be redone wider than the
 * buffer holds fails with NZ_EWORKSPACE during the call.  Samples are run in
 * as many chunks as the buffer needs, so large batches are slower than with a
 * full-size workspace, never different.
 * The buffer keeps the last call's contents; every call clears what it needs.
 * Calls on one device are serialised by a lock inside the library, so calls
 * from several host threads of one process queue up; each process has its own
 * copy of the buffer.
 */
#define NZ_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int nz_sweep_batch_static(const nz_job *jobs, int32_t njobs, int32_t *d_nstar, int32_t *d_mass,
                          int32_t *h_backoffs, const nz_tuning *tune, void *stream);

/* Size of that buffer in bytes (NZ_STATIC_SCRATCH_BYTES). */
size_t nz_static_scratch_bytes(void);

/* Statistics of the last nz_sweep_batch on the calling thread, stats[0..5]:
 * chunks, samples redone because their band ran out, because a bucket
 * overflowed, backoffs, sites occupied by the bulk prefill (summed over the
 * final runs of all samples) and sites added by the sequential sweep. */
int nz_last_batch_stats(int64_t stats[6]);

/* Per job of the last nz_sweep_batch on the calling thread (njobs must be that
 * batch's job count; HOST arrays, caller's job order): serial[j] = sites added
 * by the sequential sweep, prefilled[j] = sites occupied by the bulk prefill,
 * each summed over the final runs of job j's samples. */
int nz_last_batch_job_stats(int64_t *serial, int64_t *prefilled, int32_t njobs);

/* Phase timing of nz_sweep_batch with HIP events recorded on the caller's
 * stream around each group of launches.  nz_set_timing(1) turns it on for later
 * calls on the calling thread (0 turns it off).  nz_last_batch_timing fills
 * ms[0..5]: milliseconds in keys (with clearing), bulk connected components,
 * bucket sort, sweep, the whole call, and ms[5] = number of sweep launches. */
int nz_set_timing(int enable);
int nz_last_batch_timing(double ms[6]);

/* With timing on, the bulk labelling of free-boundary prefills split by kernel
 * (HIP events on the launch stream around every dispatch, in-chunk backoff
 * passes included): ms[0..3] = milliseconds summed over dispatches in the hook,
 * compress and size kernels (the size pass also writes the prefilled sites'
 * lattice entries) and 0 (no separate expand pass), ms[4] = number of
 * dispatches of each. */
int nz_last_batch_cc_timing(double ms[5]);

/*
 * MLP that predicts the mean and spread of n* / N for the learned prefill: three dense
 * layers 8 -> 64 -> 64 -> 2 with tanh after the first two.  Inputs per row are
 * the seven zone-mask bits and a standardised size variable exp(-ln L / nu) =
 * L^(-1/nu) (nu = 0.5720, the 5D correlation-length exponent of Sec. II.A.3);
 * outputs (u, v) estimate
 * (ln mean, ln std) of n* / N.  Weights are BF16, arithmetic FP32.
 *
 * Parameter layout (NZ_MLP_NPARAM values, row-major, "in x out"):
 *   W1[8][64] b1[64] W2[64][64] b2[64] W3[64][2] b3[2].
 * All pointers are DEVICE pointers; B >= 1 rows; stream may be NULL.
 *   params_bf16   NZ_MLP_NPARAM uint16 (bfloat16 bit patterns);
 *   x             float [B][8];  y  float [B][2];
 *   act           float [B][NZ_MLP_NACT] cache of hidden activations written by
 *                 forward and read by backward;
 *   dy            float [B][2] gradient of the loss w.r.t. y;
 *   grad          float [NZ_MLP_NPARAM], written (not accumulated);
 *   params_fp32   FP32 master weights, updated in place by nz_mlp_adam, which
 *                 also rewrites params_bf16 (round-to-nearest-even);
 *   adam_m, adam_v  float [NZ_MLP_NPARAM] moment buffers, updated in place;
 *   hyper         HOST float[5] = {lr, beta1, beta2, eps, weight_decay};
 *   step          1-based Adam step (bias correction).
 */
#define NZ_MLP_NPARAM (8 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2)
#define NZ_MLP_NACT 128
int nz_mlp_forward(const uint16_t *params_bf16, const float *x, float *y, float *act, int32_t B,
                   void *stream);
int nz_mlp_backward(const uint16_t *params_bf16, const float *x, const float *act,
                    const float *dy, float *grad, int32_t B, void *stream);
int nz_mlp_adam(float *params_fp32, uint16_t *params_bf16, const float *grad, float *adam_m,
                float *adam_v, const float hyper[5], int32_t step, void *stream);

/*
 * Learned-prefill planning (host arithmetic; no device work).
 *
 * nz_mlp_size_stats -- mean and standard deviation (population, 1 if zero) of
 *   the size variable L^(-1/nu), nu = 0.5720, over B lattices of sides L[0..B)
 *   (HOST); out[0] = mean, out[1] = std: the standardisation of the MLP's size
 *   input, taken over its training set.
 * nz_mlp_features -- the MLP's input rows x[B][8] (HOST, written): the seven
 *   bits of zone_mask[b] (zone k in column k-1) and
 *   (L[b]^(-1/nu) - size_mean) / size_std.
 * nz_prefill_target -- the training target of one lattice of side L from the
 *   n* of its samples (HOST, nsamples entries; samples with n* = 0 never
 *   span and are left out): out[0] = samples used, out[1] = mean of n* / N,
 *   out[2] = their population standard deviation, at least 0.5 / N,
 *   out[3], out[4] = the natural logarithms of out[1], out[2] (the MLP's
 *   regression targets).  NZ_EINVAL when no sample spans.
 * nz_prefill_plan -- from the MLP's outputs y[j] = (ln mean, ln std) of n* / N
 *   for job j (HOST float [njobs][2]), writes into jobs[j] (HOST):
 *     band_hi = min(N, ceil((mean + band_sigma std) N) + 1024);
 *     plain != 0: n0 = -1 (a plain sweep that only uses the band);
 *     else n0 = floor((mean - k_sigma std) N) clamped to [0, N-1] and
 *          backoff = ceil(k_sigma std N).
 *   None of these changes any n* or mass (the backoff keeps n* exact).
 */
int nz_mlp_size_stats(const int32_t *L, int32_t B, double out[2]);
int nz_mlp_features(const uint32_t *zone_mask, const int32_t *L, int32_t B, double size_mean, double size_std,
                    float *x);
int nz_prefill_target(const int32_t *nstar, int64_t nsamples, int32_t L, double out[5]);
int nz_prefill_plan(const float *y, nz_job *jobs, int32_t njobs, double k_sigma, double band_sigma, int32_t plain);

/* Weighted mean squared error of y against target over B rows and both outputs,
 * sum_b w_b / sum(w) * sum_o (y - t)^2, into loss[0], and its gradient
 * dy = 2 w_b / sum(w) * (y - t).  DEVICE pointers: y, target, dy float [B][2];
 * weight float [B] (non-negative, positive sum); loss float [1]. */
int nz_mlp_loss(const float *y, const float *target, const float *weight, float *dy, float *loss,
                int32_t B, void *stream);

#ifdef __cplusplus
}
#endif
#endif
