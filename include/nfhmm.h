/*
 * nfhmm.h -- C ABI of the MI355X (gfx950) library for variational inference
 * in the Bayesian non-negative factorial hidden Markov model (N-FHMM) of
 * Mysore & Sahani, "Variational Inference in Non-negative Factorial Hidden
 * Markov Models for Efficient Audio Source Separation".
 *
 * What one fit computes (the paper's Sections 2.2, 3.2 and 4):
 *   given the mixture spectrogram V, the per-source dictionaries beta (W),
 *   Markov transitions and initial-state probabilities of each source model,
 *   it iterates the mean-field updates of Section 3.2 -- Eq. 7 (responsibilities
 *   of every dictionary element at every frequency), Eq. 8 (surrogate state
 *   log-likelihoods), a forward-backward pass per source chain, Eq. 6
 *   (Dirichlet posterior over the mixture weights) -- records the evidence
 *   lower bound after every iteration, and finally reconstructs each source
 *   and applies the ratio mask of Section 4.
 *
 * Conventions common to every call:
 *   - All arrays are dense, C order, float32 unless stated; sizes are int64.
 *   - Element index k of the S*N*K dictionary elements is k = (s*N + n)*K + j
 *     (source s, state n, element j of that state's dictionary).  This layout
 *     is the availability mask B of Section 2.2: element k is available exactly
 *     when source s is in state n.  Every dictionary has the same K and no
 *     element is shared between states or sources.
 *   - No C++ exception crosses the ABI.  Every call returns an nfhmm_status;
 *     nfhmm_last_error() gives a message for the last failing call on a context.
 *   - A context is used by one host thread at a time, except that
 *     nfhmm_submit / nfhmm_poll / nfhmm_wait / nfhmm_cancel may be called from
 *     any thread.
 */
#ifndef NFHMM_H
#define NFHMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NFHMM_API __attribute__((visibility("default")))

#define NFHMM_MAX_STATES   64      /* N: one state per lane of a 64-wide wavefront */
#define NFHMM_MAX_ELEMENTS 12288   /* S*N*K                                           */
#define NFHMM_MAX_SOURCES  8       /* S                                               */

typedef struct nfhmm_ctx nfhmm_ctx;

typedef enum {
  NFHMM_OK           = 0,
  NFHMM_E_INVALID    = -1,  /* bad dims, non-finite or negative V, W/A/pi not normalised */
  NFHMM_E_NOMEM      = -2,  /* the job does not fit the context's device-memory budget   */
  NFHMM_E_DEVICE     = -3,  /* a HIP runtime call failed                                 */
  NFHMM_E_NONFINITE  = -4,  /* the bound became non-finite on the device for this job    */
  NFHMM_E_CANCELLED  = -5,  /* the job was cancelled before it finished                  */
  NFHMM_E_NOTFOUND   = -6   /* unknown job id                                            */
} nfhmm_status;

/* Arithmetic of the two dictionary contractions (Eq. 7 inside Eq. 6).
 * FP32: float32 operands, float32 accumulation.
 * BF16: bfloat16 operands (round-to-nearest-even copies of W, of the expected
 *       weights exp(E[ln theta]) and of V/Lambda), float32 accumulation.
 * Everything else -- digamma, Eq. 6, Eq. 8, forward-backward, the bound and the
 * separation -- is float32 in both. */
typedef enum { NFHMM_FP32 = 0, NFHMM_BF16 = 1 } nfhmm_precision;

/* One separation problem.
 *   V          [T][F]     mixture spectrogram in counts of quanta (Section 2.2; V_lt of
 *                         Eq. 6 stored frame-major).  Finite, >= 0.
 *   W          [S][N][K][F] dictionary elements beta(k) (Section 2.1), each row of F
 *                         values sums to 1 within 1e-4.
 *   A          [S][N][N]  transitions, row-stochastic: A[s][i][j] = P(D_t=j | D_{t-1}=i)
 *                         (the transpose of the paper's column rho(d)).  Zeros allowed;
 *                         rows sum to 1 within 1e-4.
 *   pi         [S][N]     initial-state probabilities; zeros allowed; sum to 1 within 1e-4.
 *   gamma      Dirichlet concentration of Section 2.2 (the paper takes 1); >= 0.
 *   iters      number of iterations (>= 0); no convergence test.
 *   alpha_init [T][S*N*K] warm start for the Dirichlet parameters alpha-hat (every entry
 *                         > 0, finite), or NULL for the default start: Eq. 6 evaluated with
 *                         responsibilities proportional to beta and d-hat = 1/N. */
typedef struct {
  int32_t S, N, K;
  int64_t F, T;
  const float *V;
  const float *W;
  const float *A;
  const float *pi;
  float gamma;
  int32_t iters;
  const float *alpha_init;
} nfhmm_problem;

/* Outputs (any pointer may be NULL to skip that output).
 *   alpha  [T][S*N*K]  alpha-hat after the last iteration: q(theta_t) = Dir(alpha[t]) (Eq. 6)
 *   post   [S][T][N]   state marginals d-hat of each source chain from the last iteration's
 *                      forward-backward (1/N everywhere when iters == 0)
 *   sep    [S][T][F]   masked separated spectrograms V*^(s) of Section 4, computed with
 *                      E[theta_tk] = alpha[t][k] / sum_k alpha[t][k]; sum_s sep[s] = V
 *   elbo   [iters]     the evidence lower bound after each iteration (float64) */
typedef struct {
  float  *alpha;
  float  *post;
  float  *sep;
  double *elbo;
} nfhmm_result;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory that the context's resident jobs may hold (0 = no cap); max_slots caps
 * the number of jobs resident at once in the serving loop (<= 0: 64).
 * Returns NFHMM_E_DEVICE if the device cannot be used; *out is NULL then. */
NFHMM_API nfhmm_status nfhmm_create(nfhmm_ctx **out, int device, size_t hbm_budget_bytes, int max_slots);

/* Cancel queued jobs, wait for running ones, free all device memory. NULL is ignored. */
NFHMM_API void nfhmm_destroy(nfhmm_ctx *ctx);

/* Message of the last failing call on ctx (thread-local to the calling thread's
 * last call); valid until the next call on ctx from that thread.  Never NULL. */
NFHMM_API const char *nfhmm_last_error(const nfhmm_ctx *ctx);

/* ------------------------------------------------------------------ host-only helpers */

/* Device bytes one job of this shape holds while resident (host arithmetic only;
 * no device needed).  0 if the dims are invalid. */
NFHMM_API size_t nfhmm_footprint_bytes(const nfhmm_problem *p, nfhmm_precision prec);

/* Check a problem whose arrays are in host memory, as nfhmm_fit does: dims within
 * the limits above, V finite and >= 0, W rows / A rows / pi summing to 1 within 1e-4,
 * no frequency bin with V > 0 where every dictionary element is 0 (the bound would
 * be -inf), alpha_init finite and > 0.  Writes a message to msg (if non-NULL).
 * Host arithmetic only; no device needed. */
NFHMM_API nfhmm_status nfhmm_validate(const nfhmm_problem *p, char *msg, size_t msglen);

/* Admission rule of the serving loop, exposed for testing: given the footprints of
 * queued jobs in arrival order, the bytes already in use, the budget (0 = none),
 * the resident job count and the slot limit, write to admit[i] 1 for the jobs that
 * are admitted now (strict first-in-first-out: admission stops at the first job that
 * does not fit) and return how many.  A job larger than the whole budget is marked
 * -1 (it can never run).  Host arithmetic only. */
NFHMM_API int nfhmm_admission_plan(int n_queued, const size_t *footprints, size_t bytes_in_use,
                         size_t budget, int resident, int max_slots, int *admit);

/* ------------------------------------------------------------------ fitting */

/* Blocking fit of one problem whose arrays are in host memory.  Inputs are
 * validated (nfhmm_validate) and copied; the caller may reuse them on return.
 * Outputs are written to the host arrays of *r.  Copies go through a pinned host
 * ring of the context (1 GiB, allocated on first use; pageable copies when it has
 * no room), and the device working memory stays cached in the context for the
 * next call of the same shapes.  An input or output array that is itself in pinned
 * (page-locked) host memory is copied to or from the device directly instead. */
NFHMM_API nfhmm_status nfhmm_fit(nfhmm_ctx *ctx, const nfhmm_problem *p, nfhmm_precision prec,
                       nfhmm_result *r);

/* Blocking fit of n independent problems (host memory) that run together: every
 * iteration's kernels cover all n jobs in the same launches.  Each job's results
 * (alpha, post, sep and the elbo trace) are bitwise identical to fitting it alone:
 * a batch that fills the chip takes the BF16 spectrum contraction in larger tiles,
 * but every tile sums the bound's per-bin terms in the same order.  Returns the
 * first failing job's status; the other jobs' outputs are complete. */
NFHMM_API nfhmm_status nfhmm_fit_batch(nfhmm_ctx *ctx, int n, const nfhmm_problem *ps,
                             nfhmm_precision prec, nfhmm_result *rs);

/* As nfhmm_fit_batch, but every array pointer in ps[] and rs[] is a device pointer
 * on the context's device (the structs themselves are in host memory) and the work
 * is ordered on `hip_stream` (a hipStream_t; NULL = the context's own stream).  Only the dims
 * are checked on the host; V >= 0 / finite and W rows summing to 1 are checked on the
 * device and reported as NFHMM_E_INVALID.  Blocks until the work is done.
 * Working memory stays cached in the context for the next call of the same shapes. */
NFHMM_API nfhmm_status nfhmm_fit_batch_device(nfhmm_ctx *ctx, int n, const nfhmm_problem *ps,
                                    nfhmm_precision prec, nfhmm_result *rs, void *hip_stream);

/* Single-problem form of nfhmm_fit_batch_device. */
NFHMM_API nfhmm_status nfhmm_fit_device(nfhmm_ctx *ctx, const nfhmm_problem *dev_p,
                              nfhmm_precision prec, nfhmm_result *dev_r, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): nfhmm_fit_device for one
 * problem, with every intermediate array in a fixed working area that the library
 * holds on each device for the life of the process (96 MiB, a static device array)
 * instead of memory it allocates.  The call allocates nothing: no hipMalloc, no
 * hipFree, no event or stream creation; the caller passes the device inputs and
 * outputs as for nfhmm_fit_device, and the work runs on `hip_stream` (NULL: the
 * context's stream) in order, one kernel after another.  Blocks until done and
 * returns the job's status as nfhmm_fit_device does.
 * Limits: the job's working set (the sum of its arrays, about 25 MB for S=2, N=40,
 * K=10, F=513, T=1000) must fit the 96 MiB, else NFHMM_E_NOMEM with nothing run.
 * Every call on one device (from any context of the process) uses the same area and
 * overwrites what the last call left there: calls that overlap in time on one GPU
 * race and must be serialised by the caller. */
NFHMM_API nfhmm_status nfhmm_fit_device_noalloc(nfhmm_ctx *ctx, const nfhmm_problem *dev_p,
                                                nfhmm_precision prec, nfhmm_result *dev_r, void *hip_stream);

/* ------------------------------------------------------------------ learning a source model */

/* EM learning of one source's N-HMM (Section 2.1): the source model the separation
 * takes as input, learned from a spectrogram of that source alone (Section 5 learns
 * one per speaker).  States D_t follow a Markov chain (A, pi); each of the quanta
 * of frame t draws an element z from theta_t(D_t) and a frequency from
 * beta(D_t, z).  Section 2.1 states that EM finds the maximum-likelihood
 * dictionaries and transitions, with theta_t as per-frame nuisance parameters, and
 * gives no steps; one iteration here is, from the parameters it starts with:
 *   E-step  P_t(f | d) = sum_z theta_t(d, z) beta(d, z, f); the frame log-likelihood
 *           sum_f V_tf ln P_t(f | d) (the multinomial constant dropped; in double);
 *           the chain's marginals gamma_t(d) and pairwise marginals xi_t(i, j)
 *   M-step  beta'(d, z, f) ~ beta(d, z, f) sum_t gamma_t(d) theta_t(d, z) V_tf / P_t(f | d)
 *           (normalised over f); theta'_t(d, z) ~ theta_t(d, z) sum_f beta(d, z, f)
 *           V_tf / P_t(f | d) (over z); A' ~ sum_t xi_t (rows); pi' = gamma_0.
 *           A row that receives no expected counts keeps its previous values.
 * Layouts as the separation's: V [T][F]; W [N][K][F] (each row of F values sums to
 * 1); theta [T][N][K] (each row of K values sums to 1); A [N][N] row-stochastic,
 * A[i][j] = P(D_t = j | D_{t-1} = i); pi [N].  Limits: 1 <= N <= 64, 1 <= K <= 32,
 * iters >= 1.  The log-likelihood ln P(V) is non-decreasing over the iterations. */
typedef struct {
  int32_t N, K;
  int64_t F, T;
  const float *V;       /* [T][F]    counts >= 0, finite                                      */
  const float *W;       /* [N][K][F] starting dictionaries, rows >= 0 summing to 1 within 1e-4 */
  const float *theta;   /* [T][N][K] starting weights, entries > 0, rows summing to 1 within 1e-4 */
  const float *A;       /* [N][N]    starting transitions, rows summing to 1 within 1e-4      */
  const float *pi;      /* [N]       starting initial-state probabilities                     */
  int32_t iters;
} nfhmm_nhmm_problem;

typedef struct {
  float *W, *theta, *A, *pi;   /* the learned parameters (same layouts); any may be NULL     */
  double *loglik;              /* [iters] ln P(V) of the parameters each iteration started
                                  from (multinomial constant dropped), or NULL              */
} nfhmm_nhmm_result;

/* Blocking EM on host arrays.  The inputs are checked as the layouts above state,
 * plus: every state's dictionary is non-zero in every bin where V > 0 (else that
 * state's likelihood is 0 at that frame and the update is undefined) ->
 * NFHMM_E_INVALID.  Inputs are copied; outputs are written on return. */
NFHMM_API nfhmm_status nfhmm_learn_nhmm(nfhmm_ctx *ctx, const nfhmm_nhmm_problem *p, nfhmm_nhmm_result *r);

/* EM of n independent source models in one run (Section 5 learns one model per
 * speaker), on host arrays checked and copied as for nfhmm_learn_nhmm: every
 * iteration's kernels cover all problems still iterating in the same launches.
 * The forward-backward of a chain of T >= 98 frames runs time-parallel (chunks of
 * 32 frames, N times the work) while the batch holds at most 2^19 state-frames
 * (sum of N * T); in larger batches every chain takes the sequential sweeps, side
 * by side.  Problems may differ in every size and iteration count; each problem's
 * results are bitwise identical to learning it alone when the batch and the
 * problem alone fall on the same side of that line, and equal up to rounding
 * otherwise.  1 <= n <= 65535; NFHMM_E_INVALID
 * (naming the problem) if any problem fails the checks, or if the batch's largest
 * N, F and T together exceed the launch limits (split the batch).  Device memory:
 * the sum of the problems' working sets. */
NFHMM_API nfhmm_status nfhmm_learn_nhmm_batch(nfhmm_ctx *ctx, int n, const nfhmm_nhmm_problem *ps,
                                              nfhmm_nhmm_result *rs);

/* The same on device pointers (inputs and outputs; the structs in host memory),
 * ordered on hip_stream (NULL: the context's stream).  Only the sizes are checked.
 * Blocks until the work is done. */
NFHMM_API nfhmm_status nfhmm_learn_nhmm_device(nfhmm_ctx *ctx, const nfhmm_nhmm_problem *dev_p,
                                               nfhmm_nhmm_result *dev_r, void *hip_stream);

/* ------------------------------------------------------------------ serving */

/* Queue one job (host memory; validated and copied before return).  Jobs are
 * admitted first-in-first-out when the device-memory budget and a slot allow; every
 * resident job advances one iteration per round of batched launches, so jobs that
 * arrive while others run join the next round.  The output arrays of *r must stay
 * valid until nfhmm_wait returns for this job; those in pinned (page-locked) host
 * memory are written by a direct device-to-host copy, the others through the
 * context's pinned staging ring.  NFHMM_E_NOMEM if the job can never fit. */
NFHMM_API nfhmm_status nfhmm_submit(nfhmm_ctx *ctx, const nfhmm_problem *p, nfhmm_precision prec,
                          nfhmm_result *r, uint64_t *job_id);

/* *done = 1 once the job's outputs are in host memory (or it failed / was cancelled). */
NFHMM_API nfhmm_status nfhmm_poll(nfhmm_ctx *ctx, uint64_t job_id, int *done);

/* Block until the job ends; returns its status and (if non-NULL) the seconds from
 * submit to the outputs being in host memory.  The job id is released afterwards. */
NFHMM_API nfhmm_status nfhmm_wait(nfhmm_ctx *ctx, uint64_t job_id, double *latency_s);

/* Cancel a queued or resident job; nfhmm_wait then returns NFHMM_E_CANCELLED. */
NFHMM_API nfhmm_status nfhmm_cancel(nfhmm_ctx *ctx, uint64_t job_id);

/* ------------------------------------------------------------------ measurement */

/* Kernel kinds that nfhmm_profile_read reports. */
typedef enum {
  NFHMM_K_SPECTRUM = 0,   /* Lambda = beta w and R = V / Lambda (normaliser of Eq. 7)       */
  NFHMM_K_COUNTS   = 1,   /* c = w (.) beta^T R (first term of Eq. 6)                      */
  NFHMM_K_CHAINS   = 2,   /* forward-backward of every source chain                         */
  NFHMM_K_UPDATE   = 3,   /* Eq. 6, digamma, Eq. 8 and the per-frame bound terms            */
  NFHMM_K_POSTERIOR = 4,  /* d-hat from the messages (+ exact log-space pass where needed)  */
  NFHMM_K_COUNT    = 5
} nfhmm_kernel_kind;

/* Enable (1) or disable (0) timing of every later iteration launch of the context:
 * a pair of HIP events brackets each launch on the stream that launch runs on.
 * Enabling clears earlier records. */
NFHMM_API nfhmm_status nfhmm_profile_enable(nfhmm_ctx *ctx, int enable);

/* Split later blocking batches (nfhmm_fit_batch*) across `lanes` stream lanes (1 or
 * 2; default 2): each lane advances its share of the jobs on its own pair of
 * streams, so one lane's update overlaps the other's contractions. */
NFHMM_API nfhmm_status nfhmm_set_lanes(nfhmm_ctx *ctx, int lanes);

/* Restrict the timing of nfhmm_profile_enable to the kinds whose bit (1 << kind)
 * is set in `mask` (default: every kind).  Fewer timed launches perturb the
 * timed run less. */
NFHMM_API nfhmm_status nfhmm_profile_select(nfhmm_ctx *ctx, unsigned mask);

/* Wait for the recorded launches of `kind`, then return their number and summed
 * device duration in milliseconds. */
NFHMM_API nfhmm_status nfhmm_profile_read(nfhmm_ctx *ctx, int kind, int64_t *launches, double *total_ms);

/* ------------------------------------------------------------------ building blocks */

/* The forward-backward pass of one chain on the device (the step after Eq. 8 of the
 * paper; the recursion it cites from Rabiner 1989), on host arrays:
 *   logev [T][N] log evidence per frame and state (finite or -inf),
 *   A [N][N] row-stochastic, pi [N];
 *   post [T][N] receives the marginals P(D_t = n | evidence), *lnZ the log normaliser. */
NFHMM_API nfhmm_status nfhmm_chain_posterior(nfhmm_ctx *ctx, int N, int64_t T, const float *logev,
                                   const float *A, const float *pi, float *post, double *lnZ);

/* The device digamma and log-gamma (float32) used by Eqs. 7-8 and the bound, evaluated
 * on n host values x >= 1e-3 (psi and lgam may be NULL). */
NFHMM_API nfhmm_status nfhmm_special_functions(nfhmm_ctx *ctx, int64_t n, const float *x, float *psi,
                                     float *lgam);

/* ------------------------------------------------------------------ time domain */

/* The spectrograms the method works on come from a short-time Fourier transform
 * (Section 5: 16 kHz audio, 64 ms windows, 16 ms hop, i.e. nfft = 1024, hop = 256,
 * F = 513 bins), and the separated sources are taken back to the time domain with
 * the phase of the mixture (Section 1).  Conventions:
 *   window    periodic Hann, w[i] = (1 - cos(2 pi i / nfft)) / 2;
 *   framing   frame t covers samples [t hop, t hop + nfft) of the signal, no padding,
 *             so a signal of n >= nfft samples has T = 1 + (n - nfft) / hop frames
 *             (integer division; the samples after the last frame are not analysed);
 *   transform X_t[k] = sum_i w[i] x[t hop + i] exp(-2 pi i k i' / nfft), k = 0..nfft/2;
 *   inverse   weighted overlap-add: y[i] = sum_t w[j] z_t[j] / sum_t w[j]^2 over the
 *             frames covering i (j = i - t hop), z_t the inverse transform of the
 *             Hermitian spectrum mag_t exp(i phase_t) (the imaginary parts of bins 0
 *             and nfft/2 dropped); y[i] = 0 where no window weight covers i.  With
 *             hop <= nfft / 2 this inverts the transform exactly where at least one
 *             frame has w[j] > 0.
 * nfft is a power of two in [64, 4096], 1 <= hop <= nfft, 1 <= B <= 65535 signals
 * (or mixtures) processed together, 1 <= T <= 2^30 frames; arrays are dense, C order, float32; errors are
 * NFHMM_E_INVALID for bad sizes and NFHMM_E_DEVICE for a failing HIP call. */

/* Frames of a signal of n samples (0 if n < nfft). */
NFHMM_API int64_t nfhmm_stft_frames(int32_t nfft, int32_t hop, int64_t n);

/* STFT of B signals x[B][n] (host arrays): mag and phase [B][T][nfft/2 + 1] receive
 * |X| and arg X (radians, (-pi, pi]). */
NFHMM_API nfhmm_status nfhmm_stft(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, const float *x,
                                  int64_t n, float *mag, float *phase);

/* Inverse STFT of B mixtures with S magnitude sets each, mag[B][S][T][nfft/2 + 1]
 * (e.g. the separated sources V* of each mixture), source (b, s) resynthesised with
 * its mixture's phase[b][T][nfft/2 + 1]: y[B][S][n] (host arrays).  B * S <= 65535;
 * T may exceed the frame count of n (frames past the end contribute nothing).  A
 * phase may lie in any turn (it is reduced to [-pi, pi] first); the result is
 * within 1e-5 of max |y| of the exact inverse where the window weight is >= 0.1,
 * up to phases of about 2^14 pi, beyond which float32 phases lose the precision. */
NFHMM_API nfhmm_status nfhmm_istft(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, int32_t S,
                                   const float *mag, const float *phase, int64_t T, float *y, int64_t n);

/* The same on device pointers, ordered on hip_stream (NULL: the context's stream);
 * they return once the work is queued and allocate nothing. */
NFHMM_API nfhmm_status nfhmm_stft_device(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, const float *x,
                                         int64_t n, float *mag, float *phase, void *hip_stream);
NFHMM_API nfhmm_status nfhmm_istft_device(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, int32_t S,
                                          const float *mag, const float *phase, int64_t T, float *y, int64_t n,
                                          void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* NFHMM_H */
