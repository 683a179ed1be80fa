/*
 * hmm.h -- C ABI of the MI355X (gfx950) tremor-HMM likelihood library.
 *
 * The library evaluates the likelihood of the tremor hidden Markov model of
 * Stoltz, Stoltz, Obara, Wang & Bryant, "A 1000-fold Acceleration of Hidden
 * Markov Model Fitting using Graphical Processing Units" (arXiv 2003.03508):
 *
 *   eq. (1)  emission matrix P(x) = diag(e_1..e_K),
 *            e_k = p_k * phi(x | mu_k, Sigma_k)  for a tremor at x in R^2,
 *            e_k = 1 - p_k                        for "no tremor";
 *            phi is the bivariate normal density (full normalising constant).
 *   eq. (2)  L = delta^T Gamma P(x_0) Gamma P(x_1) ... Gamma P(x_N) 1,
 *            Gamma applied before the first emission, as written there.
 *
 * and returns ln L in double precision.  Conventions shared by every entry
 * point:
 *
 *   - All array arguments are DEVICE pointers (memory of the device the
 *     context was created on), owned by the caller.  The library neither
 *     frees nor keeps them past the call.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *     stream) and is asynchronous: results are valid once the caller has
 *     synchronised that stream.  A context holds scratch memory that calls
 *     reuse, so calls that share a context must be issued on one stream (or be
 *     otherwise serialised); a context is not thread-safe.
 *   - Layouts: delta[K]; Gamma[K*K] row-major with Gamma[i*K+j] the probability
 *     of moving from state i to state j; p[K]; mu[2K] as (x, y) pairs in km;
 *     Sigma[3K] as (Sxx, Sxy, Syy) triples in km^2; flag[T] uint8 (1 = tremor,
 *     0 = none); xy[2T] as (x, y) pairs, read only where flag is 1.  T counts
 *     observations (the paper's N+1).
 *   - Errors the host can see (null pointers, K or T out of range, unknown
 *     algorithm) are returned as an hmm_status and nothing is enqueued.
 *     Problems only the device can see are reported in the result: NaN for
 *     invalid parameters (delta_k < 0, Gamma_ij outside [0,1], p_k outside
 *     [0,1], non-finite mu, Sigma not symmetric positive definite, any
 *     non-finite parameter) or invalid data (a flag other than 0/1, a tremor
 *     with a non-finite location); -inf when L = 0 with valid inputs.
 *     T = 0 gives ln(sum_k delta_k), the empty chain of eq. (2).
 *   - Numerics of the GPU paths: log2 e_{t,k} is evaluated in FP64, shifted
 *     by the integer s_t = floor(max_k log2 e_{t,k}) - 96 (carried exactly),
 *     and exponentiated as 2^n * 2^f with n an integer and only f in [0, 1)
 *     rounded to FP32; products accumulate in FP32 with exact power-of-two
 *     rescaling; the final combination of exponents and the logarithm are
 *     FP64.  An emission below 2^-222 of its step's largest one loses
 *     precision (FP32 subnormal) and below 2^-245 counts as zero; the FP64
 *     oracle's limit is 2^-1074.  With any transition matrix whose entries
 *     are not tiny this cannot change ln L measurably.
 */
#ifndef HMM_MI355X_H
#define HMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMM_OK = 0,
    HMM_E_INVALID_ARG = -1,  /* null pointer, K/T/n out of range, bad option      */
    HMM_E_UNSUPPORTED = -2,  /* valid request this build does not implement      */
    HMM_E_DEVICE = -3,       /* a HIP call failed (launch, allocation of scratch) */
    HMM_E_NOMEM = -4         /* scratch memory could not be allocated            */
} hmm_status;

typedef enum {
    /* Algorithm 1 (the forward algorithm) on the GPU: one wavefront walks the
     * T observations in order, v <- (v Gamma) P(x_t).  O(T K^2) work, T
     * dependent steps.  K <= 128. */
    HMM_SERIAL_F32 = 0,
    /* The paper's parallel plan (section "The likelihood algorithm", steps
     * 1-3): the chain Gamma P(x_0) ... Gamma P(x_N) is cut into segments whose
     * products are formed independently on the matrix cores (FP32 MFMA) with
     * the emissions computed in the same kernel, then the segment products are
     * combined by a tree of matrix products on the GPU.  O(T K^3) work.
     * K <= 80. */
    HMM_BLOCKED_F32 = 1,
    HMM_BLOCKED_BF16 = 2,   /* reserved: bf16 operands, FP32 accumulation */
    HMM_BLOCKED_F16 = 3     /* reserved: fp16 operands, FP32 accumulation */
} hmm_algo;

typedef struct hmm_ctx hmm_ctx;

/* Create a context on HIP device `device` (makes it current).  *out receives
 * the context.  Returns HMM_E_DEVICE if the device cannot be used. */
int hmm_ctx_create(hmm_ctx **out, int device);

/* Release the context and its scratch memory (synchronises the device). */
int hmm_ctx_destroy(hmm_ctx *ctx);

/* ln L of eq. (2) for one parameter set and one observation sequence.
 *   K      number of hidden states, 1 <= K <= 128 (K <= 80 for blocked algos)
 *   delta, Gamma, p, mu, Sigma, flag, xy   device arrays as described above
 *   T      number of observations, 0 <= T < 2^40
 *   algo   an hmm_algo value
 *   out    device pointer to one double, receives ln L
 * Returns HMM_OK when the work was enqueued. */
int hmm_loglik(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma,
               const double *p, const double *mu, const double *Sigma, int64_t T,
               const uint8_t *flag, const double *xy, int32_t algo, void *stream,
               double *out);

/* ln L of eq. (2) for n independent parameter sets, each with its own K and
 * observation sequence, in one launch sequence (batched evaluation of MCMC
 * chains or proposals).  The descriptor arrays are HOST arrays of n entries:
 *   K[s]          states of set s, 1 <= K[s] <= 80
 *   T[s]          observations of set s, 0 <= T[s] < 2^40
 *   param_off[s]  offset (in doubles) of set s's parameter block in `params`
 *   obs_off[s]    offset (in observations) of set s's sequence in flag / xy
 * Device arrays: `params` (params_len doubles) holds for every set the block
 *   delta[K] | Gamma[K*K] (row-major) | p[K] | mu[2K] | Sigma[3K]
 * flag (obs_len entries) / xy (2*obs_len) as in hmm_loglik; sets may share
 * observations (equal obs_off).  Every block and sequence must lie inside
 * its array (checked on the host: HMM_E_INVALID_ARG otherwise);
 * out[n] receives ln L of every set, with hmm_loglik's conventions (NaN for
 * invalid parameters or data of that set, -inf for L = 0).
 * algo: HMM_BLOCKED_F32 / _BF16 / _F16.  The context builds a plan (job
 * tables, per-set scratch) for these descriptors and device pointers and, by
 * default, captures the launch sequence in a HIP graph; a later call with
 * identical descriptors and pointers (the parameter VALUES may change)
 * replays the graph.  The plan depends on the segment lengths tuned by
 * hmm_autotune_batched. */
int hmm_loglik_batched(hmm_ctx *ctx, int32_t n, const int32_t *K, const int64_t *T,
                       const int64_t *param_off, const double *params, int64_t params_len,
                       const int64_t *obs_off, const uint8_t *flag, const double *xy,
                       int64_t obs_len, int32_t algo, void *stream, double *out);

/* Use (on != 0, default) or bypass HIP graph capture for batched calls. */
int hmm_ctx_set_batch_graph(hmm_ctx *ctx, int32_t on);

/* Segment-length autotuner of the batched path: for every class of sets that
 * share a kernel, times the class's launches (reps repetitions after one
 * warm-up) for segment lengths 256..4096 on the caller's own inputs and keeps
 * the fastest in the context (used by later batched calls).  Synchronous;
 * writes out[] as a side effect.  chosen_L (host, n entries, may be NULL)
 * receives the length chosen for each set. */
int hmm_autotune_batched(hmm_ctx *ctx, int32_t n, const int32_t *K, const int64_t *T,
                         const int64_t *param_off, const double *params, int64_t params_len,
                         const int64_t *obs_off, const uint8_t *flag, const double *xy,
                         int64_t obs_len, int32_t algo, double *out, int32_t reps,
                         int64_t *chosen_L);

/* The emission stage of the GPU paths (eq. 1) on its own, for inspection.
 * For every observation t it writes the integer shift s_t (shift[t]) and the
 * scaled emissions  e_hat[t*K + k] = e_{t,k} * 2^(-s_t)  in FP32, where
 * s_t = floor(log2 max_k e_{t,k}) - 96, so the largest scaled emission lies
 * in [2^96, 2^97).
 * shift: device int32[T]; e_hat: device float[T*K].  status: device int32[1],
 * receives a bit mask (1 = invalid parameters, 2 = invalid data). */
int hmm_emission(hmm_ctx *ctx, int32_t K, const double *p, const double *mu,
                 const double *Sigma, int64_t T, const uint8_t *flag, const double *xy,
                 void *stream, int32_t *shift, float *e_hat, int32_t *status);

/* Tuning knobs of the blocked path.  block_len: observations per segment
 * (0 = automatic; otherwise >= 1).  fold: products a wavefront multiplies in
 * sequence at each level of the combination tree before the workgroup's
 * binary tree (0 = automatic; otherwise 1..64).  They change the order of
 * floating-point operations only. */
int hmm_ctx_set_blocking(hmm_ctx *ctx, int64_t block_len, int32_t fold);

/* Segment length and tree shape the blocked path would use for (K, T):
 * *block_len, *n_blocks, *levels (reduction launches).  Host only; ctx may be
 * NULL for the default knobs. */
int hmm_blocked_plan(hmm_ctx *ctx, int32_t K, int64_t T, int64_t *block_len,
                     int64_t *n_blocks, int32_t *levels);

/* Kernel timing for measurement.  While enabled (on != 0), every blocked
 * call records a pair of HIP events on its stream around its segment-product
 * kernel (the dominant kernel of HMM_BLOCKED_*).  hmm_ctx_profile_read waits
 * for the recorded events, returns the number of timed launches and their
 * summed duration in milliseconds, and forgets them.  At most 65536 launches
 * are kept; later ones are not timed.  Enabling or disabling also forgets. */
int hmm_ctx_profile(hmm_ctx *ctx, int32_t on);
int hmm_ctx_profile_read(hmm_ctx *ctx, int64_t *launches, double *total_ms);

/* Human-readable name of a status code (static storage). */
const char *hmm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* HMM_MI355X_H */
