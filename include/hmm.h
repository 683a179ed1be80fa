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
 *     0 = none); xy[2T] as (x, y) pairs, read only where flag is 1, each pair
 *     loaded as one 16-byte word: xy must be 16-byte aligned (every device
 *     allocation is; a view starting at an odd double is rejected with
 *     HMM_E_INVALID_ARG).  T counts observations (the paper's N+1).
 *   - Errors the host can see (null pointers, K or T out of range, unknown
 *     algorithm, a misaligned xy) are returned as an hmm_status and nothing is
 *     enqueued.  A request whose launches would exceed HIP's 2^32 threads per
 *     launch returns HMM_E_UNSUPPORTED; with the automatic segment lengths
 *     that happens only for hmm_emission at T >= 2^32 - 64 and for
 *     hmm_viterbi above T = 2^35 (K <= 32) or 2^34 (K > 32); a segment length
 *     set with hmm_ctx_set_blocking lowers the limit of the blocked and
 *     reverse-direction paths to about 2^26 segments (2^22 workgroups of the
 *     likelihood's segment kernel).
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
 *     are not tiny this cannot change ln L measurably.  HMM_SERIAL_F32 scales
 *     the whole forward vector by one power of two per step, so a state whose
 *     forward variable falls more than ~2^126 below the largest one is lost;
 *     that needs a transition matrix that (almost) forbids moving between
 *     states (e.g. the identity).  The blocked paths keep one exponent per
 *     start state and are not limited this way.
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
    HMM_E_UNSUPPORTED = -2,  /* valid request the library does not implement     */
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
    /* The same plan with the segment products on 16-bit MFMA: the running
     * product and the emission-scaled transition matrix are rounded to bf16
     * (resp. fp16) operands, accumulation stays FP32, rescaling by powers of
     * two.  Error grows with T (about T * 2^-8 resp. T * 2^-11 relative per
     * step at worst); the FP32 path is the reference.  K <= 80. */
    HMM_BLOCKED_BF16 = 2,
    HMM_BLOCKED_F16 = 3,
    /* BF16 / FP16 operands with the transition matrix split in two 16-bit
     * parts, hi = round(Gamma) and lo = round(Gamma - hi), both multiplied
     * into the same FP32 accumulator: twice the matrix-core work, and the
     * transition matrix then carries about twice the operand precision.
     * Rounding Gamma once (HMM_BLOCKED_BF16 / _F16) makes an error that is
     * the same at every step and grows in proportion to T; the split removes
     * most of it, leaving the per-step rounding of the running product.
     * hmm_loglik only (tremor model, one set); K <= 80. */
    HMM_BLOCKED_BF16_SPLIT = 4,
    HMM_BLOCKED_F16_SPLIT = 5
} hmm_algo;

typedef struct hmm_ctx hmm_ctx;

/* Host-side check of one parameter set of eq. (1)-(2) (a debugging aid; the
 * kernels themselves only reject non-finite or out-of-range entries and
 * report them as NaN).  All pointers are HOST arrays laid out as for
 * hmm_loglik.  Checks, in this order: delta and every row of Gamma are
 * probability vectors (entries finite and >= 0, sum within tol of 1;
 * tol <= 0 selects 1e-12 * K), p_k in [0, 1], mu finite, Sigma_k symmetric
 * positive definite (Sxx > 0 and Sxx Syy - Sxy^2 > 0, all finite).  Returns
 * HMM_OK, or HMM_E_INVALID_ARG at the first failing check with its code in
 * *what (may be NULL); K < 1 or a null array also give HMM_E_INVALID_ARG
 * (*what = HMM_PARAMS_OK then).  Touches no device. */
typedef enum {
    HMM_PARAMS_OK = 0,
    HMM_PARAMS_BAD_DELTA = 1,
    HMM_PARAMS_BAD_GAMMA = 2,
    HMM_PARAMS_BAD_P = 3,
    HMM_PARAMS_BAD_MU = 4,
    HMM_PARAMS_BAD_SIGMA = 5
} hmm_params_check;

int hmm_validate_params(int32_t K, const double *delta, const double *Gamma, const double *p,
                        const double *mu, const double *Sigma, double tol, int32_t *what);

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

/* hmm_loglik without a context and without any device allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * algorithms, conventions and results as hmm_loglik with the automatic
 * segment lengths (bit-identical output), on the CURRENT HIP device.
 * Scratch: a fixed 16 MiB device array inside the library, one copy per
 * GPU, held until the process ends; its device address is looked up once
 * per device on the first call there.  Every K <= 80 (blocked) and K <= 128
 * (serial) fits at any T; a request that would need more scratch returns
 * HMM_E_UNSUPPORTED and enqueues nothing.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (two streams, two threads)
 * race and give undefined results, so serialise them.  Nothing from an
 * earlier call is read: each call rewrites every scratch word it reads. */
int hmm_loglik_noalloc(int32_t K, const double *delta, const double *Gamma,
                       const double *p, const double *mu, const double *Sigma, int64_t T,
                       const uint8_t *flag, const double *xy, int32_t algo, void *stream,
                       double *out);

/* Other emission models.  The method needs only the emission function of the
 * model (the matrix chain of eq. 2 is the same), so the same kernels serve
 * other HMMs:
 *   HMM_EMIS_POISSON  counts: e_k(y) = lambda_k^y e^(-lambda_k) / y!
 *                     e0 = lambda[K] (> 0), e1 unused (may be NULL),
 *                     obs = int32 counts[T] (>= 0)
 *   HMM_EMIS_GAUSS1D  e_k(x) = N(x; mu_k, var_k)
 *                     e0 = mu[K], e1 = var[K] (> 0), obs = double values[T]
 * hmm_loglik_kind returns ln L of eq. (2) with those emissions, with
 * hmm_loglik's conventions (invalid parameters, a negative count or a
 * non-finite value give NaN; L = 0 gives -inf; T = 0 gives ln sum delta) and
 * numerics, for the same algorithms and K limits. */
typedef enum { HMM_EMIS_POISSON = 1, HMM_EMIS_GAUSS1D = 2 } hmm_emission_kind;

int hmm_loglik_kind(hmm_ctx *ctx, int32_t kind, int32_t K, const double *delta,
                    const double *Gamma, const double *e0, const double *e1, int64_t T,
                    const void *obs, int32_t algo, void *stream, double *out);

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

/* Work distribution of the batched segment kernels.  on != 0 (default): one
 * persistent launch per kernel class, about as many workgroups as the GPU
 * holds at once, each pulling (set, segment-group) jobs from an atomic
 * counter in decreasing order of their work; on == 0: one workgroup per job.
 * Both give the same result bit for bit (the jobs and their products are the
 * same; only the order in which workgroups take them differs). */
int hmm_ctx_set_batch_persistent(hmm_ctx *ctx, int32_t on);

/* Column packing of the FP32 blocked path.  A wavefront advances
 * G = floor(32 NT / K) segments at once, their start-state columns side by
 * side in NT 32-column MFMA tiles that share the Gamma^T operand, so one step
 * costs NT ceil(K / 2) MFMAs for all G instead of ceil(K / 2) per segment.
 * NT = 4 or 5 gives floor(32 NT / K) segments and 8 wavefronts per workgroup
 * (two per SIMD), NT = 2 three segments and 16 wavefronts (four per SIMD).
 * mode 1 (default, from measurements): NT = 5 for K = 19, 20, 22 (and 17 in
 * batched calls), NT = 2 for single-set calls with K = 21, NT = 4 for the
 * other 17 <= K <= 25; other K not packed.
 * mode 2: NT = 2 for 17 <= K <= 21.  mode 4: NT = 4 for 17 <= K <= 28.
 * mode 5: NT = 5 (8 wavefronts per workgroup) for K in {17, 19, 20, 22},
 * where five tiles hold more live columns than four.  Other K are not packed
 * under modes 2, 4 and 5.  mode 0: no packing.  Packed
 * segments have balanced lengths, floor or ceil of T over their number.
 * A single-set call packs when the segment length is automatic
 * (hmm_ctx_set_blocking with block_len 0) and T >= 16 * 256 * W, W = G times
 * the wavefronts per workgroup (the packed plan then gives every CU a
 * workgroup of segments of at least 16 observations); a batched call packs the
 * sets of a K the mode covers when together they give at least 256 such
 * workgroups.  Otherwise one segment per wavefront, which fills the chip
 * better.  Single-set calls of the other emission kinds (hmm_loglik_kind)
 * pack by the same rules.  The products are the same up to FP32 rounding
 * order.
 * HMM_E_INVALID_ARG for a null context or another mode. */
int hmm_ctx_set_packing(hmm_ctx *ctx, int32_t mode);

/* Autotuner of the batched path: for every class of sets that share a
 * kernel, times the class's launches (reps repetitions after one warm-up)
 * for segment lengths 256..4096 and for the segment kernel's full and half
 * wavefront count per workgroup, on the caller's own inputs, and keeps the
 * fastest pair in the context (used by later batched calls).  Synchronous;
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

/* ------------------------------------------------------------------------
 * Metropolis-Hastings over the model parameters (section "Monte Carlo Markov
 * Chains"; prior densities of Appendix A), many chains in parallel, each
 * iteration one batched exact likelihood evaluation of all chains' proposals.
 *
 * Parameter vector theta (unconstrained, FP64) of D = K*K + 4K entries:
 *   [0, K(K-1))    row i of Gamma as log(Gamma_ij / Gamma_ii), j != i ascending
 *   [.., +K)       logit p_k
 *   [.., +2K)      mu_k as (x, y) pairs, km
 *   [.., +2K)      log of Sigma_k's diagonal (xx, yy); Sigma_xy = 0
 * delta is fixed to the uniform distribution.  Log prior (additive constants
 * dropped, Jacobians of the transforms included):
 *   Gamma rows ~ Dirichlet(0.01, ..., 0.01)        -> 0.01 * sum_ij ln Gamma_ij
 *   p_k ~ Gamma(10, rate 100) for k < K/2 (mean 0.1), Gamma(810, rate 900)
 *     otherwise (mean 0.9), variance 0.001, truncated to (0, 1)
 *                                                  -> a ln p - b p + ln(1 - p)
 *   mu_k uniform on box = {x0, x1, y0, y1} (km)    -> 0 inside, -inf outside
 *   Sigma_k ~ inverse Wishart(nu = K, I_2) restricted to diagonal matrices
 *                                  -> -(K+1)/2 (w_x + w_y) - (e^-w_x + e^-w_y)/2
 *   with w = ln Sigma_diag.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011) with key = seed and
 * counter (index, chain, iteration, purpose); uniforms are
 * ((64-bit word >> 11) + 1/2) * 2^-53 of words (0,1) and (2,3); normals are
 * Box-Muller pairs (r cos 2 pi u1, r sin 2 pi u1), r = sqrt(-2 ln u0).
 * Purposes: 1 proposal normals (index = coordinate pair), 2 mixture choice,
 * 3 acceptance uniform, 4 training minibatch rows, 5 weight initialisation,
 * 6 held-out pairs of a training call, 7-9 the t-walk (below).
 * ------------------------------------------------------------------------ */
typedef enum { MCMC_RANDOM_WALK = 0, MCMC_LEARNED = 1, MCMC_TWALK = 2 } mcmc_proposal;

/* A sampler owns device memory, a private context whose batched plan its
 * iteration graphs replay, and one captured graph per proposal kind.  Like a
 * context it is not thread-safe: calls on one sampler must be serialised
 * (one host thread, one stream). */

typedef struct mcmc_chains mcmc_chains;

/* Device buffers and sizes of a sampler (filled by mcmc_view_get; the
 * pointers stay valid until mcmc_destroy).  C = n_chains, D = dim,
 * H = history_len. */
typedef struct {
    int32_t K, n_chains, dim;
    int64_t iterations;        /* MH iterations run so far                       */
    int64_t history_len;       /* iterations kept in the history ring            */
    double *theta;             /* [C*D] current states                           */
    double *loglik, *logprior; /* [C] of the current states                      */
    double *theta_prop;        /* [C*D] last proposals                           */
    double *loglik_prop, *logprior_prop, *logq_fwd; /* [C] of the last proposals */
    long long *accepts;        /* [C] accepted moves                             */
    float *history;            /* [H*C*D] states after iteration t at slot t % H  */
    double *history_logpost;   /* [H*C] loglik + logprior after iteration t      */
    float *net_weights;        /* [net_count] proposal network, layout below     */
    int64_t net_count;
    int32_t net_hidden;        /* width of both hidden layers (256)              */
    double *center, *in_scale, *out_scale; /* [D] network standardisation        */
    int32_t lag, trained;
    double *theta2;            /* [C*D] t-walk: second point of every chain      */
    double *loglik2, *logprior2; /* [C] of the second points                     */
    long long *twalk_counts;   /* [C*8] t-walk: kernel k proposed [2k], accepted [2k+1] */
    int32_t *twalk_code;       /* [C] last t-walk proposal: bit 0 moved, bit 1 x moved
                                  (else x'), bits 2-3 kernel (0 traverse, 1 walk,
                                  2 blow, 3 hop)                                  */
    int32_t companion;         /* second points set                              */
} mcmc_view;

/* Create n_chains chains for a K-state model over the observations
 * (flag, xy, T) -- device arrays that must stay valid while the sampler is
 * used.  box: HOST double[4] {x0, x1, y0, y1}.  history: iterations kept in
 * the ring that training reads (>= 2).  All chains start at theta = 0 with
 * ln L unset: call mcmc_set_state before mcmc_step.  1 <= K <= 80. */
int mcmc_create(hmm_ctx *ctx, int32_t K, int32_t n_chains, int64_t T, const uint8_t *flag,
                const double *xy, const double *box, uint64_t seed, int64_t history,
                mcmc_chains **out);
int mcmc_destroy(mcmc_chains *chains);

/* Set every chain's state (theta: device [C*D]) and the random-walk scales
 * (rw_scale: device [D], > 0), and evaluate ln L and the log prior there. */
int mcmc_set_state(mcmc_chains *chains, const double *theta, const double *rw_scale,
                   void *stream);
int mcmc_set_rw_scale(mcmc_chains *chains, const double *rw_scale, void *stream);

/* n_iter Metropolis-Hastings iterations of every chain.  Iteration t of
 * chain c:
 *   proposal MCMC_RANDOM_WALK:  theta' = theta + rw_scale .* z
 *   proposal MCMC_LEARNED: with probability 1 - eps (uniform of purpose 2)
 *     theta'_d = theta_d + out_scale_d (o_d + exp(o_{D+d}) z_d), o the network
 *     output at X = (theta - center) / in_scale; otherwise the random walk.
 *     Needs a trained (or loaded) network; 0 < eps < 1.
 *   z: normals of purpose 1.  theta' is mapped to model parameters, ln L of
 *   all chains' proposals is computed by the batched FP32 blocked path, and
 *   theta' is accepted when ln u < ln L' + ln prior' - ln L - ln prior +
 *   ln q(theta | theta') - ln q(theta' | theta), u of purpose 3 (q is the
 *   mixture density; the q terms are zero for the random walk).
 * The state after the iteration is written to the history ring.  Enqueued
 * on `stream`. */
int mcmc_step(mcmc_chains *chains, int32_t n_iter, int32_t proposal, double eps, void *stream);

/* The t-walk (Christen & Fox, "A general purpose sampling algorithm for
 * continuous distributions (the t-walk)", Bayesian Analysis 2010), the
 * general-purpose sampler that the paper runs over this posterior (section
 * "GPUeR-hmmer"), as mcmc_step(..., MCMC_TWALK, ...).  Every chain holds two
 * points x (theta) and x' (theta2).  Iteration t of chain c:
 *   (uh, uk) = the uniform pair of purpose 7, index 0: x moves when uh < 1/2
 *     (h = x, b = x'), else x' (h = x', b = x); uk picks the kernel
 *     (traverse below p_traverse, walk below p_traverse + p_walk, blow below
 *     p_traverse + p_walk + p_blow, else hop);
 *   coordinate j is in the subset phi when u_j < min(D, n1) / D, u_j the
 *     element j % 2 of the uniform pair of purpose 8, index j / 2;
 *   on phi (elsewhere y = h):
 *     traverse  y = b + beta (b - h); (v1, v2) the uniform pair of purpose 9,
 *               index 0; beta = v2^(1/(a_t+1)) if v1 < (a_t-1)/(2 a_t), else
 *               v2^(1/(1-a_t)); ln factor = (n_phi - 2) ln beta
 *     walk      y = h + (h - b) z, z = a_w/(1+a_w) (-1 + 2v + a_w v^2), v the
 *               uniforms of purpose 9 laid out as for phi; ln factor = 0
 *     blow      y = b + s z, s = max_phi |h - b|
 *     hop       y = h + s z, s = max_phi |h - b| / 3
 *               z the Box-Muller normals of purpose 9 laid out as for phi;
 *               ln factor = ln g(h | y) - ln g(y | h), g the product over phi
 *               of the normal densities of the move (centre b for blow, the
 *               moving point for hop; the scale from the starting point);
 *               -inf when the reverse scale is 0
 *   an empty phi (or s = 0) does not move; otherwise y is accepted into the
 *   moving point when ln u < ln L(y) + ln prior(y) - ln L(h) - ln prior(h) +
 *   ln factor, u the first uniform of purpose 3, index 0.
 * The history ring records x.  One likelihood evaluation per chain and
 * iteration, by the batched FP32 blocked path.
 *   mcmc_set_companion  sets x' of every chain (theta2: device [C*D]) and
 *                       evaluates ln L and the log prior there; needs
 *                       mcmc_set_state first; required before MCMC_TWALK steps
 *   mcmc_set_twalk      tuning: HOST double[6] = {p_traverse, p_walk, p_blow,
 *                       a_t, a_w, n1}, hop taking the rest; probabilities >= 0
 *                       summing to <= 1, a_t > 1, a_w > 0, n1 > 0.  The default
 *                       is Christen & Fox's {0.4918, 0.4918, 0.0082, 6, 1.5, 4}. */
int mcmc_set_companion(mcmc_chains *chains, const double *theta2, void *stream);
int mcmc_set_twalk(mcmc_chains *chains, const double *tuning);

int mcmc_view_get(mcmc_chains *chains, mcmc_view *view);

/* Options of mcmc_train_proposal. */
typedef struct {
    int32_t steps;        /* Adam steps (0: only the start described below)          */
    int32_t batch;        /* pairs per minibatch, 1..65535                            */
    int32_t lag;          /* pair lag in iterations (fixed by the first call)         */
    double lr;            /* Adam learning rate (beta 0.9 / 0.999, eps 1e-8)          */
    double weight_decay;  /* decoupled weight decay on W1, W2, W3                     */
    int64_t window;       /* iterations of history used (0: as far as the ring goes)  */
    int64_t window_end;   /* the window ends before this iteration (0: the current)   */
    double holdout;       /* fraction of the window (its end) held out, in [0, 1)     */
    int32_t val_every;    /* Adam steps between evaluations of the held-out loss      */
    int32_t val_batch;    /* held-out pairs evaluated, 1..65535                       */
} mcmc_train_opts;

/* Train the learned proposal on lagged pairs (theta_t, theta_{t+lag}) of a
 * window of history: the `window` iterations before iteration `window_end`.
 * With holdout > 0 the window is split in time: pairs starting in its first
 * 1 - holdout part train, pairs starting in the rest are held out.  Adam
 * steps run on minibatches of training pairs (time and chain drawn with
 * Philox purpose 4, iteration word = the network's Adam step) of the
 * Gaussian negative log-likelihood of the move.  The first call after
 * creation or mcmc_reset_proposal fixes, from the training pairs, the
 * standardisation (center and in_scale: mean and standard deviation of
 * theta; out_scale: standard deviation of the lag move; scales floored at
 * 0.1 * rw_scale) and the lag, and starts the network at the least-squares
 * fit of its linear part: per coordinate, move/out_scale = a x + b + noise of
 * standard deviation s gives the skip a, the mean bias b (b3[d]) and the
 * log-sd bias ln s (b3[D+d]), with W3 = 0.  With holdout > 0, val_batch
 * held-out pairs (purpose 6) are evaluated before the first step and every
 * val_every steps; the call ends with the weights of the lowest held-out loss
 * (possibly the starting ones).
 * loss_out: device float[steps] or NULL (each step's minibatch loss);
 * val_out: device float[1 + ceil(steps / val_every)] or NULL (held-out
 * losses); best_step: host int or NULL, receives the Adam step (0-based,
 * within this call) whose weights were kept, -1 for the starting weights
 * (synchronises the stream).
 * Network: X (D) -> h1 = tanh(X W1 + b1) (256) -> h2 = tanh(h1 W2 + b2) (256)
 *          -> o = h2 W3 + b3 (2D), plus a per-coordinate linear skip on the
 *          mean outputs: o[d] += a[d] X[d] for d < D (it represents the
 *          mean reversion of lagged moves coordinate by coordinate, which the
 *          256-wide layers cannot for D > 256).  Weights flat, FP32, in the
 *          order W1 [D][256], b1, W2 [256][256], b2, W3 [256][2D], b3, a [D],
 *          each W row-major with the input index first. */
int mcmc_train_proposal(mcmc_chains *chains, const mcmc_train_opts *opts, void *stream,
                        float *loss_out, float *val_out, int32_t *best_step);

/* Forget the trained network: weights re-initialised from `seed` (Glorot
 * uniform hidden layers, zero output layer, biases and skip), Adam state
 * cleared; the next training call recomputes the standardisation and may
 * choose a new lag. */
int mcmc_reset_proposal(mcmc_chains *chains, uint64_t seed, void *stream);

/* The proposal network on its own (for checks): network outputs out[n*2D]
 * for inputs X[n*D] (device, FP32). */
int mlp_forward(mcmc_chains *chains, int32_t n, const float *X, float *out, void *stream);

/* Loss terms row_loss[B] (each with the 1/B factor) and the gradient
 * grad[net_count] (same layout as the weights) of the training loss for a
 * given minibatch: inputs X[B*D] and targets R[B*D] (moves in units of
 * out_scale), device FP32.  No update. */
int mlp_loss_grad(mcmc_chains *chains, int32_t B, const float *X, const float *R,
                  float *row_loss, float *grad, void *stream);

/* Install network weights and standardisation (device arrays) as if trained
 * with this lag. */
int mlp_set_weights(mcmc_chains *chains, const float *weights, const double *center,
                    const double *in_scale, const double *out_scale, int32_t lag, void *stream);

/* The parameter transform of the sampler on its own: for n vectors theta
 * (device [n*D]) writes the likelihood blocks params[n * K(K+7)] in the
 * layout of hmm_loglik_batched and the log priors logprior[n].  box: HOST
 * double[4].  1 <= K <= 128. */
int hmm_theta_to_params(hmm_ctx *ctx, int32_t K, int32_t n, const double *theta,
                        const double *box, double *params, double *logprior, void *stream);

/* ------------------------------------------------------------------------
 * State posteriors and the gradient of ln L (forward-backward) for the tremor
 * model of eq. (1)-(2), with s_{-1} ~ delta the state before x_0 as in eq. (2).
 * Computed around the same segment products as the blocked likelihood
 * (section "The likelihood algorithm"): the products give the forward and
 * backward messages at segment boundaries, then every segment reruns the
 * forward and backward recursions over its own observations (FP32 within a
 * segment, FP64 at the boundaries and in all sums).  1 <= K <= 80.
 *
 * hmm_posterior: device outputs
 *   gamma  float [T*K]: gamma[t*K + k] = P(s_t = k | x_0..x_{T-1})
 *          (required when T > 0; also used as scratch during the call)
 *   stats  double [K*K + K + 7K] (may be NULL):
 *          [0, K*K)     xi[i*K + j] = sum_{t=0..T-1} P(s_{t-1} = i, s_t = j | x)
 *                       (t = 0 is the step from s_{-1})
 *          [K*K, +K)    P(s_{-1} = i | x)
 *          [.., +7K)    per state k: sum_t gamma_t,k, then over tremor steps
 *                       (flag 1) sum gamma, gamma x, gamma y, gamma x^2,
 *                       gamma x y, gamma y^2 (x, y in km)
 *   loglik double [1]: ln L (the same value as hmm_loglik, blocked FP32)
 * T = 0: stats hold xi = 0, P(s_{-1}) = delta / sum delta, moments 0.
 * Invalid parameters or data: ln L and stats are NaN, gamma rows NaN.  When
 * L = 0 (ln L = -inf) the other outputs are NaN or meaningless.
 *
 * hmm_loglik_grad: ln L and its gradient with every parameter entry treated
 *   as a free variable (no row-sum constraint on Gamma or delta), from the
 *   same expectations (Fisher's identity), device double grad[K + K*K + K +
 *   2K + 3K] = [d/d delta | d/d Gamma (row-major) | d/d p | d/d mu (x, y per
 *   state) | d/d Sigma (xx, xy, yy per state; Sxy as one variable that
 *   enters both off-diagonal positions)].  Needs T*K floats of workspace.
 * Both enqueue on `stream`; HMM_E_UNSUPPORTED for K > 80.
 * ------------------------------------------------------------------------ */
int hmm_posterior(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma,
                  const double *p, const double *mu, const double *Sigma, int64_t T,
                  const uint8_t *flag, const double *xy, void *stream, float *gamma,
                  double *stats, double *loglik);
int hmm_loglik_grad(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma,
                    const double *p, const double *mu, const double *Sigma, int64_t T,
                    const uint8_t *flag, const double *xy, void *stream, double *loglik,
                    double *grad);

/* One EM (Baum-Welch) iteration for the tremor model of eq. (1)-(2): the
 * E-step is hmm_posterior's forward-backward expectations, the M-step their
 * complete-data maximum likelihood, in FP64 on the device:
 *   delta_i  = P(s_{-1} = i | x)          Gamma_ij = xi_ij / sum_j xi_ij
 *   p_k      = n1_k / n_k                 mu_k     = s_k / n1_k
 *   Sigma_k  = S2_k / n1_k - mu_k mu_k^T  (expected covariance of the
 *                                          tremor locations of state k)
 * with n_k, n1_k, s_k, S2_k the expected counts and sums of hmm_posterior's
 * moments.  An entry whose expected count is exactly zero (a Gamma row never
 * left, n_k = 0, or n1_k = 0 for mu_k and Sigma_k) keeps its input value.
 *   loglik      device double [1]: ln L of the INPUT parameters
 *   params_out  device double [K + K*K + K + 2K + 3K]: the new parameters,
 *               packed [delta | Gamma (row-major) | p | mu | Sigma (xx, xy,
 *               yy)]; it may be the packed vector the five inputs point into
 *               (delta = params_out, Gamma = delta + K, ...) for in-place
 *               iteration, and must not overlap them otherwise.
 * Invalid parameters or data: ln L and params_out NaN.  EM may drive a state
 * to a singular Sigma (one tremor location); the next call then reports the
 * parameters as invalid.  Needs T*K floats of workspace; enqueues on
 * `stream`; HMM_E_UNSUPPORTED for K > 80.
 * ------------------------------------------------------------------------ */
int hmm_em_step(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma,
                const double *p, const double *mu, const double *Sigma, int64_t T,
                const uint8_t *flag, const double *xy, void *stream, double *loglik,
                double *params_out);

/* Most likely hidden path (Viterbi) of the tremor model of eq. (1)-(2),
 * with s_{-1} ~ delta the state before x_0:
 *   max over s_{-1}, s_0, ..., s_{T-1} of ln(delta_{s_-1} prod_t Gamma_{s_t-1 s_t} e_t,s_t).
 * Exact max-plus recursion, parallel over time: max-plus products of
 * segments (log2, FP32, renormalised every step; FP64 offsets), combined in
 * groups of 16 level by level, decoded top-down, then a Viterbi pass with
 * backpointers inside every segment between its two boundary states.  Ties
 * go to the smallest state index.  1 <= K <= 80 (64 < K: two wavefronts per
 * segment, the matrix exchanged through LDS).
 *   path   device int32 [T]: s_0 .. s_{T-1} (required when T > 0)
 *   first  device int32 [1]: s_{-1}
 *   score  device double [1]: the maximum (natural log)
 * T = 0: first = argmax delta, score = ln max delta.  Invalid parameters or
 * data: score NaN, first and path -1.  FP32 scores inside segments: a path
 * whose joint log probability is within about 1e-6 relative of the best one
 * may be returned instead of it.  HMM_E_UNSUPPORTED for K > 80. */
int hmm_viterbi(hmm_ctx *ctx, int32_t K, const double *delta, const double *Gamma,
                const double *p, const double *mu, const double *Sigma, int64_t T,
                const uint8_t *flag, const double *xy, void *stream, int32_t *path,
                int32_t *first, double *score);

/* Posterior-predictive simulation (section "Forecasting"): for every draw
 * d < n, a parameter set in the packed layout delta | Gamma | p | mu | Sigma
 * (params: device double [n][K*(K+7)], delta unused; e.g. the output of
 * hmm_theta_to_params for posterior samples) and a distribution of the
 * state before the first simulated step (start: device double [n][K]; for
 * a forecast after the data, gamma of the last observed step from
 * hmm_posterior), H steps of eq. (1)-(2):
 *   s_-1 ~ start_d;  s_t ~ Gamma[s_{t-1}, .];  f_t ~ Bernoulli(p_{s_t});
 *   x_t = mu + C z (C the lower Cholesky factor of Sigma_{s_t}) if f_t = 1.
 * A categorical draw with uniform u takes the smallest k with u < w_0 + ...
 * + w_k (FP64, ascending), the last k with w_k > 0 if rounding leaves u
 * above the total; all-zero weights end the draw's path (state -1, flag 0,
 * NaN location from that step on).  Random numbers: Philox with counter
 * (0, d, t, purpose), purpose 10 the pair (u_state, u_flag) of step t,
 * 11 the Box-Muller pair (z0, z1) of step t, 12 (first uniform, step 0)
 * for s_-1.  Outputs (device, step-major): states int32 [H][n],
 * flags uint8 [H][n], xy double [H][n][2] (NaN when f = 0), first int32 [n]
 * (s_-1).  Parameters are not validated.  FP64 throughout. */
int hmm_simulate(hmm_ctx *ctx, int32_t n, int32_t K, const double *params, const double *start,
                 int32_t H, uint64_t seed, void *stream, int32_t *states, uint8_t *flags,
                 double *xy, int32_t *first);

/* Philox draws of the sampler's streams: for i < n, out[2i], out[2i+1] are
 * the two uniforms (normal = 0) or Box-Muller normals (normal = 1) of counter
 * (i, chain, iter, purpose).  out: device double[2n] (may be NULL when n = 0). */
int hmm_philox(hmm_ctx *ctx, uint64_t seed, uint32_t purpose, uint32_t iter, uint32_t chain,
               int64_t n, int32_t normal, double *out, void *stream);

/* Checkpoints of a sampler, for resuming a run: a host byte image of the
 * chain states (theta, ln L, log prior), the random-walk scale, acceptance
 * counts, the Philox seed and iteration counter, the history ring, the prior
 * box, the network with its standardisation, lag and Adam state, and the
 * t-walk's second points, tuning and kernel counts.  A sampler
 * created for the same K, chain count, history length and observations that
 * loads the image continues bit for bit as the saved one would have (the
 * observations themselves are not part of the image).
 *   mcmc_checkpoint_size   *bytes = the image size
 *   mcmc_checkpoint_save   writes the image into host[bytes] (synchronises
 *                          the stream); the state must have been set
 *   mcmc_checkpoint_load   restores from host[bytes]; HMM_E_INVALID_ARG if the
 *                          image is not a checkpoint of a sampler of this
 *                          shape (synchronises the stream) */
int mcmc_checkpoint_size(mcmc_chains *chains, int64_t *bytes);
int mcmc_checkpoint_save(mcmc_chains *chains, void *host, int64_t bytes, void *stream);
int mcmc_checkpoint_load(mcmc_chains *chains, const void *host, int64_t bytes, void *stream);

/* Human-readable name of a status code (static storage). */
const char *hmm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* HMM_MI355X_H */
