/*
 * FP64 CPU oracle for the tremor-HMM forward log-likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library (nothing here is included
 * by, or includes anything from, the package sources).
 *
 * Model (paper, section "An HMM for classifying nonvolcanic tremors"):
 *   observations x_0..x_N, each either "no tremor" or a point in R^2;
 *   K hidden states, state k has a tremor probability p_k and a bivariate
 *   normal location law N(mu_k, Sigma_k).
 *   Emission matrix, eq. (1): P(x) = diag(e_1..e_K) with
 *       e_k = p_k * phi(x | mu_k, Sigma_k)   if x is a tremor location,
 *       e_k = 1 - p_k                         if x is "no tremor".
 *   Likelihood, eq. (2): L = delta^T Gamma P(x_0) Gamma P(x_1) ... Gamma P(x_N) 1.
 *   The forward algorithm (Algorithm 1) evaluates eq. (2) left to right with a
 *   row vector: v <- delta^T, then for every observation v <- v Gamma, v <- v P(x).
 *
 * Readings taken where the paper is silent (all also listed in the design notes):
 *   - eq. (1) has lost its case labels; the first case is a tremor (flag 1),
 *     the second is "no tremor" (flag 0); the location is ignored when flag=0.
 *   - Gamma is applied before the first emission, exactly as eq. (2) and
 *     Algorithm 1 write it; delta is used as given (not renormalised).
 *   - phi keeps its full normalising constant (units of the inputs, km here).
 *   - Sigma_k is a full symmetric 2x2 matrix given as (Sxx, Sxy, Syy).
 *   - T = N+1 counts observations.  T = 0 gives log(sum_k delta_k) (the empty
 *     chain of eq. (2) is delta^T 1).
 *   - L = 0 gives -inf; invalid parameters or data give NaN (see oracle_valid).
 *   - Underflow is avoided as the paper says (logarithm and scaling, section
 *     "Step 3"); the scaling constant here is the per-step sum c_t, which is
 *     mathematically exact and only changes rounding.  One scale is shared by
 *     all states, so a state whose forward variable trails the largest by
 *     more than ~e^-745 at some step underflows to zero; this needs a
 *     transition matrix that (almost) forbids moving between states (e.g.
 *     the identity), for which the tests use the closed form instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_LN_2PI 1.8378770664093454835606594728112

/* Parameter and data validity shared by every oracle entry point.
 * delta_k >= 0, 0 <= Gamma_ij <= 1, 0 <= p_k <= 1, mu finite,
 * Sxx > 0, Syy > 0, Sxx*Syy - Sxy^2 > 0, all finite.  Returns 1 if valid. */
static int oracle_params_valid(int K, const double *delta, const double *Gamma,
                               const double *p, const double *mu, const double *Sigma)
{
    if (K < 1) return 0;
    for (int k = 0; k < K; ++k) {
        if (!isfinite(delta[k]) || delta[k] < 0.0) return 0;
        for (int j = 0; j < K; ++j) {
            double g = Gamma[(size_t)k * K + j];
            if (!isfinite(g) || g < 0.0 || g > 1.0) return 0;
        }
        if (!isfinite(p[k]) || p[k] < 0.0 || p[k] > 1.0) return 0;
        if (!isfinite(mu[2 * k]) || !isfinite(mu[2 * k + 1])) return 0;
        double sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
        if (!isfinite(sxx) || !isfinite(sxy) || !isfinite(syy)) return 0;
        if (!(sxx > 0.0) || !(syy > 0.0)) return 0;
        if (!(sxx * syy - sxy * sxy > 0.0)) return 0;
    }
    return 1;
}

/* eq. (1) in natural-log form.  out[t*K + k] = ln e_{t,k}.
 * ln e = ln p_k - ln(2 pi) - ln|Sigma_k|/2 - (x-mu_k)^T Sigma_k^{-1} (x-mu_k)/2  (tremor)
 * ln e = ln(1 - p_k)                                                         (no tremor)
 * Returns 0 on success, 1 if some data point is invalid (flag not 0/1, or a
 * tremor with a non-finite location); out is then filled with NaN. */
int oracle_log_emission(int K, const double *p, const double *mu, const double *Sigma,
                        int64_t T, const uint8_t *flag, const double *xy, double *out)
{
    for (int64_t t = 0; t < T; ++t) {
        int bad = 0;
        if (flag[t] > 1) bad = 1;
        if (flag[t] == 1 && (!isfinite(xy[2 * t]) || !isfinite(xy[2 * t + 1]))) bad = 1;
        if (bad) {
            for (int64_t i = 0; i < T * (int64_t)K; ++i) out[i] = NAN;
            return 1;
        }
        for (int k = 0; k < K; ++k) {
            double v;
            if (flag[t] == 1) {
                double sxx = Sigma[3 * k], sxy = Sigma[3 * k + 1], syy = Sigma[3 * k + 2];
                double det = sxx * syy - sxy * sxy;
                double d0 = xy[2 * t] - mu[2 * k];
                double d1 = xy[2 * t + 1] - mu[2 * k + 1];
                /* Sigma^{-1} = [[syy, -sxy], [-sxy, sxx]] / det */
                double q = (syy * d0 * d0 - 2.0 * sxy * d0 * d1 + sxx * d1 * d1) / det;
                v = log(p[k]) - ORACLE_LN_2PI - 0.5 * log(det) - 0.5 * q;
            } else {
                v = log1p(-p[k]);
            }
            out[(size_t)t * K + k] = v;
        }
    }
    return 0;
}

/* Algorithm 1 with per-step normalisation, given ln e_{t,k} directly.
 *   a <- delta^T Gamma
 *   for t = 0..T-1:
 *     if t > 0: a <- u Gamma
 *     m_t = max_k ln e_{t,k};  b_k = a_k exp(ln e_{t,k} - m_t);  c_t = sum_k b_k
 *     if c_t == 0: L = 0 -> return -inf
 *     u <- b / c_t;  ll += ln c_t + m_t
 *   return ll
 * Summations run over ascending indices. */
double oracle_forward_from_logemis(int K, const double *delta, const double *Gamma,
                                   int64_t T, const double *logE)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)K);
    double *a = (double *)malloc(sizeof(double) * (size_t)K);
    double ll = 0.0;
    if (T == 0) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += delta[k];
        free(u); free(a);
        return log(s);
    }
    for (int k = 0; k < K; ++k) u[k] = delta[k];
    for (int64_t t = 0; t < T; ++t) {
        /* a = u Gamma (for t = 0, u = delta: the Gamma before P(x_0) in eq. 2) */
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int i = 0; i < K; ++i) s += u[i] * Gamma[(size_t)i * K + j];
            a[j] = s;
        }
        const double *le = logE + (size_t)t * K;
        double m = -INFINITY;
        for (int k = 0; k < K; ++k) if (le[k] > m) m = le[k];
        if (isnan(m)) { free(u); free(a); return NAN; }
        if (m == -INFINITY) { free(u); free(a); return -INFINITY; }
        double c = 0.0;
        for (int k = 0; k < K; ++k) {
            u[k] = a[k] * exp(le[k] - m);
            c += u[k];
        }
        if (c == 0.0) { free(u); free(a); return -INFINITY; }
        for (int k = 0; k < K; ++k) u[k] /= c;
        ll += log(c) + m;
    }
    free(u); free(a);
    return ll;
}

/* Full likelihood: validity checks, eq. (1), then Algorithm 1 (natural log). */
double oracle_loglik(int K, const double *delta, const double *Gamma, const double *p,
                     const double *mu, const double *Sigma, int64_t T,
                     const uint8_t *flag, const double *xy)
{
    if (!oracle_params_valid(K, delta, Gamma, p, mu, Sigma) || T < 0) return NAN;
    double *logE = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (size_t)K);
    if (!logE) return NAN;
    if (oracle_log_emission(K, p, mu, Sigma, T, flag, xy, logE) != 0) { free(logE); return NAN; }
    double ll = oracle_forward_from_logemis(K, delta, Gamma, T, logE);
    free(logE);
    return ll;
}

/* Other emission models.  The paper notes that the method applies to other
 * HMMs by changing only the emission function (sections "Discussion" and
 * "Conclusion"); the likelihood is still eq. (2) with P(x) = diag(e_1..e_K).
 *   kind 1, Poisson counts:  e_k(y) = lambda_k^y exp(-lambda_k) / y!
 *            e0 = lambda[K] (> 0), obs = int32 counts[T] (>= 0)
 *   kind 2, 1-D Gaussian:    e_k(x) = N(x; mu_k, var_k)
 *            e0 = mu[K], e1 = var[K] (> 0), obs = double values[T] (finite)
 * out[t*K + k] = ln e_{t,k}.  Returns 0, or 1 for invalid parameters or data
 * (out then holds NaN). */
int oracle_log_emission_kind(int kind, int K, const double *e0, const double *e1, int64_t T,
                             const void *obs, double *out)
{
    int bad = 0;
    for (int k = 0; k < K; ++k) {
        if (kind == 1 && !(isfinite(e0[k]) && e0[k] > 0.0)) bad = 1;
        if (kind == 2 && !(isfinite(e0[k]) && isfinite(e1[k]) && e1[k] > 0.0)) bad = 1;
    }
    if (kind != 1 && kind != 2) bad = 1;
    for (int64_t t = 0; t < T && !bad; ++t) {
        for (int k = 0; k < K; ++k) {
            double v;
            if (kind == 1) {
                const int32_t y = ((const int32_t *)obs)[t];
                if (y < 0) { bad = 1; break; }
                v = (double)y * log(e0[k]) - e0[k] - lgamma((double)y + 1.0);
            } else {
                const double x = ((const double *)obs)[t];
                if (!isfinite(x)) { bad = 1; break; }
                const double d = x - e0[k];
                v = -0.5 * ORACLE_LN_2PI - 0.5 * log(e1[k]) - 0.5 * d * d / e1[k];
            }
            out[(size_t)t * K + k] = v;
        }
    }
    if (bad)
        for (int64_t i = 0; i < T * (int64_t)K; ++i) out[i] = NAN;
    return bad;
}

/* ln L of eq. (2) with the emissions of oracle_log_emission_kind. */
double oracle_loglik_kind(int kind, int K, const double *delta, const double *Gamma, const double *e0,
                          const double *e1, int64_t T, const void *obs)
{
    if (K < 1 || T < 0) return NAN;
    for (int k = 0; k < K; ++k) {
        if (!isfinite(delta[k]) || delta[k] < 0.0) return NAN;
        for (int j = 0; j < K; ++j) {
            const double g = Gamma[(size_t)k * K + j];
            if (!isfinite(g) || g < 0.0 || g > 1.0) return NAN;
        }
    }
    double *logE = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * (size_t)K);
    if (!logE) return NAN;
    if (oracle_log_emission_kind(kind, K, e0, e1, T, obs, logE) != 0) { free(logE); return NAN; }
    double ll = oracle_forward_from_logemis(K, delta, Gamma, T, logE);
    free(logE);
    return ll;
}

/* The same quantity in the order of the paper's parallel plan (section "The
 * likelihood algorithm", steps 1-3): the chain Gamma P(x_0) ... Gamma P(x_N)
 * is cut into segments of L factors, each segment's matrix product is formed
 * on its own (with a scalar scale factor kept as a logarithm), and the
 * segment products are then applied to delta^T left to right (the paper does
 * this last part on the host).  Everything is FP64.  By associativity the
 * result equals oracle_loglik up to rounding; the tests use this to pin that
 * the block order is exact.  Each segment's running matrix is divided by its
 * largest entry after every factor. */
double oracle_loglik_blocked(int K, const double *delta, const double *Gamma, const double *p,
                             const double *mu, const double *Sigma, int64_t T,
                             const uint8_t *flag, const double *xy, int64_t L)
{
    if (!oracle_params_valid(K, delta, Gamma, p, mu, Sigma) || T < 0 || L < 1) return NAN;
    if (T == 0) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += delta[k];
        return log(s);
    }
    size_t KK = (size_t)K * K;
    double *logE = (double *)malloc(sizeof(double) * (size_t)T * K);
    double *M = (double *)malloc(sizeof(double) * KK);
    double *W = (double *)malloc(sizeof(double) * KK);
    double *v = (double *)malloc(sizeof(double) * K);
    double *w = (double *)malloc(sizeof(double) * K);
    if (oracle_log_emission(K, p, mu, Sigma, T, flag, xy, logE) != 0) {
        free(logE); free(M); free(W); free(v); free(w);
        return NAN;
    }
    double ll = 0.0; /* accumulated log scale factors */
    for (int k = 0; k < K; ++k) v[k] = delta[k];
    for (int64_t s0 = 0; s0 < T; s0 += L) {
        int64_t s1 = s0 + L < T ? s0 + L : T;
        /* M <- identity */
        for (size_t i = 0; i < KK; ++i) M[i] = 0.0;
        for (int k = 0; k < K; ++k) M[(size_t)k * K + k] = 1.0;
        double seg_log = 0.0;
        for (int64_t t = s0; t < s1; ++t) {
            const double *le = logE + (size_t)t * K;
            double m = -INFINITY;
            for (int k = 0; k < K; ++k) if (le[k] > m) m = le[k];
            if (m == -INFINITY) { ll = -INFINITY; goto done; }
            /* W = M Gamma diag(exp(le - m)) */
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    double s = 0.0;
                    for (int r = 0; r < K; ++r) s += M[(size_t)i * K + r] * Gamma[(size_t)r * K + j];
                    W[(size_t)i * K + j] = s * exp(le[j] - m);
                }
            double mx = 0.0;
            for (size_t i = 0; i < KK; ++i) if (W[i] > mx) mx = W[i];
            if (mx == 0.0) { ll = -INFINITY; goto done; }
            for (size_t i = 0; i < KK; ++i) M[i] = W[i] / mx;
            seg_log += m + log(mx);
        }
        /* v <- v M, normalised by its sum */
        double c = 0.0;
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int i = 0; i < K; ++i) s += v[i] * M[(size_t)i * K + j];
            w[j] = s;
            c += s;
        }
        if (c == 0.0) { ll = -INFINITY; goto done; }
        for (int j = 0; j < K; ++j) v[j] = w[j] / c;
        ll += seg_log + log(c);
    }
done:
    free(logE); free(M); free(W); free(v); free(w);
    return ll;
}

/* Many independent sets at once, one set per call of oracle_loglik; used only
 * to time the oracle on several host threads.  Sets are described by offsets
 * into packed arrays exactly like the batched GPU entry point's inputs.
 * Threads (if > 1) split the sets round-robin with pthreads. */
#include <pthread.h>
typedef struct {
    int32_t n, nthreads, tid;
    const int32_t *K; const int64_t *T; const int64_t *param_off; const double *params;
    const int64_t *obs_off; const uint8_t *flag; const double *xy; double *out;
} oracle_batch_job;

static void *oracle_batch_worker(void *arg)
{
    oracle_batch_job *j = (oracle_batch_job *)arg;
    for (int32_t s = j->tid; s < j->n; s += j->nthreads) {
        int K = j->K[s];
        const double *base = j->params + j->param_off[s];
        /* packed parameter block: delta[K], Gamma[K*K], p[K], mu[2K], Sigma[3K] */
        const double *delta = base, *Gamma = delta + K, *pp = Gamma + (size_t)K * K;
        const double *mu = pp + K, *Sigma = mu + 2 * K;
        int64_t o = j->obs_off[s];
        j->out[s] = oracle_loglik(K, delta, Gamma, pp, mu, Sigma, j->T[s], j->flag + o, j->xy + 2 * o);
    }
    return NULL;
}

int oracle_loglik_batch(int32_t n, const int32_t *K, const int64_t *T, const int64_t *param_off,
                        const double *params, const int64_t *obs_off, const uint8_t *flag,
                        const double *xy, double *out, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    oracle_batch_job jobs[256];
    int started[256];
    for (int32_t i = 0; i < nthreads; ++i) {
        jobs[i] = (oracle_batch_job){n, nthreads, i, K, T, param_off, params, obs_off, flag, xy, out};
        /* a worker that cannot be started runs on this thread instead */
        started[i] = nthreads > 1 && pthread_create(&th[i], NULL, oracle_batch_worker, &jobs[i]) == 0;
        if (!started[i]) oracle_batch_worker(&jobs[i]);
    }
    for (int32_t i = 0; i < nthreads; ++i)
        if (started[i]) pthread_join(th[i], NULL);
    return 0;
}

/* State posteriors of eq. (2)'s model by the scaled forward-backward
 * recursions (the reverse-mode counterpart of Algorithm 1), FP64.
 * With s_{-1} ~ delta the state before x_0 and e^_{t,k} = exp(ln e_{t,k} - m_t):
 *   forward   u_{-1} = delta;  a_t = u_{t-1} Gamma;  b_t = a_t o e^_t;
 *             c_t = sum_k b_t,k;  u_t = b_t / c_t  (stored for every t)
 *   backward  v_{T-1} = 1;  v_{t-1,i} = sum_j Gamma_ij e^_t,j v_t,j / c_t
 * so that sum_k u_t,k v_t,k = 1 and
 *   gamma_t,k = P(s_t = k | x)              = u_t,k v_t,k
 *   xi_t(i,j) = P(s_{t-1} = i, s_t = j | x) = u_{t-1,i} Gamma_ij e^_t,j v_t,j / c_t
 * Outputs: gamma[T*K]; xi[K*K] = sum over t = 0..T-1 of xi_t (t = 0 is the
 * step from s_{-1}); pre[K] = P(s_{-1} = i | x) = sum_j xi_0(i,j);
 * mom[K*7] per state k: sum_t gamma_t,k, then over tremor steps (flag 1)
 * sum gamma, sum gamma x, sum gamma y, sum gamma x^2, sum gamma x y,
 * sum gamma y^2.  Returns ln L (the forward pass's sum of ln c_t + m_t).
 * Invalid inputs give NaN, L = 0 gives -inf; the outputs are then NaN.
 * Summations run over ascending indices (xi and the moments over ascending
 * t within the backward pass, i.e. descending t). */
double oracle_posterior(int K, const double *delta, const double *Gamma, const double *p,
                        const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
                        const double *xy, double *gamma, double *xi, double *pre, double *mom)
{
    const size_t KK = (size_t)K * K, TK = (size_t)(T > 0 ? T : 1) * K;
    for (size_t i = 0; i < KK; ++i) xi[i] = 0.0;
    for (int k = 0; k < K; ++k) pre[k] = 0.0;
    for (int i = 0; i < 7 * K; ++i) mom[i] = 0.0;
    if (!oracle_params_valid(K, delta, Gamma, p, mu, Sigma) || T < 0) goto invalid;
    {
        double *logE = (double *)malloc(sizeof(double) * TK);
        double *c = (double *)malloc(sizeof(double) * (T > 0 ? T : 1));
        double *m = (double *)malloc(sizeof(double) * (T > 0 ? T : 1));
        double *v = (double *)malloc(sizeof(double) * K);
        double *w = (double *)malloc(sizeof(double) * K);
        double ll = 0.0;
        if (oracle_log_emission(K, p, mu, Sigma, T, flag, xy, logE) != 0) {
            free(logE); free(c); free(m); free(v); free(w);
            goto invalid;
        }
        if (T == 0) {
            double s = 0.0;
            for (int k = 0; k < K; ++k) s += delta[k];
            for (int k = 0; k < K; ++k) pre[k] = delta[k] / s;
            free(logE); free(c); free(m); free(v); free(w);
            return log(s);
        }
        /* forward: gamma holds u_t */
        for (int64_t t = 0; t < T; ++t) {
            const double *u = t == 0 ? delta : gamma + (size_t)(t - 1) * K;
            double *ut = gamma + (size_t)t * K;
            const double *le = logE + (size_t)t * K;
            double mt = -INFINITY;
            for (int k = 0; k < K; ++k) if (le[k] > mt) mt = le[k];
            if (mt == -INFINITY) ll = -INFINITY;
            if (!isfinite(ll)) break;
            double ct = 0.0;
            for (int j = 0; j < K; ++j) {
                double a = 0.0;
                for (int i = 0; i < K; ++i) a += u[i] * Gamma[(size_t)i * K + j];
                ut[j] = a * exp(le[j] - mt);
                ct += ut[j];
            }
            if (ct == 0.0) { ll = -INFINITY; break; }
            for (int j = 0; j < K; ++j) ut[j] /= ct;
            c[t] = ct;
            m[t] = mt;
            ll += log(ct) + mt;
        }
        if (!isfinite(ll)) {
            free(logE); free(c); free(m); free(v); free(w);
            for (size_t i = 0; i < TK; ++i) gamma[i] = NAN;
            for (size_t i = 0; i < KK; ++i) xi[i] = NAN;
            for (int k = 0; k < K; ++k) pre[k] = NAN;
            for (int i = 0; i < 7 * K; ++i) mom[i] = NAN;
            return ll;
        }
        /* backward: v = v_t; gamma_t = u_t o v_t overwrites u_t once u_t is used */
        for (int k = 0; k < K; ++k) v[k] = 1.0;
        for (int64_t t = T - 1; t >= 0; --t) {
            const double *le = logE + (size_t)t * K;
            const double *uprev = t == 0 ? delta : gamma + (size_t)(t - 1) * K;
            double *gt = gamma + (size_t)t * K;
            /* w_j = e^_t,j v_t,j / c_t */
            for (int j = 0; j < K; ++j) w[j] = exp(le[j] - m[t]) * v[j] / c[t];
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < K; ++j) {
                    const double x = uprev[i] * Gamma[(size_t)i * K + j] * w[j];
                    xi[(size_t)i * K + j] += x;
                    if (t == 0) pre[i] += x;
                }
            for (int k = 0; k < K; ++k) {
                const double g = gt[k] * v[k];
                gt[k] = g;
                mom[7 * k] += g;
                if (flag[t] == 1) {
                    const double x = xy[2 * t], y = xy[2 * t + 1];
                    mom[7 * k + 1] += g;
                    mom[7 * k + 2] += g * x;
                    mom[7 * k + 3] += g * y;
                    mom[7 * k + 4] += g * x * x;
                    mom[7 * k + 5] += g * x * y;
                    mom[7 * k + 6] += g * y * y;
                }
            }
            /* v_{t-1,i} = sum_j Gamma_ij w_j */
            for (int i = 0; i < K; ++i) {
                double s = 0.0;
                for (int j = 0; j < K; ++j) s += Gamma[(size_t)i * K + j] * w[j];
                v[i] = s;
            }
        }
        free(logE); free(c); free(m); free(v); free(w);
        return ll;
    }
invalid:
    for (size_t i = 0; i < TK; ++i) gamma[i] = NAN;
    for (size_t i = 0; i < KK; ++i) xi[i] = NAN;
    for (int k = 0; k < K; ++k) pre[k] = NAN;
    for (int i = 0; i < 7 * K; ++i) mom[i] = NAN;
    return NAN;
}

/* Most likely hidden path (Viterbi) of eq. (2)'s model, in the log domain:
 *   V_{-1,i} = ln delta_i
 *   V_t,j = max_i (V_{t-1,i} + ln Gamma_ij) + ln e_t,j,  psi_t,j = its argmax
 * (the smallest i on ties), s_{T-1} = argmax_j V_{T-1,j} (smallest j on ties),
 * s_{t-1} = psi_t,s_t.  path[t] = s_t for t = 0..T-1, *first = s_{-1}.
 * Returns max over paths of ln(delta_s-1 prod_t Gamma e) (ln 0 = -inf), NaN
 * on invalid input (the path is then -1 everywhere). */
double oracle_viterbi(int K, const double *delta, const double *Gamma, const double *p,
                      const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
                      const double *xy, int32_t *path, int32_t *first)
{
    const size_t TK = (size_t)(T > 0 ? T : 1) * K;
    for (int64_t t = 0; t < T; ++t) path[t] = -1;
    *first = -1;
    if (!oracle_params_valid(K, delta, Gamma, p, mu, Sigma) || T < 0) return NAN;
    double *logE = (double *)malloc(sizeof(double) * TK);
    int32_t *psi = (int32_t *)malloc(sizeof(int32_t) * (TK + K));
    double *V = (double *)malloc(sizeof(double) * K);
    double *Vn = (double *)malloc(sizeof(double) * K);
    if (oracle_log_emission(K, p, mu, Sigma, T, flag, xy, logE) != 0) {
        free(logE); free(psi); free(V); free(Vn);
        return NAN;
    }
    for (int i = 0; i < K; ++i) V[i] = log(delta[i]);
    for (int64_t t = 0; t < T; ++t) {
        for (int j = 0; j < K; ++j) {
            double best = -INFINITY;
            int arg = 0;
            for (int i = 0; i < K; ++i) {
                const double s = V[i] + log(Gamma[(size_t)i * K + j]);
                if (s > best) { best = s; arg = i; }
            }
            Vn[j] = best + logE[(size_t)t * K + j];
            psi[(size_t)t * K + j] = arg;
        }
        for (int j = 0; j < K; ++j) V[j] = Vn[j];
    }
    double best = -INFINITY;
    int arg = 0;
    for (int j = 0; j < K; ++j) if (V[j] > best) { best = V[j]; arg = j; }
    if (T == 0) {
        *first = arg;
    } else {
        path[T - 1] = arg;
        for (int64_t t = T - 1; t > 0; --t) path[t - 1] = psi[(size_t)t * K + path[t]];
        *first = psi[path[0]];
    }
    free(logE); free(psi); free(V); free(Vn);
    return best;
}
