/* Driver for running the C oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by test_sanitizers.py).  It
 * exercises every entry point on a small seeded problem, the ragged block
 * lengths, the batch driver with several threads and the error conventions,
 * and prints the results so the test can compare them with the unsanitized
 * build. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_log_emission(int K, const double *p, const double *mu, const double *Sigma, int64_t T,
                        const uint8_t *flag, const double *xy, double *out);
double oracle_loglik(int K, const double *delta, const double *Gamma, const double *p, const double *mu,
                     const double *Sigma, int64_t T, const uint8_t *flag, const double *xy);
double oracle_loglik_blocked(int K, const double *delta, const double *Gamma, const double *p,
                             const double *mu, const double *Sigma, int64_t T, const uint8_t *flag,
                             const double *xy, int64_t L);
int oracle_loglik_batch(int32_t n, const int32_t *K, const int64_t *T, const int64_t *param_off,
                        const double *params, const int64_t *obs_off, const uint8_t *flag, const double *xy,
                        double *out, int32_t nthreads);

static uint64_t state = 88172645463325252ull;
static double unif(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    enum { K = 4, T = 777 };
    double delta[K], Gamma[K * K], p[K], mu[2 * K], Sigma[3 * K];
    for (int i = 0; i < K; ++i) {
        double s = 0.0;
        for (int j = 0; j < K; ++j) s += (Gamma[i * K + j] = (i == j ? 20.0 : 1.0) * (0.5 + unif()));
        for (int j = 0; j < K; ++j) Gamma[i * K + j] /= s;
        delta[i] = 1.0 / K;
        p[i] = 0.1 + 0.8 * unif();
        mu[2 * i] = 200.0 * unif();
        mu[2 * i + 1] = 200.0 * unif();
        Sigma[3 * i] = 25.0 + 400.0 * unif();
        Sigma[3 * i + 1] = 0.0;
        Sigma[3 * i + 2] = 25.0 + 400.0 * unif();
    }
    uint8_t *flag = malloc(T);
    double *xy = malloc(sizeof(double) * 2 * T);
    for (int t = 0; t < T; ++t) {
        flag[t] = unif() < 0.5;
        xy[2 * t] = flag[t] ? 200.0 * unif() : NAN;
        xy[2 * t + 1] = flag[t] ? 200.0 * unif() : NAN;
    }
    double *le = malloc(sizeof(double) * T * K);
    printf("emission %d %.17g\n", oracle_log_emission(K, p, mu, Sigma, T, flag, xy, le), le[T * K - 1]);
    printf("serial %.17g\n", oracle_loglik(K, delta, Gamma, p, mu, Sigma, T, flag, xy));
    const int64_t Ls[] = {1, 2, 3, 7, 64, T, T + 5};
    for (int i = 0; i < 7; ++i)
        printf("blocked %lld %.17g\n", (long long)Ls[i],
               oracle_loglik_blocked(K, delta, Gamma, p, mu, Sigma, T, flag, xy, Ls[i]));
    printf("empty %.17g\n", oracle_loglik(K, delta, Gamma, p, mu, Sigma, 0, flag, xy));
    double bad_p[K] = {0.5, 1.5, 0.5, 0.5};
    printf("invalid %.17g\n", oracle_loglik(K, delta, Gamma, bad_p, mu, Sigma, T, flag, xy));
    /* batch: the same set three times with different lengths, several threads */
    enum { NB = 3 };
    const int blk = K + K * K + K + 2 * K + 3 * K;
    double *params = malloc(sizeof(double) * NB * blk);
    int32_t Kb[NB];
    int64_t Tb[NB], poff[NB], ooff[NB];
    for (int s = 0; s < NB; ++s) {
        double *b = params + s * blk;
        int o = 0;
        for (int i = 0; i < K; ++i) b[o++] = delta[i];
        for (int i = 0; i < K * K; ++i) b[o++] = Gamma[i];
        for (int i = 0; i < K; ++i) b[o++] = p[i];
        for (int i = 0; i < 2 * K; ++i) b[o++] = mu[i];
        for (int i = 0; i < 3 * K; ++i) b[o++] = Sigma[i];
        Kb[s] = K;
        Tb[s] = T - 100 * s;
        poff[s] = (int64_t)s * blk;
        ooff[s] = 10 * s;
    }
    double out[NB];
    printf("batch %d", oracle_loglik_batch(NB, Kb, Tb, poff, params, ooff, flag, xy, out, 3));
    for (int s = 0; s < NB; ++s) printf(" %.17g", out[s]);
    printf("\n");
    free(params);
    free(le);
    free(xy);
    free(flag);
    return 0;
}
