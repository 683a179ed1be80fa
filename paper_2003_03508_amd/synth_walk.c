/* Hidden-path walker for the synthetic workload generator (synth.py).
 * Given the cumulative rows of a transition matrix and one uniform per step,
 * state_t is the first index j with cum[state_{t-1}][j] > u_t (clamped to
 * K-1), exactly as bisect.bisect_right on the same rows.  Sampling only: no
 * likelihood arithmetic lives here. */
#include <stdint.h>

void synth_walk(int K, const double *cum /* K*K */, int32_t s0, int64_t T, const double *u /* T */,
                int32_t *out /* T */)
{
    int32_t s = s0;
    for (int64_t t = 0; t < T; ++t) {
        const double *row = cum + (int64_t)s * K;
        const double x = u[t];
        int lo = 0, hi = K; /* first j in [lo, hi) with row[j] > x */
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (row[mid] > x) hi = mid; else lo = mid + 1;
        }
        s = lo < K ? lo : K - 1;
        out[t] = s;
    }
}
