// Blocked-path kernels for 48 < K <= 80 (tile sides 64 and 80).  Compiled
// separately from hmm_api.hip so that their MFMA accumulators may live in
// AGPRs (these kernels hold more than 256 values per lane).
#include "hmm_host.hpp"

namespace hmmh {

int run_blocked_large(const Shape &sh, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                      const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                      const Layout &ly)
{
    switch (sh.S * 100 + sh.MT) {
    case 3202:
        return dispatch_nsl<32, 2, 25, 32>(needed_slots<32, 2>(K), ctx, K, delta, T, flag, xy, st, out, pl, ly);
    case 1605:
        return dispatch_nsl<16, 5, 17, 20>(needed_slots<16, 5>(K), ctx, K, delta, T, flag, xy, st, out, pl, ly);
    default:
        return HMM_E_UNSUPPORTED;
    }
}

int run_blocked_lp_large(int MT, bool f16, int K, hmm_ctx *ctx, const double *delta, int64_t T,
                         const uint8_t *flag, const double *xy, hipStream_t st, double *out, const Plan &pl,
                         const Layout &ly)
{
    const int nsl = (MT == 4) ? needed_slots<16, 4>(K) : needed_slots<16, 5>(K);
    switch (MT * 2 + (f16 ? 1 : 0)) {
    case 8: return dispatch_lp<4, false, 13, 16>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    case 9: return dispatch_lp<4, true, 13, 16>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    case 10: return dispatch_lp<5, false, 17, 20>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    case 11: return dispatch_lp<5, true, 17, 20>(nsl, ctx, K, delta, T, flag, xy, st, out, pl, ly);
    default: return HMM_E_UNSUPPORTED;
    }
}

}  // namespace hmmh
