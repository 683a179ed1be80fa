// Blocked-path kernels compiled with their MFMA accumulators allowed in
// AGPRs: FP32 tiles of side 64 and 80 (more than 256 values per lane) and the
// 16-bit-operand kernels with 4 or 5 row tiles.
#include "hmm_host.hpp"

namespace hmmh {

namespace {

template <int S, int MT, int LO, int HI>
bool pick_f32(int nsl, KernelSet *ks)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (nsl == LO) {
            *ks = kernel_set_f32<S, MT, LO>();
            return true;
        }
        return pick_f32<S, MT, LO + 1, HI>(nsl, ks);
    }
}

template <int MT, bool F16, int LO, int HI, bool SPLIT = false>
bool pick_lp(int nsl, KernelSet *ks)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (nsl == LO) {
            *ks = kernel_set_lp<MT, F16, LO, SPLIT>();
            return true;
        }
        return pick_lp<MT, F16, LO + 1, HI, SPLIT>(nsl, ks);
    }
}

template <int MT, int LO, int HI>
bool pick_lp_algo(int algo, int nsl, KernelSet *ks)
{
    switch (algo) {
    case HMM_BLOCKED_BF16: return pick_lp<MT, false, LO, HI>(nsl, ks);
    case HMM_BLOCKED_F16: return pick_lp<MT, true, LO, HI>(nsl, ks);
    case HMM_BLOCKED_BF16_SPLIT: return pick_lp<MT, false, LO, HI, true>(nsl, ks);
    case HMM_BLOCKED_F16_SPLIT: return pick_lp<MT, true, LO, HI, true>(nsl, ks);
    default: return false;
    }
}

}  // namespace

bool kernels_large(int algo, int S, int MT, int NSL, KernelSet *ks)
{
    if (algo == HMM_BLOCKED_F32) {
        if (S == 32 && MT == 2) return pick_f32<32, 2, 25, 32>(NSL, ks);
        if (S == 16 && MT == 5) return pick_f32<16, 5, 17, 20>(NSL, ks);
        return false;
    }
    if (S != 16) return false;
    if (MT == 4) return pick_lp_algo<4, 13, 16>(algo, NSL, ks);
    if (MT == 5) return pick_lp_algo<5, 17, 20>(algo, NSL, ks);
    return false;
}

}  // namespace hmmh
