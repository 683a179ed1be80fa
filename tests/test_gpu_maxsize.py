"""The longest sequences: ln L at T > 2^32, where any 32-bit observation or
segment index would wrap.

Expected value.  When the observations repeat one block of P steps n times
and end with the block's first r steps, eq. (2) regroups as
    L = delta^T (M_P)^n M_r 1,   M_s = prod_{t < s} Gamma diag(e_t) over the block,
so ln L follows from one pass over the block and n by repeated squaring, in
FP64 with a running log scale (`periodic_loglik`).  That regrouping is pinned
on the CPU against the forward-algorithm oracle on the explicit sequence.
Tolerance: 1e-6 relative, the blocked FP32 likelihood's bound."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_03508_amd import synth


def _normalise(M, logs):
    s = M.max()
    return M / s, logs + math.log(s)


def periodic_loglik(delta, Gamma, logE, n, r):
    """ln(delta^T (M_P)^n M_r 1) for the block log emissions logE (P, K)."""
    K = Gamma.shape[0]
    M, lm = np.eye(K), 0.0
    Mr, lr = (np.eye(K), 0.0) if r == 0 else (None, None)
    for t in range(logE.shape[0]):
        c = logE[t].max()
        M = (M @ Gamma) * np.exp(logE[t] - c)[None, :]
        M, lm = _normalise(M, lm + c)
        if t + 1 == r:
            Mr, lr = M.copy(), lm
    R, lR = np.eye(K), 0.0
    B, lB = M, lm
    while n:
        if n & 1:
            R, lR = _normalise(R @ B, lR + lB)
        n >>= 1
        if n:
            B, lB = _normalise(B @ B, 2.0 * lB)
    v = np.asarray(delta) @ R @ Mr
    return lR + lr + math.log(v.sum())


@pytest.mark.parametrize("K,P,n,r", [(3, 50, 0, 17), (3, 50, 1, 0), (4, 40, 5, 7), (5, 64, 11, 63)])
def test_periodic_regrouping_matches_the_forward_oracle(K, P, n, r):
    prm, obs = synth.make(K, P, 40 + K)
    T = n * P + r
    flag = np.resize(obs.flag, T)
    xy = np.resize(obs.xy, (T, 2))
    want = oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, flag, xy)
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    got = periodic_loglik(prm.delta, prm.Gamma, le, n, r)
    assert abs(got - want) <= 1e-10 * max(1.0, abs(want)), (got, want)


@pytest.mark.gpu
@pytest.mark.parametrize("K", [25, 6])
def test_loglik_beyond_2_pow_32(K):
    from paper_2003_03508_amd import binding
    P = 100_003
    T = 2 ** 32 + 4097
    n, r = divmod(T, P)
    prm, obs = synth.make(K, P, 60 + K)
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    want = periodic_loglik(prm.delta, prm.Gamma, le, n, r)
    ctx = binding.Context(0)
    try:
        d = binding.to_device(prm, obs)
        # n + 1 copies of the block, then the first T steps (a contiguous prefix)
        d["flag"] = d["flag"].repeat(n + 1)[:T]
        d["xy"] = d["xy"].repeat(n + 1, 1)[:T]
        print(f"K={K} T={T} P={P} n={n} r={r}", flush=True)
        got = float(ctx.loglik(**d).cpu()[0])
    finally:
        ctx.close()
        d = None
        torch.cuda.empty_cache()
    assert abs(got - want) <= 1e-6 * abs(want), (got, want, abs(got - want) / abs(want))
