"""GPU EM (Baum-Welch) iteration against the FP64 oracle, through the C ABI.

The M-step is FP64 arithmetic on hmm_posterior's expectations, which match
the oracle's to about 1e-6 of each sum (positive FP32 terms summed in FP64;
the location moments are accumulated about the input mu, so the covariance
S2/n1 - mu mu' loses nothing to cancellation beyond FP64's).  Quotients of
two such sums are then good to a few 1e-6 relative:
  delta, Gamma, p     absolute 1e-5 (probabilities)
  mu                  1e-5 of the state's spread sqrt(Sxx Syy) (km)
  Sigma               1e-4 relative to sqrt(Sxx Syy)
  ln L                1e-6 relative (the blocked FP32 likelihood's bound).
Sizes: one to many segments and fold groups, ragged tails, each K padding of
the local pass (16, 32, 64, 80), and the full K = 25, T = 1e6 workload."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_03508_amd import synth

from test_gpu_parity import binding, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _packed(prm):
    return torch.as_tensor(prm.packed(), dtype=torch.float64, device="cuda").contiguous()


def _unpack(v, K):
    v = np.asarray(v, dtype=np.float64)
    o = [0, K, K + K * K, 2 * K + K * K, 4 * K + K * K, 7 * K + K * K]
    return (v[o[0]:o[1]], v[o[1]:o[2]].reshape(K, K), v[o[2]:o[3]], v[o[3]:o[4]].reshape(K, 2),
            v[o[4]:o[5]].reshape(K, 3))


def _want(prm, obs):
    r = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    new = oracle.em_mstep(r["xi"], r["pre"], r["mom"], (prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma))
    return r["loglik"], new


def _check(got, want, what):
    d, G, p, mu, S = got
    d0, G0, p0, mu0, S0 = want
    assert np.abs(d - d0).max() <= 1e-5, (what, "delta")
    assert np.abs(G - G0).max() <= 1e-5, (what, "Gamma", np.abs(G - G0).max())
    assert np.abs(p - p0).max() <= 1e-5, (what, "p")
    spread = np.sqrt(S0[:, 0] * S0[:, 2])
    assert (np.abs(mu - mu0).max(axis=1) <= 1e-5 * spread).all(), (what, "mu", np.abs(mu - mu0).max())
    assert (np.abs(S - S0).max(axis=1) <= 1e-4 * spread).all(), (what, "Sigma", np.abs(S - S0).max())


def _step(ctx, prm, obs, block_len=0):
    ctx.set_blocking(block_len, 0)
    try:
        f = torch.as_tensor(obs.flag, dtype=torch.uint8, device="cuda").contiguous()
        xy = torch.as_tensor(obs.xy, dtype=torch.float64, device="cuda").contiguous()
        out, ll = ctx.em_step(_packed(prm), prm.K, f, xy)
        torch.cuda.synchronize()
        return float(ll.cpu()[0]), _unpack(out.cpu().numpy(), prm.K)
    finally:
        ctx.set_blocking(0, 0)


@pytest.mark.parametrize("K,T,L", [(1, 300, 32), (3, 1000, 32), (3, 5003, 0), (8, 2999, 40), (20, 4000, 33),
                                   (25, 20000, 0), (33, 3001, 32), (64, 2500, 32), (70, 2500, 32), (80, 3000, 0)])
def test_em_step_matches_oracle(binding, ctx, K, T, L):
    prm, obs = synth.make(K, T, 200 + K)
    ll0, want = _want(prm, obs)
    ll, got = _step(ctx, prm, obs, L)
    assert abs(ll - ll0) <= 1e-6 * abs(ll0), (ll, ll0)
    _check(got, want, (K, T, L))


def test_em_in_place_iterations(binding, ctx):
    """Ten iterations in place on the device (no host copy between them) follow
    the oracle's EM path; ln L of every iterate matches and never decreases."""
    prm, obs = synth.make(3, 3000, 5)
    rng = np.random.default_rng(1)
    start = synth.HMMParams(np.full(3, 1 / 3), rng.dirichlet(np.ones(3) * 5, size=3),
                            np.clip(prm.p + 0.1 * rng.standard_normal(3), 0.05, 0.95),
                            prm.mu + 15 * rng.standard_normal((3, 2)), prm.Sigma * 1.5)
    n = 10
    v = _packed(start)
    trace = torch.empty(n, dtype=torch.float64, device="cuda")
    f = torch.as_tensor(obs.flag, dtype=torch.uint8, device="cuda").contiguous()
    xy = torch.as_tensor(obs.xy, dtype=torch.float64, device="cuda").contiguous()
    for i in range(n):
        ctx.em_step(v, 3, f, xy, out=v, loglik=trace[i:i + 1])
    torch.cuda.synchronize()
    got_ll = trace.cpu().numpy()
    cur, want_ll = start, []
    for i in range(n):
        ll, new = _want(cur, obs)
        want_ll.append(ll)
        cur = synth.HMMParams(*new)
    assert np.allclose(got_ll, want_ll, rtol=1e-6, atol=0), (got_ll, want_ll)
    assert all(b >= a - 1e-6 * abs(a) for a, b in zip(got_ll, got_ll[1:]))
    got = _unpack(v.cpu().numpy(), 3)
    want = (cur.delta, cur.Gamma, cur.p, cur.mu, cur.Sigma)
    # ten contractions of the FP32-sum errors: a looser bar than one step
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=1e-3, atol=1e-4), (a, b)


def test_em_zero_counts_and_edge_cases(binding, ctx):
    prm, obs = synth.make(3, 1500, 11)
    # a state that never emits a tremor: p stays 0, mu and Sigma are kept bit for bit
    z = synth.HMMParams(prm.delta, prm.Gamma, np.where(np.arange(3) == 1, 0.0, prm.p), prm.mu, prm.Sigma)
    ll0, want = _want(z, obs)
    ll, got = _step(ctx, z, obs)
    assert abs(ll - ll0) <= 1e-6 * abs(ll0)
    _check(got, want, "p1=0")
    assert got[2][1] == 0.0 and np.array_equal(got[3][1], prm.mu[1]) and np.array_equal(got[4][1], prm.Sigma[1])
    # T = 0: delta renormalised, everything else kept
    d0 = np.array([0.2, 0.2, 0.4])
    e = synth.Observations(flag=obs.flag[:0], xy=obs.xy[:0])
    ll, got = _step(ctx, synth.HMMParams(d0, prm.Gamma, prm.p, prm.mu, prm.Sigma), e)
    assert abs(ll - math.log(0.8)) < 1e-12
    assert np.allclose(got[0], d0 / 0.8, rtol=1e-15) and np.array_equal(got[1], prm.Gamma)
    assert np.array_equal(got[2], prm.p) and np.array_equal(got[3], prm.mu) and np.array_equal(got[4], prm.Sigma)
    # K = 1: the sample mean and covariance of the tremor locations
    p1, o1 = synth.make(1, 2000, 3)
    ll, got = _step(ctx, p1, o1, 32)
    x = o1.xy[o1.flag.astype(bool)]
    C = np.cov(x.T, bias=True)
    assert abs(got[2][0] - o1.flag.mean()) < 1e-7
    assert np.allclose(got[3][0], x.mean(axis=0), rtol=1e-6)
    assert np.allclose(got[4][0], [C[0, 0], C[0, 1], C[1, 1]], rtol=1e-4, atol=1e-4 * math.sqrt(C[0, 0] * C[1, 1]))
    assert got[1][0, 0] == 1.0 and got[0][0] == 1.0
    # invalid parameters: NaN
    bad = synth.HMMParams(prm.delta, prm.Gamma, np.where(np.arange(3) == 0, 1.5, prm.p), prm.mu, prm.Sigma)
    ll, got = _step(ctx, bad, obs)
    assert math.isnan(ll) and all(np.isnan(a).all() for a in got)


def test_em_argument_errors(binding, ctx):
    prm, obs = synth.make(81, 100, 12)
    f = torch.as_tensor(obs.flag, dtype=torch.uint8, device="cuda").contiguous()
    xy = torch.as_tensor(obs.xy, dtype=torch.float64, device="cuda").contiguous()
    with pytest.raises(binding.HMMError):
        ctx.em_step(_packed(prm), 81, f, xy)
    prm, obs = synth.make(3, 100, 12)
    v = _packed(prm)
    f = torch.as_tensor(obs.flag, dtype=torch.uint8, device="cuda").contiguous()
    xy = torch.as_tensor(obs.xy, dtype=torch.float64, device="cuda").contiguous()
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    a = v.data_ptr()
    rc = binding._lib.hmm_em_step(ctx._h, 3, a, a + 24, a + 96, a + 120, a + 168, 100, f.data_ptr(), xy.data_ptr(),
                                  None, ll.data_ptr(), None)
    assert rc == binding.HMM_E_INVALID_ARG
    with pytest.raises(ValueError):
        ctx.em_step(v[:-1].contiguous(), 3, f, xy)


def test_em_step_full_size(binding, ctx):
    """K = 25, T = 1e6 (the likelihood benchmark's workload)."""
    w = synth.WORKLOADS["k25_t1e6"]
    prm, obs = synth.make(w["K"], w["T"], w["seed"])
    ll0, want = _want(prm, obs)
    ll, got = _step(ctx, prm, obs)
    assert abs(ll - ll0) <= 1e-6 * abs(ll0), (ll, ll0)
    _check(got, want, "k25_t1e6")
