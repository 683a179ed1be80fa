"""GPU forward-backward (state posteriors, expected transitions, weighted
moments, gradient of ln L) against the FP64 oracle, through the C ABI.

Tolerances (FP32 recursions inside segments, FP64 messages and sums):
  gamma_t,k          absolute 1e-4 (a probability);
  xi, pre, moments   relative 2e-5 of the largest entry of their block
                     (sums of T FP32 terms in FP64);
  ln L               1e-6 relative (the blocked FP32 likelihood's bound);
  gradient           relative 1e-4 of each block's scale (built in FP64 from
                     the expectations above).
Sizes span one to many segments and groups, ragged tails, every K padding of
the local pass (16, 32, 64, and 80 with two states per lane), and the full
K = 25, T = 1e6 workload."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_03508_amd import synth

from test_gpu_parity import binding, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _run(binding, ctx, prm, obs, block_len=0):
    ctx.set_blocking(block_len, 0)
    try:
        r = ctx.posterior(**binding.to_device(prm, obs))
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().astype(np.float64) for k, v in r.items()}
    finally:
        ctx.set_blocking(0, 0)


def _check(got, want, T, what):
    assert abs(got["loglik"][0] - want["loglik"]) <= 1e-6 * max(1.0, abs(want["loglik"])), what
    if T:
        err = np.abs(got["gamma"] - want["gamma"]).max()
        assert err <= 1e-4, (what, "gamma", err)
    for name in ("xi", "pre", "mom"):
        scale = np.abs(want[name]).max() + 1e-300
        err = np.abs(got[name] - want[name]).max() / scale
        assert err <= 2e-5, (what, name, err)


@pytest.mark.parametrize("K,T,L", [(1, 200, 32), (3, 1000, 32), (3, 5003, 0), (8, 2999, 40), (20, 4000, 33),
                                   (25, 20000, 0), (33, 3001, 32), (48, 2000, 64), (64, 2500, 32),
                                   (65, 2100, 32), (72, 3001, 0), (80, 2600, 40)])
def test_posterior_matches_oracle(binding, ctx, K, T, L):
    prm, obs = synth.make(K, T, 100 + K)
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    _check(_run(binding, ctx, prm, obs, L), want, T, (K, T, L))


def test_posterior_with_correlated_sigma_and_uneven_delta(binding, ctx):
    prm, obs = synth.make(5, 3000, 7)
    prm.Sigma[:, 1] = 0.4 * np.sqrt(prm.Sigma[:, 0] * prm.Sigma[:, 2])
    prm.delta = np.array([0.5, 0.2, 0.1, 0.15, 0.05])
    _, obs = synth.make(5, 3000, 7)
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    _check(_run(binding, ctx, prm, obs, 50), want, 3000, "correlated")


def test_full_size_k25_t1e6(binding, ctx):
    prm, obs = synth.make(**synth.WORKLOADS["k25_t1e6"])
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    got = _run(binding, ctx, prm, obs)
    _check(got, want, obs.T, "k25_t1e6")
    assert np.allclose(got["gamma"].sum(axis=1), 1.0, atol=1e-5)


@pytest.mark.parametrize("K,T,L", [(3, 2000, 32), (20, 20000, 0), (25, 100000, 0), (80, 6000, 0)])
def test_gradient_matches_oracle(binding, ctx, K, T, L):
    prm, obs = synth.make(K, T, 200 + K)
    prm.Sigma[:, 1] = 0.2 * np.sqrt(prm.Sigma[:, 0] * prm.Sigma[:, 2])
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    g_want = oracle.grad_from_stats(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, want["xi"], want["pre"],
                                    want["mom"])
    ctx.set_blocking(L, 0)
    try:
        ll, g = ctx.loglik_grad(**binding.to_device(prm, obs))
        torch.cuda.synchronize()
    finally:
        ctx.set_blocking(0, 0)
    assert abs(float(ll.item()) - want["loglik"]) <= 1e-6 * abs(want["loglik"])
    for name in ("delta", "Gamma", "p", "mu", "Sigma"):
        got = g[name].cpu().numpy().reshape(np.shape(g_want[name]))
        scale = np.abs(g_want[name]).max()
        assert np.abs(got - g_want[name]).max() <= 1e-4 * scale, (name, np.abs(got - g_want[name]).max(), scale)


def test_edge_cases(binding, ctx):
    prm, obs = synth.make(4, 100, 9)
    # T = 0: only the state before x_0 is left
    e = synth.Observations(flag=obs.flag[:0], xy=obs.xy[:0])
    r = _run(binding, ctx, prm, e)
    assert abs(r["loglik"][0] - math.log(prm.delta.sum())) < 1e-12
    assert np.allclose(r["pre"], prm.delta / prm.delta.sum()) and not r["xi"].any() and not r["mom"].any()
    # T = 1
    one = synth.Observations(flag=obs.flag[:1], xy=obs.xy[:1])
    want = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, one.flag, one.xy)
    _check(_run(binding, ctx, prm, one), want, 1, "T=1")
    # K = 1: gamma = 1, xi = T
    p1, o1 = synth.make(1, 777, 10)
    r = _run(binding, ctx, p1, o1, 32)
    assert np.allclose(r["gamma"], 1.0) and abs(r["xi"][0, 0] - 777) < 1e-3
    # invalid parameters: NaN everywhere
    bad = synth.HMMParams(**{**prm.__dict__, "p": np.where(np.arange(4) == 0, 1.5, prm.p)})
    r = _run(binding, ctx, bad, obs)
    assert math.isnan(r["loglik"][0]) and np.isnan(r["gamma"]).all() and np.isnan(r["xi"]).all()


def test_identity_transitions_closed_form(binding, ctx):
    """Gamma = I: the posterior of the constant state, delta_k prod_t e_t,k
    normalised, at every step.  Data from a sticky chain over states with
    nearby centres: every single step keeps the states' emissions within the
    blocked path's range (2^-256 of the best), while over the whole sequence
    the past and the future favour different states by far more than the
    floating-point range."""
    K, T = 3, 4000
    prm, _ = synth.make(K, T, 11)
    prm.mu[:] = prm.mu.mean(axis=0) + 0.1 * (prm.mu - prm.mu.mean(axis=0))
    obs = synth.sample_path(np.random.default_rng(12), prm, T)
    prm.Gamma = np.eye(K)
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy).sum(axis=0) + np.log(prm.delta)
    w = np.exp(le - le.max())
    w /= w.sum()
    r = _run(binding, ctx, prm, obs, 64)
    assert np.abs(r["gamma"] - w).max() <= 1e-4
    assert np.allclose(r["xi"], np.diag(T * w), rtol=1e-4, atol=1e-3 * T)


def test_argument_errors(binding, ctx):
    import ctypes
    prm, obs = synth.make(81, 100, 12)
    with pytest.raises(binding.HMMError):
        ctx.posterior(**binding.to_device(prm, obs))
    prm, obs = synth.make(3, 100, 12)
    d = binding.to_device(prm, obs)
    lib = binding._lib
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = lib.hmm_posterior(ctx._h, 3, d["delta"].data_ptr(), d["Gamma"].data_ptr(), d["p"].data_ptr(),
                           d["mu"].data_ptr(), d["Sigma"].data_ptr(), 100, d["flag"].data_ptr(),
                           d["xy"].data_ptr(), None, None, None, out.data_ptr())
    assert rc == binding.HMM_E_INVALID_ARG
    rc = lib.hmm_loglik_grad(ctx._h, 3, d["delta"].data_ptr(), d["Gamma"].data_ptr(), d["p"].data_ptr(),
                             d["mu"].data_ptr(), d["Sigma"].data_ptr(), 100, d["flag"].data_ptr(),
                             d["xy"].data_ptr(), None, out.data_ptr(), None)
    assert rc == binding.HMM_E_INVALID_ARG
