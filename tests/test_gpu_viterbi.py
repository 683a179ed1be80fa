"""GPU Viterbi against the FP64 oracle, through the C ABI.

The maximum itself (score) must match the oracle's to 1e-6 relative (the FP32
likelihood's bound).  Paths are compared by what is unique: the joint log
probability of the returned path, recomputed in FP64 along it, must equal the
oracle's maximum within that tolerance, and every transition of the path must
be allowed (Gamma > 0).  Where the two paths differ, both are maxima up to
FP32 rounding (counted; exact ties are rare with continuous data)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_03508_amd import synth

from test_gpu_parity import binding, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _path_score(prm, obs, first, path):
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    s = np.concatenate([[first], path]).astype(np.int64)
    with np.errstate(divide="ignore"):
        return (math.log(prm.delta[first]) + np.log(prm.Gamma[s[:-1], s[1:]]).sum()
                + le[np.arange(len(path)), path].sum())


def _run(binding, ctx, prm, obs, L=0):
    ctx.set_blocking(L, 0)
    try:
        path, first, score = ctx.viterbi(**binding.to_device(prm, obs))
        torch.cuda.synchronize()
        return path.cpu().numpy(), int(first.item()), float(score.item())
    finally:
        ctx.set_blocking(0, 0)


def _check(binding, ctx, prm, obs, L=0, what=""):
    want, wpath, wfirst = oracle.viterbi(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    path, first, score = _run(binding, ctx, prm, obs, L)
    tol = 1e-6 * max(1.0, abs(want))
    assert abs(score - want) <= tol, (what, score, want)
    assert path.shape == wpath.shape and path.min() >= 0 and path.max() < prm.K
    along = _path_score(prm, obs, first, path)
    assert abs(along - want) <= tol, (what, along, want)
    return int((path != wpath).sum()) + int(first != wfirst)


@pytest.mark.parametrize("K,T,L", [(1, 300, 32), (2, 50, 32), (3, 1000, 32), (3, 5003, 0), (8, 2999, 40),
                                   (16, 4000, 33), (17, 3001, 32), (25, 20000, 0), (25, 20000, 32),
                                   (32, 2500, 32), (5, 1, 0), (33, 2000, 32), (48, 3001, 40),
                                   (64, 2500, 0), (65, 2100, 32), (72, 3001, 0), (80, 2600, 40), (80, 700, 0)])
def test_viterbi_matches_oracle(binding, ctx, K, T, L):
    prm, obs = synth.make(K, T, 300 + K)
    diff = _check(binding, ctx, prm, obs, L, (K, T, L))
    assert diff <= max(2, T // 1000)


def test_viterbi_mixing_and_sparse_transitions(binding, ctx):
    rng = np.random.default_rng(5)
    prm, obs = synth.make(6, 4000, 31)
    prm.Gamma = rng.dirichlet(np.full(6, 0.3), size=6)
    prm.Gamma[prm.Gamma < 1e-3] = 0.0
    prm.Gamma /= prm.Gamma.sum(axis=1, keepdims=True)
    prm.delta = rng.dirichlet(np.ones(6))
    obs = synth.sample_path(np.random.default_rng(6), prm, 4000)
    _check(binding, ctx, prm, obs, 48, "sparse")


def test_viterbi_full_size_k25_t1e6(binding, ctx):
    prm, obs = synth.make(**synth.WORKLOADS["k25_t1e6"])
    diff = _check(binding, ctx, prm, obs, 0, "k25_t1e6")
    assert diff <= 1000


def test_viterbi_edge_cases(binding, ctx):
    prm, obs = synth.make(4, 100, 9)
    e = synth.Observations(flag=obs.flag[:0], xy=obs.xy[:0])
    path, first, score = _run(binding, ctx, prm, e)
    assert path.size == 0 and first == int(np.argmax(prm.delta))
    assert abs(score - math.log(prm.delta.max())) < 1e-12
    bad = synth.HMMParams(**{**prm.__dict__, "p": np.where(np.arange(4) == 0, 1.5, prm.p)})
    path, first, score = _run(binding, ctx, bad, obs)
    assert math.isnan(score) and first == -1 and (path == -1).all()

@pytest.mark.parametrize("what", ["flag 2", "nan location", "inf location"])
def test_viterbi_invalid_data(binding, ctx, what):
    """Invalid observations (a flag other than 0/1, a tremor with a
    non-finite location) anywhere in the sequence give a NaN score and -1
    for s_-1 and the whole path, as invalid parameters do."""
    prm, obs = synth.make(5, 3000, 13)
    flag, xy = obs.flag.copy(), obs.xy.copy()
    t = 2222
    if what == "flag 2":
        flag[t] = 2
    else:
        flag[t] = 1
        xy[t] = (np.nan, 1.0) if what == "nan location" else (1.0, np.inf)
    bad = synth.Observations(flag=flag, xy=xy)
    assert math.isnan(oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, flag, xy))
    path, first, score = _run(binding, ctx, prm, bad, 64)
    assert math.isnan(score) and first == -1 and (path == -1).all()
    # the same context then gives the valid answer again
    _check(binding, ctx, prm, obs, 64, "after invalid data")


def test_viterbi_identity_transitions(binding, ctx):
    """Gamma = I: the path stays in argmax_k ln delta_k + sum_t ln e_t,k."""
    K, T = 3, 3000
    prm, _ = synth.make(K, T, 11)
    prm.mu[:] = prm.mu.mean(axis=0) + 0.1 * (prm.mu - prm.mu.mean(axis=0))
    obs = synth.sample_path(np.random.default_rng(12), prm, T)
    prm.Gamma = np.eye(K)
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy).sum(axis=0) + np.log(prm.delta)
    path, first, score = _run(binding, ctx, prm, obs, 64)
    assert (path == np.argmax(le)).all() and first == np.argmax(le)
    assert abs(score - le.max()) <= 1e-6 * abs(le.max())
