"""Pins of the posterior-predictive simulation oracle: transition, tremor and
location statistics of long simulated paths against the parameters they come
from (chi-square and moment tests), the start distribution, the categorical
rule's edge cases, and the Philox stream layout."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import forecast, philox
from paper_2003_03508_amd import synth


def _params(K, seed, sxy=0.5):
    prm, _ = synth.make(K, 10, seed)
    prm.Sigma[:, 1] = sxy * np.sqrt(prm.Sigma[:, 0] * prm.Sigma[:, 2])
    return prm


def _numpy_draws(rng, H):
    u = rng.random((H, 2))
    z = rng.standard_normal((H, 2))
    return (lambda t: (u[t, 0], u[t, 1], z[t, 0], z[t, 1])), rng.random()


def test_categorical_rule():
    assert forecast.categorical([0.2, 0.3, 0.5], 0.0) == 0
    assert forecast.categorical([0.2, 0.3, 0.5], 0.2) == 1      # u < c_k, strict
    assert forecast.categorical([0.2, 0.3, 0.5], 0.2 - 1e-12) == 0
    assert forecast.categorical([0.2, 0.3, 0.5], 0.5 - 1e-12) == 1
    assert forecast.categorical([0.2, 0.3, 0.5], 0.999) == 2
    assert forecast.categorical([0.0, 1.0, 0.0], 0.5) == 1
    assert forecast.categorical([0.5, 0.5 - 1e-17, 0.0], 1.0 - 1e-18) == 1   # rounding: last positive


def test_simulated_path_statistics_match_the_parameters():
    """One long path (H = 60,000) of a 3-state model with mixing transitions
    and correlated Sigma: transition counts vs Gamma rows (chi-square), tremor
    rates vs p (binomial), location means and covariances vs mu, Sigma."""
    K, H = 3, 60000
    prm = _params(K, 2)
    rng = np.random.default_rng(1)
    prm.Gamma = rng.dirichlet(np.full(K, 2.0), size=K)
    step, u0 = _numpy_draws(np.random.default_rng(2), H)
    st, fl, xy, first = forecast.simulate_one(synth.HMMParams.packed(prm), np.ones(K) / K, K, H, step, u0)
    s = np.concatenate([[first], st])
    for i in range(K):
        nxt = s[1:][s[:-1] == i]
        obs = np.bincount(nxt, minlength=K)
        chi2, pval = stats.chisquare(obs, prm.Gamma[i] * obs.sum())
        assert pval > 1e-4, (i, obs, prm.Gamma[i])
        m = st == i
        k1 = fl[m].sum()
        assert abs(k1 - prm.p[i] * m.sum()) < 5 * math.sqrt(m.sum() * prm.p[i] * (1 - prm.p[i]))
        pts = xy[m & (fl == 1)]
        n = pts.shape[0]
        S = np.array([[prm.Sigma[i, 0], prm.Sigma[i, 1]], [prm.Sigma[i, 1], prm.Sigma[i, 2]]])
        se = np.sqrt(np.diag(S) / n)
        assert np.all(np.abs(pts.mean(axis=0) - prm.mu[i]) < 5 * se)
        C = np.cov(pts.T)
        assert np.all(np.abs(C - S) < 6 * np.sqrt((S ** 2 + np.outer(np.diag(S), np.diag(S))) / n))
    assert np.isnan(xy[fl == 0]).all() and not np.isnan(xy[fl == 1]).any()


def test_start_distribution_and_first_step():
    """s_-1 ~ start and s_0 ~ start Gamma over many short draws."""
    K, n = 4, 20000
    prm = _params(K, 3)
    start = np.array([0.1, 0.6, 0.0, 0.3])
    blk = synth.HMMParams.packed(prm)
    rng = np.random.default_rng(4)
    f0, s0 = [], []
    for _ in range(n):
        step, u0 = _numpy_draws(rng, 1)
        st, _, _, first = forecast.simulate_one(blk, start, K, 1, step, u0)
        f0.append(first)
        s0.append(st[0])
    c = np.bincount(f0, minlength=K)
    assert c[2] == 0
    assert stats.chisquare(c[[0, 1, 3]], start[[0, 1, 3]] * n).pvalue > 1e-4
    want = start @ prm.Gamma
    assert stats.chisquare(np.bincount(s0, minlength=K), want * n).pvalue > 1e-4


def test_dead_end_stops_the_path():
    K = 2
    prm = _params(K, 5)
    prm.Gamma = np.array([[0.0, 1.0], [0.0, 0.0]])      # state 1 has no way out
    step, u0 = _numpy_draws(np.random.default_rng(7), 5)
    st, fl, xy, first = forecast.simulate_one(synth.HMMParams.packed(prm), np.array([1.0, 0.0]), K, 5, step, u0)
    assert first == 0 and st[0] == 1 and (st[1:] == -1).all() and not fl[1:].any() and np.isnan(xy[1:]).all()
    st, fl, xy, first = forecast.simulate_one(synth.HMMParams.packed(prm), np.zeros(2), K, 5, step, u0)
    assert first == -1 and (st == -1).all()


def test_philox_stream_layout():
    step, u0 = forecast.philox_draws(9, 3)
    assert u0 == philox.uniform2(9, 12, 0, 3, 0)[0]
    assert step(5)[:2] == philox.uniform2(9, 10, 5, 3, 0)
    assert step(5)[2:] == philox.normal2(9, 11, 5, 3, 0)
