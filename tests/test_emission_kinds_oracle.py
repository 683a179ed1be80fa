"""Pins of the oracle's other emission models (Poisson counts, 1-D Gaussian):
emissions against SciPy, closed forms of the likelihood, brute-force path
enumeration and the error conventions."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

import oracle
from paper_2003_03508_amd import synth


@pytest.mark.parametrize("kind", [1, 2])
def test_log_emission_matches_scipy(kind):
    s = synth.make_kind(kind, 5, 300, seed=10 + kind)
    got = oracle.log_emission_kind(kind, s.e0, s.e1, s.obs)
    if kind == 1:
        want = stats.poisson.logpmf(s.obs[:, None], s.e0[None, :])
    else:
        want = stats.norm.logpdf(s.obs[:, None], s.e0[None, :], np.sqrt(s.e1)[None, :])
    assert np.allclose(got, want, rtol=1e-13, atol=1e-12)


def _brute(delta, Gamma, logE):
    """log sum over every hidden path s_-1..s_{T-1} (eq. 2 applies Gamma first)."""
    T, K = logE.shape
    terms = []
    for path in itertools.product(range(K), repeat=T + 1):
        v = math.log(delta[path[0]]) if delta[path[0]] > 0 else -math.inf
        for t in range(T):
            v += math.log(Gamma[path[t], path[t + 1]]) + logE[t, path[t + 1]]
        terms.append(v)
    return logsumexp(terms)


@pytest.mark.parametrize("kind", [1, 2])
def test_loglik_brute_force(kind):
    s = synth.make_kind(kind, 3, 6, seed=20 + kind)
    logE = oracle.log_emission_kind(kind, s.e0, s.e1, s.obs)
    want = _brute(s.delta, s.Gamma, logE)
    got = oracle.loglik_kind(kind, s.delta, s.Gamma, s.e0, s.e1, s.obs)
    assert abs(got - want) <= 1e-12 * abs(want)


@pytest.mark.parametrize("kind", [1, 2])
def test_loglik_closed_forms(kind):
    s = synth.make_kind(kind, 1, 500, seed=30 + kind)
    # K = 1: the sum of the log emissions
    want = float(np.sum(oracle.log_emission_kind(kind, s.e0, s.e1, s.obs)))
    got = oracle.loglik_kind(kind, s.delta, s.Gamma, s.e0, s.e1, s.obs)
    assert abs(got - want) <= 1e-12 * abs(want)
    # Gamma = I: ln sum_k delta_k prod_t e_{t,k}
    s = synth.make_kind(kind, 4, 200, seed=40 + kind)
    logE = oracle.log_emission_kind(kind, s.e0, s.e1, s.obs)
    want = logsumexp(np.log(s.delta) + logE.sum(axis=0))
    got = oracle.loglik_kind(kind, s.delta, np.eye(4), s.e0, s.e1, s.obs)
    assert abs(got - want) <= 1e-12 * abs(want)


def test_poisson_closed_form_counts():
    # one state, counts y: sum_t (y_t ln lambda - lambda - ln y_t!)
    y = np.array([0, 1, 5, 12, 3], dtype=np.int32)
    lam = 4.5
    want = float(np.sum(y * math.log(lam) - lam - np.array([math.lgamma(v + 1) for v in y])))
    got = oracle.loglik_kind(1, [1.0], [[1.0]], [lam], None, y)
    assert abs(got - want) <= 1e-13 * abs(want)


def test_error_conventions():
    d, G = [0.5, 0.5], [[0.9, 0.1], [0.2, 0.8]]
    assert math.isnan(oracle.loglik_kind(1, d, G, [1.0, 0.0], None, [1, 2]))        # lambda <= 0
    assert math.isnan(oracle.loglik_kind(1, d, G, [1.0, 2.0], None, [1, -2]))       # negative count
    assert math.isnan(oracle.loglik_kind(2, d, G, [0.0, 1.0], [1.0, -1.0], [0.5]))  # var <= 0
    assert math.isnan(oracle.loglik_kind(2, d, G, [0.0, 1.0], [1.0, 1.0], [math.inf]))
    assert abs(oracle.loglik_kind(2, d, G, [0.0, 1.0], [1.0, 1.0], np.zeros(0))) < 1e-15  # T = 0
