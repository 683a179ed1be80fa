"""Pins of the forward-backward, Viterbi and gradient oracles: every posterior
quantity against enumeration of all hidden paths with SciPy's densities, the
gradient assembled from the posterior expectations against central finite
differences of the likelihood oracle (Fisher's identity), closed forms
(one state, Gamma = I) and the recursions' identities."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2003_03508_amd import synth


def _emis(p, mu, Sigma, flag, xy):
    """e_{t,k} from SciPy (independent of the oracle's eq. (1) code)."""
    T, K = flag.shape[0], p.shape[0]
    E = np.empty((T, K))
    for t in range(T):
        for k in range(K):
            if flag[t]:
                S = [[Sigma[k, 0], Sigma[k, 1]], [Sigma[k, 1], Sigma[k, 2]]]
                E[t, k] = p[k] * stats.multivariate_normal(mu[k], S).pdf(xy[t])
            else:
                E[t, k] = 1 - p[k]
    return E


def _brute(delta, Gamma, E):
    """Posterior marginals, pairwise sums, s_-1 posterior, best path by enumeration."""
    T, K = E.shape
    Z = 0.0
    g = np.zeros((T, K))
    xi = np.zeros((K, K))
    pre = np.zeros(K)
    best, arg = -1.0, None
    for path in itertools.product(range(K), repeat=T + 1):
        w = delta[path[0]]
        for t in range(T):
            w *= Gamma[path[t], path[t + 1]] * E[t, path[t + 1]]
        Z += w
        pre[path[0]] += w
        for t in range(T):
            g[t, path[t + 1]] += w
            xi[path[t], path[t + 1]] += w
        if w > best:
            best, arg = w, path
    return g / Z, xi / Z, pre / Z, math.log(Z), math.log(best), arg


def _small(K, T, seed, sxy=0.0):
    prm, obs = synth.make(K, T, seed)
    Sigma = prm.Sigma.copy()
    Sigma[:, 1] = sxy * np.sqrt(Sigma[:, 0] * Sigma[:, 2])
    return prm, obs, Sigma


@pytest.mark.parametrize("K,T,seed,sxy,mixing", [(2, 5, 0, 0.0, False), (3, 4, 1, 0.4, False),
                                                 (3, 5, 2, -0.3, False), (1, 5, 3, 0.2, False),
                                                 (3, 5, 9, 0.1, True), (2, 6, 10, 0.0, True)])
def test_posterior_and_viterbi_match_path_enumeration(K, T, seed, sxy, mixing):
    prm, obs, Sigma = _small(K, T, seed, sxy)
    rng = np.random.default_rng(seed)
    delta = rng.dirichlet(np.ones(K))      # delta != stationary
    if mixing:                             # small diagonal: the best path changes state
        prm.Gamma = rng.dirichlet(np.ones(K), size=K) * 0.6 + 0.4 * np.roll(np.eye(K), 1, axis=1)
    E = _emis(prm.p, prm.mu, Sigma, obs.flag, obs.xy.reshape(-1, 2))
    g, xi, pre, lz, lbest, arg = _brute(delta, prm.Gamma, E)
    r = oracle.posterior(delta, prm.Gamma, prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert abs(r["loglik"] - lz) < 1e-11 * max(1, abs(lz))
    assert np.allclose(r["gamma"], g, rtol=1e-10, atol=1e-13)
    assert np.allclose(r["xi"], xi, rtol=1e-10, atol=1e-13)
    assert np.allclose(r["pre"], pre, rtol=1e-10, atol=1e-13)
    f = obs.flag.astype(bool)
    x = obs.xy.reshape(-1, 2)
    for k in range(K):
        w = g[:, k]
        want = [w.sum(), w[f].sum(), (w * x[:, 0])[f].sum(), (w * x[:, 1])[f].sum(),
                (w * x[:, 0] ** 2)[f].sum(), (w * x[:, 0] * x[:, 1])[f].sum(), (w * x[:, 1] ** 2)[f].sum()]
        assert np.allclose(r["mom"][k], want, rtol=1e-9, atol=1e-12)
    score, path, first = oracle.viterbi(delta, prm.Gamma, prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert abs(score - lbest) < 1e-10 * max(1, abs(lbest))
    assert (first,) + tuple(path) == tuple(arg)


def _fd(f, x, h):
    x = np.array(x, dtype=np.float64)
    out = np.empty(x.size)
    for i in range(x.size):
        a, b = x.copy().ravel(), x.copy().ravel()
        step = h * max(1.0, abs(a[i]))
        a[i] += step
        b[i] -= step
        out[i] = (f(a.reshape(x.shape)) - f(b.reshape(x.shape))) / (2 * step)
    return out.reshape(x.shape)


@pytest.mark.parametrize("K,T,seed,sxy", [(3, 300, 4, 0.3), (4, 200, 5, -0.5)])
def test_gradient_from_posterior_matches_finite_differences(K, T, seed, sxy):
    """Fisher's identity: the gradient built from the forward-backward
    expectations equals d ln L / d theta of the (forward-only) likelihood
    oracle, entry by entry, with no constraint tying the entries."""
    prm, obs, Sigma = _small(K, T, seed, sxy)
    delta = np.random.default_rng(seed).dirichlet(np.ones(K))
    args = dict(delta=delta, Gamma=prm.Gamma, p=prm.p, mu=prm.mu, Sigma=Sigma)
    r = oracle.posterior(delta, prm.Gamma, prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    g = oracle.grad_from_stats(delta, prm.Gamma, prm.p, prm.mu, Sigma, r["xi"], r["pre"], r["mom"])

    def ll(name):
        def f(v):
            a = dict(args)
            a[name] = v
            return oracle.loglik(a["delta"], a["Gamma"], a["p"], a["mu"], a["Sigma"], obs.flag, obs.xy)
        return f
    for name, h in (("delta", 1e-6), ("Gamma", 1e-6), ("p", 1e-7), ("mu", 1e-6), ("Sigma", 1e-6)):
        want = _fd(ll(name), args[name], h)
        got = g[name].reshape(want.shape)
        assert np.allclose(got, want, rtol=2e-5, atol=2e-5 * np.abs(want).max()), (name, got, want)


def test_one_state_and_identity_closed_forms():
    prm, obs, Sigma = _small(1, 50, 6)
    r = oracle.posterior([1.0], [[1.0]], prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert np.allclose(r["gamma"], 1.0) and np.allclose(r["xi"], [[50.0]]) and np.allclose(r["pre"], 1.0)
    score, path, first = oracle.viterbi([1.0], [[1.0]], prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert first == 0 and np.all(path == 0) and abs(score - r["loglik"]) < 1e-9 * abs(score)
    # Gamma = I: the state never changes; its posterior is delta_k prod_t e_t,k normalised
    K, T = 3, 40
    prm, obs, Sigma = _small(K, T, 7)
    prm.mu[:] = prm.mu.mean(axis=0) + 0.2 * (prm.mu - prm.mu.mean(axis=0))   # keep states comparable
    delta = np.array([0.2, 0.5, 0.3])
    le = np.log(_emis(prm.p, prm.mu, Sigma, obs.flag, obs.xy.reshape(-1, 2))).sum(axis=0) + np.log(delta)
    w = np.exp(le - le.max())
    w /= w.sum()
    r = oracle.posterior(delta, np.eye(K), prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert np.allclose(r["gamma"], np.tile(w, (T, 1)), rtol=1e-8, atol=1e-12)
    assert np.allclose(r["xi"], np.diag(T * w), rtol=1e-8, atol=1e-10)
    score, path, first = oracle.viterbi(delta, np.eye(K), prm.p, prm.mu, Sigma, obs.flag, obs.xy)
    assert np.all(path == np.argmax(le)) and first == np.argmax(le)
    assert abs(score - le.max()) < 1e-9 * abs(score)


def test_posterior_identities_and_errors():
    prm, obs = synth.make(4, 3000, 8)
    r = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    assert abs(r["loglik"] - oracle.loglik(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag,
                                           obs.xy)) < 1e-9 * abs(r["loglik"])
    assert np.allclose(r["gamma"].sum(axis=1), 1.0, atol=1e-12)
    assert abs(r["xi"].sum() - 3000) < 1e-8
    assert np.allclose(r["xi"].sum(axis=0), r["gamma"].sum(axis=0), rtol=1e-12)      # into s_t
    assert np.allclose(r["xi"].sum(axis=1) - r["pre"] + r["gamma"][-1],               # out of s_t-1
                       r["gamma"].sum(axis=0), rtol=1e-10)
    assert np.allclose(r["mom"][:, 0], r["gamma"].sum(axis=0), rtol=1e-12)
    # the Viterbi path's joint probability, recomputed along the path, is the score
    score, path, first = oracle.viterbi(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    le = oracle.log_emission(prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    s = np.concatenate([[first], path])
    along = math.log(prm.delta[first]) + np.log(prm.Gamma[s[:-1], s[1:]]).sum() + le[np.arange(3000), path].sum()
    assert abs(along - score) < 1e-9 * abs(score)
    assert score <= r["loglik"]
    # empty sequence, invalid parameters
    e = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag[:0], obs.xy[:0])
    assert abs(e["loglik"]) < 1e-15 and np.allclose(e["pre"], prm.delta)
    bad = prm.p.copy()
    bad[0] = 1.5
    b = oracle.posterior(prm.delta, prm.Gamma, bad, prm.mu, prm.Sigma, obs.flag, obs.xy)
    assert math.isnan(b["loglik"]) and np.isnan(b["gamma"]).all()
