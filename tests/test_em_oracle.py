"""Pins of the EM (Baum-Welch) M-step oracle: with one state it is the sample
maximum likelihood in closed form; iterating EM never decreases ln L (the EM
inequality); from a perturbed start on a long synthetic record it recovers
the generating parameters; the new parameters are stationary points of the
expected complete-data log-likelihood (finite differences)."""
import math

import numpy as np

import oracle
from paper_2003_03508_amd import synth


def test_one_state_is_the_sample_mle():
    prm, obs = synth.make(1, 2000, 3)
    r = oracle.posterior([1.0], [[1.0]], prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    d, G, p, mu, S = oracle.em_mstep(r["xi"], r["pre"], r["mom"])
    f = obs.flag.astype(bool)
    x = obs.xy.reshape(-1, 2)[f]
    assert abs(p[0] - f.mean()) < 1e-12
    assert np.allclose(mu[0], x.mean(axis=0), rtol=1e-12)
    C = np.cov(x.T, bias=True)
    assert np.allclose(S[0], [C[0, 0], C[0, 1], C[1, 1]], rtol=1e-9)
    assert np.allclose(G, [[1.0]]) and np.allclose(d, [1.0])


def _em(prm, obs, n):
    d, G, p, mu, S = prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma
    lls = []
    for _ in range(n):
        r = oracle.posterior(d, G, p, mu, S, obs.flag, obs.xy)
        lls.append(r["loglik"])
        d, G, p, mu, S = oracle.em_mstep(r["xi"], r["pre"], r["mom"])
    return lls, (d, G, p, mu, S)


def test_em_never_decreases_the_likelihood():
    prm, obs = synth.make(3, 3000, 5)
    rng = np.random.default_rng(1)
    start = synth.HMMParams(np.full(3, 1 / 3), rng.dirichlet(np.ones(3) * 5, size=3),
                            np.clip(prm.p + 0.1 * rng.standard_normal(3), 0.05, 0.95),
                            prm.mu + 15 * rng.standard_normal((3, 2)), prm.Sigma * 1.5)
    lls, _ = _em(start, obs, 12)
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(lls, lls[1:])), lls
    assert lls[-1] > lls[0] + 10


def test_em_recovers_generating_parameters():
    prm, obs = synth.make(2, 40000, 7)
    start = synth.HMMParams(prm.delta, np.array([[0.8, 0.2], [0.3, 0.7]]), np.clip(prm.p * 0.8, 0.05, 0.95),
                            prm.mu + 5.0, prm.Sigma * 1.3)
    _, (d, G, p, mu, S) = _em(start, obs, 40)
    assert np.allclose(G, prm.Gamma, atol=0.02)
    assert np.allclose(p, prm.p, atol=0.02)
    assert np.allclose(mu, prm.mu, atol=1.5)
    assert np.allclose(S[:, [0, 2]], prm.Sigma[:, [0, 2]], rtol=0.1)


def test_mstep_is_a_stationary_point_of_q():
    """Q(theta) = sum_ij xi_ij ln Gamma_ij + sum_i pre_i ln delta_i
    + sum_k [n1 ln p + (n - n1) ln(1 - p) + tremor Gaussian terms from the
    moments]; its partial derivatives in the free directions (rows of Gamma
    and delta moved along the simplex, p, mu, Sigma) vanish at the M-step."""
    prm, obs = synth.make(3, 2000, 9)
    r = oracle.posterior(prm.delta, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    xi, pre, mom = r["xi"], r["pre"], r["mom"]
    d, G, p, mu, S = oracle.em_mstep(xi, pre, mom)

    def Q(d, G, p, mu, S):
        q = float((xi * np.log(G)).sum() + (pre * np.log(d)).sum())
        for k in range(3):
            n, n1 = mom[k, 0], mom[k, 1]
            q += n1 * math.log(p[k]) + (n - n1) * math.log1p(-p[k])
            M = np.array([[S[k, 0], S[k, 1]], [S[k, 1], S[k, 2]]])
            Mi = np.linalg.inv(M)
            s1 = mom[k, 2:4]
            S2 = np.array([[mom[k, 4], mom[k, 5]], [mom[k, 5], mom[k, 6]]])
            C = S2 - np.outer(s1, mu[k]) - np.outer(mu[k], s1) + n1 * np.outer(mu[k], mu[k])
            q += -n1 * math.log(2 * math.pi) - 0.5 * n1 * math.log(np.linalg.det(M)) - 0.5 * np.trace(Mi @ C)
        return q
    q0 = Q(d, G, p, mu, S)

    def slope(f, h, scale):
        """|central difference of Q along a move f(e)| over a natural scale
        of that block's second derivative times the step"""
        return abs(f(h) - f(-h)) / (2 * h) / scale
    for k in range(3):
        n, n1 = mom[k, 0], mom[k, 1]

        def fp(e, k=k):
            pp = p.copy(); pp[k] += e
            return Q(d, G, pp, mu, S)
        assert slope(fp, 1e-6 * min(p[k], 1 - p[k]), n / (p[k] * (1 - p[k]))) < 1e-6
        for a in range(2):
            def fm(e, k=k, a=a):
                mp = mu.copy(); mp[k, a] += e
                return Q(d, G, p, mp, S)
            assert slope(fm, 1e-4, n1 / math.sqrt(S[k, 0] * S[k, 2])) < 1e-6
        for a in range(3):
            def fs(e, k=k, a=a):
                sp = S.copy(); sp[k, a] += e
                return Q(d, G, p, mu, sp)
            assert slope(fs, 1e-4 * math.sqrt(S[k, 0] * S[k, 2]), n1 / (S[k, 0] + S[k, 2])) < 1e-6
        # Gamma row k: move mass between two entries (stays on the simplex)
        def fg(e, k=k):
            Gp = G.copy(); Gp[k, 0] += e; Gp[k, 1] -= e
            return Q(d, Gp, p, mu, S)
        assert slope(fg, 1e-4 * min(G[k, 0], G[k, 1]), xi[k].sum()) < 1e-6

    def fd(e):
        dp = d.copy(); dp[0] += e; dp[1] -= e
        return Q(dp, G, p, mu, S)
    assert slope(fd, 1e-4 * min(d[0], d[1]), 1.0) < 1e-6
    # and Q is concave there: random moves in each block lower it
    rng = np.random.default_rng(3)
    assert Q(d, G, p, mu + rng.normal(0, 0.5, mu.shape), S) < q0
    assert Q(d, G, np.clip(p + rng.normal(0, 0.01, 3), 0.01, 0.99), mu, S) < q0
    assert Q(d, G, p, mu, S * np.array([1.05, 1.0, 0.97])) < q0
    Gr = G * np.exp(rng.normal(0, 0.05, G.shape))
    assert Q(d, Gr / Gr.sum(axis=1, keepdims=True), p, mu, S) < q0


def test_zero_counts_keep_the_previous_values():
    """A state with p_k = 0 has n1_k = 0 (no tremor hour can be its): mu_k
    and Sigma_k are left as they were, p_k stays 0.  With T = 0 only delta
    is renormalised."""
    prm, obs = synth.make(3, 1500, 11)
    p = prm.p.copy()
    p[1] = 0.0
    r = oracle.posterior(prm.delta, prm.Gamma, p, prm.mu, prm.Sigma, obs.flag, obs.xy)
    assert r["mom"][1, 1] == 0.0
    d, G, pn, mu, S = oracle.em_mstep(r["xi"], r["pre"], r["mom"], (prm.delta, prm.Gamma, p, prm.mu, prm.Sigma))
    assert pn[1] == 0.0 and np.array_equal(mu[1], prm.mu[1]) and np.array_equal(S[1], prm.Sigma[1])
    assert np.all(np.isfinite(mu)) and np.allclose(G.sum(axis=1), 1.0)
    _, G2, _, mu2, _ = oracle.em_mstep(r["xi"], r["pre"], r["mom"])
    assert np.all(np.isnan(mu2[1]))
    d0 = np.array([0.2, 0.2, 0.4])
    r = oracle.posterior(d0, prm.Gamma, prm.p, prm.mu, prm.Sigma, obs.flag[:0], obs.xy[:0])
    d, G, pn, mu, S = oracle.em_mstep(r["xi"], r["pre"], r["mom"], (d0, prm.Gamma, prm.p, prm.mu, prm.Sigma))
    assert np.allclose(d, d0 / d0.sum()) and np.array_equal(G, prm.Gamma) and np.array_equal(pn, prm.p)
    assert np.array_equal(mu, prm.mu) and np.array_equal(S, prm.Sigma)
