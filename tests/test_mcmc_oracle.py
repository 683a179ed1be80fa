"""Pins of the sampler's CPU oracle (Philox streams, parameter transform and
prior, Metropolis-Hastings step, proposal network) and of the ESS estimator,
against published test vectors, library densities, closed forms, finite
differences and known posteriors."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import mcmc as omcmc
from oracle import mlp as omlp
from oracle import philox
from paper_2003_03508_amd import ess as E
from paper_2003_03508_amd import mcmc as hm
from paper_2003_03508_amd import synth


# --------------------------------------------------------------------------- Philox
# Known-answer vectors of Philox4x32-10 published with the Random123 library
# (Salmon et al., SC 2011).
KAT = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
       ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
       ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert philox.philox4x32(ctr, key) == want


def test_philox_uniform_and_normal_moments():
    u = np.array([philox.uniform2(7, 3, it, 2, 0) for it in range(20000)]).ravel()
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    z = np.array(philox.normals(11, 1, 5, 3, 40000))
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_u01_extremes():
    assert philox.u01(0, 0) == 0.5 / 2 ** 53
    assert philox.u01(0xFFFFFFFF, 0xFFFFFFFF) == (2 ** 53 - 0.5) / 2 ** 53


# --------------------------------------------------------------------------- transform and prior
def _rand_theta(rng, K, box):
    th = np.concatenate([rng.normal(0, 1.5, K * (K - 1)), rng.normal(0, 2, K),
                         np.column_stack([rng.uniform(box[0], box[1], K), rng.uniform(box[2], box[3], K)]).ravel(),
                         rng.normal(4, 1, 2 * K)])
    return th


@pytest.mark.parametrize("K", [1, 2, 3, 5])
def test_transform_round_trip(K):
    rng = np.random.default_rng(K)
    box = (0, 200, 0, 200)
    th = _rand_theta(rng, K, box)
    d, G, p, mu, S = omcmc.to_params(K, th)
    assert np.allclose(G.sum(axis=1), 1, atol=1e-15)
    assert np.all(G > 0) and np.all((p > 0) & (p < 1))
    assert np.allclose(d, 1 / K)
    # the host-side inverse recovers theta, which pins the index order
    assert np.allclose(hm.theta_from_params(G, p, mu, S), th, atol=1e-12)
    # logistic and exponentials by their definitions
    a = K * (K - 1)
    assert np.allclose(p, 1 / (1 + np.exp(-th[a:a + K])))
    assert np.allclose(S[:, 1], 0) and np.allclose(np.log(S[:, [0, 2]]).ravel(), th[a + 3 * K:])


def _alr_log_jacobian(eta, i):
    """ln |det d(g_j, j != i)/d eta| of the row map by central differences."""
    K = eta.shape[0] + 1

    def g_free(e):
        logits = np.insert(e, i, 0.0)
        w = np.exp(logits - logits.max())
        return np.delete(w / w.sum(), i)

    J = np.empty((K - 1, K - 1))
    h = 1e-6
    for j in range(K - 1):
        ep, em = eta.copy(), eta.copy()
        ep[j] += h
        em[j] -= h
        J[:, j] = (g_free(ep) - g_free(em)) / (2 * h)
    return np.linalg.slogdet(J)[1]


def _prior_by_libraries(K, th, box):
    """Log prior of theta from SciPy densities plus numerically differentiated
    Jacobians (up to an additive constant)."""
    d, G, p, mu, S = omcmc.to_params(K, th)
    lg, _, _, lw = omcmc.split(K, th)
    tot = 0.0
    for i in range(K):
        if K > 1:
            tot += stats.dirichlet.logpdf(G[i], np.full(K, 0.01)) + _alr_log_jacobian(lg[i], i)
    for k in range(K):
        a, b = omcmc.gamma_shape_rate(k, K)
        # truncation to (0, 1) only adds a constant
        tot += stats.gamma.logpdf(p[k], a, scale=1 / b) + math.log(p[k] * (1 - p[k]))
        if K >= 2:
            tot += stats.invwishart.logpdf(np.diag([S[k, 0], S[k, 2]]), df=K, scale=np.eye(2))
        else:
            # nu = 1 is below SciPy's inverse-Wishart range; on diagonal matrices
            # the kernel is a product of inverse-gamma((nu + 1)/2, 1/2) densities
            tot += sum(stats.invgamma.logpdf(S[k, j], (K + 1) / 2, scale=0.5) for j in (0, 2))
        tot += lw[k, 0] + lw[k, 1]
    return tot


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_log_prior_matches_library_densities(K):
    rng = np.random.default_rng(100 + K)
    box = (-10, 210, -5, 190)
    ths = [_rand_theta(rng, K, box) for _ in range(4)]
    ours = np.array([omcmc.log_prior(K, t, box) for t in ths])
    ref = np.array([_prior_by_libraries(K, t, box) for t in ths])
    # equal up to one additive constant
    assert np.allclose(ours - ours[0], ref - ref[0], rtol=0, atol=1e-6 * (1 + np.abs(ref - ref[0])))


def test_log_prior_box_and_gamma_halves():
    K = 4
    box = (0, 100, 0, 100)
    th = _rand_theta(np.random.default_rng(1), K, box)
    assert math.isfinite(omcmc.log_prior(K, th, box))
    a = K * (K - 1)
    bad = th.copy()
    bad[a + K] = 100.5          # mu_0 x outside
    assert omcmc.log_prior(K, bad, box) == -math.inf
    got = [omcmc.gamma_shape_rate(k, K) for k in range(K)]
    assert np.allclose(got, [(10.0, 100.0)] * 2 + [(810.0, 900.0)] * 2, rtol=1e-14)
    assert np.allclose(omcmc.gamma_shape_rate(0, 1), (810.0, 900.0), rtol=1e-14)


# --------------------------------------------------------------------------- MH step
def _k1_problem(T=300, seed=5):
    prm, obs = synth.make(1, T, seed)
    box = hm.box_of(obs.flag, obs.xy)
    return prm, obs, box


def _run_oracle_chain(K, theta0, rw, obs, box, seed, chain, n_iter, net=None, eps=None):
    th = np.array(theta0, dtype=np.float64)
    lp = omcmc.log_prior(K, th, box)
    ll = omcmc.loglik(K, th, obs.flag, obs.xy)
    out = np.empty((n_iter, th.shape[0]))
    acc = 0
    for it in range(n_iter):
        r = omcmc.mh_step(K, th, ll, lp, seed, it, chain, rw, obs.flag, obs.xy, box, net=net, eps=eps)
        if r["accept"]:
            th, ll, lp = r["prop"], r["ll"], r["lp"]
            acc += 1
        out[it] = th
    return out, acc / n_iter


def _k1_exact(obs, box):
    """Posterior means of p, mu_x and ln Sigma_xx for K = 1.

    p: quadrature of p^n1 (1-p)^n0 times the Gamma(810, rate 900) prior on
    (0, 1).  With the inverse-Wishart kernel on diagonal matrices the x axis
    separates: after integrating mu_x (box far wider than its posterior),
    Sigma_xx ~ inverse gamma(alpha = (n1 + nu)/2, beta = (S + 1)/2), S the
    scatter of the tremor x coordinates, so E[mu_x] = mean x and
    E[ln Sigma_xx] = ln beta - digamma(alpha)."""
    from scipy.special import digamma
    f = obs.flag.astype(bool)
    n1, n0 = int(f.sum()), int((~f).sum())
    a, b = omcmc.gamma_shape_rate(0, 1)
    logf = lambda q: (n1 + a - 1) * math.log(q) + n0 * math.log1p(-q) - b * q
    grid = np.linspace(1e-6, 1 - 1e-6, 20001)
    vals = np.array([logf(q) for q in grid])
    m, mode = vals.max(), grid[np.argmax(vals)]
    Z = integrate.quad(lambda q: math.exp(logf(q) - m), 0, 1, points=[mode], limit=200)[0]
    Ep = integrate.quad(lambda q: q * math.exp(logf(q) - m), 0, 1, points=[mode], limit=200)[0] / Z
    x = obs.xy.reshape(-1, 2)[f, 0]
    S = float(((x - x.mean()) ** 2).sum())
    nu = 1
    Ew = math.log((S + 1) / 2) - digamma((n1 + nu) / 2)
    return Ep, float(x.mean()), Ew


def _k1_rw_scale(obs):
    f = obs.flag.astype(bool)
    n1 = f.sum()
    x = obs.xy.reshape(-1, 2)[f]
    sd = np.array([0.15, x[:, 0].std() / math.sqrt(n1), x[:, 1].std() / math.sqrt(n1),
                   math.sqrt(2 / n1), math.sqrt(2 / n1)])
    return 1.2 * sd


def _check_k1_means(d, obs, box):
    Ep, Emx, Ew = _k1_exact(obs, box)
    p = 1 / (1 + np.exp(-d[:, :, 0]))
    for est, want in ((p, Ep), (d[:, :, 1], Emx), (d[:, :, 3], Ew)):
        assert abs(est.mean() - want) < 4 * E.mcse_mean(est), (est.mean(), want, E.mcse_mean(est))


def test_mh_oracle_k1_posterior_means():
    # few observations, so that the prior and its Jacobians move the
    # posterior by many Monte Carlo standard errors
    prm, obs, box = _k1_problem(T=60)
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    rw = _k1_rw_scale(obs)
    chains = []
    for c in range(8):
        draws, acc = _run_oracle_chain(1, th0, rw, obs, box, seed=21, chain=c, n_iter=2500)
        assert 0.1 < acc < 0.7
        chains.append(draws[500:])
    _check_k1_means(np.stack(chains), obs, box)


def test_mh_oracle_hastings_term_corrects_a_biased_proposal():
    """A deliberately drifting 'learned' move still samples the posterior
    because the mixture density enters the ratio in both directions (without
    that term, or with its sign flipped, the means move by > 10 MCSE)."""
    prm, obs, box = _k1_problem()
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    rw = _k1_rw_scale(obs)

    def net(theta):
        return 0.5 * rw, np.log(0.6 * rw) + 0.0 * theta   # constant drift

    chains = []
    for c in range(4):
        draws, acc = _run_oracle_chain(1, th0, rw, obs, box, seed=33, chain=c, n_iter=3000, net=net, eps=0.2)
        chains.append(draws[500:])
    _check_k1_means(np.stack(chains), obs, box)


def test_mh_oracle_step_fields_are_consistent():
    prm, obs, box = _k1_problem(T=100)
    th = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    rw = _k1_rw_scale(obs)
    lp = omcmc.log_prior(1, th, box)
    ll = omcmc.loglik(1, th, obs.flag, obs.xy)
    r = omcmc.mh_step(1, th, ll, lp, 3, 0, 0, rw, obs.flag, obs.xy, box)
    z = np.array(philox.normals(3, philox.PROPOSAL, 0, 0, 5))
    assert np.allclose(r["prop"], th + rw * z, rtol=0, atol=1e-15)
    assert r["log_ratio"] == pytest.approx(r["ll"] + r["lp"] - ll - lp)
    assert r["accept"] == (r["log_u"] < r["log_ratio"])


# --------------------------------------------------------------------------- network
def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    D, H, B = 3, 5, 4
    w = rng.normal(0, 0.5, omlp.count(D, H))
    X = rng.normal(size=(B, D))
    R = rng.normal(size=(B, D))
    g = omlp.grad(w, X, R, D, H)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (omlp.loss(wp, X, R, D, H) - omlp.loss(wm, X, R, D, H)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_mlp_loss_is_gaussian_nll():
    rng = np.random.default_rng(1)
    D, H, B = 4, 6, 5
    w = rng.normal(0, 0.5, omlp.count(D, H))
    X = rng.normal(size=(B, D))
    R = rng.normal(size=(B, D))
    O, _ = omlp.forward(w, X, D, H)
    nll = -stats.norm.logpdf(R, loc=O[:, :D], scale=np.exp(O[:, D:])).sum(axis=1) - 0.5 * D * math.log(2 * math.pi)
    assert np.allclose(omlp.loss_rows(w, X, R, D, H), nll / B, rtol=1e-12, atol=1e-12)


def test_mlp_layout_and_forward_by_hand():
    D, H = 2, 3
    assert omlp.count(D, H) == D * H + H + H * H + H + H * 2 * D + 2 * D + D
    rng = np.random.default_rng(2)
    w = rng.normal(size=omlp.count(D, H))
    x = rng.normal(size=D)
    W1 = w[:D * H].reshape(D, H)
    b1 = w[D * H:D * H + H]
    o = D * H + H
    W2 = w[o:o + H * H].reshape(H, H)
    b2 = w[o + H * H:o + H * H + H]
    o += H * H + H
    W3 = w[o:o + H * 2 * D].reshape(H, 2 * D)
    b3 = w[o + H * 2 * D:o + H * 2 * D + 2 * D]
    a = w[o + H * 2 * D + 2 * D:]
    assert a.shape == (D,)
    h1 = [math.tanh(sum(x[i] * W1[i, j] for i in range(D)) + b1[j]) for j in range(H)]
    h2 = [math.tanh(sum(h1[i] * W2[i, j] for i in range(H)) + b2[j]) for j in range(H)]
    out = [sum(h2[i] * W3[i, j] for i in range(H)) + b3[j] + (a[j] * x[j] if j < D else 0.0)
           for j in range(2 * D)]
    got, _ = omlp.forward(w, x[None, :], D, H)
    assert np.allclose(got[0], out, rtol=1e-14, atol=1e-14)


# --------------------------------------------------------------------------- ESS
@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ess_ar1_closed_form(phi):
    rng = np.random.default_rng(int(phi * 10))
    m, n = 4, 40000
    e = rng.standard_normal((m, n))
    x = np.empty((m, n))
    x[:, 0] = e[:, 0] / math.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    want = m * n * (1 - phi) / (1 + phi)
    assert abs(E.ess(x) / want - 1) < 0.1


def test_ess_detects_chains_stuck_apart():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 5000)) * 0.1 + np.arange(4)[:, None]
    assert E.ess(x) < 100


def test_relabel_recovers_permutation():
    rng = np.random.default_rng(4)
    ref = rng.uniform(0, 200, (6, 2))
    perms = [rng.permutation(6) for _ in range(5)]
    draws = np.stack([ref[p] + rng.normal(0, 0.5, (6, 2)) for p in perms])
    got = E.relabel(draws, ref)
    for p, g in zip(perms, got):
        assert np.all(p[g] == np.arange(6))
