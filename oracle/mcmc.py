"""Metropolis-Hastings over the tremor-HMM parameters, plain FP64 (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the section "Monte Carlo Markov Chains" (accept or reject a proposed
state by the ratio of likelihood times prior at the proposed and the current
state) and the prior densities of the same section and Appendix A:

  * each row of Gamma ~ symmetric Dirichlet with concentration 0.01 (read
    row-wise: a Dirichlet over all K^2 entries would not give stochastic
    rows);
  * p_k ~ Gamma with mean 0.1 and variance 0.001 for the first floor(K/2)
    states and mean 0.9, variance 0.001 for the rest (shape m^2/v, rate m/v),
    read as truncated to (0, 1);
  * mu_k ~ uniform on a rectangle containing all observations;
  * Sigma_k ~ inverse Wishart with K degrees of freedom and identity scale
    (read as the 2x2 identity), evaluated on diagonal matrices.

Unconstrained coordinates theta (the MCMC state):
  [0, K(K-1))  row i of Gamma as log(Gamma_ij / Gamma_ii), j != i ascending
  [.., +K)     logit p_k
  [.., +2K)    mu_k (x, y)
  [.., +2K)    log Sigma_k,xx, log Sigma_k,yy  (Sigma_xy = 0)
delta is uniform and not sampled.  The log prior of theta is the log density
of the constrained parameters plus the log absolute Jacobian determinant of
the map theta -> parameters; additive constants are dropped.
"""
import math

import numpy as np

from . import loglik as _loglik
from . import philox

ALPHA = 0.01


def dim(K):
    return K * K + 4 * K


def split(K, theta):
    theta = np.asarray(theta, dtype=np.float64)
    a = K * (K - 1)
    return (theta[:a].reshape(K, K - 1), theta[a:a + K], theta[a + K:a + 3 * K].reshape(K, 2),
            theta[a + 3 * K:a + 5 * K].reshape(K, 2))


def to_params(K, theta):
    """theta -> (delta, Gamma, p, mu, Sigma) in the likelihood's layout."""
    lg, lgt, mu, lw = split(K, theta)
    Gamma = np.empty((K, K))
    for i in range(K):
        logits = np.insert(lg[i], i, 0.0)          # reference entry Gamma_ii
        m = logits.max()
        w = np.exp(logits - m)
        Gamma[i] = w / w.sum()
    p = 1.0 / (1.0 + np.exp(-lgt))
    Sigma = np.zeros((K, 3))
    Sigma[:, 0] = np.exp(lw[:, 0])
    Sigma[:, 2] = np.exp(lw[:, 1])
    delta = np.full(K, 1.0 / K)
    return delta, Gamma, p, mu.copy(), Sigma


def gamma_shape_rate(k, K):
    m = 0.1 if k < K // 2 else 0.9
    v = 0.001
    return m * m / v, m / v


def log_prior(K, theta, box):
    """Log prior density of theta (with the Jacobian of every transform)."""
    lg, lgt, mu, lw = split(K, theta)
    total = 0.0
    # Gamma rows: Dirichlet(alpha) density (alpha - 1) sum_j ln g_ij, plus the
    # log Jacobian of the additive-log-ratio map, sum_j ln g_ij over all K
    # entries of the row.
    for i in range(K):
        logits = np.insert(lg[i], i, 0.0)
        m = logits.max()
        lng = logits - (m + math.log(np.exp(logits - m).sum()))
        total += (ALPHA - 1.0) * lng.sum() + lng.sum()
    # p_k: Gamma(a, b) density (a - 1) ln p - b p, Jacobian of the logistic
    # map ln p + ln(1 - p); ln p = -log(1 + e^-z), ln(1 - p) = -log(1 + e^z).
    for k in range(K):
        z = float(lgt[k])
        lnp = -np.logaddexp(0.0, -z)
        ln1p = -np.logaddexp(0.0, z)
        a, b = gamma_shape_rate(k, K)
        total += (a - 1.0) * lnp - b * math.exp(lnp) + lnp + ln1p
    # mu_k: uniform on the box
    x0, x1, y0, y1 = box
    for k in range(K):
        if not (x0 <= mu[k, 0] <= x1 and y0 <= mu[k, 1] <= y1):
            return -math.inf
    # Sigma_k = diag(s_x, s_y): inverse-Wishart(nu = K, I) kernel
    # |S|^(-(nu + 3)/2) exp(-tr(S^-1)/2), Jacobian of s = e^w: w_x + w_y.
    nu = K
    for k in range(K):
        wx, wy = float(lw[k, 0]), float(lw[k, 1])
        total += -(nu + 3) / 2.0 * (wx + wy) - 0.5 * (math.exp(-wx) + math.exp(-wy)) + (wx + wy)
    return total


def loglik(K, theta, flag, xy):
    d, G, p, mu, S = to_params(K, theta)
    return _loglik(d, G, p, mu, S, flag, xy)


def log_normal_move(a, b, mean_shift, log_sd):
    """sum_d ln N(b_d | a_d + mean_shift_d, exp(log_sd_d)^2)."""
    z = (b - a - mean_shift) * np.exp(-log_sd)
    return float(np.sum(-0.5 * z * z - log_sd - 0.5 * math.log(2 * math.pi)))


def log_mixture(eps, lq_net, lq_rw):
    return float(np.logaddexp(math.log1p(-eps) + lq_net, math.log(eps) + lq_rw))


def mh_step(K, theta, ll, lp, seed, it, chain, rw, flag, xy, box, net=None, eps=None):
    """One Metropolis-Hastings iteration of one chain.

    net: None for the random walk, else a callable theta -> (mean_shift,
    log_sd) of the learned move, used with probability 1 - eps.  Returns a
    dict with the proposal, its log prior and likelihood, the proposal
    densities, ln of the acceptance ratio, ln u and the decision.
    """
    theta = np.asarray(theta, dtype=np.float64)
    rw = np.asarray(rw, dtype=np.float64)
    D = theta.shape[0]
    z = np.array(philox.normals(seed, philox.PROPOSAL, it, chain, D))
    use_net = False
    if net is not None:
        um, _ = philox.uniform2(seed, philox.MIXTURE, it, chain, 0)
        use_net = um >= eps
    if use_net:
        shift, lsd = net(theta)
        prop = theta + shift + np.exp(lsd) * z
    else:
        prop = theta + rw * z
    lp_p = log_prior(K, prop, box)
    ll_p = loglik(K, prop, flag, xy)
    lq_f = lq_r = 0.0
    if net is not None:
        zero = np.zeros(D)
        s_f, l_f = net(theta)
        s_r, l_r = net(prop)
        lq_f = log_mixture(eps, log_normal_move(theta, prop, s_f, l_f),
                           log_normal_move(theta, prop, zero, np.log(rw)))
        lq_r = log_mixture(eps, log_normal_move(prop, theta, s_r, l_r),
                           log_normal_move(prop, theta, zero, np.log(rw)))
    la = (ll_p + lp_p) - (ll + lp) + (lq_r - lq_f)
    u, _ = philox.uniform2(seed, philox.ACCEPT, it, chain, 0)
    lu = math.log(u)
    accept = bool(lu < la)
    return dict(prop=prop, lp=lp_p, ll=ll_p, lq_fwd=lq_f, lq_rev=lq_r, log_ratio=la, log_u=lu,
                accept=accept, use_net=use_net)
