"""Second, independent oracle: the forward algorithm in the log domain.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

It evaluates the same eq. (2) likelihood as the C oracle but shares none of its
code: emissions come from SciPy's bivariate normal log-pdf (a textbook routine)
and the recursion (Algorithm 1) is run on log forward variables with
logsumexp, so no scaling constants appear at all:
    log a_0(j)   = logsumexp_i(log delta_i + log Gamma_ij) + log e_0(j)
    log a_t(j)   = logsumexp_i(log a_{t-1}(i) + log Gamma_ij) + log e_t(j)
    log L        = logsumexp_j log a_{T-1}(j)
Pure NumPy; meant for T up to ~1e4.
"""
import numpy as np
from scipy.special import logsumexp
from scipy.stats import multivariate_normal


def log_emission(p, mu, Sigma, flag, xy):
    """ln e_{t,k} of eq. (1): ln p_k + ln phi(x|mu_k,Sigma_k) if flag=1 else ln(1-p_k)."""
    p = np.asarray(p, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, 2)
    Sigma = np.asarray(Sigma, dtype=np.float64).reshape(-1, 3)
    flag = np.asarray(flag)
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    T, K = flag.shape[0], p.shape[0]
    out = np.empty((T, K))
    tremor = flag == 1
    with np.errstate(divide="ignore"):
        for k in range(K):
            S = np.array([[Sigma[k, 0], Sigma[k, 1]], [Sigma[k, 1], Sigma[k, 2]]])
            out[:, k] = np.log1p(-p[k])
            if tremor.any():
                out[tremor, k] = np.log(p[k]) + multivariate_normal(mean=mu[k], cov=S).logpdf(
                    xy[tremor]).reshape(-1)
    return out


def forward_from_logemis(delta, Gamma, logE):
    delta = np.asarray(delta, dtype=np.float64)
    Gamma = np.asarray(Gamma, dtype=np.float64)
    logE = np.asarray(logE, dtype=np.float64)
    with np.errstate(divide="ignore"):
        lG = np.log(Gamma)
        la = np.log(delta)
    if logE.shape[0] == 0:
        return float(logsumexp(la))
    for t in range(logE.shape[0]):
        la = logsumexp(la[:, None] + lG, axis=0) + logE[t]
    return float(logsumexp(la))


def loglik(delta, Gamma, p, mu, Sigma, flag, xy):
    return forward_from_logemis(delta, Gamma, log_emission(p, mu, Sigma, flag, xy))
