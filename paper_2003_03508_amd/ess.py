"""Effective sample size of MCMC output (host diagnostics for the sampler).

The paper judges its chains by trace plots and the number of effective
independent samples (section "Monte Carlo Markov Chains") without naming an
estimator.  Used here: the multi-chain estimator of Gelman et al. (Bayesian
Data Analysis, 3rd ed., section 11.5) with Geyer's initial monotone sequence
truncation (Geyer, "Practical Markov chain Monte Carlo", Statistical Science
1992):

    rho_t = 1 - (W - mean_c acov_c(t)) / var+,   var+ = (n-1)/n W + B/n
    P_k = rho_2k + rho_2k+1, summed while positive, made non-increasing,
    tau = -1 + 2 sum_k P_k,  ESS = m n / tau

for m chains of n draws (W: mean within-chain variance, B/n: variance of the
chain means).  Also the relabelling of mixture-like states used to compare
posterior summaries with known generating parameters.
"""
import numpy as np


def _autocov(x):
    """Biased autocovariance of a 1-D series for lags 0..n-1 (FFT)."""
    n = x.shape[0]
    y = x - x.mean()
    f = np.fft.rfft(y, n=2 * n)
    ac = np.fft.irfft(f * np.conj(f), n=2 * n)[:n]
    return ac / n


def ess(draws):
    """ESS of a scalar quantity; draws is (n,) or (m chains, n)."""
    x = np.asarray(draws, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    m, n = x.shape
    if n < 4:
        return float("nan")
    acov = np.stack([_autocov(c) for c in x])
    W = np.mean(acov[:, 0] * n / (n - 1))
    Bn = np.var(x.mean(axis=1), ddof=1) if m > 1 else 0.0
    var_plus = W * (n - 1) / n + Bn
    if not var_plus > 0:
        return float("nan")
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    pairs = rho[: 2 * (n // 2)].reshape(-1, 2).sum(axis=1)
    total = 0.0
    prev = np.inf
    for P in pairs:
        if P <= 0:
            break
        P = min(P, prev)
        total += P
        prev = P
    tau = max(-1.0 + 2.0 * total, 1.0 / np.log10(max(m * n, 10)))
    return float(m * n / tau)


def ess_columns(draws):
    """ESS of every column: draws is (m, n, d) -> (d,)."""
    x = np.asarray(draws, dtype=np.float64)
    return np.array([ess(x[:, :, j]) for j in range(x.shape[2])])


def mcse_mean(draws):
    """Monte Carlo standard error of the posterior mean of a scalar."""
    x = np.asarray(draws, dtype=np.float64)
    e = ess(x)
    return float(np.std(x.reshape(-1), ddof=1) / np.sqrt(e))


def relabel(mu_draws, mu_ref):
    """Permutation per draw that best matches state means to reference means.

    mu_draws: (..., K, 2); mu_ref: (K, 2).  Returns integer array (..., K) with
    perm[..., j] = the sampled state matched to reference state j (Hungarian
    assignment on squared distances).
    """
    from scipy.optimize import linear_sum_assignment
    mu = np.asarray(mu_draws, dtype=np.float64)
    shp = mu.shape[:-2]
    K = mu.shape[-2]
    flat = mu.reshape(-1, K, 2)
    out = np.empty((flat.shape[0], K), dtype=np.int64)
    for i, m in enumerate(flat):
        cost = ((mu_ref[:, None, :] - m[None, :, :]) ** 2).sum(-1)
        r, c = linear_sum_assignment(cost)
        out[i, r] = c
    return out.reshape(shp + (K,))
