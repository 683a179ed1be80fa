"""Host helpers of the sampler: the inverse of its parameter transform (to
start chains at given parameter values), the prior box from the observations
and the random-walk scale heuristics.  The transform itself, the prior, the
proposals and the accept/reject step run on the GPU (``binding.Chains``).

Unconstrained layout (length K*K + 4K): Gamma rows as log(Gamma_ij/Gamma_ii)
for j != i ascending, then logit p_k, then mu_k (x, y), then log of Sigma_k's
diagonal (xx, yy).
"""
import numpy as np


def dim(K):
    return K * K + 4 * K


def theta_from_params(Gamma, p, mu, Sigma):
    """Unconstrained vector of a parameter set (Sigma as (Sxx, Sxy, Syy) rows; Sxy ignored)."""
    Gamma = np.asarray(Gamma, dtype=np.float64)
    K = Gamma.shape[0]
    rows = []
    for i in range(K):
        lg = np.log(Gamma[i]) - np.log(Gamma[i, i])
        rows.append(np.delete(lg, i))
    p = np.asarray(p, dtype=np.float64)
    Sigma = np.asarray(Sigma, dtype=np.float64).reshape(K, 3)
    parts = [np.concatenate(rows) if K > 1 else np.zeros(0), np.log(p) - np.log1p(-p),
             np.asarray(mu, dtype=np.float64).reshape(-1), np.log(Sigma[:, [0, 2]]).reshape(-1)]
    return np.concatenate(parts)


def box_of(flag, xy):
    """(x0, x1, y0, y1): the bounding rectangle of the tremor locations."""
    f = np.asarray(flag).astype(bool)
    pts = np.asarray(xy, dtype=np.float64).reshape(-1, 2)[f]
    if pts.shape[0] == 0:
        return (-1e300, 1e300, -1e300, 1e300)
    return (float(pts[:, 0].min()), float(pts[:, 0].max()), float(pts[:, 1].min()), float(pts[:, 1].max()))


def block_slices(K):
    """Index ranges of the four parameter groups: Gamma, p, mu, log Sigma."""
    a = K * (K - 1)
    return dict(gamma=slice(0, a), p=slice(a, a + K), mu=slice(a + K, a + 3 * K),
                logsigma=slice(a + 3 * K, a + 5 * K))
