"""FP64 CPU oracle for the tremor-HMM forward log-likelihood.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library in ``paper_2003_03508_amd`` and never imports it.

Contents
  * ``hmm_oracle.c`` -- plain FP64 scaled forward algorithm (Algorithm 1 of the
    paper applied to eq. (2), emissions from eq. (1)), plus the same quantity
    in the block-product order of the paper's three-step parallel plan.
    Loaded here through ctypes.
  * ``logspace.py`` -- a second, independent forward algorithm in the log
    domain (NumPy, logsumexp), with emissions from SciPy's bivariate normal.
  * ``brute.py``    -- enumeration of every hidden path in exact rationals.
  * ``loglik_kind`` -- eq. (2) with Poisson-count or 1-D Gaussian emissions
    (other HMMs differ from the tremor model only in the emission function).
  * ``posterior`` / ``viterbi`` -- state posteriors by forward-backward (with
    expected transition counts and weighted moments) and the most likely path.
  * ``grad_from_stats`` -- the gradient of ln L from those expectations.
  * ``em_mstep`` -- the EM (Baum-Welch) maximisation step from them.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmm_oracle.c")
_LIB = os.path.join(_HERE, "libhmm_oracle.so")


def build(force=True):
    """Compile the C oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-D_GNU_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_log_emission.restype = ctypes.c_int
        L.oracle_log_emission.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int64, u8p, dp, dp]
        L.oracle_forward_from_logemis.restype = ctypes.c_double
        L.oracle_forward_from_logemis.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, dp]
        L.oracle_loglik.restype = ctypes.c_double
        L.oracle_loglik.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int64, u8p, dp]
        L.oracle_loglik_blocked.restype = ctypes.c_double
        L.oracle_loglik_blocked.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int64,
                                            u8p, dp, ctypes.c_int64]
        L.oracle_log_emission_kind.restype = ctypes.c_int
        L.oracle_log_emission_kind.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_void_p,
                                               dp]
        L.oracle_loglik_kind.restype = ctypes.c_double
        L.oracle_loglik_kind.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.c_int64,
                                         ctypes.c_void_p]
        L.oracle_posterior.restype = ctypes.c_double
        L.oracle_posterior.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int64, u8p, dp, dp, dp, dp, dp]
        L.oracle_viterbi.restype = ctypes.c_double
        L.oracle_viterbi.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int64, u8p, dp, i32p, i32p]
        L.oracle_loglik_batch.restype = ctypes.c_int
        L.oracle_loglik_batch.argtypes = [ctypes.c_int32, i32p, i64p, i64p, dp, i64p, u8p, dp, dp,
                                          ctypes.c_int32]
        _lib = L
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def log_emission(p, mu, Sigma, flag, xy):
    """ln e_{t,k} of eq. (1) as a (T, K) float64 array (NaN everywhere on bad data)."""
    p, pp = _f64(p)
    mu, mup = _f64(mu)
    Sigma, sp = _f64(Sigma)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    K, T = p.shape[0], flag.shape[0]
    out = np.empty((T, K), dtype=np.float64)
    lib().oracle_log_emission(K, pp, mup, sp, T, fp, xp,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def forward_from_logemis(delta, Gamma, logE):
    """Algorithm 1 (scaled) on given ln e_{t,k}; returns ln L."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    logE, lp = _f64(logE)
    K = delta.shape[0]
    T = logE.shape[0] if logE.size else 0
    return lib().oracle_forward_from_logemis(K, dp_, gp, T, lp)


def loglik(delta, Gamma, p, mu, Sigma, flag, xy):
    """ln L of eq. (2): validity checks, eq. (1), scaled Algorithm 1, FP64."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    p, pp = _f64(p)
    mu, mup = _f64(mu)
    Sigma, sp = _f64(Sigma)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    return lib().oracle_loglik(delta.shape[0], dp_, gp, pp, mup, sp, flag.shape[0], fp, xp)


def loglik_blocked(delta, Gamma, p, mu, Sigma, flag, xy, L):
    """ln L in the segment-product order of the paper's parallel plan (FP64)."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    p, pp = _f64(p)
    mu, mup = _f64(mu)
    Sigma, sp = _f64(Sigma)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    return lib().oracle_loglik_blocked(delta.shape[0], dp_, gp, pp, mup, sp, flag.shape[0],
                                       fp, xp, int(L))


def loglik_batch(K, T, param_off, params, obs_off, flag, xy, nthreads=1):
    """ln L for many packed sets (same packing as the batched GPU call)."""
    K = np.ascontiguousarray(K, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.int64)
    param_off = np.ascontiguousarray(param_off, dtype=np.int64)
    obs_off = np.ascontiguousarray(obs_off, dtype=np.int64)
    params, pp = _f64(params)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    n = K.shape[0]
    out = np.empty(n, dtype=np.float64)
    lib().oracle_loglik_batch(
        n, K.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        T.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        param_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pp,
        obs_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), fp, xp,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(nthreads))
    return out


POISSON, GAUSS1D = 1, 2


def _kind_args(kind, e0, e1, obs):
    e0, p0 = _f64(e0)
    e1, p1 = _f64(e1 if e1 is not None else np.zeros_like(e0))
    if kind == POISSON:
        obs = np.ascontiguousarray(obs, dtype=np.int32)
    else:
        obs = np.ascontiguousarray(obs, dtype=np.float64)
    return e0, p0, e1, p1, obs


def log_emission_kind(kind, e0, e1, obs):
    """ln e_{t,k} (T, K) of the Poisson (kind 1: e0 = lambda, obs = int counts) or
    1-D Gaussian (kind 2: e0 = mu, e1 = var, obs = values) emission model."""
    e0, p0, e1, p1, obs = _kind_args(kind, e0, e1, obs)
    K, T = e0.shape[0], obs.shape[0]
    out = np.empty((T, K), dtype=np.float64)
    lib().oracle_log_emission_kind(kind, K, p0, p1, T, obs.ctypes.data,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def loglik_kind(kind, delta, Gamma, e0, e1, obs):
    """ln L of eq. (2) with the Poisson or 1-D Gaussian emission model (FP64)."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    e0, p0, e1, p1, obs = _kind_args(kind, e0, e1, obs)
    return lib().oracle_loglik_kind(kind, delta.shape[0], dp_, gp, p0, p1, obs.shape[0], obs.ctypes.data)


def posterior(delta, Gamma, p, mu, Sigma, flag, xy):
    """State posteriors by the scaled forward-backward recursions (FP64).

    Returns dict: loglik, gamma (T, K) = P(s_t = k | x), xi (K, K) = expected
    transition counts summed over t = 0..T-1 (t = 0 from the state s_-1 before
    x_0), pre (K,) = P(s_-1 = k | x), mom (K, 7) = per state sum gamma, then
    over tremor steps sum gamma, gamma x, gamma y, gamma x^2, gamma x y, gamma y^2."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    p, pp = _f64(p)
    mu, mup = _f64(mu)
    Sigma, sp = _f64(Sigma)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    K, T = delta.shape[0], flag.shape[0]
    gamma = np.empty((max(T, 1), K))
    xi = np.empty((K, K))
    pre = np.empty(K)
    mom = np.empty((K, 7))
    P = ctypes.POINTER(ctypes.c_double)
    ll = lib().oracle_posterior(K, dp_, gp, pp, mup, sp, T, fp, xp, gamma.ctypes.data_as(P),
                                xi.ctypes.data_as(P), pre.ctypes.data_as(P), mom.ctypes.data_as(P))
    return dict(loglik=ll, gamma=gamma[:T], xi=xi, pre=pre, mom=mom)


def viterbi(delta, Gamma, p, mu, Sigma, flag, xy):
    """Most likely hidden path: (score = max ln P(path, x), path int32 (T,), s_-1)."""
    delta, dp_ = _f64(delta)
    Gamma, gp = _f64(Gamma)
    p, pp = _f64(p)
    mu, mup = _f64(mu)
    Sigma, sp = _f64(Sigma)
    flag, fp = _u8(flag)
    xy, xp = _f64(np.asarray(xy).reshape(-1, 2))
    K, T = delta.shape[0], flag.shape[0]
    path = np.empty(max(T, 1), dtype=np.int32)
    first = ctypes.c_int32()
    score = lib().oracle_viterbi(K, dp_, gp, pp, mup, sp, T, fp, xp,
                                 path.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(first))
    return score, path[:T], first.value


def grad_from_stats(delta, Gamma, p, mu, Sigma, xi, pre, mom):
    """Gradient of ln L with respect to (delta, Gamma, p, mu, Sigma), every entry
    a free variable (Sigma as its three entries Sxx, Sxy, Syy), from the
    posterior expectations (Fisher's identity: grad ln L = E[grad ln P(s, x) | x]):
      d/d delta_i    = pre_i / delta_i
      d/d Gamma_ij   = xi_ij / Gamma_ij
      d/d p_k        = n1_k / p_k - (n_k - n1_k) / (1 - p_k)
      d/d mu_k       = Sigma_k^-1 (s_k - n1_k mu_k)
      d/d Sigma_k    = G = (1/2) Sigma^-1 (C_k - n1_k Sigma) Sigma^-1 as a matrix,
                       C_k = sum gamma f (x - mu)(x - mu)^T; Sxy enters twice: 2 G_xy
    with n_k = sum gamma, n1_k = sum over tremor steps, s_k = sum gamma f x."""
    delta = np.asarray(delta, dtype=np.float64)
    Gamma = np.asarray(Gamma, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, 2)
    Sigma = np.asarray(Sigma, dtype=np.float64).reshape(-1, 3)
    K = delta.shape[0]
    g_delta = pre / delta
    g_Gamma = xi / Gamma
    n, n1 = mom[:, 0], mom[:, 1]
    g_p = n1 / p - (n - n1) / (1.0 - p)
    g_mu = np.empty((K, 2))
    g_S = np.empty((K, 3))
    for k in range(K):
        S = np.array([[Sigma[k, 0], Sigma[k, 1]], [Sigma[k, 1], Sigma[k, 2]]])
        Si = np.linalg.inv(S)
        s = mom[k, 2:4]
        m = mu[k]
        g_mu[k] = Si @ (s - n1[k] * m)
        M2 = np.array([[mom[k, 4], mom[k, 5]], [mom[k, 5], mom[k, 6]]])
        C = M2 - np.outer(s, m) - np.outer(m, s) + n1[k] * np.outer(m, m)
        G = 0.5 * Si @ (C - n1[k] * S) @ Si
        g_S[k] = (G[0, 0], 2.0 * G[0, 1], G[1, 1])
    return dict(delta=g_delta, Gamma=g_Gamma, p=g_p, mu=g_mu, Sigma=g_S)


def em_mstep(xi, pre, mom, prev=None):
    """Maximisation step of EM (Baum-Welch) for eq. (2)'s model from the
    posterior expectations of `posterior`: the complete-data maximum
    likelihood with counts replaced by their expectations,
      delta_i   = P(s_-1 = i | x)
      Gamma_ij  = xi_ij / sum_j xi_ij
      p_k       = n1_k / n_k            (expected tremor rate of state k)
      mu_k      = s_k / n1_k            (weighted mean of its tremor locations)
      Sigma_k   = S2_k / n1_k - mu_k mu_k^T  (weighted covariance)
    with n_k = sum_t gamma_t,k, n1_k, s_k, S2_k the sums over tremor steps of
    gamma, gamma x and gamma x x^T.  An expected count of exactly zero leaves
    its quotient undefined; with `prev` = (delta, Gamma, p, mu, Sigma) such
    entries keep their previous value (a Gamma row never left, n_k = 0 for
    p_k, n1_k = 0 for mu_k and Sigma_k), without it they are NaN.
    Returns (delta, Gamma, p, mu, Sigma)."""
    xi = np.asarray(xi, dtype=np.float64)
    pre = np.asarray(pre, dtype=np.float64)
    mom = np.asarray(mom, dtype=np.float64)
    K = pre.shape[0]
    n, n1 = mom[:, 0], mom[:, 1]
    rows = xi.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        delta = pre / pre.sum()
        Gamma = xi / rows[:, None]
        p = n1 / n
        mu = mom[:, 2:4] / n1[:, None]
        Sigma = np.empty((K, 3))
        Sigma[:, 0] = mom[:, 4] / n1 - mu[:, 0] ** 2
        Sigma[:, 1] = mom[:, 5] / n1 - mu[:, 0] * mu[:, 1]
        Sigma[:, 2] = mom[:, 6] / n1 - mu[:, 1] ** 2
    if prev is not None:
        d0, G0, p0, mu0, S0 = (np.asarray(a, dtype=np.float64) for a in prev)
        if pre.sum() == 0.0:
            delta = d0.reshape(K).copy()
        G0 = G0.reshape(K, K)
        for k in range(K):
            if rows[k] == 0.0:
                Gamma[k] = G0[k]
            if n[k] == 0.0:
                p[k] = p0.reshape(K)[k]
            if n1[k] == 0.0:
                mu[k] = mu0.reshape(K, 2)[k]
                Sigma[k] = S0.reshape(K, 3)[k]
    return delta, Gamma, p, mu, Sigma
