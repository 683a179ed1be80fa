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
