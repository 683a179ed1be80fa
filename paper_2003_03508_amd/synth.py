"""Seeded synthetic tremor-HMM workloads.

This module only draws random inputs; it contains none of the likelihood
arithmetic, so both the GPU library's tests and the CPU oracle can be fed from
it.  It stands in for the paper's Shikoku tremor catalogue (105,000 hourly
points, section "Tremor dataset of the Shikoku region") and for the simulator
the paper used to make synthetic data (section "OpenCL algorithm vs Forward
algorithm"), neither of which is available: hourly binary tremor occurrence
plus a 2-D location in km, generated from the HMM of the paper's model
section.

Recipe (one parameter set, ``numpy.random.default_rng(seed)``, draws in this
order):
  1. Gamma rows ~ Dirichlet(alpha), alpha = 1 off the diagonal, 50 on it.
  2. delta = uniform 1/K (not drawn).
  3. p_k ~ U(0.05, 0.9).
  4. mu_k ~ U([0, 200]^2) km.
  5. sigma_k ~ U(5, 30)^2 km (x then y), Sigma_k = diag(sigma_x^2, sigma_y^2),
     stored as (Sxx, Sxy, Syy) with Sxy = 0.
  6. s_{-1} ~ delta, then s_t ~ Gamma[s_{t-1}, :] for t = 0..T-1 (the state
     before the first observation, as eq. (2) applies Gamma before P(x_0)).
  7. f_t ~ Bernoulli(p_{s_t}); x_t ~ N(mu_{s_t}, Sigma_{s_t}) if f_t = 1,
     else (NaN, NaN).
Uniforms for steps 6-7 are drawn as whole arrays (u_state[T+1], u_flag[T],
z[T, 2]) before the path is walked.
"""
import bisect
import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_WALK_SRC = os.path.join(_HERE, "synth_walk.c")
_WALK_LIB = os.path.join(_HERE, "libsynth_walk.so")
_walk = None


def build_walker():
    """Compile the C path walker (gcc); the generator uses it when present."""
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", _WALK_LIB + ".tmp", _WALK_SRC], check=True)
    os.replace(_WALK_LIB + ".tmp", _WALK_LIB)


def _walker():
    global _walk
    if _walk is None:
        if not os.path.exists(_WALK_LIB) or os.path.getmtime(_WALK_LIB) < os.path.getmtime(_WALK_SRC):
            try:
                build_walker()
            except (OSError, subprocess.CalledProcessError):
                _walk = False
                return _walk
        lib = ctypes.CDLL(_WALK_LIB)
        lib.synth_walk.restype = None
        lib.synth_walk.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p]
        _walk = lib
    return _walk


def _walk_path(rows, s0, u):
    """state_t = bisect_right(rows[state_{t-1}], u[t]) clamped to K-1."""
    K, T = len(rows), u.shape[0]
    out = np.empty(T, dtype=np.int32)
    lib = _walker()
    if lib:
        cum = np.ascontiguousarray(np.array(rows, dtype=np.float64))
        u = np.ascontiguousarray(u, dtype=np.float64)
        lib.synth_walk(K, cum.ctypes.data, int(s0), T, u.ctypes.data, out.ctypes.data)
        return out
    s = s0
    us = u.tolist()
    for t in range(T):
        s = bisect.bisect_right(rows[s], us[t])
        if s >= K:
            s = K - 1
        out[t] = s
    return out


@dataclass
class HMMParams:
    delta: np.ndarray   # (K,)
    Gamma: np.ndarray   # (K, K) row-stochastic
    p: np.ndarray       # (K,)
    mu: np.ndarray      # (K, 2)
    Sigma: np.ndarray   # (K, 3) as (Sxx, Sxy, Syy)

    @property
    def K(self):
        return int(self.delta.shape[0])

    def packed(self):
        """delta | Gamma (row-major) | p | mu | Sigma as one float64 vector."""
        return np.concatenate([self.delta.ravel(), self.Gamma.ravel(), self.p.ravel(),
                               self.mu.ravel(), self.Sigma.ravel()]).astype(np.float64)


@dataclass
class Observations:
    flag: np.ndarray    # (T,) uint8, 1 = tremor
    xy: np.ndarray      # (T, 2) float64, NaN where flag = 0
    states: np.ndarray = field(default=None)  # (T,) hidden states (for diagnostics)

    @property
    def T(self):
        return int(self.flag.shape[0])

    def digest(self):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.flag).tobytes())
        h.update(np.ascontiguousarray(self.xy).tobytes())
        return h.hexdigest()


def draw_params(rng, K, diag_alpha=50.0, off_alpha=1.0):
    alpha = np.full((K, K), off_alpha)
    np.fill_diagonal(alpha, diag_alpha)
    Gamma = np.stack([rng.dirichlet(alpha[i]) for i in range(K)])
    delta = np.full(K, 1.0 / K)
    p = rng.uniform(0.05, 0.9, size=K)
    mu = rng.uniform(0.0, 200.0, size=(K, 2))
    sig = rng.uniform(5.0, 30.0, size=(K, 2))
    Sigma = np.stack([sig[:, 0] ** 2, np.zeros(K), sig[:, 1] ** 2], axis=1)
    return HMMParams(delta, Gamma, p, mu, Sigma)


def sample_path(rng, prm, T):
    K = prm.K
    u_state = rng.random(T + 1)
    u_flag = rng.random(T)
    z = rng.standard_normal((T, 2))
    cum_delta = np.cumsum(prm.delta)
    cum_delta[-1] = 1.0
    rows = []
    for i in range(K):
        c = np.cumsum(prm.Gamma[i])
        c[-1] = 1.0
        rows.append(c.tolist())
    s = min(bisect.bisect_right(cum_delta.tolist(), u_state[0]), K - 1)
    states = _walk_path(rows, s, u_state[1:])
    flag = (u_flag < prm.p[states]).astype(np.uint8)
    sd = np.sqrt(np.stack([prm.Sigma[:, 0], prm.Sigma[:, 2]], axis=1))
    xy = prm.mu[states] + sd[states] * z
    xy[flag == 0] = np.nan
    return Observations(flag, np.ascontiguousarray(xy), states)


def make(K, T, seed):
    """One parameter set and one path with the recipe above."""
    rng = np.random.default_rng(seed)
    prm = draw_params(rng, K)
    obs = sample_path(rng, prm, T)
    return prm, obs


@dataclass
class KindSet:
    """An HMM with a non-tremor emission model: kind 1 Poisson counts
    (e0 = lambda, obs = int32 counts), kind 2 1-D Gaussian (e0 = mu, e1 = var,
    obs = float64 values)."""
    kind: int
    delta: np.ndarray
    Gamma: np.ndarray
    e0: np.ndarray
    e1: np.ndarray
    obs: np.ndarray
    states: np.ndarray = field(default=None)

    @property
    def K(self):
        return int(self.delta.shape[0])

    @property
    def T(self):
        return int(self.obs.shape[0])


def make_kind(kind, K, T, seed):
    """Synthetic HMM of another emission family, same transition recipe.

    ``numpy.random.default_rng(seed)``, draws in this order: Gamma rows ~
    Dirichlet(1 off the diagonal, 50 on it); delta = 1/K; kind 1: lambda_k ~
    U(0.5, 20); kind 2: mu_k ~ U(0, 100), sd_k ~ U(1, 10); the path as in
    ``sample_path`` (state uniforms for s_-1..s_{T-1}); then the observations:
    counts ~ Poisson(lambda_s) (kind 1) or x = mu_s + sd_s z (kind 2)."""
    rng = np.random.default_rng(seed)
    alpha = np.full((K, K), 1.0)
    np.fill_diagonal(alpha, 50.0)
    Gamma = np.stack([rng.dirichlet(alpha[i]) for i in range(K)])
    delta = np.full(K, 1.0 / K)
    if kind == 1:
        e0 = rng.uniform(0.5, 20.0, size=K)
        e1 = np.zeros(K)
    elif kind == 2:
        e0 = rng.uniform(0.0, 100.0, size=K)
        e1 = rng.uniform(1.0, 10.0, size=K) ** 2
    else:
        raise ValueError("kind must be 1 (Poisson) or 2 (1-D Gaussian)")
    u_state = rng.random(T + 1)
    rows = []
    for i in range(K):
        c = np.cumsum(Gamma[i])
        c[-1] = 1.0
        rows.append(c.tolist())
    cum_delta = np.cumsum(delta)
    cum_delta[-1] = 1.0
    s0 = min(bisect.bisect_right(cum_delta.tolist(), u_state[0]), K - 1)
    states = _walk_path(rows, s0, u_state[1:])
    if kind == 1:
        obs = rng.poisson(e0[states]).astype(np.int32)
    else:
        obs = e0[states] + np.sqrt(e1[states]) * rng.standard_normal(T)
    return KindSet(kind, delta, Gamma, e0, e1, np.ascontiguousarray(obs), states)


# Workloads with the shapes the paper's method is benchmarked on.
WORKLOADS = {
    "k3_t1e4": dict(K=3, T=10_000, seed=0),
    "k25_t1e6": dict(K=25, T=1_000_000, seed=1),
    "k80_t4m": dict(K=80, T=4_194_304, seed=2),
    "k20_t5e5": dict(K=20, T=500_000, seed=4),
    "k25_t105k": dict(K=25, T=105_000, seed=6),   # the size of the paper's Shikoku record
}


def batch(n=256, K_lo=8, K_hi=64, T_lo=100_000, T_hi=1_000_000, seed=3, T_scale=1.0):
    """n independent sets, K ~ U{K_lo..K_hi}, T ~ U[T_lo, T_hi] (times T_scale),
    each drawn by ``make`` with its own seed.  Draw order: from
    default_rng(seed): K[n], T[n], per-set seeds[n].  Returns (packed arrays,
    list of (params, observations))."""
    rng = np.random.default_rng(seed)
    Ks = rng.integers(K_lo, K_hi + 1, size=n)
    Ts = (rng.integers(T_lo, T_hi + 1, size=n) * T_scale).astype(np.int64)
    seeds = rng.integers(0, 2**62, size=n)
    sets = [make(int(Ks[i]), int(Ts[i]), int(seeds[i])) for i in range(n)]
    return pack(sets), sets


def pack_digest(packed):
    """sha256 of a packed batch (descriptors, parameter blocks, observations)."""
    h = hashlib.sha256()
    for key in ("K", "T", "param_off", "obs_off", "params", "flag", "xy"):
        h.update(np.ascontiguousarray(packed[key]).tobytes())
    return h.hexdigest()


def pack(sets):
    """Pack (params, obs) pairs: returns dict of K, T, param_off, params, obs_off, flag, xy."""
    Ks = np.array([prm.K for prm, _ in sets], dtype=np.int32)
    Ts = np.array([obs.T for _, obs in sets], dtype=np.int64)
    blocks = [prm.packed() for prm, _ in sets]
    param_off = np.zeros(len(sets), dtype=np.int64)
    if len(sets) > 1:
        param_off[1:] = np.cumsum([b.shape[0] for b in blocks])[:-1]
    obs_off = np.zeros(len(sets), dtype=np.int64)
    if len(sets) > 1:
        obs_off[1:] = np.cumsum(Ts)[:-1]
    params = np.concatenate(blocks) if blocks else np.zeros(0)
    flag = np.concatenate([obs.flag for _, obs in sets]) if sets else np.zeros(0, np.uint8)
    xy = np.concatenate([obs.xy for _, obs in sets]) if sets else np.zeros((0, 2))
    return dict(K=Ks, T=Ts, param_off=param_off, params=params, obs_off=obs_off,
                flag=flag, xy=xy)
