"""Posterior-predictive simulation of the tremor HMM (section "Forecasting"),
plain FP64 Python (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For each draw d (a parameter set of the posterior sample) and a start
distribution pi_d over the state s_{-1} before the first simulated hour
(for a forecast after the data: P(s_{T-1} | x_0..x_{T-1})), H steps follow
the model of eq. (1)-(2), Gamma applied before every emission:
    s_{-1} ~ pi_d,  s_t ~ Gamma[s_{t-1}, .],  f_t ~ Bernoulli(p_{s_t}),
    x_t = mu_{s_t} + C_{s_t} z_t  when f_t = 1 (C the lower Cholesky factor of
          Sigma: C = [[sqrt(Sxx), 0], [Sxy / sqrt(Sxx), sqrt(Syy - Sxy^2 / Sxx)]]),
    x_t = (nan, nan) otherwise.
A categorical draw with weights w and uniform u takes the smallest k with
u < w_0 + ... + w_k (sums in ascending order, FP64); if rounding leaves u
above the total, the last k with w_k > 0.  A Bernoulli(p) draw is 1 when
u < p.  A categorical draw over weights that are all zero ends the draw's
path: that step and every later one get state -1, flag 0 and no location.

Random numbers (Philox, see philox.py), counter (index 0, draw, step, purpose):
    purpose 10, step t: (u_state, u_flag) of step t
    purpose 11, step t: Box-Muller normals (z0, z1) of step t
    purpose 12, step 0: (u_init, unused) for s_{-1}
Parameter blocks use the packed layout delta | Gamma | p | mu | Sigma
(delta unused here).
"""
import math

import numpy as np

from . import philox

STEP, NORMAL, INIT = 10, 11, 12


def categorical(w, u):
    c = 0.0
    last = -1
    for k, wk in enumerate(w):
        c += wk
        if wk > 0.0:
            last = k
        if u < c:
            return k
    return last


def unpack(block, K):
    b = np.asarray(block, dtype=np.float64)
    G = b[K:K + K * K].reshape(K, K)
    p = b[K + K * K:2 * K + K * K]
    mu = b[2 * K + K * K:4 * K + K * K].reshape(K, 2)
    S = b[4 * K + K * K:7 * K + K * K].reshape(K, 3)
    return G, p, mu, S


def philox_draws(seed, draw):
    """draw_fn(t) -> (u_state, u_flag, z0, z1) and u_init for one draw."""
    def step(t):
        us, uf = philox.uniform2(seed, STEP, t, draw, 0)
        z0, z1 = philox.normal2(seed, NORMAL, t, draw, 0)
        return us, uf, z0, z1
    return step, philox.uniform2(seed, INIT, 0, draw, 0)[0]


def simulate_one(block, start, K, H, step_fn, u_init):
    """(states (H,), flags (H,), xy (H, 2), s_-1) of one draw."""
    G, p, mu, S = unpack(block, K)
    s = categorical(start, u_init)
    first = s
    states = np.full(H, -1, dtype=np.int32)
    flags = np.zeros(H, dtype=np.uint8)
    xy = np.full((H, 2), np.nan)
    for t in range(H):
        if s < 0:
            break
        us, uf, z0, z1 = step_fn(t)
        s = categorical(G[s], us)
        if s < 0:
            break
        states[t] = s
        f = 1 if uf < p[s] else 0
        flags[t] = f
        if f:
            sxx, sxy, syy = S[s]
            c00 = math.sqrt(sxx)
            c10 = sxy / c00
            c11 = math.sqrt(syy - sxy * sxy / sxx)
            xy[t, 0] = mu[s, 0] + c00 * z0
            xy[t, 1] = mu[s, 1] + c10 * z0 + c11 * z1
    return states, flags, xy, first


def simulate(blocks, starts, K, H, seed):
    """All draws on the Philox streams: states (H, n), flags (H, n), xy (H, n, 2), first (n,)."""
    n = len(blocks)
    states = np.empty((H, n), dtype=np.int32)
    flags = np.empty((H, n), dtype=np.uint8)
    xy = np.empty((H, n, 2))
    first = np.empty(n, dtype=np.int32)
    for d in range(n):
        step, u0 = philox_draws(seed, d)
        st, fl, x, f0 = simulate_one(blocks[d], starts[d], K, H, step, u0)
        states[:, d], flags[:, d], xy[:, d], first[d] = st, fl, x, f0
    return states, flags, xy, first
