"""Pins of the t-walk oracle (Christen & Fox 2010): each kernel's Hastings
factor against the proposal densities measured numerically from the oracle's
own move maps, invariance of Gaussian targets under each kernel mixture, and
the posterior of the one-state tremor HMM against quadrature."""
import math

import numpy as np
import pytest

from oracle import twalk
from paper_2003_03508_amd import mcmc as hm

from test_mcmc_oracle import _check_k1_means, _k1_problem


def _draws(rng, n):
    return twalk.Draws(uh=rng.random(), uk=rng.random(), u_phi=rng.random(n), u_t=(rng.random(), rng.random()),
                       u_w=rng.random(n), z=rng.normal(size=n), u_acc=rng.random())


def _forced(dr, kind, tw=twalk.DEFAULT, n=None):
    """The same draws with the kernel choice forced to `kind` and every
    coordinate in the subset."""
    lo = (0.0, tw[0], tw[0] + tw[1], tw[0] + tw[1] + tw[2], 1.0)
    dr.uk = 0.5 * (lo[kind] + lo[kind + 1])
    dr.u_phi = np.zeros_like(dr.u_phi)
    return dr


# --------------------------------------------------------------------------- Hastings factors
def _traverse_beta(h, b, u1, u2):
    dr = twalk.Draws(uh=0.0, uk=0.0, u_phi=np.zeros(h.shape[0]), u_t=(u1, u2), u_w=None, z=None, u_acc=0.5)
    _, y, _, _ = twalk.propose(h, b, dr)
    return float((y[0] - b[0]) / (b[0] - h[0]))


def _traverse_density(beta, h, b):
    """Density of beta under the oracle's traverse sampler, measured from its
    map: the branch threshold on u1 by bisection, then 1/|d beta/d u2| by a
    central difference at the u2 that gives beta (also by bisection)."""
    lo, hi = 1e-12, 1 - 1e-12
    for _ in range(80):           # largest u1 that still gives beta < 1
        mid = 0.5 * (lo + hi)
        if _traverse_beta(h, b, mid, 0.5) < 1.0:
            lo = mid
        else:
            hi = mid
    p_small = lo
    u1 = 0.5 * p_small if beta < 1.0 else 0.5 * (1.0 + p_small)
    prob = p_small if beta < 1.0 else 1.0 - p_small
    f = lambda u2: _traverse_beta(h, b, u1, u2)
    a, c = 1e-15, 1 - 1e-15
    inc = f(0.9) > f(0.1)
    for _ in range(200):
        m = 0.5 * (a + c)
        if (f(m) < beta) == inc:
            a = m
        else:
            c = m
    u = 0.5 * (a + c)
    eps = 1e-7 * max(u, 1e-3)
    dbdu = (f(u + eps) - f(u - eps)) / (2 * eps)
    return prob / abs(dbdu)


@pytest.mark.parametrize("n,seed", [(3, 0), (7, 1), (12, 2)])
def test_traverse_factor_is_jacobian_times_density_ratio(n, seed):
    """Reversible-jump form of the traverse ratio: the map (h, beta) ->
    (y, beta') with y = b + beta (b - h) has the inverse beta' = 1/beta;
    factor = g(beta') / g(beta) * |det d(y, beta')/d(h, beta)|, the
    determinant by finite differences and g measured from the sampler."""
    rng = np.random.default_rng(seed)
    h, b = rng.normal(size=n), rng.normal(size=n)
    for u1, u2 in ((0.2, 0.3), (0.9, 0.6), (0.05, 0.97), (0.7, 0.02)):
        dr = twalk.Draws(uh=0.0, uk=0.0, u_phi=np.zeros(n), u_t=(u1, u2), u_w=None, z=None, u_acc=0.5)
        kind, y, lf, moved = twalk.propose(h, b, dr)
        assert kind == twalk.TRAVERSE and moved
        beta = float((y[0] - b[0]) / (b[0] - h[0]))
        # inverse: moving y with b fixed by 1/beta returns h
        assert np.allclose(b + (1 / beta) * (b - y), h, atol=1e-12)

        def psi(v):
            hh, bb = v[:n], v[n]
            return np.concatenate([b + bb * (b - hh), [1.0 / bb]])
        v0 = np.concatenate([h, [beta]])
        J = np.empty((n + 1, n + 1))
        for j in range(n + 1):
            e = np.zeros(n + 1)
            e[j] = 1e-6 * max(1.0, abs(v0[j]))
            J[:, j] = (psi(v0 + e) - psi(v0 - e)) / (2 * e[j])
        logdet = np.linalg.slogdet(J)[1]
        g_fwd = _traverse_density(beta, h, b)
        g_rev = _traverse_density(1.0 / beta, h, b)
        want = math.log(g_rev) - math.log(g_fwd) + logdet
        assert abs(lf - want) < 1e-4 * max(1.0, abs(want)), (u1, u2, lf, want)


def _walk_z(u):
    n = 1
    h, b = np.array([1.0]), np.array([0.0])
    dr = twalk.Draws(uh=0.0, uk=0.6, u_phi=np.zeros(n), u_t=None, u_w=np.array([u]), z=None, u_acc=0.5)
    _, y, _, _ = twalk.propose(h, b, dr)
    return float(y[0] - 1.0)              # (y - h) / (h - b) with h - b = 1


def _walk_density(z):
    """Density of the walk's z from its map: bisection for u, then
    1/|dz/du| by a central difference; zero outside the map's range."""
    zlo, zhi = _walk_z(1e-15), _walk_z(1 - 1e-15)
    if not zlo <= z <= zhi:
        return 0.0
    a, c = 1e-15, 1 - 1e-15
    for _ in range(200):
        m = 0.5 * (a + c)
        if _walk_z(m) < z:
            a = m
        else:
            c = m
    u = min(max(0.5 * (a + c), 1e-6), 1 - 1e-6)
    return 1e-6 * 2 / abs(_walk_z(u + 1e-6) - _walk_z(u - 1e-6))


@pytest.mark.parametrize("seed", [0, 1])
def test_walk_is_symmetric(seed):
    """q(y | h) = prod g(z_j) / |h_j - b_j| equals q(h | y) with the reverse
    z'_j = (h_j - y_j) / (y_j - b_j); the oracle's factor is 0."""
    rng = np.random.default_rng(seed)
    n = 6
    for _ in range(4):
        h, b = rng.normal(size=n), rng.normal(size=n)
        dr = _forced(_draws(rng, n), twalk.WALK)
        kind, y, lf, moved = twalk.propose(h, b, dr)
        assert kind == twalk.WALK and moved and lf == 0.0
        z = (y - h) / (h - b)
        zr = (h - y) / (y - b)
        lq_f = sum(math.log(_walk_density(v)) for v in z) - np.log(np.abs(h - b)).sum()
        lq_r = sum(math.log(_walk_density(v)) for v in zr) - np.log(np.abs(y - b)).sum()
        assert abs(lq_r - lq_f) < 1e-5, (lq_r, lq_f)


@pytest.mark.parametrize("kind", [twalk.BLOW, twalk.HOP])
def test_blow_and_hop_factors_match_measured_gaussian_densities(kind):
    """The move is Gaussian in the subset coordinates: its centre and scale
    are read off the oracle's own outputs for two different normal vectors,
    in both directions, and the factor is ln q(h | y) - ln q(y | h)."""
    rng = np.random.default_rng(4 + kind)
    n = 9
    for _ in range(5):
        h, b = rng.normal(size=n), 3 * rng.normal(size=n)
        dr = _forced(_draws(rng, n), kind)
        dr.u_phi = (rng.random(n) < 0.5).astype(float)          # 0 = in the subset
        phi = dr.u_phi < min(n, 4) / n
        if not phi.any():
            continue
        k2, y, lf, moved = twalk.propose(h, b, dr)
        assert k2 == kind and moved
        assert np.array_equal(y[~phi], h[~phi])

        def centre_scale(src):
            d1 = twalk.Draws(**{**dr.__dict__, "z": np.full(n, 0.5)})
            d2 = twalk.Draws(**{**dr.__dict__, "z": np.full(n, 1.5)})
            y1 = twalk.propose(src, b, d1)[1][phi]
            s = twalk.propose(src, b, d2)[1][phi] - y1
            assert np.allclose(s, s[0])
            return y1 - 0.5 * s, s[0]

        def logq(v, c, s):
            return float(np.sum(-0.5 * ((v - c) / s) ** 2 - math.log(s) - 0.5 * math.log(2 * math.pi)))
        c_f, s_f = centre_scale(h)
        c_r, s_r = centre_scale(y)
        # Christen & Fox's scales: the largest subset distance to b (blow),
        # a third of it (hop); centred at b (blow) or at the moving point (hop)
        shrink = 1.0 if kind == twalk.BLOW else 1.0 / 3.0
        assert abs(s_f - shrink * np.abs(h - b)[phi].max()) < 1e-12 * abs(s_f)
        assert np.allclose(c_f, b[phi] if kind == twalk.BLOW else h[phi], rtol=0, atol=1e-12)
        want = logq(h[phi], c_r, s_r) - logq(y[phi], c_f, s_f)
        assert abs(lf - want) < 1e-9 * max(1.0, abs(want)), (lf, want)


def test_empty_subset_and_zero_scale_do_not_move():
    rng = np.random.default_rng(7)
    n = 10
    h, b = rng.normal(size=n), rng.normal(size=n)
    for kind in range(4):
        dr = _forced(_draws(rng, n), kind)
        dr.u_phi = np.ones(n)                  # min(n, 4)/n = 0.4 < 1: nothing selected
        _, y, lf, moved = twalk.propose(h, b, dr)
        assert not moved and np.array_equal(y, h) and lf == 0.0
    for kind in (twalk.BLOW, twalk.HOP):       # h = b on the subset: scale 0
        dr = _forced(_draws(rng, n), kind)
        _, y, _, moved = twalk.propose(h, h.copy(), dr)
        assert not moved and np.array_equal(y, h)
    x = rng.normal(size=n)
    lp = lambda v: -0.5 * float(v @ v)
    dr = _forced(_draws(rng, n), twalk.WALK)
    dr.u_phi = np.ones(n)
    x2, xp2, _, _, info = twalk.step(x, b, lp(x), lp(b), lp, dr)
    assert not info["accept"] and x2 is x and xp2 is b


def test_kernel_choice_point_choice_and_subset_size():
    assert [twalk.kernel_of(u) for u in (0.0, 0.4917, 0.4919, 0.9835, 0.9837, 0.9917, 0.9919, 0.99999)] == \
        [0, 0, 1, 1, 2, 2, 3, 3]
    rng = np.random.default_rng(8)
    n = 40
    sel, moved_x = [], []
    x, xp = rng.normal(size=n), rng.normal(size=n)
    for _ in range(2000):
        dr = _forced(_draws(rng, n), twalk.WALK)
        dr.u_phi = rng.random(n)
        dr.u_acc = 1e-300                          # accept every finite ratio
        x2, xp2, _, _, info = twalk.step(x, xp, 0.0, 0.0, lambda v: 0.0, dr)
        moved_x.append(info["move_x"])
        sel.append(int((info["y"] != (x if info["move_x"] else xp)).sum()))
    # n1 = 4 of n coordinates on average (binomial sd 1.9 / sqrt(2000) = 0.04),
    # and either point with probability 1/2 (sd 0.011)
    assert abs(np.mean(sel) - 4.0) < 0.2, np.mean(sel)
    assert abs(np.mean(moved_x) - 0.5) < 0.05


# --------------------------------------------------------------------------- invariance
def _gauss_target(n=6, seed=3):
    r = np.random.default_rng(seed)
    A = r.normal(size=(n, n))
    S = A @ A.T / n + 0.5 * np.eye(n)
    return r.normal(size=n) * 2, S


def _run_gauss(tw, chains=4, iters=15000, burn=2000, seed=0, n=6):
    m, S = _gauss_target(n)
    P = np.linalg.inv(S)
    lp = lambda v: -0.5 * (v - m) @ P @ (v - m)
    rng = np.random.default_rng(seed)
    out, acc = [], 0
    for _ in range(chains):
        x, xp = m + rng.normal(size=n), m + rng.normal(size=n)
        lx, lxp = lp(x), lp(xp)
        tr = []
        for _ in range(iters):
            x, xp, lx, lxp, info = twalk.step(x, xp, lx, lxp, lp, _draws(rng, n), tw)
            acc += info["accept"]
            tr.append(x.copy())
        out.append(np.array(tr[burn:]))
    d = np.stack(out)
    C, N, _ = d.shape
    nb = 30
    bl = N // nb

    def zscores(v, want):
        bm = v[:, :nb * bl].reshape(C, nb, bl, n).mean(2).reshape(-1, n)
        se = bm.std(0, ddof=1) / math.sqrt(bm.shape[0])
        return (v.reshape(-1, n).mean(0) - want) / se
    return acc / (chains * iters), zscores(d, m), zscores((d - m) ** 2, np.diag(S))


@pytest.mark.parametrize("name,tw", [("traverse+walk", (0.5, 0.5, 0.0, 6.0, 1.5, 4.0)),
                                     ("blow", (0.0, 0.0, 1.0, 6.0, 1.5, 4.0)),
                                     ("hop", (0.0, 0.0, 0.0, 6.0, 1.5, 4.0)),
                                     ("default", twalk.DEFAULT)])
def test_correlated_gaussian_is_invariant(name, tw):
    """Means and variances of a correlated 6-D Gaussian within 4.5 batch-means
    standard errors (a wrong ratio, e.g. the current point's density taken
    from the other point, moves variances by 7-10)."""
    acc, zm, zv = _run_gauss(tw)
    assert 0.05 < acc < 0.8, acc
    assert np.abs(zm).max() < 4.5 and np.abs(zv).max() < 4.5, (zm, zv)


def test_k1_posterior_means():
    prm, obs, box = _k1_problem(T=60)
    th0 = hm.theta_from_params(prm.Gamma, prm.p, prm.mu, prm.Sigma)
    f = twalk.hmm_logpost(1, obs.flag, obs.xy, box)
    rng = np.random.default_rng(12)
    n = th0.shape[0]
    chains = []
    for _ in range(6):
        x = th0 + 0.05 * rng.normal(size=n)
        xp = th0 + 0.05 * rng.normal(size=n)
        lx, lxp = f(x), f(xp)
        tr = []
        for _ in range(4000):
            x, xp, lx, lxp, _ = twalk.step(x, xp, lx, lxp, f, _draws(rng, n))
            tr.append(x.copy())
        chains.append(np.array(tr[800:]))
    _check_k1_means(np.stack(chains), obs, box)


def test_philox_draws_follow_the_documented_streams():
    from oracle import philox
    seed, it, c, n = 77, 5, 3, 5
    dr = twalk.philox_draws(seed, it, c, n)
    assert (dr.uh, dr.uk) == philox.uniform2(seed, 7, it, c, 0)
    assert dr.u_phi[3] == philox.uniform2(seed, 8, it, c, 1)[1]
    assert dr.u_w[4] == philox.uniform2(seed, 9, it, c, 2)[0]
    assert tuple(dr.u_t) == philox.uniform2(seed, 9, it, c, 0)
    assert dr.z[1] == philox.normal2(seed, 9, it, c, 0)[1]
    assert dr.u_acc == philox.uniform2(seed, 3, it, c, 0)[0]
