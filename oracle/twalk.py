"""The t-walk (Christen & Fox, "A general purpose sampling algorithm for
continuous distributions (the t-walk)", Bayesian Analysis 5(2), 2010), the
general-purpose sampler the paper runs over its HMM posterior (section
"GPUeR-hmmer"), plain FP64 (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The t-walk runs two points (x, x') with target pi(x) pi(x').  Each iteration
moves one of them, h, with the other point b fixed, by one of four kernels,
only on a random subset phi of the n coordinates (each coordinate
independently with probability min(n, n1)/n), and accepts with
    A = pi(y) / pi(h) * (Hastings factor of the kernel).
Coordinates outside phi keep their value; an empty phi (or a zero scale for
blow and hop) leaves the state unchanged and counts as a rejection.  A blow or
hop proposal y with a zero reverse scale (y_j = b_j on all of phi) cannot
move back, so its factor is 0 (log -inf) and it is rejected.
  traverse: beta from g_t(beta) prop. to beta^a_t on (0, 1] and beta^-a_t
      above 1 (beta = u^(1/(a_t+1)) with probability (a_t-1)/(2 a_t), else
      u^(1/(1-a_t))), y_j = b_j + beta (b_j - h_j).  The map
      (h_phi, beta) -> (y_phi, 1/beta) has Jacobian beta^n_phi / beta^2 and
      g_t(1/beta) = g_t(beta), so the factor is beta^(n_phi - 2).
  walk: z_j = a_w/(1+a_w) (-1 + 2u_j + a_w u_j^2) (density prop. to
      1/sqrt(1+z) on [-a_w/(1+a_w), a_w]), y_j = h_j + (h_j - b_j) z_j; the
      reverse move has z' = -z/(1+z) and the same density, so the factor is 1.
  blow: s(u) = max_phi |u_j - b_j|, y_j = b_j + s(h) N(0, 1);
      factor g(h | y) / g(y | h), g(v | u) = prod_phi N(v_j; b_j, s(u)^2).
  hop: s(u) = max_phi |u_j - b_j| / 3, y_j = h_j + s(h) N(0, 1);
      factor g(h | y) / g(y | h), g(v | u) = prod_phi N(v_j; u_j, s(u)^2).
Tuning (Christen & Fox's defaults): kernel probabilities traverse 0.4918,
walk 0.4918, blow 0.0082, hop the rest; a_t = 6, a_w = 1.5, n1 = 4.

The random numbers of one iteration are a `Draws` record, so that the same
steps run on the library's Philox streams (`philox_draws`) or, in the
oracle's own statistical pins, on any other generator:
  uh, uk    which point moves (x when uh < 1/2) and which kernel (uk)
  u_phi[n]  subset uniforms
  u_t[2]    traverse: the branch and the beta uniform
  u_w[n]    walk uniforms
  z[n]      blow / hop normals
  u_acc     the acceptance uniform
Philox streams (see philox.py), counter (index, chain, iteration, purpose):
  purpose 7: (uh, uk) = the uniform pair of index 0
  purpose 8: u_phi, coordinate j = element j % 2 of the pair of index j // 2
  purpose 9: u_w as u_phi; u_t = the pair of index 0; z = Box-Muller normals,
             coordinate j = element j % 2 of the pair of index j // 2
  purpose 3: u_acc = the first uniform of index 0 (as for Metropolis-Hastings).
"""
import math
from dataclasses import dataclass

import numpy as np

from . import philox

CHOICE, SUBSET, VARIATE = 7, 8, 9
TRAVERSE, WALK, BLOW, HOP = 0, 1, 2, 3
NAMES = ("traverse", "walk", "blow", "hop")
# (p_traverse, p_walk, p_blow, a_t, a_w, n1); hop takes 1 - p_traverse - p_walk - p_blow
DEFAULT = (0.4918, 0.4918, 0.0082, 6.0, 1.5, 4.0)


@dataclass
class Draws:
    uh: float
    uk: float
    u_phi: np.ndarray
    u_t: tuple
    u_w: np.ndarray
    z: np.ndarray
    u_acc: float


def _pairs(fn, n):
    out = []
    for i in range((n + 1) // 2):
        out.extend(fn(i))
    return np.array(out[:n], dtype=np.float64)


def philox_draws(seed, it, chain, n):
    """The draws of iteration `it` of chain `chain` from the Philox streams."""
    uh, uk = philox.uniform2(seed, CHOICE, it, chain, 0)
    return Draws(
        uh=uh, uk=uk,
        u_phi=_pairs(lambda i: philox.uniform2(seed, SUBSET, it, chain, i), n),
        u_t=philox.uniform2(seed, VARIATE, it, chain, 0),
        u_w=_pairs(lambda i: philox.uniform2(seed, VARIATE, it, chain, i), n),
        z=_pairs(lambda i: philox.normal2(seed, VARIATE, it, chain, i), n),
        u_acc=philox.uniform2(seed, philox.ACCEPT, it, chain, 0)[0])


def kernel_of(uk, tw=DEFAULT):
    if uk < tw[0]:
        return TRAVERSE
    if uk < tw[0] + tw[1]:
        return WALK
    if uk < tw[0] + tw[1] + tw[2]:
        return BLOW
    return HOP


def _log_normal_kernel(v, m, s):
    """sum_j ln N(v_j; m_j, s^2) without the 2 pi constant (it cancels)."""
    return -v.shape[0] * math.log(s) - float(np.sum((v - m) ** 2)) / (2.0 * s * s)


def propose(h, b, dr, tw=DEFAULT):
    """(kernel, y, log Hastings factor, moved) for moving h with b fixed."""
    h = np.asarray(h, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = h.shape[0]
    a_t, a_w, n1 = tw[3], tw[4], tw[5]
    kind = kernel_of(dr.uk, tw)
    phi = dr.u_phi < min(n, n1) / n
    nphi = int(phi.sum())
    y = h.copy()
    if nphi == 0:
        return kind, y, 0.0, False
    if kind == TRAVERSE:
        u1, u2 = dr.u_t
        if u1 < (a_t - 1.0) / (2.0 * a_t):
            beta = u2 ** (1.0 / (a_t + 1.0))
        else:
            beta = u2 ** (1.0 / (1.0 - a_t))
        y[phi] = b[phi] + beta * (b[phi] - h[phi])
        return kind, y, (nphi - 2) * math.log(beta), True
    if kind == WALK:
        u = dr.u_w
        z = a_w / (1.0 + a_w) * (-1.0 + 2.0 * u + a_w * u * u)
        y[phi] = h[phi] + (h[phi] - b[phi]) * z[phi]
        return kind, y, 0.0, True
    hp, bp, zp = h[phi], b[phi], dr.z[phi]
    shrink = 1.0 if kind == BLOW else 1.0 / 3.0
    s_fwd = shrink * float(np.max(np.abs(hp - bp)))
    if not s_fwd > 0.0:
        return kind, y, 0.0, False
    if kind == BLOW:
        yp = bp + s_fwd * zp
        s_rev = shrink * float(np.max(np.abs(yp - bp)))
        lg_fwd = _log_normal_kernel(yp, bp, s_fwd)
        lg_rev = _log_normal_kernel(hp, bp, s_rev) if s_rev > 0.0 else -math.inf
    else:
        yp = hp + s_fwd * zp
        s_rev = shrink * float(np.max(np.abs(yp - bp)))
        lg_fwd = _log_normal_kernel(yp, hp, s_fwd)
        lg_rev = _log_normal_kernel(hp, yp, s_rev) if s_rev > 0.0 else -math.inf
    y[phi] = yp
    return kind, y, lg_rev - lg_fwd, True


def step(x, xp, lpost_x, lpost_xp, logpost, dr, tw=DEFAULT):
    """One t-walk iteration.  logpost: point -> log target.  Returns the new
    (x, xp, lpost_x, lpost_xp) and a dict describing the move."""
    move_x = dr.uh < 0.5
    h, b, lh = (x, xp, lpost_x) if move_x else (xp, x, lpost_xp)
    kind, y, lcorr, moved = propose(h, b, dr, tw)
    info = dict(kind=kind, move_x=move_x, y=y, moved=moved, log_factor=lcorr,
                log_ratio=None, accept=False)
    if not moved:
        return x, xp, lpost_x, lpost_xp, info
    ly = logpost(y)
    la = ly - lh + lcorr
    acc = bool(math.log(dr.u_acc) < la)
    info.update(log_ratio=la, log_u=math.log(dr.u_acc), accept=acc, logpost_y=ly)
    if acc:
        if move_x:
            x, lpost_x = y, ly
        else:
            xp, lpost_xp = y, ly
    return x, xp, lpost_x, lpost_xp, info


def hmm_logpost(K, flag, xy, box):
    """theta -> ln L + ln prior of the tremor HMM (the target of the sampler)."""
    from . import mcmc as _mcmc

    def f(theta):
        lp = _mcmc.log_prior(K, theta, box)
        return _mcmc.loglik(K, theta, flag, xy) + lp
    return f
