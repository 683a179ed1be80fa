"""Brute-force likelihood by enumerating every hidden path (tiny K and T only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

eq. (2) expanded as a sum over paths.  With s_{-1} the state before the first
observation (eq. 2 applies Gamma before P(x_0)):
    L = sum over (s_{-1}, s_0, ..., s_{T-1}) of
        delta_{s_{-1}} * prod_t Gamma_{s_{t-1}, s_t} * e_{t, s_t}
There are K^(T+1) paths.  With ``fractions.Fraction`` inputs the sum is exact.
"""
import itertools
import math
from fractions import Fraction


def likelihood(delta, Gamma, E):
    """Exact (if inputs are Fractions) L for E[t][k] = e_{t,k}."""
    K = len(delta)
    T = len(E)
    total = 0 * delta[0]
    for path in itertools.product(range(K), repeat=T + 1):
        w = delta[path[0]]
        for t in range(T):
            w = w * Gamma[path[t]][path[t + 1]] * E[t][path[t + 1]]
        total = total + w
    return total


def log_fraction(x):
    """ln of a positive Fraction without converting through float (no underflow)."""
    x = Fraction(x)
    if x <= 0:
        return -math.inf
    return math.log(x.numerator) - math.log(x.denominator)
