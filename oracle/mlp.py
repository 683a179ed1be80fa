"""The learned proposal's network and loss, plain FP64 NumPy (CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Network (two hidden layers of width H, tanh, and a per-coordinate linear
skip on the mean outputs):
    h1 = tanh(x W1 + b1),  h2 = tanh(h1 W2 + b2),  o = h2 W3 + b3,
    o[:D] += a * x
with x of length D and o of length 2D: o[:D] is the mean of the move and
o[D:] its log standard deviation, both in units of the output scale.
Weights are one flat vector in the order W1 (D x H), b1, W2 (H x H), b2,
W3 (H x 2D), b3, a (D), each W row-major with the input index first.

Loss of a minibatch of B rows (x_b, r_b), r the observed move:
    loss = (1/B) sum_b sum_d [ (r_bd - o_bd)^2 exp(-2 o_b,D+d) / 2 + o_b,D+d ]
i.e. the Gaussian negative log-likelihood of the moves up to the constant
(D/2) ln 2 pi per row.  The gradient is obtained by the chain rule, layer by
layer (reverse mode), in FP64.
"""
import numpy as np


def sizes(D, H):
    return [(D, H), (H,), (H, H), (H,), (H, 2 * D), (2 * D,), (D,)]


def count(D, H):
    return sum(int(np.prod(s)) for s in sizes(D, H))


def unpack(w, D, H):
    w = np.asarray(w, dtype=np.float64)
    out, off = [], 0
    for s in sizes(D, H):
        n = int(np.prod(s))
        out.append(w[off:off + n].reshape(s))
        off += n
    assert off == w.shape[0]
    return out


def forward(w, X, D, H):
    """Outputs (B, 2D) and the hidden activations."""
    W1, b1, W2, b2, W3, b3, a = unpack(w, D, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    O = h2 @ W3 + b3
    O[:, :D] += a * X
    return O, (h1, h2)


def loss_rows(w, X, R, D, H):
    """Per-row loss terms (each including the 1/B factor)."""
    O, _ = forward(w, X, D, H)
    R = np.asarray(R, dtype=np.float64)
    B = O.shape[0]
    m, s = O[:, :D], O[:, D:]
    e = R - m
    return np.sum(0.5 * e * e * np.exp(-2.0 * s) + s, axis=1) / B


def loss(w, X, R, D, H):
    return float(np.sum(loss_rows(w, X, R, D, H)))


def grad(w, X, R, D, H):
    """Gradient of `loss` with respect to the flat weight vector."""
    W1, b1, W2, b2, W3, b3, a = unpack(w, D, H)
    X = np.asarray(X, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    O, (h1, h2) = forward(w, X, D, H)
    B = O.shape[0]
    e = R - O[:, :D]
    q = np.exp(-2.0 * O[:, D:])
    dO = np.concatenate([-e * q, 1.0 - e * e * q], axis=1) / B
    ga = (dO[:, :D] * X).sum(axis=0)
    gW3 = h2.T @ dO
    gb3 = dO.sum(axis=0)
    dh2 = (dO @ W3.T) * (1.0 - h2 * h2)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (1.0 - h1 * h1)
    gW1 = X.T @ dh1
    gb1 = dh1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, ga)])


def move(w, theta, center, in_scale, out_scale, D, H):
    """(mean shift, log sd) of the learned move at theta, in theta units."""
    x = (np.asarray(theta, dtype=np.float64) - center) / in_scale
    o, _ = forward(w, x[None, :], D, H)
    o = o[0]
    return out_scale * o[:D], np.log(out_scale) + o[D:]
